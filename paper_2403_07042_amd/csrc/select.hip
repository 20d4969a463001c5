// State-space selection (Sec. III.B): move a state onto a subset of its
// basis.  The kept block P rho P is renormalised to the trace the state had
// (1 - sink), so the probability of the removed states is redistributed
// over the kept ones and the sink is carried unchanged.
//
//   select_trace_kernel  (one workgroup, FP64): tr of the kept block and of
//                        the whole state; writes the new state's scalars
//   compact_kernel       rho_to[i][j] = scale * rho_from[keep_i][keep_j],
//                        zero in the padding (rows / columns >= n_to)
//   select_decide_kernel (one workgroup): the keep/delete decision from two
//                        population vectors, the kept indices compacted in
//                        increasing order
#include "device.hpp"

namespace qme {

static constexpr int kSelThreads = 256;

template <typename T>
__global__ __launch_bounds__(kSelThreads) void select_trace_kernel(CompactArgs<T> p) {
  __shared__ double s_kept[kSelThreads], s_all[kSelThreads];
  double kept = 0.0, all = 0.0;
  for (int64_t i = threadIdx.x; i < p.n_to; i += kSelThreads) {
    const int64_t k = p.keep[i];
    kept += double(p.from_re[k * p.ld_from + k]);
  }
  for (int64_t u = threadIdx.x; u < p.n_from; u += kSelThreads)
    all += double(p.from_re[u * p.ld_from + u]);
  s_kept[threadIdx.x] = kept;
  s_all[threadIdx.x] = all;
  __syncthreads();
  for (int w = kSelThreads / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
      s_kept[threadIdx.x] += s_kept[threadIdx.x + w];
      s_all[threadIdx.x] += s_all[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double sink = p.aux_from[0];
    p.aux_to[0] = sink;
    p.aux_to[1] = s_kept[0];
    p.aux_to[2] = s_all[0] - s_kept[0];      // probability of the removed states
    p.aux_to[3] = p.aux_from[3];
    p.aux_to[4] = (1.0 - sink) / s_kept[0];
    p.aux_to[5] = p.aux_to[6] = p.aux_to[7] = 0.0;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void compact_kernel(CompactArgs<T> p) {
  const int64_t i = blockIdx.y;
  const int64_t j = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (j >= p.ld_to) return;
  const int64_t o = i * p.ld_to + j;
  T re = T(0), im = T(0);
  if (i < p.n_to && j < p.n_to) {
    const double scale = p.aux_to[4];
    const int64_t src = int64_t(p.keep[i]) * p.ld_from + p.keep[j];
    re = T(scale * double(p.from_re[src]));
    im = T(scale * double(p.from_im[src]));
  }
  p.to_re[o] = re;
  p.to_im[o] = im;
}

template <typename T>
hipError_t launch_compact(const CompactArgs<T> &a, hipStream_t s) {
  if (a.n_to < 1 || a.n_to > a.n_from || a.ld_to < a.n_to || a.ld_to > 65535)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(select_trace_kernel<T>, dim3(1), dim3(kSelThreads), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(compact_kernel<T>, dim3(unsigned((a.ld_to + 255) / 256), unsigned(a.ld_to)),
                     dim3(256), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_compact<float>(const CompactArgs<float> &, hipStream_t);
template hipError_t launch_compact<double>(const CompactArgs<double> &, hipStream_t);

// Growth speed |p_now - p_prev| / interval against eps in FP64, the same
// operations as the host decision (qme_select_states), so both keep the same
// states.  The states are taken in chunks of the workgroup's size; a chunk's
// kept states are numbered by the wave ballots and the waves' counts, after
// every state of the earlier chunks.
static constexpr int kDecideThreads = 1024;

template <typename T>
__global__ __launch_bounds__(kDecideThreads) void select_decide_kernel(DecideArgs<T> a) {
  constexpr int kWaves = kDecideThreads / 64;
  __shared__ int s_count[kWaves];
  __shared__ int s_bad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  bool bad = false;
  int64_t base = 0;                       // states kept in earlier chunks
  for (int64_t s0 = 0; s0 < a.n; s0 += kDecideThreads) {
    const int64_t s = s0 + tid;
    bool keep = false;
    if (s < a.n) {
      const double pn = double(a.re[s * a.ld + s]);
      const double pp = a.p_prev[s];
      bad = bad || !isfinite(pn) || !isfinite(pp);
      keep = fabs(pn - pp) / a.interval >= a.eps;
      a.p_now[s] = pn;
    }
    const uint64_t m = __ballot(keep);
    const int below = __popcll(m & ((uint64_t(1) << lane) - 1));
    if (lane == 0) s_count[wave] = __popcll(m);
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < kWaves; ++w) {
      const int c = s_count[w];
      before += w < wave ? c : 0;
      total += c;
    }
    if (keep) a.keep[base + before + below] = int32_t(s);
    base += total;
    __syncthreads();                      // the counts are rewritten by the next chunk
  }
  if (bad) s_bad = 1;
  __syncthreads();
  if (tid == 0) *a.n_keep = s_bad ? -1 : base;
}

template <typename T>
hipError_t launch_select_decide(const DecideArgs<T> &a, hipStream_t s) {
  if (a.n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(select_decide_kernel<T>, dim3(1), dim3(kDecideThreads), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_select_decide<float>(const DecideArgs<float> &, hipStream_t);
template hipError_t launch_select_decide<double>(const DecideArgs<double> &, hipStream_t);

}  // namespace qme
