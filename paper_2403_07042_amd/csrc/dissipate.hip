// Decoherence step, Hermitian symmetrisation and trace renormalisation.
//
// Given the rotated state Z = U rho_k U^dag (only tiles on or below the
// diagonal are valid), one step of the Lindblad term of Sec. II, Eq. 3 with
// monomial decoherence operators in gather form:
//   (A_j Z A_j^dag)[u,v] = c_j[u] c_j[v] Z[pi_j[u], pi_j[v]],
//   (A_j^dag A_j)[u,u]   = a_j[u]^2,  d[u] = sum_j gamma_j a_j[u]^2,
//   rho_d[u,v] = Z[u,v] (1 - dt (d[u] + d[v]) / 2)
//              + dt sum_j cg_j[u] cg_j[v] Z[pi_j[u], pi_j[v]]   (cg = sqrt(gamma) c).
//
// trace_kernel (one workgroup) needs only the diagonal of Z: it forms
// tr rho_d = sum_w trw[w] Z[w,w] (the jump terms regrouped by the diagonal
// element they read, weights fixed per context) and the probability leaving
// the basis in FP64, updates the sink and the renormalisation factor
// (1 - sink) / tr rho_d.  dissipate_kernel
// then writes X = scale * rho_d for u >= v and its conjugate mirror, so X is
// exactly Hermitian; all arithmetic is FP64 whatever the storage type.
#include "dissipate_tile.hpp"

namespace qme {

// 256 threads: the same reduction order as the persistent batched step
static constexpr int kTraceThreads = 256;

template <typename T>
__global__ __launch_bounds__(kTraceThreads) void trace_kernel(DissArgs<T> p) {
  __shared__ double s_tr[kTraceThreads], s_lost[kTraceThreads], s_rot[kTraceThreads];
  trace_body<T, kTraceThreads>(p, s_tr, s_lost, s_rot);
}

// FUSE: every block forms the trace sums itself (the same reduction as
// trace_kernel, so the factor is bitwise the same; its loads overlap the
// tile's own) and block 0 stores the step's scalars; otherwise the factor
// comes from the trace pass.
template <typename T, bool SPARSE, bool FUSE>
__global__ __launch_bounds__(kDissThreads) void dissipate_kernel(DissArgs<T> p) {
  __shared__ T s_re[TD][TD + 1];
  __shared__ T s_im[TD][TD + 1];
  __shared__ GatherLds g;
  __shared__ double s_t[3][kDissThreads / 64];
  dissipate_tile<T, SPARSE, FUSE>(p, blockIdx.x, [&]() {
    if constexpr (FUSE)
      return trace_body<T, kDissThreads>(p, s_t[0], s_t[1], s_t[2], blockIdx.x == 0);
    else
      return p.aux_out[4];
  }, s_re, s_im, &g);
}

__global__ void scalars_home_kernel(double *aux) {
  aux[sink_slot(0)] = aux[sink_slot(1)];
  aux[steps_slot(0)] = aux[steps_slot(1)];
}

hipError_t launch_scalars_home(double *aux, hipStream_t s) {
  return launch_kernel(scalars_home_kernel, dim3(1), dim3(1), 0, s, aux);
}

template <typename T>
__global__ void diag_kernel(const T *x_re, int64_t ld, int64_t n, double *out) {
  const int64_t u = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (u < n) out[u] = double(x_re[u * ld + u]);
}

template <typename T>
hipError_t launch_trace(const DissArgs<T> &a, hipStream_t s) {
  return launch_kernel(trace_kernel<T>, dim3(1), dim3(kTraceThreads), 0, s, a);
}

template <typename T>
hipError_t launch_dissipate(const DissArgs<T> &a, hipStream_t s) {
  const int tiles = int((a.n + TD - 1) / TD);
  const int blocks = tiles * (tiles + 1) / 2;
  const bool sparse = a.n_csr > 0 || a.koff_ptr;
  if (a.fuse_trace)
    return sparse ? launch_kernel(dissipate_kernel<T, true, true>, dim3(blocks), dim3(kDissThreads), 0, s, a)
                  : launch_kernel(dissipate_kernel<T, false, true>, dim3(blocks), dim3(kDissThreads), 0, s, a);
  return sparse ? launch_kernel(dissipate_kernel<T, true, false>, dim3(blocks), dim3(kDissThreads), 0, s, a)
                : launch_kernel(dissipate_kernel<T, false, false>, dim3(blocks), dim3(kDissThreads), 0, s, a);
}

template <typename T>
hipError_t launch_diag(const T *x_re, int64_t ld, int64_t n, double *out, hipStream_t s) {
  const int blocks = int((n + 255) / 256);
  hipLaunchKernelGGL(diag_kernel<T>, dim3(blocks), dim3(256), 0, s, x_re, ld, n, out);
  return hipGetLastError();
}

template hipError_t launch_trace<float>(const DissArgs<float> &, hipStream_t);
template hipError_t launch_trace<double>(const DissArgs<double> &, hipStream_t);
template hipError_t launch_dissipate<float>(const DissArgs<float> &, hipStream_t);
template hipError_t launch_dissipate<double>(const DissArgs<double> &, hipStream_t);
template hipError_t launch_diag<float>(const float *, int64_t, int64_t, double *, hipStream_t);
template hipError_t launch_diag<double>(const double *, int64_t, int64_t, double *, hipStream_t);

}  // namespace qme
