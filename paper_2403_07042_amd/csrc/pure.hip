// Pure-state steps of a closed model (Sec. IV.B: one photon on the plane of
// cavities without leakage).  With no decoherence operator acting on the
// basis the dissipator and the sink vanish and a pure start stays pure:
// rho_k = psi_k psi_k^dag, and the step's rotation U rho U^dag followed by
// the trace renormalisation is psi <- U psi / |psi| -- O(N^2) work per step
// instead of the two O(N^3) products.
//
// pure_step_kernel: one wavefront per row i of dU (= U - I, the context's
// propagator planes, ld x ld, zero padded) for each of NV vectors:
//   y_v[i] = (x_v[i] + sum_j dU[i][j] x_v[j]) / |x_v|.
// The row streams from HBM in 16-byte loads (coalesced: lane l of the wave
// takes columns (64 m + l) E .. + E - 1 of chunk m); x is re-read from the
// caches by every row.  Each lane accumulates its columns in the storage
// type; the wave then sums the lane partials in FP64 (butterfly) and forms
// y in FP64.  |x_v|^2 is summed in FP64 by every wave over the x elements it
// loads (all of x, in the same lane partition and order in every wave), so
// every row divides by the bitwise-same norm without any cross-workgroup
// step.  Rows and columns >= n are padding: x is read as zero there and the
// padding rows of y are written as zero.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "ctx.hpp"
#include "device.hpp"
#include "model.hpp"
#include "qme.h"

namespace qme {

static constexpr int kPureThreads = 128;   // two rows per workgroup
static constexpr int kPureLoads = 2;       // 16-byte loads per lane, row plane and pass

template <typename T>
struct alignas(16) Pack16 {
  T v[16 / sizeof(T)];
};

template <typename T>
__device__ __forceinline__ Pack16<T> load16(const T *p) {
  return *reinterpret_cast<const Pack16<T> *>(p);
}

template <typename T, int NV>
__global__ __launch_bounds__(kPureThreads) void pure_step_kernel(PureArgs<T> p) {
  constexpr int E = 16 / int(sizeof(T));
  constexpr int M = kPureLoads;
  constexpr int PASS = 64 * E * M;   // columns per pass of a wave: 512 FP32, 256 FP64
  const int lane = threadIdx.x & 63;
  const int64_t row = int64_t(blockIdx.x) * (kPureThreads / 64) + (threadIdx.x >> 6);
  if (row >= p.ld) return;
  if (row >= p.n) {
    if (lane < NV) {
      p.y_re[lane * p.ld + row] = T(0);
      p.y_im[lane * p.ld + row] = T(0);
    }
    return;
  }
  const T *ur = p.u_re + row * p.ld;
  const T *ui = p.u_im + row * p.ld;
  T acc_re[NV], acc_im[NV];
  double nrm[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    acc_re[v] = acc_im[v] = T(0);
    nrm[v] = 0.0;
  }
  for (int64_t c0 = 0; c0 < p.ld; c0 += PASS) {
    Pack16<T> a[M], b[M], xr[NV][M], xi[NV][M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int64_t col = c0 + int64_t(m * 64 + lane) * E;
      if (col < p.ld) {
        a[m] = load16(ur + col);
        b[m] = load16(ui + col);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          xr[v][m] = load16(p.x_re + v * p.ld + col);
          xi[v][m] = load16(p.x_im + v * p.ld + col);
        }
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          a[m].v[e] = b[m].v[e] = T(0);
#pragma unroll
          for (int v = 0; v < NV; ++v) xr[v][m].v[e] = xi[v][m].v[e] = T(0);
        }
      }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int64_t col = c0 + int64_t(m * 64 + lane) * E;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const bool in = col + e < p.n;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const T x_re = in ? xr[v][m].v[e] : T(0);
          const T x_im = in ? xi[v][m].v[e] : T(0);
          nrm[v] += double(x_re) * double(x_re) + double(x_im) * double(x_im);
          acc_re[v] = fma(a[m].v[e], x_re, acc_re[v]);
          acc_re[v] = fma(-b[m].v[e], x_im, acc_re[v]);
          acc_im[v] = fma(a[m].v[e], x_im, acc_im[v]);
          acc_im[v] = fma(b[m].v[e], x_re, acc_im[v]);
        }
      }
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double sr = double(acc_re[v]), si = double(acc_im[v]), sn = nrm[v];
    for (int off = 32; off > 0; off >>= 1) {
      sr += __shfl_xor(sr, off);
      si += __shfl_xor(si, off);
      sn += __shfl_xor(sn, off);
    }
    if (lane == v) {
      const double scale = 1.0 / sqrt(sn);
      const int64_t o = v * p.ld + row;
      p.y_re[o] = T(scale * (double(p.x_re[o]) + sr));
      p.y_im[o] = T(scale * (double(p.x_im[o]) + si));
    }
  }
}

template <typename T, int NV>
static hipError_t launch_nv(const PureArgs<T> &a, hipStream_t s) {
  const unsigned blocks = unsigned(a.ld / (kPureThreads / 64));
  hipLaunchKernelGGL((pure_step_kernel<T, NV>), dim3(blocks), dim3(kPureThreads), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pure_step(const PureArgs<T> &a, int nv, hipStream_t s) {
  if (a.n < 1 || a.ld < a.n || a.ld % (kPureThreads / 64) != 0 || a.ld % (16 / sizeof(T)) != 0)
    return hipErrorInvalidValue;
  switch (nv) {
    case 1: return launch_nv<T, 1>(a, s);
    case 2: return launch_nv<T, 2>(a, s);
    case 3: return launch_nv<T, 3>(a, s);
    case 4: return launch_nv<T, 4>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_pure_step<float>(const PureArgs<float> &, int, hipStream_t);
template hipError_t launch_pure_step<double>(const PureArgs<double> &, int, hipStream_t);

}  // namespace qme

using namespace qme;

#define PURE_OK(call)                                                         \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) {                                                   \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));           \
      return QME_E_DEVICE;                                                    \
    }                                                                         \
  } while (0)

namespace {

size_t pure_bytes(const qme_ctx *c, int32_t n_vec) {
  const size_t b = 2 * size_t(n_vec) * size_t(c->ld) * size_t(c->elem);
  return (b + 255) / 256 * 256;
}

// Validation shared by the pure-state calls: context, vector count and
// precision (FP32 / FP64 storage; BF16X3 contexts have no pure form).
qme_status pure_check(const qme_ctx *c, int32_t n_vec) {
  if (!c) { set_error("ctx is NULL"); return QME_E_ARG; }
  if (n_vec < 1 || n_vec > QME_PURE_MAX_VECTORS) {
    set_error("n_vec must be in [1, QME_PURE_MAX_VECTORS]");
    return QME_E_ARG;
  }
  if (c->precision == QME_BF16X3) {
    set_error("pure-state steps run in FP32 or FP64 contexts");
    return QME_E_UNSUPPORTED;
  }
  return QME_OK;
}

// No decoherence operator acts on the basis: no gather channel, and every
// rate-weighted A^dag A diagonal and leak weight is zero.
bool closed_model(const qme_ctx *c) {
  if (c->jt.n_gather != 0) return false;
  for (double x : c->jt.d)
    if (x != 0.0) return false;
  for (double x : c->jt.leak)
    if (x != 0.0) return false;
  return true;
}

template <typename T>
qme_status pure_run(qme_ctx *c, void *state, int32_t n_vec, int64_t n_steps, void *ws,
                    hipStream_t s) {
  const size_t plane = size_t(n_vec) * size_t(c->ld);
  T *a = static_cast<T *>(state), *b = static_cast<T *>(ws);
  if (n_steps % 2) {
    // odd count: start from a copy in the workspace so the last step writes the state
    PURE_OK(hipMemcpyAsync(ws, state, 2 * plane * sizeof(T), hipMemcpyDeviceToDevice, s));
    std::swap(a, b);
  }
  for (int64_t k = 0; k < n_steps; ++k) {
    PureArgs<T> args{a, a + plane, b, b + plane, static_cast<const T *>(c->du_re),
                     static_cast<const T *>(c->du_im), c->ld, c->n};
    PURE_OK(launch_pure_step<T>(args, n_vec, s));
    std::swap(a, b);
  }
  return QME_OK;
}

}  // namespace

extern "C" qme_status qme_pure_layout(const qme_ctx *c, int32_t n_vec, size_t *state_bytes,
                                      size_t *workspace_bytes) {
  set_error("");
  const qme_status st = pure_check(c, n_vec);
  if (st != QME_OK) return st;
  if (state_bytes) *state_bytes = pure_bytes(c, n_vec);
  if (workspace_bytes) *workspace_bytes = pure_bytes(c, n_vec);
  return QME_OK;
}

extern "C" qme_status qme_pure_set(const qme_ctx *c, void *state, int32_t n_vec,
                                   const double *psi_re, const double *psi_im, void *hip_stream) {
  try {
    set_error("");
    qme_status st = pure_check(c, n_vec);
    if (st != QME_OK) return st;
    if (!state || !psi_re || !psi_im) { set_error("NULL argument"); return QME_E_ARG; }
    st = check_device(c);
    if (st != QME_OK) return st;
    const size_t plane = size_t(n_vec) * size_t(c->ld);
    std::vector<char> buf(pure_bytes(c, n_vec), 0);
    for (int32_t v = 0; v < n_vec; ++v) {
      double norm = 0.0;
      for (int64_t i = 0; i < c->n; ++i) {
        const double xr = psi_re[size_t(v) * c->n + i], xi = psi_im[size_t(v) * c->n + i];
        if (!std::isfinite(xr) || !std::isfinite(xi)) { set_error("psi is not finite"); return QME_E_ARG; }
        norm += xr * xr + xi * xi;
        const size_t o = size_t(v) * c->ld + i;
        if (c->elem == 8) {
          reinterpret_cast<double *>(buf.data())[o] = xr;
          reinterpret_cast<double *>(buf.data())[plane + o] = xi;
        } else {
          reinterpret_cast<float *>(buf.data())[o] = float(xr);
          reinterpret_cast<float *>(buf.data())[plane + o] = float(xi);
        }
      }
      if (!(norm > 0.0)) { set_error("psi has a zero vector"); return QME_E_ARG; }
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    PURE_OK(hipMemcpyAsync(state, buf.data(), buf.size(), hipMemcpyHostToDevice, s));
    PURE_OK(hipStreamSynchronize(s));
    return QME_OK;
  } catch (const std::bad_alloc &) {
    set_error("out of host memory");
    return QME_E_SIZE;
  } catch (const std::exception &e) {
    set_error(std::string("internal error: ") + e.what());
    return QME_E_STATE;
  }
}

extern "C" qme_status qme_pure_get(const qme_ctx *c, const void *state, int32_t n_vec,
                                   double *psi_re, double *psi_im, void *hip_stream) {
  try {
    set_error("");
    qme_status st = pure_check(c, n_vec);
    if (st != QME_OK) return st;
    if (!state) { set_error("NULL argument"); return QME_E_ARG; }
    st = check_device(c);
    if (st != QME_OK) return st;
    const size_t plane = size_t(n_vec) * size_t(c->ld);
    std::vector<char> buf(pure_bytes(c, n_vec));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    PURE_OK(hipMemcpyAsync(buf.data(), state, buf.size(), hipMemcpyDeviceToHost, s));
    PURE_OK(hipStreamSynchronize(s));
    for (int32_t v = 0; v < n_vec; ++v)
      for (int64_t i = 0; i < c->n; ++i) {
        const size_t o = size_t(v) * c->ld + i, dst = size_t(v) * c->n + i;
        const double xr = c->elem == 8 ? reinterpret_cast<double *>(buf.data())[o]
                                       : double(reinterpret_cast<float *>(buf.data())[o]);
        const double xi = c->elem == 8 ? reinterpret_cast<double *>(buf.data())[plane + o]
                                       : double(reinterpret_cast<float *>(buf.data())[plane + o]);
        if (psi_re) psi_re[dst] = xr;
        if (psi_im) psi_im[dst] = xi;
      }
    return QME_OK;
  } catch (const std::bad_alloc &) {
    set_error("out of host memory");
    return QME_E_SIZE;
  } catch (const std::exception &e) {
    set_error(std::string("internal error: ") + e.what());
    return QME_E_STATE;
  }
}

extern "C" qme_status qme_pure_step(qme_ctx *c, void *state, int32_t n_vec, int64_t n_steps,
                                    void *ws, void *hip_stream) {
  try {
    TraceRange range("qme_pure_step");
    set_error("");
    qme_status st = pure_check(c, n_vec);
    if (st != QME_OK) return st;
    if (!state || !ws) { set_error("NULL argument"); return QME_E_ARG; }
    if (n_steps < 0) { set_error("n_steps < 0"); return QME_E_ARG; }
    if ((reinterpret_cast<uintptr_t>(state) | reinterpret_cast<uintptr_t>(ws)) & 255) {
      set_error("state and workspace must be 256-byte aligned");
      return QME_E_ARG;
    }
    if (!closed_model(c)) {
      set_error("pure-state steps need a closed model (no decoherence operator acting on the basis)");
      return QME_E_STATE;
    }
    st = check_device(c);
    if (st != QME_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    return c->elem == 8 ? pure_run<double>(c, state, n_vec, n_steps, ws, s)
                        : pure_run<float>(c, state, n_vec, n_steps, ws, s);
  } catch (const std::bad_alloc &) {
    set_error("out of host memory");
    return QME_E_SIZE;
  } catch (const std::exception &e) {
    set_error(std::string("internal error: ") + e.what());
    return QME_E_STATE;
  }
}
