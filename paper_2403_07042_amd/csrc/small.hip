// Whole time steps of a small system (n <= 32) in one launch of one
// workgroup: the propagator increment and the state stay in LDS for every
// step, so a step costs no kernel launches and no HBM traffic.
//
// The step is the same as the tiled path's (Sec. II, Eqs. 2-3, with the
// "unitary evolution" products of Sec. IV.B):
//   T   = rho + dU rho                (rho Hermitian: B[k][j] = conj(rho[j][k]))
//   Z   = T + T conj(dU)              on and below the diagonal
//   trace / sink / renormalisation    FP64, the same reduction tree
//   rho' = scale * Herm(Z + dt D(Z))  FP64, written in both triangles
// Products accumulate in the storage type with scalar FMAs (k ascending);
// the decoherence arithmetic is operation-for-operation that of the tiled
// decoherence pass, so only the products' rounding order differs from it.
#include "device.hpp"

#include <algorithm>

namespace qme {

constexpr int kSmallLd = kSmallN + 1;     // padded LDS row
constexpr int kSmallThreads = 256;
constexpr int kSmallGather = 16;          // channels whose tables are staged in LDS
constexpr int64_t kSmallStepsPerLaunch = 4096;

template <typename T>
__global__ __launch_bounds__(kSmallThreads) void small_steps_kernel(SmallArgs<T> p) {
  __shared__ T sU[2][kSmallN * kSmallLd];
  __shared__ T sA[2][kSmallN * kSmallLd];
  __shared__ T sB[2][kSmallN * kSmallLd];
  __shared__ double s_d[kSmallN], s_leak[kSmallN], s_trw[kSmallN];
  __shared__ int32_t s_pi[kSmallGather][kSmallN];
  __shared__ double s_cg[kSmallGather][kSmallN];
  __shared__ double s_scale;

  const int n = p.n, tid = threadIdx.x, nn = n * n;
  const int64_t ld = p.ld;
  const bool staged = p.n_gather <= kSmallGather;
  for (int e = tid; e < nn; e += kSmallThreads) {
    const int i = e / n, j = e - (e / n) * n;
    sU[0][i * kSmallLd + j] = p.u_re[i * ld + j];
    sU[1][i * kSmallLd + j] = p.u_im[i * ld + j];
    sA[0][i * kSmallLd + j] = p.re[i * ld + j];
    sA[1][i * kSmallLd + j] = p.im[i * ld + j];
  }
  for (int u = tid; u < n; u += kSmallThreads) {
    s_d[u] = p.d[u];
    s_leak[u] = p.leak[u];
    s_trw[u] = p.trw[u];
  }
  if (staged)
    for (int e = tid; e < p.n_gather * n; e += kSmallThreads) {
      const int j = e / n, u = e - (e / n) * n;
      s_pi[j][u] = p.pi[int64_t(j) * n + u];
      s_cg[j][u] = p.cg[int64_t(j) * n + u];
    }
  double sink = p.aux[0], rot = p.aux[1], lost = p.aux[2], steps = p.aux[3], scale = p.aux[4];
  __syncthreads();

  T(*rho)[kSmallN * kSmallLd] = sA;
  T(*tb)[kSmallN * kSmallLd] = sB;
  const double dt = p.dt;
  for (int64_t s = 0; s < p.steps; ++s) {
    // T = rho + dU rho
    for (int e = tid; e < nn; e += kSmallThreads) {
      const int i = e / n, j = e - (e / n) * n;
      T cr = T(0), ci = T(0);
      for (int k = 0; k < n; ++k) {
        const T ar = sU[0][i * kSmallLd + k], ai = sU[1][i * kSmallLd + k];
        const T mr = rho[0][j * kSmallLd + k], mi = rho[1][j * kSmallLd + k];
        cr = fma(ar, mr, cr);
        cr = fma(ai, mi, cr);
        ci = fma(ai, mr, ci);
        ci = fma(-ar, mi, ci);
      }
      tb[0][i * kSmallLd + j] = cr + rho[0][i * kSmallLd + j];
      tb[1][i * kSmallLd + j] = ci + rho[1][i * kSmallLd + j];
    }
    __syncthreads();
    // Z = T + T conj(dU), lower triangle, into rho's buffer (rho is dead)
    T(*z)[kSmallN * kSmallLd] = rho;
    for (int e = tid; e < nn; e += kSmallThreads) {
      const int i = e / n, j = e - (e / n) * n;
      if (j > i) continue;
      T cr = T(0), ci = T(0);
      for (int k = 0; k < n; ++k) {
        const T ar = tb[0][i * kSmallLd + k], ai = tb[1][i * kSmallLd + k];
        const T mr = sU[0][j * kSmallLd + k], mi = sU[1][j * kSmallLd + k];
        cr = fma(ar, mr, cr);
        cr = fma(ai, mi, cr);
        ci = fma(ai, mr, ci);
        ci = fma(-ar, mi, ci);
      }
      z[0][i * kSmallLd + j] = cr + tb[0][i * kSmallLd + j];
      z[1][i * kSmallLd + j] = ci + tb[1][i * kSmallLd + j];
    }
    __syncthreads();
    // trace, lost probability and renormalisation (wave 0; lanes >= n add 0)
    if (tid < 64) {
      double tr = 0.0, lo = 0.0, ro = 0.0;
      if (tid < n) {
        const int u = tid;
        const double zu = double(z[0][u * kSmallLd + u]);
        tr = s_trw[u] * zu;
        lo = s_leak[u] * zu;
        ro = zu;
      }
      for (int w = kSmallN / 2; w > 0; w >>= 1) {
        tr += __shfl_down(tr, w);
        lo += __shfl_down(lo, w);
        ro += __shfl_down(ro, w);
      }
      if (tid == 0) {
        sink = sink + dt * lo;
        steps = steps + 1.0;
        rot = ro;
        lost = lo;
        scale = (1.0 - sink) / tr;
        s_scale = scale;
      }
    }
    __syncthreads();
    // rho' = scale * (Z + dt D(Z)) on and below the diagonal, mirrored, into tb
    const double sc = s_scale;
    for (int e = tid; e < nn; e += kSmallThreads) {
      const int u = e / n, v = e - (e / n) * n;
      if (v > u) continue;
      const double zr = double(z[0][u * kSmallLd + v]), zi = double(z[1][u * kSmallLd + v]);
      const double f = 1.0 - 0.5 * dt * (s_d[u] + s_d[v]);
      double xr = f * zr, xi = f * zi;
      for (int j = 0; j < p.n_gather; ++j) {
        const int32_t pu = staged ? s_pi[j][u] : p.pi[int64_t(j) * n + u];
        const int32_t pv = staged ? s_pi[j][v] : p.pi[int64_t(j) * n + v];
        if (pu >= 0 && pv >= 0) {
          const double cu = staged ? s_cg[j][u] : p.cg[int64_t(j) * n + u];
          const double cv = staged ? s_cg[j][v] : p.cg[int64_t(j) * n + v];
          const double w = dt * cu * cv;
          double gr, gi;
          if (pu >= pv) {
            gr = double(z[0][pu * kSmallLd + pv]);
            gi = double(z[1][pu * kSmallLd + pv]);
          } else {
            gr = double(z[0][pv * kSmallLd + pu]);
            gi = -double(z[1][pv * kSmallLd + pu]);
          }
          xr += w * gr;
          xi += w * gi;
        }
      }
      xr *= sc;
      xi *= sc;
      if (u == v) xi = 0.0;
      tb[0][u * kSmallLd + v] = T(xr);
      tb[1][u * kSmallLd + v] = T(xi);
      if (u != v) {
        tb[0][v * kSmallLd + u] = T(xr);
        tb[1][v * kSmallLd + u] = T(-xi);
      }
    }
    __syncthreads();
    T(*t)[kSmallN * kSmallLd] = rho;
    rho = tb;
    tb = t;
  }
  for (int e = tid; e < nn; e += kSmallThreads) {
    const int i = e / n, j = e - (e / n) * n;
    p.re[i * ld + j] = rho[0][i * kSmallLd + j];
    p.im[i * ld + j] = rho[1][i * kSmallLd + j];
  }
  if (tid == 0) {
    p.aux[0] = sink;
    p.aux[1] = rot;
    p.aux[2] = lost;
    p.aux[3] = steps;
    p.aux[4] = scale;
  }
}

template <typename T>
hipError_t launch_small_steps(const SmallArgs<T> &a, hipStream_t s) {
  if (a.n < 1 || a.n > kSmallN || a.ld < a.n || a.steps < 0) return hipErrorInvalidValue;
  for (int64_t done = 0; done < a.steps; done += kSmallStepsPerLaunch) {
    SmallArgs<T> b = a;
    b.steps = std::min<int64_t>(kSmallStepsPerLaunch, a.steps - done);
    hipError_t e = launch_kernel(small_steps_kernel<T>, dim3(1), dim3(kSmallThreads), 0, s, b);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t launch_small_steps<float>(const SmallArgs<float> &, hipStream_t);
template hipError_t launch_small_steps<double>(const SmallArgs<double> &, hipStream_t);

}  // namespace qme
