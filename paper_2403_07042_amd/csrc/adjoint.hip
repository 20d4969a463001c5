// Adjoint of the time step: gradients of a final diagonal observable with
// respect to the couplings g, the hoppings mu and the decoherence rates gamma.
//
// The paper's fourth modelling point (Sec. II) is to fit Hamiltonian
// parameters to experiment; these gradients make that fit possible.  With
// the step map rho_{k+1} = E(U rho_k U^dag), E = I + dt D (Sec. II, Eqs. 2-3;
// the renormalisation is the identity in exact arithmetic) and the objective
// f = sum_s o_s Re rho_K[s,s], the adjoint recursion is
//   lam_K = diag(o)
//   mu_k  = E^dag(lam_{k+1}) = lam + dt sum_j gamma_j (A^dag lam A - 1/2 {A^dag A, lam})
//   X_k   = U^dag mu_k,  lam_k = X_k U,  G = sum_k rho_k X_k
//   df/dgamma_j = dt sum_k Re tr(lam_{k+1} D_j(U rho_k U^dag))
//   df/dtheta_p = 2 dt Im tr(L(-i H dt, G) H_p)     (H_p = dH/dtheta_p)
// where L is the Frechet derivative of the exponential (evaluated on the
// host in FP64).  States are recomputed per segment from checkpoints taken
// every K steps of the forward pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <optional>
#include <string>
#include <vector>

#include "ctx.hpp"
#include "device.hpp"
#include "model.hpp"
#include "qme.h"

namespace qme {

static constexpr int kAdjThreads = 256;

template <typename T>
__device__ __forceinline__ void herm_at(const T *re, const T *im, int64_t ld, int64_t a, int64_t b,
                                        double &r, double &i) {
  if (a >= b) {
    r = double(re[a * ld + b]);
    i = double(im[a * ld + b]);
  } else {
    r = double(re[b * ld + a]);
    i = -double(im[b * ld + a]);
  }
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

template <typename T>
__global__ __launch_bounds__(kAdjThreads) void adj_dissipate_kernel(AdjArgs<T> p, int a0, int na,
                                                                     int first) {
  constexpr int TD = kAdjTile;
  __shared__ T s_re[TD][TD + 1];
  __shared__ T s_im[TD][TD + 1];
  __shared__ double s_col[kAdjThreads / TD][TD];
  __shared__ double s_g[kAdjThreads / TD][kMaxArrival];
  const int t = blockIdx.x;
  int bi = int((sqrtf(8.0f * float(t) + 1.0f) - 1.0f) * 0.5f);
  while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
  while (bi * (bi + 1) / 2 > t) --bi;
  const int bj = t - bi * (bi + 1) / 2;
  const bool diag_tile = bi == bj;
  const double dt = p.dt;
  const int c = threadIdx.x & (TD - 1);   // lane = column
  const int r0 = threadIdx.x / TD;        // wave = row phase
  const int64_t v = int64_t(bj) * TD + c;
  const int64_t n = p.n, ld = p.ld;

  double colacc = 0.0;
  double gacc[kMaxArrival];
#pragma unroll
  for (int a = 0; a < kMaxArrival; ++a) gacc[a] = 0.0;
  const double dv = v < n ? p.d[v] : 0.0;

  // rows rr = r0 + 4 k; the element loads of G rows are issued together
  // (unconditionally, an element outside the tile reading entry 0) ahead of
  // their rows' stores, which could alias them as far as the compiler knows
  constexpr int RSTEP = kAdjThreads / TD;
  constexpr int G = 4;
  static_assert(TD % (G * RSTEP) == 0, "row groups tile the adjoint tile");
  for (int rq = r0; rq < TD; rq += G * RSTEP) {
   T g_lre[G], g_lim[G], g_zre[G], g_zim[G];
   double g_du[G];
#pragma unroll
   for (int gq = 0; gq < G; ++gq) {
     const int64_t u = int64_t(bi) * TD + rq + gq * RSTEP;
     const bool valid = u < n && v < n && !(diag_tile && v > u);
     const int64_t o = valid ? u * ld + v : 0;
     g_lre[gq] = p.l_re[o];
     g_lim[gq] = p.l_im[o];
     g_zre[gq] = p.z_re[o];
     g_zim[gq] = p.z_im[o];
     g_du[gq] = p.d[valid ? u : 0];
   }
#pragma unroll
   for (int gq = 0; gq < G; ++gq) {
    const int rr = rq + gq * RSTEP;
    const int64_t u = int64_t(bi) * TD + rr;
    const bool valid = u < n && v < n && !(diag_tile && v > u);
    double e = 0.0;
    if (valid) {
      const int64_t o = u * ld + v;
      const double lr = double(g_lre[gq]), li = double(g_lim[gq]);
      if (first) {
        const double f = 1.0 - 0.5 * dt * (g_du[gq] + dv);
        double mr = f * lr, mi = f * li;
        for (int j = 0; j < p.n_gather; ++j) {
          const int32_t tu = p.tau[int64_t(j) * n + u];
          const int32_t tv = p.tau[int64_t(j) * n + v];
          if (tu >= 0 && tv >= 0) {
            const double w = dt * p.ca[int64_t(j) * n + u] * p.ca[int64_t(j) * n + v];
            double gr, gi;
            herm_at(p.l_re, p.l_im, ld, tu, tv, gr, gi);
            mr += w * gr;
            mi += w * gi;
          }
        }
        if (p.n_csr > 0 || p.koff_ptr) {
          // sparse channels: gamma A^T lam A and -1/2 {K_off, lam}
          double ar = 0.0, ai = 0.0;
          for (int ch = 0; ch < p.n_csr; ++ch) {
            const int64_t *ptr = p.csrt_ptr + int64_t(ch) * (n + 1);
            double cr = 0.0, ci = 0.0;
            for (int64_t x = ptr[u]; x < ptr[u + 1]; ++x) {
              const int32_t k = p.csrt_col[x];
              const double a = p.csrt_val[x];
              for (int64_t y = ptr[v]; y < ptr[v + 1]; ++y) {
                double gr, gi;
                herm_at(p.l_re, p.l_im, ld, k, p.csrt_col[y], gr, gi);
                const double w = a * p.csrt_val[y];
                cr += w * gr;
                ci += w * gi;
              }
            }
            ar += p.csr_gamma[ch] * cr;
            ai += p.csr_gamma[ch] * ci;
          }
          if (p.koff_ptr) {
            double kr = 0.0, ki = 0.0;
            for (int64_t x = p.koff_ptr[u]; x < p.koff_ptr[u + 1]; ++x) {
              double gr, gi;
              herm_at(p.l_re, p.l_im, ld, p.koff_col[x], v, gr, gi);
              kr += p.koff_val[x] * gr;
              ki += p.koff_val[x] * gi;
            }
            for (int64_t y = p.koff_ptr[v]; y < p.koff_ptr[v + 1]; ++y) {
              double gr, gi;
              herm_at(p.l_re, p.l_im, ld, u, p.koff_col[y], gr, gi);
              kr += p.koff_val[y] * gr;
              ki += p.koff_val[y] * gi;
            }
            ar -= 0.5 * kr;
            ai -= 0.5 * ki;
          }
          mr += dt * ar;
          mi += dt * ai;
        }
        if (u == v) mi = 0.0;
        p.mu_re[o] = T(mr);
        p.mu_im[o] = T(mi);
        if (diag_tile) {
          if (u != v) {
            p.mu_re[v * ld + u] = T(mr);
            p.mu_im[v * ld + u] = T(-mi);
          }
        } else {
          s_re[rr][c] = T(mr);
          s_im[rr][c] = T(mi);
        }
        // e(u, v) = Re(Z[u,v] lam[v,u]) = Re(Z[u,v] conj(lam[u,v]))
        const double zr = double(g_zre[gq]), zi = double(g_zim[gq]);
        e = zr * lr + zi * li;
        if (u != v) colacc += e;
      }
      const double w2 = (u == v) ? 1.0 : 2.0;
      for (int a = 0; a < kMaxArrival; ++a) {
        if (a >= na) break;
        const int64_t base = int64_t(a0 + a) * n;
        const int32_t pu = p.upi[base + u], pv = p.upi[base + v];
        if (pu >= 0 && pv >= 0) {
          double gr, gi;
          herm_at(p.z_re, p.z_im, ld, pu, pv, gr, gi);
          // Re(lam[v,u] Z[pu,pv]) = Re(conj(lam[u,v]) g)
          gacc[a] += w2 * p.uc[base + u] * p.uc[base + v] * (lr * gr + li * gi);
        }
      }
    }
    if (first) {
      const double rs = wave_sum(e);
      if (c == 0 && u < n) p.rowbuf[int64_t(bj) * n + u] = rs;
    }
   }
  }
  if (first) {
    s_col[r0][c] = colacc;
  }
  for (int a = 0; a < kMaxArrival; ++a) {
    if (a >= na) break;
    const double g = wave_sum(gacc[a]);
    if (c == 0) s_g[r0][a] = g;
  }
  __syncthreads();
  if (first && r0 == 0 && v < n) {
    double sacc = 0.0;
    for (int w = 0; w < kAdjThreads / TD; ++w) sacc += s_col[w][c];
    p.colbuf[int64_t(bi) * n + v] = sacc;
  }
  if (int(threadIdx.x) < na) {
    double sacc = 0.0;
    for (int w = 0; w < kAdjThreads / TD; ++w) sacc += s_g[w][threadIdx.x];
    p.gbuf[int64_t(blockIdx.x) * p.n_arrival + a0 + threadIdx.x] = sacc;
  }
  if (!first || diag_tile) return;
  // mirror tile (bj, bi) of mu
  const int64_t ucol = int64_t(bi) * TD + c;
  for (int a = r0; a < TD; a += kAdjThreads / TD) {
    const int64_t vrow = int64_t(bj) * TD + a;
    if (vrow >= n || ucol >= n) continue;
    p.mu_re[vrow * ld + ucol] = s_re[c][a];
    p.mu_im[vrow * ld + ucol] = -s_im[c][a];
  }
}

template <typename T>
__global__ __launch_bounds__(kAdjThreads) void adj_sparse_gamma_kernel(AdjSparseArgs<T> p) {
  constexpr int TD = kAdjTile;
  __shared__ double s_w[kAdjThreads / 64];
  const int t = blockIdx.x, q = blockIdx.y;
  int bi = int((sqrtf(8.0f * float(t) + 1.0f) - 1.0f) * 0.5f);
  while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
  while (bi * (bi + 1) / 2 > t) --bi;
  const int bj = t - bi * (bi + 1) / 2;
  const int c = threadIdx.x & (TD - 1);
  const int r0 = threadIdx.x / TD;
  const int64_t v = int64_t(bj) * TD + c;
  const int64_t n = p.n, ld = p.ld;
  const int64_t *aptr = p.csr_ptr + int64_t(q) * (n + 1);
  const int64_t *kptr = p.kj_ptr + int64_t(q) * (n + 1);
  double acc = 0.0;
  for (int rr = r0; rr < TD; rr += kAdjThreads / TD) {
    const int64_t u = int64_t(bi) * TD + rr;
    if (u >= n || v >= n || (bi == bj && v > u)) continue;
    double er = 0.0, ei = 0.0;
    for (int64_t x = aptr[u]; x < aptr[u + 1]; ++x) {      // (A Z A^T)[u,v]
      const int32_t k = p.csr_col[x];
      const double a = p.csr_val[x];
      for (int64_t y = aptr[v]; y < aptr[v + 1]; ++y) {
        double zr, zi;
        herm_at(p.z_re, p.z_im, ld, k, p.csr_col[y], zr, zi);
        const double w = a * p.csr_val[y];
        er += w * zr;
        ei += w * zi;
      }
    }
    double kr = 0.0, ki = 0.0;
    for (int64_t x = kptr[u]; x < kptr[u + 1]; ++x) {      // (K_off Z)[u,v]
      double zr, zi;
      herm_at(p.z_re, p.z_im, ld, p.kj_col[x], v, zr, zi);
      kr += p.kj_val[x] * zr;
      ki += p.kj_val[x] * zi;
    }
    for (int64_t y = kptr[v]; y < kptr[v + 1]; ++y) {      // (Z K_off)[u,v]
      double zr, zi;
      herm_at(p.z_re, p.z_im, ld, u, p.kj_col[y], zr, zi);
      kr += p.kj_val[y] * zr;
      ki += p.kj_val[y] * zi;
    }
    er -= 0.5 * kr;
    ei -= 0.5 * ki;
    const int64_t o = u * ld + v;
    const double lr = double(p.l_re[o]), li = double(p.l_im[o]);
    acc += (u == v ? 1.0 : 2.0) * (lr * er + li * ei);
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = s_w[0];
    for (int w = 1; w < kAdjThreads / 64; ++w) sum += s_w[w];
    p.part[int64_t(q) * gridDim.x + t] = sum;
  }
}

__global__ __launch_bounds__(256) void sparse_gamma_reduce_kernel(const double *part, int blocks,
                                                                  const int32_t *channel,
                                                                  double dt, double *grad) {
  __shared__ double s[256];
  const int q = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < blocks; b += 256) acc += part[int64_t(q) * blocks + b];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) grad[channel[q]] += dt * s[0];
}

__global__ void q_reduce_kernel(const double *rowbuf, const double *colbuf, int64_t n,
                                int tiles, double *q) {
  const int64_t u = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int tu = int(u / kAdjTile);
  // the same sums in the same order, the loads of G terms issued together
  constexpr int G = 8;
  double acc = 0.0;
  for (int b0 = 0; b0 <= tu; b0 += G) {
    double x[G];
#pragma unroll
    for (int g = 0; g < G; ++g) x[g] = rowbuf[int64_t(b0 + g <= tu ? b0 + g : 0) * n + u];
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (b0 + g <= tu) acc += x[g];
  }
  for (int b0 = tu; b0 < tiles; b0 += G) {
    double x[G];
#pragma unroll
    for (int g = 0; g < G; ++g) x[g] = colbuf[int64_t(b0 + g < tiles ? b0 + g : 0) * n + u];
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (b0 + g < tiles) acc += x[g];
  }
  q[u] = acc;
}

__global__ __launch_bounds__(256) void gamma_reduce_kernel(const double *gbuf, int blocks,
                                                           int n_arrival, const int32_t *arrival_of,
                                                           const double *ada, const double *q,
                                                           int64_t n, double dt, double *grad) {
  __shared__ double s_a[256], s_b[256];
  const int j = blockIdx.x;
  double anti = 0.0, jump = 0.0;
  for (int64_t u = threadIdx.x; u < n; u += 256) anti += ada[int64_t(j) * n + u] * q[u];
  const int a = arrival_of[j];
  if (a >= 0)
    for (int b = threadIdx.x; b < blocks; b += 256) jump += gbuf[int64_t(b) * n_arrival + a];
  s_a[threadIdx.x] = anti;
  s_b[threadIdx.x] = jump;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
      s_a[threadIdx.x] += s_a[threadIdx.x + w];
      s_b[threadIdx.x] += s_b[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) grad[j] += dt * (s_b[0] - s_a[0]);
}

template <typename T>
__global__ void set_diag_kernel(T *x_re, T *x_im, int64_t ld, int64_t n, const double *o) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ld * ld) return;
  const int64_t i = e / ld, j = e % ld;
  x_re[e] = (i == j && i < n) ? T(o[i]) : T(0);
  x_im[e] = T(0);
}

// ---------------------------------------------- Frechet finalisation (FP64)
// W = L(B, G) for B = -i tau H by the series of the adjoint of the Frechet
// derivative of exp: M_1 = G, R_1 = G B, M_{k+1} = (B M_k + R_k) / (k+1),
// R_{k+1} = R_k B / (k+1), W = sum_k M_k.  H is sparse (CSR, symmetric), so
// every product is a sparse-times-dense pass.

template <typename T>
__global__ void widen_kernel(const T *gr, const T *gi, double *dr, double *di, int64_t total) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < total) {
    dr[e] = double(gr[e]);
    di[e] = double(gi[e]);
  }
}

// out = inv (B X + R), W += out      (row i of B X uses row i of H)
__global__ void frechet_left_kernel(const int64_t *ptr, const int32_t *col, const double *val,
                                    double tau, const double *xr, const double *xi,
                                    const double *rr, const double *ri, double *outr,
                                    double *outi, double *wr, double *wi, int64_t n, int64_t ld,
                                    double inv) {
  const int64_t i = blockIdx.y;
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double ar = 0.0, ai = 0.0;
  for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q) {
    const int64_t o = int64_t(col[q]) * ld + j;
    ar += val[q] * xr[o];
    ai += val[q] * xi[o];
  }
  const int64_t o = i * ld + j;
  // B X = -i tau (H X): real part tau Im(HX), imaginary part -tau Re(HX)
  const double vr = inv * (tau * ai + rr[o]);
  const double vi = inv * (-tau * ar + ri[o]);
  outr[o] = vr;
  outi[o] = vi;
  wr[o] += vr;
  wi[o] += vi;
}

// out = inv X B                      ((X H)[i][j] = sum over row j of H)
__global__ void frechet_right_kernel(const int64_t *ptr, const int32_t *col, const double *val,
                                     double tau, const double *xr, const double *xi,
                                     double *outr, double *outi, int64_t n, int64_t ld,
                                     double inv) {
  const int64_t i = blockIdx.y;
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double ar = 0.0, ai = 0.0;
  for (int64_t q = ptr[j]; q < ptr[j + 1]; ++q) {
    const int64_t o = i * ld + col[q];
    ar += val[q] * xr[o];
    ai += val[q] * xi[o];
  }
  const int64_t o = i * ld + j;
  outr[o] = inv * tau * ai;
  outi[o] = -inv * tau * ar;
}

// out[e] = Im W[col_e][row_e] * val_e  (tr(W H_p) gathers W transposed)
__global__ void term_gather_kernel(const double *wi, const int32_t *trow, const int32_t *tcol,
                                   const double *tval, int64_t ne, int64_t ld, double *out) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < ne) out[e] = wi[int64_t(tcol[e]) * ld + trow[e]] * tval[e];
}

template <typename T>
hipError_t launch_adj_dissipate(const AdjArgs<T> &a, hipStream_t s) {
  const int tiles = int((a.n + kAdjTile - 1) / kAdjTile);
  const int blocks = tiles * (tiles + 1) / 2;
  int a0 = 0;
  bool first = true;
  do {
    const int na = std::min(kMaxArrival, a.n_arrival - a0);
    hipLaunchKernelGGL(adj_dissipate_kernel<T>, dim3(blocks), dim3(kAdjThreads), 0, s, a, a0,
                       std::max(na, 0), first ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    first = false;
    a0 += kMaxArrival;
  } while (a0 < a.n_arrival);
  return hipSuccess;
}

template <typename T>
hipError_t launch_adj_sparse_gamma(const AdjSparseArgs<T> &a, hipStream_t s) {
  if (a.n_csr == 0) return hipSuccess;
  const int tiles = int((a.n + kAdjTile - 1) / kAdjTile);
  const int blocks = tiles * (tiles + 1) / 2;
  hipLaunchKernelGGL(adj_sparse_gamma_kernel<T>, dim3(blocks, a.n_csr), dim3(kAdjThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sparse_gamma_reduce(const double *part, int blocks, int n_csr,
                                      const int32_t *channel, double dt, double *grad,
                                      hipStream_t s) {
  if (n_csr == 0) return hipSuccess;
  hipLaunchKernelGGL(sparse_gamma_reduce_kernel, dim3(n_csr), dim3(256), 0, s, part, blocks,
                     channel, dt, grad);
  return hipGetLastError();
}

hipError_t launch_q_reduce(const double *rowbuf, const double *colbuf, int64_t n, double *q,
                           hipStream_t s) {
  const int tiles = int((n + kAdjTile - 1) / kAdjTile);
  hipLaunchKernelGGL(q_reduce_kernel, dim3(int((n + 63) / 64)), dim3(64), 0, s, rowbuf,
                     colbuf, n, tiles, q);
  return hipGetLastError();
}

hipError_t launch_gamma_reduce(const double *gbuf, int blocks, int n_arrival,
                               const int32_t *arrival_of, const double *ada, const double *q,
                               int64_t n, int n_jumps, double dt, double *grad, hipStream_t s) {
  if (n_jumps == 0) return hipSuccess;
  hipLaunchKernelGGL(gamma_reduce_kernel, dim3(n_jumps), dim3(256), 0, s, gbuf, blocks,
                     std::max(n_arrival, 1), arrival_of, ada, q, n, dt, grad);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_set_diag(T *x_re, T *x_im, int64_t ld, int64_t n, const double *o,
                           hipStream_t s) {
  const int64_t total = ld * ld;
  hipLaunchKernelGGL(set_diag_kernel<T>, dim3(int((total + 255) / 256)), dim3(256), 0, s, x_re,
                     x_im, ld, n, o);
  return hipGetLastError();
}

template hipError_t launch_adj_sparse_gamma<float>(const AdjSparseArgs<float> &, hipStream_t);
template hipError_t launch_adj_sparse_gamma<double>(const AdjSparseArgs<double> &, hipStream_t);
template hipError_t launch_adj_dissipate<float>(const AdjArgs<float> &, hipStream_t);
template hipError_t launch_adj_dissipate<double>(const AdjArgs<double> &, hipStream_t);
template hipError_t launch_set_diag<float>(float *, float *, int64_t, int64_t, const double *,
                                           hipStream_t);
template hipError_t launch_set_diag<double>(double *, double *, int64_t, int64_t,
                                            const double *, hipStream_t);

}  // namespace qme

// ------------------------------------------------------------ host driver

namespace qme {

struct AdjLayout {
  int64_t nseg = 0, seg = 0;
  size_t S = 0, cp = 0, R = 0, Zs = 0, Y = 0, lam = 0, mu = 0, X = 0, G = 0;
  size_t rowbuf = 0, colbuf = 0, gbuf = 0, q = 0, o = 0, grad = 0, diag = 0, total = 0;
  size_t gsp = 0;   // sparse channels' rate-gradient partials
  size_t fw = 0, fm = 0, fm2 = 0, fr = 0, fr2 = 0, fterm = 0;
  int tiles = 0, blocks = 0;
};

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

static AdjLayout adj_layout(const qme_ctx *c, int64_t n_steps, int32_t every) {
  AdjLayout L;
  L.seg = std::max<int64_t>(1, std::min<int64_t>(every, std::max<int64_t>(n_steps, 1)));
  L.nseg = n_steps > 0 ? (n_steps + L.seg - 1) / L.seg : 0;
  const size_t sb = align256(state_bytes(c));
  const size_t p2 = align256(2 * plane_elems(c) * size_t(c->elem));
  const int64_t n = c->n;
  L.tiles = int((n + kAdjTile - 1) / kAdjTile);
  L.blocks = L.tiles * (L.tiles + 1) / 2;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t at = off; off += align256(bytes); return at; };
  L.S = take(sb);
  L.cp = take(sb * size_t(std::max<int64_t>(L.nseg, 1)));
  L.R = take(sb * size_t(L.seg + 1));
  L.Zs = take(p2 * size_t(L.seg));
  L.Y = take(p2);
  L.lam = take(p2);
  L.mu = take(p2);
  L.X = take(p2);
  L.G = take(p2);
  L.rowbuf = take(sizeof(double) * size_t(L.tiles) * n);
  L.colbuf = take(sizeof(double) * size_t(L.tiles) * n);
  L.gbuf = take(sizeof(double) * size_t(L.blocks) * size_t(std::max(1, c->n_arrival)));
  L.gsp = take(sizeof(double) * size_t(L.blocks) * size_t(std::max(1, c->jt.n_csr)));
  L.q = take(sizeof(double) * n);
  L.o = take(sizeof(double) * n);
  L.grad = take(sizeof(double) * std::max<size_t>(1, c->model.jumps.size()));
  L.diag = take(sizeof(double) * n);
  const size_t p2d = 2 * plane_elems(c) * sizeof(double);
  L.fw = take(p2d);
  L.fm = take(p2d);
  L.fm2 = take(p2d);
  L.fr = take(p2d);
  L.fr2 = take(p2d);
  L.fterm = take(sizeof(double) * std::max<size_t>(1, size_t(c->term_offset.back())));
  L.total = off;
  return L;
}

// part: 2 * ld^2 elements of dead planes for a tail split of a lower product
template <typename T>
static hipError_t gemm(const qme_ctx *c, int tile, const GemmOps &o, const T *a_re, const T *a_im,
                       const T *m_re, const T *m_im, const T *x_re, const T *x_im, T *c_re,
                       T *c_im, hipStream_t s, T *part = nullptr) {
  CgemmArgs<T> g{a_re, a_im, m_re, m_im, x_re, x_im, c_re, c_im, c->ld, T(1), T(1)};
  if (o.lower && part && c->tail_split) {
    const int kt = c->precision == QME_FP32 && tile == 32 ? 32 : 16;
    const SplitPlan sp = plan_tail_split(int(c->ld / tile), tile, kt, c->ld, c->cus, 2 * plane_elems(c));
    g.full = sp.full;
    g.split = sp.split;
    g.part = part;
  }
  if constexpr (sizeof(T) == 4) return launch_cgemm_f32(g, tile, o, s);
  else return launch_cgemm_f64(g, tile, o, s);
}

#define ADJ_OK(call)                                                          \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) {                                                   \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));           \
      return QME_E_DEVICE;                                                    \
    }                                                                         \
  } while (0)

template <typename T>
static qme_status adjoint_impl(qme_ctx *c, const void *state0, int64_t n_steps, int32_t every,
                               const double *obs, double *value, double *grad, char *ws,
                               hipStream_t s) {
  const AdjLayout L = adj_layout(c, n_steps, every);
  const size_t pe = plane_elems(c);
  const size_t sb = state_bytes(c), sba = align256(sb);
  const size_t p2 = align256(2 * pe * size_t(c->elem));
  const int64_t n = c->n;
  const int nj = int(c->model.jumps.size());
  char *S = ws + L.S;
  auto planes = [&](size_t off) {
    T *re = reinterpret_cast<T *>(ws + off);
    return std::make_pair(re, re + pe);
  };
  auto [lam_re, lam_im] = planes(L.lam);
  auto [mu_re, mu_im] = planes(L.mu);
  auto [x_re, x_im] = planes(L.X);
  auto [g_re, g_im] = planes(L.G);
  const T *u_re = static_cast<const T *>(c->du_re), *u_im = static_cast<const T *>(c->du_im);

  // forward pass with checkpoints; the last segment is run straight into the
  // recompute buffers R / Zs, so it is not recomputed in the backward pass
  std::optional<TraceRange> phase;   // roctx range of the current phase
  phase.emplace("qme_adjoint: forward with checkpoints");
  char *R = ws + L.R;
  // the decoherence passes write rows/columns < n only: the padding of the
  // recomputed states must be zero for the products that read them
  ADJ_OK(hipMemsetAsync(R, 0, sba * size_t(L.seg + 1), s));
  ADJ_OK(hipMemcpyAsync(S, state0, sb, hipMemcpyDeviceToDevice, s));
  for (int64_t g = 0; g < L.nseg; ++g) {
    ADJ_OK(hipMemcpyAsync(ws + L.cp + size_t(g) * sba, S, sb, hipMemcpyDeviceToDevice, s));
    const int64_t len = std::min<int64_t>(L.seg, n_steps - g * L.seg);
    if (g + 1 < L.nseg) {
      for (int64_t i = 0; i < len; ++i) ADJ_OK(step_once<T>(c, S, S, ws + L.Y, ws + L.Zs, s));
    } else {
      ADJ_OK(hipMemcpyAsync(R, S, sb, hipMemcpyDeviceToDevice, s));
      for (int64_t i = 0; i < len; ++i)
        ADJ_OK(step_once<T>(c, R + size_t(i) * sba, R + size_t(i + 1) * sba, ws + L.Y,
                            ws + L.Zs + size_t(i) * p2, s));
      const int64_t last = n_steps - g * L.seg;
      if (last != len) { set_error("internal: segment length mismatch"); return QME_E_STATE; }
      ADJ_OK(hipMemcpyAsync(S, R + size_t(len) * sba, sb, hipMemcpyDeviceToDevice, s));
    }
  }
  // objective
  double *diag = reinterpret_cast<double *>(ws + L.diag);
  ADJ_OK(launch_diag<T>(reinterpret_cast<const T *>(S), c->ld, n, diag, s));
  std::vector<double> pops(n);
  ADJ_OK(hipMemcpyAsync(pops.data(), diag, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  ADJ_OK(hipStreamSynchronize(s));
  double f = 0.0;
  for (int64_t u = 0; u < n; ++u) f += obs[u] * pops[u];
  if (value) *value = f;

  // lam_K = diag(o), G = 0, rate gradients = 0
  double *o_dev = reinterpret_cast<double *>(ws + L.o);
  double *ggam = reinterpret_cast<double *>(ws + L.grad);
  ADJ_OK(hipMemcpyAsync(o_dev, obs, sizeof(double) * n, hipMemcpyHostToDevice, s));
  ADJ_OK(launch_set_diag<T>(lam_re, lam_im, c->ld, n, o_dev, s));
  ADJ_OK(hipMemsetAsync(ws + L.G, 0, p2, s));
  // the adjoint decoherence pass writes rows/columns < n only: the padding
  // of mu must be zero for the products that read it
  ADJ_OK(hipMemsetAsync(ws + L.mu, 0, p2, s));
  ADJ_OK(hipMemsetAsync(ggam, 0, sizeof(double) * std::max(1, nj), s));

  AdjArgs<T> aa{lam_re, lam_im, mu_re, mu_im, nullptr, nullptr, c->ld, n, c->model.dt, c->d,
                c->tau, c->ca, c->jt.n_gather, c->upi, c->uc, c->n_arrival,
                reinterpret_cast<double *>(ws + L.rowbuf), reinterpret_cast<double *>(ws + L.colbuf),
                reinterpret_cast<double *>(ws + L.gbuf)};
  aa.n_csr = c->jt.n_csr;
  aa.csrt_ptr = c->csrt_ptr;
  aa.csrt_col = c->csrt_col;
  aa.csrt_val = c->csrt_val;
  aa.csr_gamma = c->csr_gamma;
  aa.koff_ptr = c->jt.koff_col.empty() ? nullptr : c->koff_ptr;
  aa.koff_col = c->koff_col;
  aa.koff_val = c->koff_val;
  AdjSparseArgs<T> sa{lam_re, lam_im, nullptr, nullptr, c->ld, n, c->jt.n_csr, c->csr_ptr,
                      c->csr_col, c->csr_val, c->kj_ptr, c->kj_col, c->kj_val,
                      reinterpret_cast<double *>(ws + L.gsp)};
  double *q = reinterpret_cast<double *>(ws + L.q);
  GemmOps ox, ol, og;
  ox.conj_a = true;   // X = mu + conj(dU) mu   (mu^H = mu)
  ox.conj_b = true;
  ol.lower = true;    // lam = X + X dU          (dU^T = dU)
  og.b_rows = true;   // G += rho X
  ox.direct = ol.direct = og.direct = c->direct;
  ox.cus = ol.cus = og.cus = c->cus;

  phase.reset();
  phase.emplace("qme_adjoint: backward (segment recompute + adjoint steps)");
  for (int64_t g = L.nseg - 1; g >= 0; --g) {
    const int64_t len = std::min<int64_t>(L.seg, n_steps - g * L.seg);
    if (g + 1 < L.nseg) {   // recompute the segment from its checkpoint
      ADJ_OK(hipMemcpyAsync(R, ws + L.cp + size_t(g) * sba, sb, hipMemcpyDeviceToDevice, s));
      for (int64_t i = 0; i < len; ++i)
        ADJ_OK(step_once<T>(c, R + size_t(i) * sba, R + size_t(i + 1) * sba, ws + L.Y,
                            ws + L.Zs + size_t(i) * p2, s));
    }
    for (int64_t i = len - 1; i >= 0; --i) {
      auto [z_re, z_im] = planes(L.Zs + size_t(i) * p2);
      aa.z_re = z_re;
      aa.z_im = z_im;
      ADJ_OK(launch_adj_dissipate<T>(aa, s));
      ADJ_OK(launch_q_reduce(aa.rowbuf, aa.colbuf, n, q, s));
      ADJ_OK(launch_gamma_reduce(aa.gbuf, L.blocks, c->n_arrival, c->arrival_of, c->ada, q, n,
                                 nj, c->model.dt, ggam, s));
      sa.z_re = z_re;
      sa.z_im = z_im;
      ADJ_OK(launch_adj_sparse_gamma<T>(sa, s));
      ADJ_OK(launch_sparse_gamma_reduce(sa.part, L.blocks, c->jt.n_csr, c->csr_channel,
                                        c->model.dt, ggam, s));
      ADJ_OK(gemm<T>(c, c->tile1, ox, u_re, u_im, mu_re, mu_im, mu_re, mu_im, x_re, x_im, s));
      // mu is dead once X is formed: it holds the split partials
      ADJ_OK(gemm<T>(c, c->tile2, ol, x_re, x_im, u_re, u_im, x_re, x_im, lam_re, lam_im, s, mu_re));
      const T *r_re = reinterpret_cast<const T *>(R + size_t(i) * sba), *r_im = r_re + pe;
      ADJ_OK(gemm<T>(c, c->tile1, og, r_re, r_im, x_re, x_im, g_re, g_im, g_re, g_im, s));
    }
  }

  phase.reset();
  phase.emplace("qme_adjoint: Frechet finalisation");
  std::vector<double> gam(std::max(1, nj));
  ADJ_OK(hipMemcpyAsync(gam.data(), ggam, sizeof(double) * gam.size(), hipMemcpyDeviceToHost, s));
  const size_t n_terms = c->term_offset.size() - 1;
  const double dt = c->model.dt;
  if (c->squarings == 0) {
    // finalisation on the device in FP64
    const int64_t ld = c->ld;
    auto dpl = [&](size_t off) {
      double *re = reinterpret_cast<double *>(ws + off);
      return std::make_pair(re, re + pe);
    };
    auto [w_re, w_im] = dpl(L.fw);
    auto [m_re, m_im] = dpl(L.fm);
    auto [m2_re, m2_im] = dpl(L.fm2);
    auto [r_re, r_im] = dpl(L.fr);
    auto [r2_re, r2_im] = dpl(L.fr2);
    const int64_t total = int64_t(pe);
    const dim3 eb(256), eg(unsigned((total + 255) / 256));
    hipLaunchKernelGGL(widen_kernel<T>, eg, eb, 0, s, g_re, g_im, m_re, m_im, total);
    ADJ_OK(hipGetLastError());
    hipLaunchKernelGGL(widen_kernel<T>, eg, eb, 0, s, g_re, g_im, w_re, w_im, total);
    ADJ_OK(hipGetLastError());
    const double tau = dt;
    const dim3 sg(unsigned((n + 255) / 256), unsigned(n));
    hipLaunchKernelGGL(frechet_right_kernel, sg, eb, 0, s, c->h_ptr, c->h_col, c->h_val, tau,
                       m_re, m_im, r_re, r_im, n, ld, 1.0);
    ADJ_OK(hipGetLastError());
    // number of terms: theta^k / k! below 1e-18 with theta = tau |H|_1
    const double theta = tau * c->h_norm1;
    int kmax = 1;
    for (double term = theta; kmax < 60 && (term > 1e-18 || double(kmax) < theta);) {
      ++kmax;
      term *= theta / double(kmax);
    }
    for (int k = 1; k <= kmax; ++k) {
      const double inv = 1.0 / double(k + 1);
      hipLaunchKernelGGL(frechet_left_kernel, sg, eb, 0, s, c->h_ptr, c->h_col, c->h_val, tau,
                         m_re, m_im, r_re, r_im, m2_re, m2_im, w_re, w_im, n, ld, inv);
      ADJ_OK(hipGetLastError());
      hipLaunchKernelGGL(frechet_right_kernel, sg, eb, 0, s, c->h_ptr, c->h_col, c->h_val, tau,
                         r_re, r_im, r2_re, r2_im, n, ld, inv);
      ADJ_OK(hipGetLastError());
      std::swap(m_re, m2_re);
      std::swap(m_im, m2_im);
      std::swap(r_re, r2_re);
      std::swap(r_im, r2_im);
    }
    const int64_t ne = c->term_offset.back();
    std::vector<double> te(std::max<int64_t>(1, ne));
    double *fterm = reinterpret_cast<double *>(ws + L.fterm);
    if (ne > 0) {
      hipLaunchKernelGGL(term_gather_kernel, dim3(unsigned((ne + 255) / 256)), eb, 0, s, w_im,
                         c->t_row, c->t_col, c->t_val, ne, ld, fterm);
      ADJ_OK(hipGetLastError());
      ADJ_OK(hipMemcpyAsync(te.data(), fterm, sizeof(double) * ne, hipMemcpyDeviceToHost, s));
    }
    ADJ_OK(hipStreamSynchronize(s));
    for (size_t p = 0; p < n_terms; ++p) {
      double im = 0.0;
      for (int64_t e = c->term_offset[p]; e < c->term_offset[p + 1]; ++e) im += te[e];
      grad[p] = 2.0 * dt * im;
    }
  } else {
    // scaling and squaring was needed: finalise on the host in FP64
    std::vector<T> gh(2 * pe);
    ADJ_OK(hipMemcpyAsync(gh.data(), g_re, sizeof(T) * 2 * pe, hipMemcpyDeviceToHost, s));
    ADJ_OK(hipStreamSynchronize(s));
    std::vector<double> gr(size_t(n) * n), gi(size_t(n) * n), wr, wi;
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < n; ++j) {
        gr[size_t(i) * n + j] = double(gh[size_t(i) * c->ld + j]);
        gi[size_t(i) * n + j] = double(gh[pe + size_t(i) * c->ld + j]);
      }
    std::string err;
    if (!frechet_adjoint(c->model, c->h, gr, gi, wr, wi, err)) {
      set_error(err);
      return QME_E_NUMERIC;
    }
    const std::vector<TermCoo> terms = hamiltonian_terms(c->model);
    for (size_t p = 0; p < terms.size(); ++p) {
      // tr(W H_p) = sum_{(r,c)} W[c][r] H_p[r][c]; only its imaginary part is used
      double im = 0.0;
      for (size_t e = 0; e < terms[p].val.size(); ++e)
        im += wi[size_t(terms[p].col[e]) * n + terms[p].row[e]] * terms[p].val[e];
      grad[p] = 2.0 * dt * im;
    }
  }
  for (int j = 0; j < nj; ++j) grad[n_terms + j] = gam[j];
  return QME_OK;
}

}  // namespace qme

using namespace qme;

extern "C" qme_status qme_adjoint_workspace_size(const qme_ctx *c, int64_t n_steps,
                                                 int32_t checkpoint_every, size_t *bytes) {
  set_error("");
  if (!c || !bytes) { set_error("NULL argument"); return QME_E_ARG; }
  if (n_steps < 0 || checkpoint_every < 1) { set_error("n_steps < 0 or checkpoint_every < 1"); return QME_E_ARG; }
  *bytes = adj_layout(c, n_steps, checkpoint_every).total;
  return QME_OK;
}

extern "C" qme_status qme_adjoint(qme_ctx *c, const void *state0, int64_t n_steps,
                                  int32_t checkpoint_every, const double *obs, double *value,
                                  double *grad, void *ws, size_t ws_bytes, void *hip_stream) {
  try {
    TraceRange range("qme_adjoint");
    set_error("");
    if (!c || !state0 || !obs || !grad || !ws) { set_error("NULL argument"); return QME_E_ARG; }
    if (n_steps < 0 || checkpoint_every < 1) { set_error("n_steps < 0 or checkpoint_every < 1"); return QME_E_ARG; }
    if ((reinterpret_cast<uintptr_t>(ws) | reinterpret_cast<uintptr_t>(state0)) & 255) {
      set_error("state and workspace must be 256-byte aligned");
      return QME_E_ARG;
    }
    for (int64_t u = 0; u < c->n; ++u)
      if (!std::isfinite(obs[u])) { set_error("observable is not finite"); return QME_E_ARG; }
    if (ws_bytes < adj_layout(c, n_steps, checkpoint_every).total) {
      set_error("adjoint workspace too small (see qme_adjoint_workspace_size)");
      return QME_E_SIZE;
    }
    qme_status st = check_device(c);
    if (st != QME_OK) return st;
    // the recomputed forward steps are not qme_step's kernels: no profiling
    // records (and no armed launch timer) during the call
    struct ProfilingOff {
      qme_ctx *c;
      bool was;
      ~ProfilingOff() {
        c->profiling = was;
        launch_timer() = nullptr;
      }
    } profiling_off{c, c->profiling};
    c->profiling = false;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    char *w = static_cast<char *>(ws);
    if (c->elem == 8) return adjoint_impl<double>(c, state0, n_steps, checkpoint_every, obs, value, grad, w, s);
    return adjoint_impl<float>(c, state0, n_steps, checkpoint_every, obs, value, grad, w, s);
  } catch (const std::bad_alloc &) {
    set_error("out of host memory");
    return QME_E_SIZE;
  } catch (const std::exception &e) {
    set_error(std::string("internal error: ") + e.what());
    return QME_E_STATE;
  }
}
