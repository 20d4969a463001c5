// Device-side bodies of the decoherence step (shared by the per-step
// kernels in dissipate.hip and the persistent batched step).
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
// Decoherence operators that are not monomial (general-form models) enter in
// sparse form (DissArgs::n_csr, koff): per element the jump term of channel
// j is gamma_j sum_{k in row u of A_j} sum_{l in row v of A_j} a_uk a_vl
// Z[k,l], and the off-diagonal part of K = sum gamma A^dag A adds
// -1/2 (K Z + Z K)[u,v] beside the diagonal factor.
//
// trace_kernel (one workgroup) needs only the diagonal of Z: it forms
// tr rho_d = sum_w trw[w] Z[w,w] (the jump terms regrouped by the diagonal
// element they read, weights fixed per context) and the probability leaving
// the basis in FP64, updates the sink and the renormalisation factor
// (1 - sink) / tr rho_d.  dissipate_kernel
// then writes X = scale * rho_d for u >= v and its conjugate mirror, so X is
// exactly Hermitian; all arithmetic is FP64 whatever the storage type.
#pragma once

#include "device.hpp"

namespace qme {

static constexpr int TD = 32;          // tile edge of the decoherence pass
static constexpr int kDissThreads = 256;

template <typename T>
__device__ __forceinline__ void zlower(const DissArgs<T> &p, int64_t a, int64_t b, double &re,
                                       double &im) {
  // element (a, b) of the Hermitian Z from its lower triangle
  if (a >= b) {
    re = double(p.z_re[a * p.ld + b]);
    im = double(p.z_im[a * p.ld + b]);
  } else {
    re = double(p.z_re[b * p.ld + a]);
    im = -double(p.z_im[b * p.ld + a]);
  }
}

// One workgroup of NT threads: FP64 trace of rho_d, lost probability,
// sink and renormalisation factor of one step (see the file comment).
template <typename T, int NT>
__device__ __forceinline__ void trace_body(const DissArgs<T> &p, double *s_tr, double *s_lost,
                                           double *s_rot) {
  // tr rho_d = sum_u rho_d[u,u] = sum_w trw[w] Z[w,w]: the jump terms
  // c_j[u]^2 Z[pi_j u, pi_j u] regrouped by the state w = pi_j u they read
  const int tid = thread_index();
  double tr = 0.0, lost = 0.0, rot = 0.0;
  // the lost probability's off-diagonal terms (restricted sparse channels):
  // lost += value Re Z[col,row], and the trace loses dt times the same
  for (int64_t e = tid; e < p.n_loff; e += NT) {
    double zr, zi;
    zlower(p, p.loff_col[e], p.loff_row[e], zr, zi);
    const double x = p.loff_val[e] * zr;
    lost += x;
    tr -= p.dt * x;
  }
  // u = tid + k NT in increasing k; the loads of G values of k are
  // issued together (one batch at N = 2048), the sums keep that order
  constexpr int G = 8;
  for (int64_t u0 = tid; u0 < p.n; u0 += int64_t(G) * NT) {
    double z[G], wk[G], lk[G];
#pragma unroll
    for (int gi = 0; gi < G; ++gi) {
      const int64_t u = u0 + int64_t(gi) * NT;
      const bool ok = u < p.n;
      z[gi] = !ok ? 0.0 : p.zdiag ? p.zdiag[u] : double(p.z_re[u * p.ld + u]);
      wk[gi] = ok ? p.trw[u] : 0.0;
      lk[gi] = ok ? p.leak[u] : 0.0;
    }
#pragma unroll
    for (int gi = 0; gi < G; ++gi) {
      tr += wk[gi] * z[gi];
      lost += lk[gi] * z[gi];
      rot += z[gi];
    }
  }
  // wave sums by butterfly (every lane ends with the same value), then the
  // NT / 64 wave sums in wave order
  for (int off = 32; off > 0; off >>= 1) {
    tr += __shfl_xor(tr, off);
    lost += __shfl_xor(lost, off);
    rot += __shfl_xor(rot, off);
  }
  if ((tid & 63) == 0) {
    s_tr[tid >> 6] = tr;
    s_lost[tid >> 6] = lost;
    s_rot[tid >> 6] = rot;
  }
  __syncthreads();
  if (tid == 0) {
    double t = s_tr[0], l = s_lost[0], r = s_rot[0];
    for (int w = 1; w < NT / 64; ++w) {
      t += s_tr[w];
      l += s_lost[w];
      r += s_rot[w];
    }
    const double sink = p.aux_in[0] + p.dt * l;
    const double steps = p.aux_in[3] + 1.0;
    p.aux_out[0] = sink;
    p.aux_out[1] = r;
    p.aux_out[2] = l;
    p.aux_out[3] = steps;
    p.aux_out[4] = (1.0 - sink) / t;
  }
}

// Gather tables of up to kGatherChunk channels for one tile's rows (u) and
// columns (v), staged in LDS once per tile.
constexpr int kGatherChunk = 8;
struct GatherLds {
  int32_t pu[kGatherChunk][TD], pv[kGatherChunk][TD];
  double cu[kGatherChunk][TD], cv[kGatherChunk][TD];
};

// One TD x TD lower-triangle tile t of the decoherence pass (256 threads);
// s_re / s_im: LDS staging of TD x (TD + 1) elements for the mirrored write;
// g: LDS for the gather tables (used when 0 < n_gather <= kGatherChunk).
// SPARSE: the variant with the sparse channels' terms (DissArgs::n_csr,
// koff); models without them take the other, which needs fewer registers.
template <typename T, bool SPARSE = false>
__device__ __forceinline__ void dissipate_tile(const DissArgs<T> &p, int t, T (*s_re)[TD + 1],
                                               T (*s_im)[TD + 1], GatherLds *g) {
  int bi = int((sqrtf(8.0f * float(t) + 1.0f) - 1.0f) * 0.5f);
  while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
  while (bi * (bi + 1) / 2 > t) --bi;
  const int bj = t - bi * (bi + 1) / 2;
  const bool diag_tile = bi == bj;
  const double scale = p.aux_out[4];
  const double dt = p.dt;
  const int tid = thread_index();
  const int c = tid & (TD - 1);
  const int r0 = tid / TD;
  const int64_t v = int64_t(bj) * TD + c;
  const bool staged = p.n_gather > 0 && p.n_gather <= kGatherChunk;
  if (staged) {
    for (int e = tid; e < p.n_gather * TD; e += kDissThreads) {
      const int j = e / TD, i = e - (e / TD) * TD;
      const int64_t u = int64_t(bi) * TD + i, w = int64_t(bj) * TD + i;
      const int64_t base = int64_t(j) * p.n;
      g->pu[j][i] = u < p.n ? p.pi[base + u] : -1;
      g->cu[j][i] = u < p.n ? p.cg[base + u] : 0.0;
      g->pv[j][i] = w < p.n ? p.pi[base + w] : -1;
      g->cv[j][i] = w < p.n ? p.cg[base + w] : 0.0;
    }
    __syncthreads();
  }

  double dv = 0.0;
  if (v < p.n) dv = p.d[v];
  // G of this thread's rows at a time (rows r0 + kRows * i): all their loads
  // (the element, its row's rate, then each channel's gathered elements) are
  // issued before any of them is used, so a thread keeps G requests in
  // flight; each element's arithmetic is unchanged.
  constexpr int kRows = kDissThreads / TD;
  constexpr int G = 4;
  for (int rb = r0; rb < TD; rb += kRows * G) {
    bool ok[G];
    double xr[G], xi[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const int rr = rb + q * kRows;
      const int64_t u = int64_t(bi) * TD + rr;
      ok[q] = rr < TD && u < p.n && v < p.n && !(diag_tile && v > u);
      double zr = 0.0, zi = 0.0, du = 0.0;
      if (ok[q]) {
        const int64_t o = u * p.ld + v;
        zr = double(p.z_re[o]);
        zi = double(p.z_im[o]);
        du = p.d[u];
      }
      const double f = 1.0 - 0.5 * dt * (du + dv);
      xr[q] = f * zr;
      xi[q] = f * zi;
    }
    for (int j = 0; j < p.n_gather; ++j) {
      double gr[G], gi[G], w[G];
      bool use[G];
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const int rr = rb + q * kRows;
        const int64_t u = int64_t(bi) * TD + rr;
        int32_t pu = -1, pv = -1;
        double cu = 0.0, cv = 0.0;
        if (ok[q]) {
          if (staged) {
            pu = g->pu[j][rr];
            pv = g->pv[j][c];
            cu = g->cu[j][rr];
            cv = g->cv[j][c];
          } else {
            pu = p.pi[int64_t(j) * p.n + u];
            pv = p.pi[int64_t(j) * p.n + v];
            cu = p.cg[int64_t(j) * p.n + u];
            cv = p.cg[int64_t(j) * p.n + v];
          }
        }
        use[q] = pu >= 0 && pv >= 0;
        w[q] = dt * cu * cv;
        gr[q] = gi[q] = 0.0;
        if (use[q]) zlower(p, pu, pv, gr[q], gi[q]);
      }
#pragma unroll
      for (int q = 0; q < G; ++q) {
        if (use[q]) {
          xr[q] += w[q] * gr[q];
          xi[q] += w[q] * gi[q];
        }
      }
    }
    if (SPARSE && (p.n_csr > 0 || p.koff_ptr)) {
      // sparse channels and K's off-diagonal part
#pragma unroll
      for (int q = 0; q < G; ++q) {
        if (!ok[q]) continue;
        const int64_t u = int64_t(bi) * TD + rb + q * kRows;
        double ar = 0.0, ai = 0.0;
        for (int ch = 0; ch < p.n_csr; ++ch) {
          const int64_t *ptr = p.csr_ptr + int64_t(ch) * (p.n + 1);
          double cr = 0.0, ci = 0.0;
          for (int64_t x = ptr[u]; x < ptr[u + 1]; ++x) {
            const int32_t k = p.csr_col[x];
            const double a = p.csr_val[x];
            for (int64_t y = ptr[v]; y < ptr[v + 1]; ++y) {
              double zr, zi;
              zlower(p, k, p.csr_col[y], zr, zi);
              const double w = a * p.csr_val[y];
              cr += w * zr;
              ci += w * zi;
            }
          }
          ar += p.csr_gamma[ch] * cr;
          ai += p.csr_gamma[ch] * ci;
        }
        if (p.koff_ptr) {
          double kr = 0.0, ki = 0.0;
          for (int64_t x = p.koff_ptr[u]; x < p.koff_ptr[u + 1]; ++x) {   // (K Z)[u,v]
            double zr, zi;
            zlower(p, p.koff_col[x], v, zr, zi);
            kr += p.koff_val[x] * zr;
            ki += p.koff_val[x] * zi;
          }
          for (int64_t y = p.koff_ptr[v]; y < p.koff_ptr[v + 1]; ++y) {   // (Z K)[u,v]
            double zr, zi;
            zlower(p, u, p.koff_col[y], zr, zi);
            kr += p.koff_val[y] * zr;
            ki += p.koff_val[y] * zi;
          }
          ar -= 0.5 * kr;
          ai -= 0.5 * ki;
        }
        xr[q] += dt * ar;
        xi[q] += dt * ai;
      }
    }
#pragma unroll
    for (int q = 0; q < G; ++q) {
      if (!ok[q]) continue;
      const int rr = rb + q * kRows;
      const int64_t u = int64_t(bi) * TD + rr;
      const int64_t o = u * p.ld + v;
      double yr = xr[q] * scale, yi = xi[q] * scale;
      if (u == v) yi = 0.0;
      p.x_re[o] = T(yr);
      p.x_im[o] = T(yi);
      if (diag_tile) {
        if (u != v) {
          p.x_re[v * p.ld + u] = T(yr);
          p.x_im[v * p.ld + u] = T(-yi);
        }
      } else {
        s_re[rr][c] = T(yr);
        s_im[rr][c] = T(yi);
      }
    }
  }
  if (diag_tile) return;
  __syncthreads();
  // mirror tile (bj, bi): element (a, b) = conj(X[bi*TD + b][bj*TD + a])
  const int64_t ucol = int64_t(bi) * TD + c;
  for (int a = r0; a < TD; a += kDissThreads / TD) {
    const int64_t vrow = int64_t(bj) * TD + a;
    if (vrow >= p.n || ucol >= p.n) continue;
    p.x_re[vrow * p.ld + ucol] = s_re[c][a];
    p.x_im[vrow * p.ld + ucol] = -s_im[c][a];
  }
}

}  // namespace qme
