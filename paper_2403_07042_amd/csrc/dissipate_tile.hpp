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
// Returns the factor to every thread; `write`: store the step's scalars.
template <typename T, int NT>
__device__ __forceinline__ double trace_body(const DissArgs<T> &p, double *s_tr, double *s_lost,
                                             double *s_rot, bool write = true) {
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
  // issued together (one batch at N = 2048), the sums keep that order.
  // Every load is unconditional (an index past n reads entry 0 and its
  // value is replaced by 0 after), so no branch makes a load wait.
  constexpr int G = 8;
  auto sums = [&](auto diag) {
    for (int64_t u0 = tid; u0 < p.n; u0 += int64_t(G) * NT) {
      double z[G], wk[G], lk[G];
#pragma unroll
      for (int gi = 0; gi < G; ++gi) {
        const int64_t u = u0 + int64_t(gi) * NT;
        const int64_t uc = u < p.n ? u : 0;
        z[gi] = diag(uc);
        wk[gi] = p.trw[uc];
        lk[gi] = p.leak[uc];
      }
#pragma unroll
      for (int gi = 0; gi < G; ++gi) {
        const bool ok = u0 + int64_t(gi) * NT < p.n;
        z[gi] = ok ? z[gi] : 0.0;
        wk[gi] = ok ? wk[gi] : 0.0;
        lk[gi] = ok ? lk[gi] : 0.0;
      }
#pragma unroll
      for (int gi = 0; gi < G; ++gi) {
        tr += wk[gi] * z[gi];
        lost += lk[gi] * z[gi];
        rot += z[gi];
      }
    }
  };
  if (p.zdiag)
    sums([&](int64_t u) { return p.zdiag[u]; });
  else
    sums([&](int64_t u) { return double(p.z_re[u * p.ld + u]); });
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
    const double sink = p.aux_in[sink_slot(p.slot_in)] + p.dt * l;
    const double steps = p.aux_in[steps_slot(p.slot_in)] + 1.0;
    const double scale = (1.0 - sink) / t;
    if (write) {
      p.aux_out[sink_slot(p.slot_out)] = sink;
      p.aux_out[1] = r;
      p.aux_out[2] = l;
      p.aux_out[steps_slot(p.slot_out)] = steps;
      p.aux_out[4] = scale;
    }
    s_tr[0] = scale;
  }
  __syncthreads();
  return s_tr[0];
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
//
// Each thread owns four consecutive columns of one row of the tile, so the
// rotated state is read and the new state written with 16-byte accesses;
// the tile is staged in LDS and its conjugate mirror (and, for a diagonal
// tile, its strict upper part) written row by row from there.  Gathered
// elements are loaded for two channels at a time before they are used, and
// a channel that maps the element onto itself (dephasing) reuses its value.
// Each element's arithmetic is that of the file comment, in channel order.
// scale_of(): the step's renormalisation factor, called by every thread.
// EARLY: call it once the tile's own elements and gather tables are in
// flight (when it forms the trace, its loads then overlap theirs); otherwise
// first (the values held across the call cost registers, which a factor that
// is only read need not pay).
template <typename T, bool SPARSE = false, bool EARLY = false, typename ScaleOf>
__device__ __forceinline__ void dissipate_tile(const DissArgs<T> &p, int t, ScaleOf scale_of,
                                               T (*s_re)[TD + 1], T (*s_im)[TD + 1],
                                               GatherLds *g) {
  typedef T vec4 __attribute__((ext_vector_type(4)));
  int bi = int((sqrtf(8.0f * float(t) + 1.0f) - 1.0f) * 0.5f);
  while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
  while (bi * (bi + 1) / 2 > t) --bi;
  const int bj = t - bi * (bi + 1) / 2;
  const bool diag_tile = bi == bj;
  const double dt = p.dt;
  const int tid = thread_index();
  const int r = tid >> 3;                 // row of the tile
  const int c0 = (tid & 7) * 4;           // first of the thread's four columns
  const int64_t ld = p.ld, n = p.n;
  const int64_t u = int64_t(bi) * TD + r;
  const int64_t v0 = int64_t(bj) * TD + c0;
  const bool staged = p.n_gather > 0 && p.n_gather <= kGatherChunk;
  double scale = 0.0;
  // the gather tables (every load unconditional: indices clamped into the
  // table, the value replaced after)
  static_assert(kGatherChunk * TD <= kDissThreads, "one table entry per thread");
  const bool stager = staged && tid < p.n_gather * TD;
  const int sj = tid / TD, si = tid - (tid / TD) * TD;
  const int64_t ta = int64_t(bi) * TD + si, tb = int64_t(bj) * TD + si;
  int32_t pa = -1, pb = -1;
  double ca = 0.0, cb = 0.0;
  if constexpr (EARLY) {
    // one entry per thread, held in registers across the factor
    if (stager) {
      const int64_t base = int64_t(sj) * n;
      const int64_t ac = ta < n ? ta : n - 1, bc = tb < n ? tb : n - 1;
      pa = p.pi[base + ac];
      pb = p.pi[base + bc];
      ca = p.cg[base + ac];
      cb = p.cg[base + bc];
    }
  } else {
    scale = scale_of();
    if (staged) {
      for (int e = tid; e < p.n_gather * TD; e += kDissThreads) {
        const int j = e / TD, i = e - (e / TD) * TD;
        const int64_t a = int64_t(bi) * TD + i, b = int64_t(bj) * TD + i;
        const int64_t base = int64_t(j) * n;
        const int64_t ac = a < n ? a : n - 1, bc = b < n ? b : n - 1;
        const int32_t la = p.pi[base + ac], lb = p.pi[base + bc];
        const double da = p.cg[base + ac], db = p.cg[base + bc];
        g->pu[j][i] = a < n ? la : -1;
        g->cu[j][i] = a < n ? da : 0.0;
        g->pv[j][i] = b < n ? lb : -1;
        g->cv[j][i] = b < n ? db : 0.0;
      }
      __syncthreads();
    }
  }

  // the four elements, the decay factors
  const bool row_ok = u < n;
  bool ok[4];
  T zr[4], zi[4];
  double xr[4], xi[4];
  if (row_ok && v0 + 3 < n) {
    const vec4 a = *reinterpret_cast<const vec4 *>(p.z_re + u * ld + v0);
    const vec4 b = *reinterpret_cast<const vec4 *>(p.z_im + u * ld + v0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      zr[i] = a[i];
      zi[i] = b[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool in = row_ok && v0 + i < n;
      zr[i] = in ? p.z_re[u * ld + v0 + i] : T(0);
      zi[i] = in ? p.z_im[u * ld + v0 + i] : T(0);
    }
  }
  const double du = row_ok ? p.d[u] : 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t v = v0 + i;
    ok[i] = row_ok && v < n && !(diag_tile && v > u);
    const double dv = v < n ? p.d[v] : 0.0;
    const double f = 1.0 - 0.5 * dt * ((ok[i] ? du : 0.0) + dv);
    xr[i] = f * (ok[i] ? double(zr[i]) : 0.0);
    xi[i] = f * (ok[i] ? double(zi[i]) : 0.0);
  }

  if constexpr (EARLY) {
    scale = scale_of();
    if (stager) {
      g->pu[sj][si] = ta < n ? pa : -1;
      g->cu[sj][si] = ta < n ? ca : 0.0;
      g->pv[sj][si] = tb < n ? pb : -1;
      g->cv[sj][si] = tb < n ? cb : 0.0;
    }
    if (staged) __syncthreads();
  }

  // monomial channels (gather form)
  if (staged) {
    constexpr int B = 2;
    for (int j0 = 0; j0 < p.n_gather; j0 += B) {
      T gr[B][4], gi[B][4];
      bool use[B][4];
      // the gathered elements: every load unconditional (an element not
      // needed reads Z[0][0]) and the values chosen after, so the 2 B x 4
      // loads of a thread are in flight together instead of one round trip
      // each behind the branches
      bool self[B][4], low[B][4];
#pragma unroll
      for (int jb = 0; jb < B; ++jb) {
        const bool ch = j0 + jb < p.n_gather;
        // (a channel that maps every state to itself reads nothing)
        const bool moves = ch && !((p.self_mask >> (j0 + jb)) & 1u);
        const int32_t pu = ch && row_ok ? g->pu[j0 + jb][r] : -1;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int32_t pv = ch && ok[i] ? g->pv[j0 + jb][c0 + i] : -1;
          use[jb][i] = pu >= 0 && pv >= 0;
          self[jb][i] = pu == u && pv == v0 + i;          // the element itself
          // element (pu, pv) of the Hermitian Z from its lower triangle
          low[jb][i] = pu >= pv;
          const int64_t o = !use[jb][i] || self[jb][i] ? 0
                            : low[jb][i]               ? int64_t(pu) * ld + pv
                                                       : int64_t(pv) * ld + pu;
          gr[jb][i] = gi[jb][i] = T(0);
          if (moves) {
            gr[jb][i] = p.z_re[o];
            gi[jb][i] = p.z_im[o];
          }
        }
      }
#pragma unroll
      for (int jb = 0; jb < B; ++jb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const T re = gr[jb][i], im = gi[jb][i];
          gr[jb][i] = !use[jb][i] ? T(0) : self[jb][i] ? zr[i] : re;
          gi[jb][i] = !use[jb][i] ? T(0) : self[jb][i] ? zi[i] : low[jb][i] ? im : -im;
        }
#pragma unroll
      for (int jb = 0; jb < B; ++jb) {
        if (j0 + jb >= p.n_gather) break;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (use[jb][i]) {
            const double w = dt * g->cu[j0 + jb][r] * g->cv[j0 + jb][c0 + i];
            xr[i] += w * double(gr[jb][i]);
            xi[i] += w * double(gi[jb][i]);
          }
        }
      }
    }
  } else {
    for (int j = 0; j < p.n_gather; ++j) {
      const int32_t pu = row_ok ? p.pi[int64_t(j) * n + u] : -1;
      const double cu = row_ok ? p.cg[int64_t(j) * n + u] : 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (!ok[i]) continue;
        const int64_t v = v0 + i;
        const int32_t pv = p.pi[int64_t(j) * n + v];
        if (pu < 0 || pv < 0) continue;
        const double w = dt * cu * p.cg[int64_t(j) * n + v];
        double gr, gi;
        zlower(p, pu, pv, gr, gi);
        xr[i] += w * gr;
        xi[i] += w * gi;
      }
    }
  }

  if (SPARSE && (p.n_csr > 0 || p.koff_ptr)) {
    // sparse channels and K's off-diagonal part
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (!ok[i]) continue;
      const int64_t v = v0 + i;
      double ar = 0.0, ai = 0.0;
      for (int ch = 0; ch < p.n_csr; ++ch) {
        const int64_t *ptr = p.csr_ptr + int64_t(ch) * (n + 1);
        double cr = 0.0, ci = 0.0;
        for (int64_t x = ptr[u]; x < ptr[u + 1]; ++x) {
          const int32_t k = p.csr_col[x];
          const double a = p.csr_val[x];
          for (int64_t y = ptr[v]; y < ptr[v + 1]; ++y) {
            double gr, gi;
            zlower(p, k, p.csr_col[y], gr, gi);
            const double w = a * p.csr_val[y];
            cr += w * gr;
            ci += w * gi;
          }
        }
        ar += p.csr_gamma[ch] * cr;
        ai += p.csr_gamma[ch] * ci;
      }
      if (p.koff_ptr) {
        double kr = 0.0, ki = 0.0;
        for (int64_t x = p.koff_ptr[u]; x < p.koff_ptr[u + 1]; ++x) {   // (K Z)[u,v]
          double gr, gi;
          zlower(p, p.koff_col[x], v, gr, gi);
          kr += p.koff_val[x] * gr;
          ki += p.koff_val[x] * gi;
        }
        for (int64_t y = p.koff_ptr[v]; y < p.koff_ptr[v + 1]; ++y) {   // (Z K)[u,v]
          double gr, gi;
          zlower(p, u, p.koff_col[y], gr, gi);
          kr += p.koff_val[y] * gr;
          ki += p.koff_val[y] * gi;
        }
        ar -= 0.5 * kr;
        ai -= 0.5 * ki;
      }
      xr[i] += dt * ar;
      xi[i] += dt * ai;
    }
  }

  // the scaled lower elements: to the state and to LDS for the mirror
  T yr[4], yi[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    yr[i] = T(xr[i] * scale);
    yi[i] = u == v0 + i ? T(0) : T(xi[i] * scale);
    s_re[r][c0 + i] = yr[i];
    s_im[r][c0 + i] = yi[i];
  }
  if (ok[0] && ok[1] && ok[2] && ok[3]) {
    vec4 a, b;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = yr[i];
      b[i] = yi[i];
    }
    *reinterpret_cast<vec4 *>(p.x_re + u * ld + v0) = a;
    *reinterpret_cast<vec4 *>(p.x_im + u * ld + v0) = b;
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (!ok[i]) continue;
      p.x_re[u * ld + v0 + i] = yr[i];
      p.x_im[u * ld + v0 + i] = yi[i];
    }
  }
  __syncthreads();
  // mirror: element (a, b) of tile (bj, bi) is conj(X[bi*TD + b][bj*TD + a]);
  // for a diagonal tile only its strict upper part (b > a)
  const int64_t mrow = int64_t(bj) * TD + r;       // row a = r of the mirror tile
  const int64_t mcol = int64_t(bi) * TD + c0;      // columns b = c0 .. c0 + 3
  if (mrow >= n) return;
  bool mok[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) mok[i] = mcol + i < n && (!diag_tile || c0 + i > r);
  T mr[4], mi[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    mr[i] = s_re[c0 + i][r];
    mi[i] = -s_im[c0 + i][r];
  }
  if (mok[0] && mok[1] && mok[2] && mok[3]) {
    vec4 a, b;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = mr[i];
      b[i] = mi[i];
    }
    *reinterpret_cast<vec4 *>(p.x_re + mrow * ld + mcol) = a;
    *reinterpret_cast<vec4 *>(p.x_im + mrow * ld + mcol) = b;
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (!mok[i]) continue;
      p.x_re[mrow * ld + mcol + i] = mr[i];
      p.x_im[mrow * ld + mcol + i] = mi[i];
    }
  }
}

}  // namespace qme
