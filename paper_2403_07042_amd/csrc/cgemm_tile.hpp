// Device-side bodies of the planar complex GEMM tiles (shared by the
// per-product kernels in cgemm.hip and the persistent batched step).
// See cgemm.hip for the operand forms and the design.
#pragma once

#include "device.hpp"

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef double doublex2 __attribute__((ext_vector_type(2)));

namespace qme {

static constexpr int kThreads = 256;   // 4 waves per tile

enum : int { kConjA = 1, kConjB = 2, kBRow = 4 };

// Tile index -> (bi, bj).  Block b runs on XCD b % 8, and each XCD has its
// own L2, so the mapping gives every XCD a compact block of output tiles
// whose operand row panels it can share:
//   full grid, tiles % 8 == 0: the 8 XCDs own a 4 x 2 grid of blocks of
//     (tiles/4) x (tiles/2) tiles; inside a block, groups of up to 8 tile
//     rows, column by column;
//   lower triangle, tiles % 8 == 0: a contiguous run of the triangle walked
//     in 8 x 8-tile super-blocks (row-major over the lower super-blocks,
//     triangular inside diagonal ones, column by column inside the others);
//   otherwise: XCD-contiguous runs of 4-row groups (full) or the plain
//     row-major triangle (lower).
// The mapping only reorders whole tiles: results do not depend on it.
__device__ __forceinline__ void tri_rowmajor(int t, int &r, int &c) {
  r = int((sqrtf(8.0f * float(t) + 1.0f) - 1.0f) * 0.5f);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  c = t - r * (r + 1) / 2;
}

__device__ __forceinline__ void tile_coords(int t, int tiles, bool lower, int &bi, int &bj) {
  if (lower) {
    const int nb = tiles * (tiles + 1) / 2;
    if ((tiles & 7) != 0 || (nb & 7) != 0) {
      tri_rowmajor(t, bi, bj);
      return;
    }
    int tt = (t & 7) * (nb >> 3) + (t >> 3);
    for (int sr = 0;; ++sr) {               // super-block row sr: sr off-diagonal + 1 diagonal
      const int row_tiles = sr * 64 + 36;
      if (tt >= row_tiles) { tt -= row_tiles; continue; }
      const int sc = tt / 64;
      if (sc < sr) {
        const int in = tt - sc * 64;
        bi = sr * 8 + (in & 7);
        bj = sc * 8 + (in >> 3);
      } else {
        int r, c;
        tri_rowmajor(tt - sr * 64, r, c);
        bi = sr * 8 + r;
        bj = sr * 8 + c;
      }
      return;
    }
  }
  const int nb = tiles * tiles;
  if ((tiles & 7) == 0) {
    const int x = t & 7, l = t >> 3;
    const int R = tiles >> 2, C = tiles >> 1;
    const int G = R < 8 ? R : 8;
    const int g = l / (G * C), in = l - g * (G * C);
    const int rows = min(G, R - g * G);
    bi = (x >> 1) * R + g * G + in % rows;
    bj = (x & 1) * C + in / rows;
    return;
  }
  int tt = t;
  if ((nb & 7) == 0) tt = (t & 7) * (nb >> 3) + (t >> 3);
  const int group = 4;
  int gsz = group * tiles;
  int g = tt / gsz;
  int first = g * group;
  int rows = min(group, tiles - first);
  int in = tt - g * gsz;
  bi = first + in % rows;
  bj = in / rows;
}

// Work of one block of a product launch.  Blocks [0, full) are whole tiles
// (tile index = block).  With a split (S > 1) the remaining tiles are cut
// along k: block full + q computes k-chunk q % S (K-tile iterations
// [s*nk/S, (s+1)*nk/S)) of tile full + q / S and writes its raw accumulator
// to partial slot q; a reduce pass sums the S slots of a tile in chunk order.
struct TileWork {
  int tile, kb, ke, slot;   // slot < 0: whole tile, normal epilogue
};
__device__ __forceinline__ TileWork tile_work(int b, int nk, int full, int S) {
  if (S <= 1 || b < full) return {b, 0, nk, -1};
  const int q = b - full, s = q % S;
  return {full + q / S, s * nk / S, (s + 1) * nk / S, q};
}

// One complex multiply-add in three real products (Gauss's 3M form) with
// the conjugations folded into the operand sums; A' = Ar + i sA Ai,
// B' = Br + i sB Bi:
//   P1 += Ar Br,   P2 += Ai Bi,   P3 += (Ar + sA Ai)(Br + sB Bi)
//   Re A'B' = P1 - sA sB P2,      Im A'B' = P3 - P1 - sA sB P2
// (combine3 forms the two after the k loop; both are linear in the
// accumulators, so k-chunk partials can be combined before they are summed).
// asum / bsum: Ar + sA Ai and Br + sB Bi, formed once per fragment.
template <typename V, typename S, typename F>
__device__ __forceinline__ void cmac3(V &p1, V &p2, V &p3, S ar, S ai, S asum, S br, S bi, S bsum,
                                      F mfma) {
  p1 = mfma(ar, br, p1);
  p2 = mfma(ai, bi, p2);
  p3 = mfma(asum, bsum, p3);
}
template <int OPS, typename V>
__device__ __forceinline__ void combine3(const V &p1, const V &p2, const V &p3, V &cr, V &ci) {
  constexpr bool flip = bool(OPS & kConjA) != bool(OPS & kConjB);   // sA sB = -1
  if (flip) {
    cr = p1 + p2;
    ci = (p3 - p1) + p2;
  } else {
    cr = p1 - p2;
    ci = (p3 - p1) - p2;
  }
}
template <int OPS, typename S>
__device__ __forceinline__ S opsum_a(S r, S i) { return (OPS & kConjA) ? r - i : r + i; }
template <int OPS, typename S>
__device__ __forceinline__ S opsum_b(S r, S i) { return (OPS & kConjB) ? r - i : r + i; }

// Value of one output element: alpha acc + beta X, or with a device scale
// s (the previous step's renormalisation) s acc + s X formed in FP64.
// The epilogues load a block's X elements before they store any of its
// results: C may alias X as far as the compiler knows, so a load placed
// after a store waits for it, and one load per element would cost one
// memory round trip per element.
template <typename T>
__device__ __forceinline__ void epi_load_x(const CgemmArgs<T> &p, bool has_x, int64_t o, T &xr,
                                           T &xi) {
  xr = has_x ? p.x_re[o] : T(0);
  xi = has_x ? p.x_im[o] : T(0);
}

// epi_value with the X element already loaded (the same arithmetic)
template <typename T>
__device__ __forceinline__ void epi_combine(const CgemmArgs<T> &p, bool has_x, bool scaled, double s,
                                            T ar, T ai, T x_r, T x_i, T &vr, T &vi) {
  if (scaled) {
    double xr = s * double(ar), xi = s * double(ai);
    if (has_x) {
      xr += s * double(x_r);
      xi += s * double(x_i);
    }
    vr = T(xr);
    vi = T(xi);
  } else {
    vr = p.alpha * ar;
    vi = p.alpha * ai;
    if (has_x) {
      vr += p.beta * x_r;
      vi += p.beta * x_i;
    }
  }
}

template <typename T>
__device__ __forceinline__ void epi_value(const CgemmArgs<T> &p, bool has_x, bool scaled, double s,
                                          int64_t o, T ar, T ai, T &vr, T &vi) {
  if (scaled) {
    double xr = s * double(ar), xi = s * double(ai);
    if (has_x) {
      xr += s * double(p.x_re[o]);
      xi += s * double(p.x_im[o]);
    }
    vr = T(xr);
    vi = T(xi);
  } else {
    vr = p.alpha * ar;
    vi = p.alpha * ai;
    if (has_x) {
      vr += p.beta * p.x_re[o];
      vi += p.beta * p.x_im[o];
    }
  }
}

// Folded decoherence epilogue of a lower-triangle tile (see CgemmArgs):
// element (rl, cl) of tile (bi, bj) with Z = (vr, vi).  The element is
// written and staged in LDS for the conjugate mirror; the strict upper part
// of a diagonal tile is left to fold_mirror.
// du, dv: fold_d of the element's row and column (0 past fold_n).
template <typename T, int BM>
__device__ __forceinline__ void fold_elem(const CgemmArgs<T> &p, int bi, int bj, int rl, int cl,
                                          T vr, T vi, double du, double dv, T (*s_re)[BM + 1],
                                          T (*s_im)[BM + 1]) {
  if (bi == bj && cl > rl) return;
  const int64_t row = int64_t(bi) * BM + rl, col = int64_t(bj) * BM + cl;
  const double zr = double(vr), zi = double(vi);
  const double f = 1.0 - 0.5 * p.fold_dt * (du + dv);
  double xr = f * zr, xi = f * zi;
  if (row == col) {
    xi = 0.0;
    if (row < p.fold_n) p.zdiag[row] = zr;
  }
  const int64_t o = row * p.ld + col;
  p.c_re[o] = T(xr);
  p.c_im[o] = T(xi);
  s_re[rl][cl] = T(xr);
  s_im[rl][cl] = T(xi);
}

// The conjugate mirror of a folded tile from its LDS copy (after a barrier):
// element (bj*BM + a, bi*BM + b) = conj(tile[b][a]), rows written contiguously.
template <typename T, int BM>
__device__ __forceinline__ void fold_mirror(const CgemmArgs<T> &p, int bi, int bj,
                                            T (*s_re)[BM + 1], T (*s_im)[BM + 1]) {
  for (int idx = thread_index(); idx < BM * BM; idx += kThreads) {
    const int a = idx / BM, b = idx - (idx / BM) * BM;
    if (bi == bj && b <= a) continue;
    const int64_t o = (int64_t(bj) * BM + a) * p.ld + int64_t(bi) * BM + b;
    p.c_re[o] = s_re[b][a];
    p.c_im[o] = -s_im[b][a];
  }
}

// ----------------------------------------------------------------- FP32
// v_mfma_f32_32x32x2_f32: A 32x2 (lane l: row l%32, k-slot l/32), B 2x32
// (lane l: k-slot l/32, col l%32), D 32x32 in 16 registers (lane l: col l%32,
// register r: row 8*(r/4) + 4*(l/32) + r%4).


// Slot of the k-chunks (4 floats) of LDS row r in the unpadded A / NT-B
// layout of the direct-load tile (16 floats per row): chunk c sits at slot
// c ^ dma_swz(r).
__device__ __forceinline__ int dma_swz(int r) { return ((r >> 1) & 3) ^ ((r >> 3) & 1); }

// The FP64 tiles' rows of 16 doubles (eight 16-byte chunks): chunk c of row
// r at slot c ^ f64_swz(r), distinct bank groups for the 8 (or 16)
// consecutive rows one 128-bit read phase serves on a 32- (or 64-) bank LDS.
__device__ __forceinline__ int f64_swz(int r) { return (r & 7) ^ ((r >> 3) & 1); }

// LDS elements a tile body needs (A and B tiles, double-buffered, re/im).
template <int BM, int OPS>
constexpr int cgemm_f32_smem() {
  constexpr int KT = 16, LDK = KT + 4, LDJ = BM + 4;
  constexpr int BSZ = (OPS & kBRow) ? KT * LDJ : BM * LDK;
  return 4 * BM * LDK + 4 * BSZ;
}
// (at least the folded epilogue's staging: the tile, BM + 1 per row, and
// the row and column factors)
// (16x16-MFMA tiles: rows of 128 bytes, KT = 16 doubles or 32 floats)
template <typename T, int BM, int OPS>
constexpr int cgemm_s_smem() {
  constexpr int E = 16 / sizeof(T), KT = 8 * E, LDK = KT, LDJ = BM + E;
  constexpr int BSZ = (OPS & kBRow) ? KT * LDJ : BM * LDK;
  constexpr int stages = 4 * BM * LDK + 4 * BSZ;
  constexpr int fold = 2 * BM * (BM + 1) + 2 * BM * int(sizeof(double) / sizeof(T));
  return stages > fold ? stages : fold;
}
template <int BM, int OPS>
constexpr int cgemm_f64_smem() { return cgemm_s_smem<double, BM, OPS>(); }

// Writes a finished FP32 tile: the raw accumulator into a split partial, or
// C = alpha * acc + beta * X, or the folded decoherence step (the operand LDS
// is free after the k loop's last barrier).
template <int BM, int OPS, bool FOLD, int F, int WM, int XG = 8>
__device__ __forceinline__ void f32_tile_epilogue(const CgemmArgs<float> &p, int bi, int bj,
                                                  float *smem, const floatx16 (&cr)[F][F],
                                                  const floatx16 (&ci)[F][F], float *part) {
  const int64_t ld = p.ld;
  const int tid = thread_index();
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 31, h = lane >> 5;
  if (part) {   // k-chunk of a split tile: raw accumulator, tile-local row-major
#pragma unroll
    for (int a = 0; a < F; ++a)
#pragma unroll
      for (int b = 0; b < F; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int o = (wm * WM + a * 32 + 8 * (r >> 2) + 4 * h + (r & 3)) * BM + wn * WM + b * 32 + li;
          part[o] = cr[a][b][r];
          part[BM * BM + o] = ci[a][b][r];
        }
    return;
  }
  // epilogue: C = alpha * acc + beta * X (or the folded decoherence step);
  // the operand LDS is free after the k loop's last barrier
  const bool has_x = p.beta != 0.0f;
  // the tile staged for the mirror (2 BM (BM + 1) elements) and the factors
  // d of its rows and columns (2 BM doubles) fit the operand LDS
  constexpr bool kCanFold =
      FOLD && 2 * BM * (BM + 1) * sizeof(float) + 2 * BM * sizeof(double) <=
                  cgemm_f32_smem<BM, OPS>() * sizeof(float);
  const bool fold = kCanFold && p.fold_d != nullptr;
  float (*f_re)[BM + 1] = reinterpret_cast<float (*)[BM + 1]>(smem);
  float (*f_im)[BM + 1] = reinterpret_cast<float (*)[BM + 1]>(smem + BM * (BM + 1));
  double *f_d = reinterpret_cast<double *>(smem + 2 * BM * (BM + 1));
  // the scale read once, before the stores (which could alias it)
  const bool scaled = p.scale != nullptr || p.scale_set;
  const double sc = p.scale ? *p.scale : p.scale_set ? p.scale_value : 1.0;
  if (fold) {
    if (tid < 2 * BM) {
      const int64_t u = tid < BM ? int64_t(bi) * BM + tid : int64_t(bj) * BM + tid - BM;
      f_d[tid] = u < p.fold_n ? p.fold_d[u] : 0.0;
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < F; ++a) {
#pragma unroll
    for (int b = 0; b < F; ++b) {
      const int cl = wn * WM + b * 32 + li;
      const int64_t col = int64_t(bj) * BM + cl;
      // X in groups of XG elements (XG registers a plane: the whole block's
      // would cost the four-waves-per-SIMD occupancy)
#pragma unroll
      for (int g = 0; g < 16; g += XG) {
      float xr[XG], xi[XG];
#pragma unroll
      for (int e = 0; e < XG; ++e) {
        const int r = g + e;
        const int64_t row = int64_t(bi) * BM + wm * WM + a * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        epi_load_x(p, has_x, row * ld + col, xr[e], xi[e]);
      }
#pragma unroll
      for (int e = 0; e < XG; ++e) {
        const int r = g + e;
        const int rl = wm * WM + a * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        const int64_t row = int64_t(bi) * BM + rl;
        const int64_t o = row * ld + col;
        float vr, vi;
        epi_combine(p, has_x, scaled, sc, cr[a][b][r], ci[a][b][r], xr[e], xi[e], vr, vi);
        if (fold) {
          fold_elem<float, BM>(p, bi, bj, rl, cl, vr, vi, f_d[rl], f_d[BM + cl], f_re, f_im);
        } else {
          p.c_re[o] = vr;
          p.c_im[o] = vi;
        }
      }
      }
    }
  }
  if (fold) {
    __syncthreads();
    fold_mirror<float, BM>(p, bi, bj, f_re, f_im);
  }
}

// FOLD: the kernel may apply the folded decoherence epilogue (lower-triangle
// launches; see CgemmArgs::fold_d).
template <int BM, int OPS, bool FOLD = false>
__device__ __forceinline__ void cgemm_f32_tile(const CgemmArgs<float> &p, int bi, int bj, float *smem,
                                               int kb = 0, int ke = -1, float *part = nullptr) {
  constexpr bool BROW = OPS & kBRow;
  constexpr int KT = 16;
  constexpr int LDK = KT + 4;          // padded LDS row of A / NT-B (floats)
  constexpr int LDJ = BM + 4;          // padded LDS row of NN-B (floats)
  constexpr int WM = BM / 2;           // wave tile
  constexpr int F = WM / 32;           // 32x32 blocks per wave side
  constexpr int PASSES = BM / 64;      // 64 rows per load pass (4 float4 per row)
  constexpr int BSZ = BROW ? KT * LDJ : BM * LDK;
  constexpr int BPASS = BROW ? (KT * BM / 4) / kThreads : PASSES;
  float (*sA)[2][BM * LDK] = reinterpret_cast<float (*)[2][BM * LDK]>(smem);
  float (*sB)[2][BSZ] = reinterpret_cast<float (*)[2][BSZ]>(smem + 4 * BM * LDK);

  const int64_t ld = p.ld;
  const int tid = thread_index();
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 31, h = lane >> 5;

  const int lr = tid >> 2, lk = (tid & 3) * 4;
  const float *ga_re = p.a_re + (int64_t(bi) * BM + lr) * ld + lk;
  const float *ga_im = p.a_im + (int64_t(bi) * BM + lr) * ld + lk;
  // NT: rows j of M;  NN: rows k of B, columns bj*BM + ...
  const int br_k = tid / (BM / 4), br_j = (tid % (BM / 4)) * 4;
  const float *gb_re = BROW ? p.m_re + int64_t(br_k) * ld + int64_t(bj) * BM + br_j
                            : p.m_re + (int64_t(bj) * BM + lr) * ld + lk;
  const float *gb_im = BROW ? p.m_im + int64_t(br_k) * ld + int64_t(bj) * BM + br_j
                            : p.m_im + (int64_t(bj) * BM + lr) * ld + lk;

  floatx4 ra[PASSES][2], rb[BPASS > 0 ? BPASS : 1][2];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PASSES; ++q) {
      const int64_t off = int64_t(q) * 64 * ld + k0;
      ra[q][0] = *reinterpret_cast<const floatx4 *>(ga_re + off);
      ra[q][1] = *reinterpret_cast<const floatx4 *>(ga_im + off);
    }
#pragma unroll
    for (int q = 0; q < BPASS; ++q) {
      const int64_t off = BROW ? (int64_t(k0) + q * (kThreads / (BM / 4))) * ld
                               : int64_t(q) * 64 * ld + k0;
      rb[q][0] = *reinterpret_cast<const floatx4 *>(gb_re + off);
      rb[q][1] = *reinterpret_cast<const floatx4 *>(gb_im + off);
    }
  };
  auto lstore = [&](int st) {
#pragma unroll
    for (int q = 0; q < PASSES; ++q) {
      const int o = (q * 64 + lr) * LDK + lk;
      *reinterpret_cast<floatx4 *>(&sA[st][0][o]) = ra[q][0];
      *reinterpret_cast<floatx4 *>(&sA[st][1][o]) = ra[q][1];
    }
#pragma unroll
    for (int q = 0; q < BPASS; ++q) {
      const int o = BROW ? (br_k + q * (kThreads / (BM / 4))) * LDJ + br_j
                         : (q * 64 + lr) * LDK + lk;
      *reinterpret_cast<floatx4 *>(&sB[st][0][o]) = rb[q][0];
      *reinterpret_cast<floatx4 *>(&sB[st][1][o]) = rb[q][1];
    }
  };

  floatx16 p1[F][F], p2[F][F], p3[F][F];
#pragma unroll
  for (int a = 0; a < F; ++a)
#pragma unroll
    for (int b = 0; b < F; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) { p1[a][b][r] = 0.0f; p2[a][b][r] = 0.0f; p3[a][b][r] = 0.0f; }

  auto mfma = [](float x, float y, floatx16 acc) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, acc, 0, 0, 0);
  };

  const int nk = ke < 0 ? int(ld / KT) : ke;
  gload(kb * KT);
  lstore(0);
  __syncthreads();
  for (int kt = kb; kt < nk; ++kt) {
    const int st = (kt - kb) & 1;
    // wave priority by progress: a workgroup in an earlier quarter of its k
    // loop issues before one further along (co-resident workgroups would
    // otherwise finish in dispatch order, the last ones at low occupancy)
    if (p.rank_prio) {
      switch (((kt - kb) * 4) / (nk - kb)) {
        case 0: __builtin_amdgcn_s_setprio(3); break;
        case 1: __builtin_amdgcn_s_setprio(2); break;
        case 2: __builtin_amdgcn_s_setprio(1); break;
        default: __builtin_amdgcn_s_setprio(0); break;
      }
    }
    if (kt + 1 < nk) gload((kt + 1) * KT);
    float ar[F][8], ai[F][8], br[F][8], bi_[F][8];
#pragma unroll
    for (int f = 0; f < F; ++f) {
      const int oa = (wm * WM + f * 32 + li) * LDK + h * 8;
      floatx4 x0 = *reinterpret_cast<const floatx4 *>(&sA[st][0][oa]);
      floatx4 x1 = *reinterpret_cast<const floatx4 *>(&sA[st][0][oa + 4]);
      floatx4 y0 = *reinterpret_cast<const floatx4 *>(&sA[st][1][oa]);
      floatx4 y1 = *reinterpret_cast<const floatx4 *>(&sA[st][1][oa + 4]);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        ar[f][e] = x0[e]; ar[f][e + 4] = x1[e];
        ai[f][e] = y0[e]; ai[f][e + 4] = y1[e];
      }
      if constexpr (BROW) {
        const int col = wn * WM + f * 32 + li;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          br[f][s] = sB[st][0][(h * 8 + s) * LDJ + col];
          bi_[f][s] = sB[st][1][(h * 8 + s) * LDJ + col];
        }
      } else {
        const int om = (wn * WM + f * 32 + li) * LDK + h * 8;
        floatx4 z0 = *reinterpret_cast<const floatx4 *>(&sB[st][0][om]);
        floatx4 z1 = *reinterpret_cast<const floatx4 *>(&sB[st][0][om + 4]);
        floatx4 w0 = *reinterpret_cast<const floatx4 *>(&sB[st][1][om]);
        floatx4 w1 = *reinterpret_cast<const floatx4 *>(&sB[st][1][om + 4]);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          br[f][e] = z0[e]; br[f][e + 4] = z1[e];
          bi_[f][e] = w0[e]; bi_[f][e + 4] = w1[e];
        }
      }
    }
    float as_[F][8], bs_[F][8];
#pragma unroll
    for (int f = 0; f < F; ++f)
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        as_[f][s] = opsum_a<OPS>(ar[f][s], ai[f][s]);
        bs_[f][s] = opsum_b<OPS>(br[f][s], bi_[f][s]);
      }
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int a = 0; a < F; ++a)
#pragma unroll
        for (int b = 0; b < F; ++b)
          cmac3(p1[a][b], p2[a][b], p3[a][b], ar[a][s], ai[a][s], as_[a][s], br[b][s], bi_[b][s],
                bs_[b][s], mfma);
    if (kt + 1 < nk) lstore(st ^ 1);
    __syncthreads();
  }
  floatx16 cr[F][F], ci[F][F];
#pragma unroll
  for (int a = 0; a < F; ++a)
#pragma unroll
    for (int b = 0; b < F; ++b) combine3<OPS>(p1[a][b], p2[a][b], p3[a][b], cr[a][b], ci[a][b]);

  f32_tile_epilogue<BM, OPS, FOLD, F, WM>(p, bi, bj, smem, cr, ci, part);
}

// NT forms with direct global -> LDS loads (global_load_lds_dwordx4: each
// wave instruction writes 64 lanes x 16 bytes to one contiguous 1 KB of LDS,
// lane L at base + 16 L).  A stage holds, per operand and plane, BM rows of
// KT = 16 floats without padding; the k-chunk c (4 floats) of row r sits at
// slot c ^ dma_swz(r), which puts the 8 (or 16) consecutive rows that one
// 128-bit read phase serves on distinct 16-byte bank groups of a 32-bank (or
// 64-bank) LDS; the swizzle is applied on the load side by choosing which
// global chunk each lane fetches.  Per K tile a wave reads its fragments,
// starts the loads of the next K tile into the other stage (its reads of that
// stage ended before the last barrier), runs its products, waits for its
// loads and meets the others at one barrier.  Each lane's fragments hold the
// same k values as in cgemm_f32_tile, so the two bodies give bitwise-identical
// results.
template <int BM, int OPS, bool FOLD = false>
__device__ __forceinline__ void cgemm_f32_tile_dma(const CgemmArgs<float> &p, int bi, int bj,
                                                   float *smem, int kb = 0, int ke = -1,
                                                   float *part = nullptr) {
  static_assert(!(OPS & kBRow), "direct loads serve the NT forms");
  constexpr int KT = 16;
  constexpr int WM = BM / 2;
  constexpr int F = WM / 32;
  constexpr int PLANE = BM * KT;                  // floats per operand plane per stage
  constexpr int STAGE = 4 * PLANE;                // A re, A im, B re, B im
  static_assert(2 * STAGE <= cgemm_f32_smem<BM, OPS>(), "stages exceed the LDS allocation");
  typedef __attribute__((address_space(1))) void gvoid;
  typedef __attribute__((address_space(3))) void lvoid;

  const int64_t ld = p.ld;
  const int tid = thread_index();
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 31, h = lane >> 5;

  // this lane's load: row (16 per wave instruction, BM / 64 instructions per
  // plane and wave) and the logical chunk that belongs at its slot
  const int lrow = lane >> 2;
  const int lchunk = (lane & 3) ^ dma_swz(lrow);     // rows come in aligned 16s
  constexpr int PASS = BM / 64;                   // rows 16 * (4 * q + wave) + lrow, q < PASS
  auto issue = [&](int st, int k0) {
    float *base = smem + st * STAGE;
#pragma unroll
    for (int q = 0; q < PASS; ++q) {
      const int r = 16 * (4 * q + wave) + lrow;
      const int64_t ga = (int64_t(bi) * BM + r) * ld + k0 + 4 * lchunk;
      const int64_t gb = (int64_t(bj) * BM + r) * ld + k0 + 4 * lchunk;
      const int lo = 16 * (4 * q + wave) * KT;    // this wave's 1 KB block
      __builtin_amdgcn_global_load_lds((gvoid *)(p.a_re + ga), (lvoid *)(base + lo), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((gvoid *)(p.a_im + ga), (lvoid *)(base + PLANE + lo), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((gvoid *)(p.m_re + gb), (lvoid *)(base + 2 * PLANE + lo), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((gvoid *)(p.m_im + gb), (lvoid *)(base + 3 * PLANE + lo), 16, 0, 0);
    }
  };

  floatx16 p1[F][F], p2[F][F], p3[F][F];
#pragma unroll
  for (int a = 0; a < F; ++a)
#pragma unroll
    for (int b = 0; b < F; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) { p1[a][b][r] = 0.0f; p2[a][b][r] = 0.0f; p3[a][b][r] = 0.0f; }
  auto mfma = [](float x, float y, floatx16 acc) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, acc, 0, 0, 0);
  };

  const int nk = ke < 0 ? int(ld / KT) : ke;
  issue(0, kb * KT);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int kt = kb; kt < nk; ++kt) {
    const int st = (kt - kb) & 1;
    const float *base = smem + st * STAGE;
    float ar[F][8], ai[F][8], br[F][8], bi_[F][8];
#pragma unroll
    for (int f = 0; f < F; ++f) {
      const int ra_ = wm * WM + f * 32 + li, swa = dma_swz(ra_);
      const int rb_ = wn * WM + f * 32 + li, swb = dma_swz(rb_);
      const int a0 = ra_ * KT + 4 * ((2 * h) ^ swa), a1 = ra_ * KT + 4 * ((2 * h + 1) ^ swa);
      const int b0 = rb_ * KT + 4 * ((2 * h) ^ swb), b1 = rb_ * KT + 4 * ((2 * h + 1) ^ swb);
      const floatx4 x0 = *reinterpret_cast<const floatx4 *>(base + a0);
      const floatx4 x1 = *reinterpret_cast<const floatx4 *>(base + a1);
      const floatx4 y0 = *reinterpret_cast<const floatx4 *>(base + PLANE + a0);
      const floatx4 y1 = *reinterpret_cast<const floatx4 *>(base + PLANE + a1);
      const floatx4 z0 = *reinterpret_cast<const floatx4 *>(base + 2 * PLANE + b0);
      const floatx4 z1 = *reinterpret_cast<const floatx4 *>(base + 2 * PLANE + b1);
      const floatx4 w0 = *reinterpret_cast<const floatx4 *>(base + 3 * PLANE + b0);
      const floatx4 w1 = *reinterpret_cast<const floatx4 *>(base + 3 * PLANE + b1);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        ar[f][e] = x0[e]; ar[f][e + 4] = x1[e];
        ai[f][e] = y0[e]; ai[f][e + 4] = y1[e];
        br[f][e] = z0[e]; br[f][e + 4] = z1[e];
        bi_[f][e] = w0[e]; bi_[f][e + 4] = w1[e];
      }
    }
    if (kt + 1 < nk) issue(st ^ 1, (kt + 1) * KT);
    float as_[F][8], bs_[F][8];
#pragma unroll
    for (int f = 0; f < F; ++f)
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        as_[f][s] = opsum_a<OPS>(ar[f][s], ai[f][s]);
        bs_[f][s] = opsum_b<OPS>(br[f][s], bi_[f][s]);
      }
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int a = 0; a < F; ++a)
#pragma unroll
        for (int b = 0; b < F; ++b)
          cmac3(p1[a][b], p2[a][b], p3[a][b], ar[a][s], ai[a][s], as_[a][s], br[b][s], bi_[b][s],
                bs_[b][s], mfma);
    // keep the products ahead of the wait (the scheduler would hoist the
    // barrier over them and expose the load latency)
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  floatx16 cr[F][F], ci[F][F];
#pragma unroll
  for (int a = 0; a < F; ++a)
#pragma unroll
    for (int b = 0; b < F; ++b) combine3<OPS>(p1[a][b], p2[a][b], p3[a][b], cr[a][b], ci[a][b]);
  f32_tile_epilogue<BM, OPS, FOLD, F, WM>(p, bi, bj, smem, cr, ci, part);
}

// ------------------------------------------- 16x16-MFMA tiles (FP64, FP32)
// v_mfma_f64_16x16x4_f64 / v_mfma_f32_16x16x4_f32: A 16x4 (lane l: row l%16,
// k-slot l/16), B 4x16 (lane l: k-slot l/16, col l%16), D 16x16 in 4
// registers (lane l: col l%16; register r: row l/16 + 4*r for f64, row
// 4*(l/16) + r for f32).  LDS rows are 128 bytes (16 doubles or 32 floats:
// eight 16-byte chunks, swizzled); each lane reads two chunks per K tile, in
// two halves with one half's fragments live.

template <typename T>
__device__ __forceinline__ int s_row(int h, int r) {
  return sizeof(T) == 8 ? h + 4 * r : 4 * h + r;
}

// Writes a finished 16x16-MFMA tile (the layout of cgemm_s_tile): the raw
// accumulator into a split partial, or C = alpha * acc + beta * X, or the
// folded decoherence step (FITS: the LDS at smem holds its staging).
template <typename T, int BM, int OPS, bool FOLD, int F, int WM, bool FITS>
__device__ __forceinline__ void s_tile_epilogue(const CgemmArgs<T> &p, int bi, int bj, T *smem,
                                                const T __attribute__((ext_vector_type(4))) (&cr)[F][F],
                                                const T __attribute__((ext_vector_type(4))) (&ci)[F][F],
                                                T *part) {
  const int64_t ld = p.ld;
  const int tid = thread_index();
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, h = lane >> 4;

  if (part) {   // k-chunk of a split tile: raw accumulator, tile-local row-major
#pragma unroll
    for (int a = 0; a < F; ++a)
#pragma unroll
      for (int b = 0; b < F; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int o = (wm * WM + a * 16 + s_row<T>(h, r)) * BM + wn * WM + b * 16 + li;
          part[o] = cr[a][b][r];
          part[BM * BM + o] = ci[a][b][r];
        }
    return;
  }
  const bool has_x = p.beta != T(0);
  constexpr bool kCanFold = FOLD && FITS;
  const bool fold = kCanFold && p.fold_d != nullptr;
  T (*f_re)[BM + 1] = reinterpret_cast<T (*)[BM + 1]>(smem);
  T (*f_im)[BM + 1] = reinterpret_cast<T (*)[BM + 1]>(smem + BM * (BM + 1));
  double *f_d = reinterpret_cast<double *>(smem + 2 * BM * (BM + 1));
  const bool scaled = p.scale != nullptr || p.scale_set;
  const double sc = p.scale ? *p.scale : p.scale_set ? p.scale_value : 1.0;
  if (fold) {
    if (tid < 2 * BM) {
      const int64_t u = tid < BM ? int64_t(bi) * BM + tid : int64_t(bj) * BM + tid - BM;
      f_d[tid] = u < p.fold_n ? p.fold_d[u] : 0.0;
    }
    __syncthreads();
  }
  T xr[F][F][4], xi[F][F][4];
#pragma unroll
  for (int a = 0; a < F; ++a)
#pragma unroll
    for (int b = 0; b < F; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = int64_t(bi) * BM + wm * WM + a * 16 + s_row<T>(h, r);
        const int64_t col = int64_t(bj) * BM + wn * WM + b * 16 + li;
        epi_load_x(p, has_x, row * ld + col, xr[a][b][r], xi[a][b][r]);
      }
#pragma unroll
  for (int a = 0; a < F; ++a) {
#pragma unroll
    for (int b = 0; b < F; ++b) {
      const int cl = wn * WM + b * 16 + li;
      const int64_t col = int64_t(bj) * BM + cl;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rl = wm * WM + a * 16 + s_row<T>(h, r);
        const int64_t row = int64_t(bi) * BM + rl;
        const int64_t o = row * ld + col;
        T vr, vi;
        epi_combine(p, has_x, scaled, sc, cr[a][b][r], ci[a][b][r], xr[a][b][r], xi[a][b][r], vr, vi);
        if (fold) {
          fold_elem<T, BM>(p, bi, bj, rl, cl, vr, vi, f_d[rl], f_d[BM + cl], f_re, f_im);
        } else {
          p.c_re[o] = vr;
          p.c_im[o] = vi;
        }
      }
    }
  }
  if (fold) {
    __syncthreads();
    fold_mirror<T, BM>(p, bi, bj, f_re, f_im);
  }
}

template <typename T, int BM, int OPS, bool FOLD = false>
__device__ __forceinline__ void cgemm_s_tile(const CgemmArgs<T> &p, int bi, int bj, T *smem,
                                             int kb = 0, int ke = -1, T *part = nullptr) {
  constexpr bool BROW = OPS & kBRow;
  constexpr int E = 16 / sizeof(T);    // elements per 16-byte chunk
  constexpr int KT = 8 * E;            // K tile: one 128-byte row
  constexpr int LDK = KT;              // LDS row of A / NT-B, 16-byte chunks swizzled
  constexpr int LDJ = BM + E;
  constexpr int WM = BM / 2;
  constexpr int F = WM / 16;           // 16x16 blocks per wave side
  constexpr int PASSES = BM / 32;      // 32 rows per pass (8 chunks per row)
  constexpr int BSZ = BROW ? KT * LDJ : BM * LDK;
  constexpr int BPASS = BROW ? (KT * BM / E) / kThreads : PASSES;
  constexpr int BSTEP = kThreads / (BM / E);   // NN-B rows per load pass
  typedef T vec __attribute__((ext_vector_type(E)));
  typedef T acc4 __attribute__((ext_vector_type(4)));
  T (*sA)[2][BM * LDK] = reinterpret_cast<T (*)[2][BM * LDK]>(smem);
  T (*sB)[2][BSZ] = reinterpret_cast<T (*)[2][BSZ]>(smem + 4 * BM * LDK);

  const int64_t ld = p.ld;
  const int tid = thread_index();
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, h = lane >> 4;

  const int lr = tid >> 3, lk = (tid & 7) * E;
  const T *ga_re = p.a_re + (int64_t(bi) * BM + lr) * ld + lk;
  const T *ga_im = p.a_im + (int64_t(bi) * BM + lr) * ld + lk;
  const int br_k = tid / (BM / E), br_j = (tid % (BM / E)) * E;
  const T *gb_re = BROW ? p.m_re + int64_t(br_k) * ld + int64_t(bj) * BM + br_j
                        : p.m_re + (int64_t(bj) * BM + lr) * ld + lk;
  const T *gb_im = BROW ? p.m_im + int64_t(br_k) * ld + int64_t(bj) * BM + br_j
                        : p.m_im + (int64_t(bj) * BM + lr) * ld + lk;

  vec ra[PASSES][2], rb[BPASS > 0 ? BPASS : 1][2];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PASSES; ++q) {
      const int64_t off = int64_t(q) * 32 * ld + k0;
      ra[q][0] = *reinterpret_cast<const vec *>(ga_re + off);
      ra[q][1] = *reinterpret_cast<const vec *>(ga_im + off);
    }
#pragma unroll
    for (int q = 0; q < BPASS; ++q) {
      const int64_t off = BROW ? (int64_t(k0) + q * BSTEP) * ld : int64_t(q) * 32 * ld + k0;
      rb[q][0] = *reinterpret_cast<const vec *>(gb_re + off);
      rb[q][1] = *reinterpret_cast<const vec *>(gb_im + off);
    }
  };
  auto lstore = [&](int st) {
#pragma unroll
    for (int q = 0; q < PASSES; ++q) {
      const int o = (q * 32 + lr) * LDK + E * ((lk / E) ^ f64_swz(q * 32 + lr));
      *reinterpret_cast<vec *>(&sA[st][0][o]) = ra[q][0];
      *reinterpret_cast<vec *>(&sA[st][1][o]) = ra[q][1];
    }
#pragma unroll
    for (int q = 0; q < BPASS; ++q) {
      const int o = BROW ? (br_k + q * BSTEP) * LDJ + br_j
                         : (q * 32 + lr) * LDK + E * ((lk / E) ^ f64_swz(q * 32 + lr));
      *reinterpret_cast<vec *>(&sB[st][0][o]) = rb[q][0];
      *reinterpret_cast<vec *>(&sB[st][1][o]) = rb[q][1];
    }
  };

  acc4 p1[F][F], p2[F][F], p3[F][F];
#pragma unroll
  for (int a = 0; a < F; ++a)
#pragma unroll
    for (int b = 0; b < F; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) { p1[a][b][r] = T(0); p2[a][b][r] = T(0); p3[a][b][r] = T(0); }

  auto mfma = [](T x, T y, acc4 acc) {
    if constexpr (sizeof(T) == 8)
      return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc, 0, 0, 0);
    else
      return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, acc, 0, 0, 0);
  };

  const int nk = ke < 0 ? int(ld / KT) : ke;
  gload(kb * KT);
  lstore(0);
  __syncthreads();
  for (int kt = kb; kt < nk; ++kt) {
    const int st = (kt - kb) & 1;
    if (kt + 1 < nk) gload((kt + 1) * KT);
    // two halves of the K tile (lane k values 2hE .. 2hE + E - 1, then the
    // next E), one half's fragments live at a time
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
      T ar[F][E], ai[F][E], br[F][E], bi_[F][E];
#pragma unroll
      for (int f = 0; f < F; ++f) {
        const int ra_ = wm * WM + f * 16 + li;
        const int oa = ra_ * LDK + E * ((2 * h + hf) ^ f64_swz(ra_));
        const vec x = *reinterpret_cast<const vec *>(&sA[st][0][oa]);
        const vec y = *reinterpret_cast<const vec *>(&sA[st][1][oa]);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          ar[f][e] = x[e];
          ai[f][e] = y[e];
        }
        if constexpr (BROW) {
          const int col = wn * WM + f * 16 + li;
#pragma unroll
          for (int e = 0; e < E; ++e) {
            br[f][e] = sB[st][0][(h * 2 * E + hf * E + e) * LDJ + col];
            bi_[f][e] = sB[st][1][(h * 2 * E + hf * E + e) * LDJ + col];
          }
        } else {
          const int rb_ = wn * WM + f * 16 + li;
          const int om = rb_ * LDK + E * ((2 * h + hf) ^ f64_swz(rb_));
          const vec z = *reinterpret_cast<const vec *>(&sB[st][0][om]);
          const vec w = *reinterpret_cast<const vec *>(&sB[st][1][om]);
#pragma unroll
          for (int e = 0; e < E; ++e) {
            br[f][e] = z[e];
            bi_[f][e] = w[e];
          }
        }
      }
      T as_[F][E], bs_[F][E];
#pragma unroll
      for (int f = 0; f < F; ++f)
#pragma unroll
        for (int e = 0; e < E; ++e) {
          as_[f][e] = opsum_a<OPS>(ar[f][e], ai[f][e]);
          bs_[f][e] = opsum_b<OPS>(br[f][e], bi_[f][e]);
        }
#pragma unroll
      for (int e = 0; e < E; ++e)
#pragma unroll
        for (int a = 0; a < F; ++a)
#pragma unroll
          for (int b = 0; b < F; ++b)
            cmac3(p1[a][b], p2[a][b], p3[a][b], ar[a][e], ai[a][e], as_[a][e], br[b][e], bi_[b][e],
                  bs_[b][e], mfma);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (kt + 1 < nk) lstore(st ^ 1);
    __syncthreads();
  }
  acc4 cr[F][F], ci[F][F];
#pragma unroll
  for (int a = 0; a < F; ++a)
#pragma unroll
    for (int b = 0; b < F; ++b) combine3<OPS>(p1[a][b], p2[a][b], p3[a][b], cr[a][b], ci[a][b]);
  s_tile_epilogue<T, BM, OPS, FOLD, F, WM,
                  2 * BM * (BM + 1) + 2 * BM * int(sizeof(double) / sizeof(T)) <=
                      cgemm_s_smem<T, BM, OPS>()>(p, bi, bj, smem, cr, ci, part);
}

// FP32 32-tiles of small products (ld <= kPanelLd): the tile's whole row
// panels of A and M, every K tile, go straight into LDS at once
// (global_load_lds_dwordx4, each wave instruction one contiguous 1 KB, lane L
// at 16 L; the chunks placed as cgemm_s_tile places them), so the block waits
// for memory once instead of once per K tile; the K tiles are then
// multiplied with cgemm_s_tile's fragments and MFMA order and the tile
// written by its epilogue, so the results are bitwise those of cgemm_s_tile
// without a split.  `pre(p)` runs while the loads are in flight (the folded
// steps' trace; it may set the epilogue's factor in its copy of the args).
constexpr int cgemm_panel_smem() { return 4 * 32 * kPanelLd; }   // floats (96 KB)

template <int OPS, bool FOLD, typename Pre>
__device__ __forceinline__ void cgemm_s_panel(const CgemmArgs<float> &args, int bi, int bj,
                                              float *smem, Pre pre) {
  CgemmArgs<float> p = args;
  static_assert(!(OPS & kBRow), "whole-panel loads serve the NT forms");
  using T = float;
  constexpr int BM = 32, E = 4, KT = 32, LDK = KT, WM = 16, F = 1;
  constexpr int PLANE = BM * LDK;       // floats of one operand plane of one K tile
  constexpr int STAGE = 4 * PLANE;      // A re, A im, M re, M im
  typedef T vec __attribute__((ext_vector_type(E)));
  typedef T acc4 __attribute__((ext_vector_type(4)));
  typedef __attribute__((address_space(1))) void gvoid;
  typedef __attribute__((address_space(3))) void lvoid;

  const int64_t ld = p.ld;
  const int nk = int(ld / KT);
  const int tid = thread_index();
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, h = lane >> 4;
  {
    // wave w fills rows 8w .. 8w + 7 of every plane and K tile: lane L at
    // row 8w + L / 8, slot L % 8, which holds chunk (L % 8) ^ f64_swz(row)
    const int row = 8 * wave + (lane >> 3);
    const int chunk = (lane & 7) ^ f64_swz(row);
    const int64_t ga = (int64_t(bi) * BM + row) * ld + E * chunk;
    const int64_t gb = (int64_t(bj) * BM + row) * ld + E * chunk;
    for (int kt = 0; kt < nk; ++kt) {
      float *base = smem + kt * STAGE + 8 * wave * LDK;
      const int64_t k0 = int64_t(kt) * KT;
      __builtin_amdgcn_global_load_lds((gvoid *)(p.a_re + ga + k0), (lvoid *)(base), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((gvoid *)(p.a_im + ga + k0), (lvoid *)(base + PLANE), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((gvoid *)(p.m_re + gb + k0), (lvoid *)(base + 2 * PLANE), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((gvoid *)(p.m_im + gb + k0), (lvoid *)(base + 3 * PLANE), 16, 0, 0);
    }
  }
  pre(p);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  acc4 p1[F][F], p2[F][F], p3[F][F];
#pragma unroll
  for (int a = 0; a < F; ++a)
#pragma unroll
    for (int b = 0; b < F; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) { p1[a][b][r] = T(0); p2[a][b][r] = T(0); p3[a][b][r] = T(0); }
  auto mfma = [](T x, T y, acc4 acc) { return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, acc, 0, 0, 0); };

  for (int kt = 0; kt < nk; ++kt) {
    const T *sa_re = smem + kt * STAGE, *sa_im = sa_re + PLANE;
    const T *sb_re = sa_re + 2 * PLANE, *sb_im = sa_re + 3 * PLANE;
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
      T ar[F][E], ai[F][E], br[F][E], bi_[F][E];
#pragma unroll
      for (int f = 0; f < F; ++f) {
        const int ra_ = wm * WM + f * 16 + li;
        const int oa = ra_ * LDK + E * ((2 * h + hf) ^ f64_swz(ra_));
        const vec x = *reinterpret_cast<const vec *>(&sa_re[oa]);
        const vec y = *reinterpret_cast<const vec *>(&sa_im[oa]);
        const int rb_ = wn * WM + f * 16 + li;
        const int om = rb_ * LDK + E * ((2 * h + hf) ^ f64_swz(rb_));
        const vec z = *reinterpret_cast<const vec *>(&sb_re[om]);
        const vec w = *reinterpret_cast<const vec *>(&sb_im[om]);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          ar[f][e] = x[e];
          ai[f][e] = y[e];
          br[f][e] = z[e];
          bi_[f][e] = w[e];
        }
      }
      T as_[F][E], bs_[F][E];
#pragma unroll
      for (int f = 0; f < F; ++f)
#pragma unroll
        for (int e = 0; e < E; ++e) {
          as_[f][e] = opsum_a<OPS>(ar[f][e], ai[f][e]);
          bs_[f][e] = opsum_b<OPS>(br[f][e], bi_[f][e]);
        }
#pragma unroll
      for (int e = 0; e < E; ++e)
#pragma unroll
        for (int a = 0; a < F; ++a)
#pragma unroll
          for (int b = 0; b < F; ++b)
            cmac3(p1[a][b], p2[a][b], p3[a][b], ar[a][e], ai[a][e], as_[a][e], br[b][e], bi_[b][e],
                  bs_[b][e], mfma);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  __syncthreads();   // the panels are read before the epilogue may stage the fold there
  acc4 cr[F][F], ci[F][F];
#pragma unroll
  for (int a = 0; a < F; ++a)
#pragma unroll
    for (int b = 0; b < F; ++b) combine3<OPS>(p1[a][b], p2[a][b], p3[a][b], cr[a][b], ci[a][b]);
  s_tile_epilogue<T, BM, OPS, FOLD, F, WM, true>(p, bi, bj, smem, cr, ci, nullptr);
}

template <int BM, int OPS, bool FOLD = false>
__device__ __forceinline__ void cgemm_f64_tile(const CgemmArgs<double> &p, int bi, int bj, double *smem,
                                               int kb = 0, int ke = -1, double *part = nullptr) {
  cgemm_s_tile<double, BM, OPS, FOLD>(p, bi, bj, smem, kb, ke, part);
}

}  // namespace qme
