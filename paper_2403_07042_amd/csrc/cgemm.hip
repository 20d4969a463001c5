// Planar complex GEMM on CDNA4 matrix cores (gfx950).
//
//   C = alpha * opA(A) * opB(B) + beta * X
//
//   opA(A) = A or conj(A)                         (CONJ_A)
//   B by rows of M ("NT"):  opB = M^T or M^H       (CONJ_B), B[k][j] = M[j][k]
//   B row-major ("NN"):     opB = B or conj(B)     (CONJ_B), B[k][j] = B[k][j]
//
// The products of a time step ("unitary evolution" stage, Sec. IV.B /
// Table III) and of its adjoint, with dU = U - I so the identity part of U
// is added exactly through X:
//   forward  T     = rho + dU rho           A = dU,  M = rho (rho = rho^H)   NT, M^H
//            rho_u = T + T conj(dU)         A = T,   M = dU  (dU symmetric)  NT, M^H, lower
//   adjoint  X     = mu + conj(dU) mu       A = dU conj, M = mu (Hermitian)  NT, M^H
//            lam   = X + X dU               A = X,   M = dU                  NT, M^T, lower
//            G    += rho X                  A = rho, B = X                   NN
//
// Design (one workgroup per BM x BM output tile, 4 waves in a 2 x 2 grid):
//   * operands read by rows (k contiguous for A and NT-B, j contiguous for
//     NN-B) with 16-byte global loads, staged through double-buffered LDS;
//   * for A and NT-B the k index inside a K tile is permuted per lane group
//     so each lane fetches its k values with two ds_read_b128;
//   * FP32 has two tile bodies with the same arithmetic: loads staged
//     through registers into padded LDS rows, or loaded straight into
//     swizzled LDS rows (global_load_lds); launches with fewer blocks than
//     two per CU take the second (GemmOps::direct);
//   * FP64 rows are swizzled, unpadded, and each K tile's fragments are
//     read in two halves, which fits five waves per SIMD at 32-tiles;
//   * a complex multiply-add is three real MFMA products (Gauss's 3M form:
//     Ar Br, Ai Bi and (Ar + sA Ai)(Br + sB Bi), combined after the k loop),
//     25 % fewer matrix-core operations than the four-product form; the
//     conjugations fold into the operand sums and the final combination;
//   * LOWER launches only the tiles on or below the diagonal (Hermitian
//     output), in an XCD-aware order, with the tiles past the last full
//     wave of CUs cut along k (tail split) and, for folded steps, the
//     decoherence factor applied in the epilogue (CgemmArgs::fold_d);
//   * a launch with at most half as many tiles as CUs has every tile cut
//     along k (small-launch split); split tiles are summed in chunk order by
//     a reduce pass.
#include "cgemm_tile.hpp"
#include "dissipate_tile.hpp"   // trace_body: the folded steps' trace in the first product

#include <algorithm>

namespace qme {

// DIRECT: operands loaded straight into LDS (NT forms only).
template <int BM, int OPS, bool LOWER, bool DIRECT = false>
__global__ __launch_bounds__(kThreads) void cgemm_f32_kernel(CgemmArgs<float> p) {
  // 32-tiles: the 16x16-MFMA body (K tile 32); 64/128: the 32x32 bodies (K tile 16)
  constexpr int kSmem = BM == 32 ? cgemm_s_smem<float, 32, OPS>() : cgemm_f32_smem<BM, OPS>();
  __shared__ __align__(16) float smem[kSmem];
  static_assert(!DIRECT || (!(OPS & kBRow) && BM != 32), "direct loads serve the NT forms");
  // whole tile, or (split launches) one k-chunk of a tile into its partial slot
  const TileWork w = tile_work(blockIdx.x, int(p.ld / (BM == 32 ? 32 : 16)), p.full, p.split);
  int bi, bj;
  tile_coords(w.tile, int(p.ld / BM), LOWER, bi, bj);
  float *part = w.slot < 0 ? nullptr : p.part + size_t(w.slot) * 2 * BM * BM;
  if constexpr (BM == 32) {
    cgemm_s_tile<float, 32, OPS, LOWER>(p, bi, bj, smem, w.kb, w.ke, part);
  } else {
    auto run = [&](const CgemmArgs<float> &a) {
      if constexpr (DIRECT)
        cgemm_f32_tile_dma<BM, OPS, LOWER>(a, bi, bj, smem, w.kb, w.ke, part);
      else
        cgemm_f32_tile<BM, OPS, LOWER>(a, bi, bj, smem, w.kb, w.ke, part);
    };
    if (!LOWER && p.tr_aux) {
      // folded steps: the previous step's factor, summed here by every block
      // as the trace pass sums it (block 0 stores the scalars), in the
      // operand LDS before the k loop uses it; the epilogue takes it by value
      double *st = reinterpret_cast<double *>(smem);
      DissArgs<float> da{nullptr, nullptr, nullptr, nullptr, p.ld, p.tr_n, p.tr_dt, nullptr,
                         p.tr_leak, nullptr, nullptr, 0, p.tr_aux, p.tr_aux, p.tr_w, p.tr_zdiag};
      da.slot_in = p.tr_slot_in;
      da.slot_out = p.tr_slot_out;
      const double f = trace_body<float, kThreads>(da, st, st + kThreads / 64,
                                                   st + 2 * (kThreads / 64), blockIdx.x == 0);
      __syncthreads();                      // every thread has read it before the LDS is reused
      CgemmArgs<float> q = p;
      q.scale_value = f;
      q.scale_set = 1;
      run(q);
    } else {
      run(p);
    }
  }
}

// FP32 32-tiles of products with ld <= kPanelLd (never split): the whole
// row panels in LDS at once (cgemm_s_panel), one workgroup per CU.  With
// tr_aux (folded steps) every block forms the previous step's trace while
// its panel loads are in flight, as the 64-tile first products do.
template <int OPS, bool LOWER>
__global__ __launch_bounds__(kThreads) void cgemm_f32_panel_kernel(CgemmArgs<float> p) {
  __shared__ __align__(16) float smem[cgemm_panel_smem()];
  __shared__ double s_tr[3][kThreads / 64];
  int bi, bj;
  tile_coords(blockIdx.x, int(p.ld / 32), LOWER, bi, bj);
  cgemm_s_panel<OPS, LOWER>(p, bi, bj, smem, [&](CgemmArgs<float> &q) {
    if (LOWER || !q.tr_aux) return;
    DissArgs<float> da{nullptr, nullptr, nullptr, nullptr, q.ld, q.tr_n, q.tr_dt, nullptr,
                       q.tr_leak, nullptr, nullptr, 0, q.tr_aux, q.tr_aux, q.tr_w, q.tr_zdiag};
    da.slot_in = q.tr_slot_in;
    da.slot_out = q.tr_slot_out;
    q.scale_value = trace_body<float, kThreads>(da, s_tr[0], s_tr[1], s_tr[2], blockIdx.x == 0);
    q.scale_set = 1;
  });
}

template <int BM, int OPS, bool LOWER>
// five waves per SIMD for the 32-tile NT forms (the step's products); the
// forms reading B by rows need more registers and keep the default bound
__global__ __launch_bounds__(kThreads, (BM == 32 && !(OPS & kBRow)) ? 5 : 1) void cgemm_f64_kernel(
    CgemmArgs<double> p) {
  __shared__ double smem[cgemm_f64_smem<BM, OPS>()];
  const TileWork w = tile_work(blockIdx.x, int(p.ld / 16), p.full, p.split);
  int bi, bj;
  tile_coords(w.tile, int(p.ld / BM), LOWER, bi, bj);
  cgemm_f64_tile<BM, OPS, LOWER>(p, bi, bj, smem, w.kb, w.ke,
                                 w.slot < 0 ? nullptr : p.part + size_t(w.slot) * 2 * BM * BM);
}

// C = alpha * sum_s part[tile, s] + beta * X over the split tiles: one
// 64-thread block per (split tile, 64 * V elements).  The chunks are loaded
// in groups of 16 (one group for the split counts the planner makes) and X
// with the first group, so a block waits for one memory round trip before
// the additions, which run in chunk (k) order.
template <typename T, int BM, bool LOWER>
__global__ __launch_bounds__(64) void split_reduce_kernel(CgemmArgs<T> p) {
  constexpr int V = 16 / sizeof(T);
  constexpr int PER_TILE = BM * BM / (64 * V);
  constexpr int G = 16;
  typedef T vec __attribute__((ext_vector_type(V)));
  const int tl = blockIdx.x / PER_TILE;
  const int e = (blockIdx.x % PER_TILE) * 64 * V + threadIdx.x * V;
  int bi, bj;
  tile_coords(p.full + tl, int(p.ld / BM), LOWER, bi, bj);
  const int64_t o = (int64_t(bi) * BM + e / BM) * p.ld + int64_t(bj) * BM + e % BM;
  const bool has_x = p.beta != T(0);
  const T *src = p.part + size_t(tl) * p.split * 2 * BM * BM + e;
  vec lr[G], li[G];
  auto load_group = [&](int c0) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      // every load unconditional (a chunk past the last re-reads it; its
      // value is not added), so they are in flight together
      const int c = c0 + g < p.split ? c0 + g : p.split - 1;
      lr[g] = *reinterpret_cast<const vec *>(src + size_t(c) * 2 * BM * BM);
      li[g] = *reinterpret_cast<const vec *>(src + size_t(c) * 2 * BM * BM + BM * BM);
    }
  };
  load_group(0);
  // X behind the first group (one wait covers both), before any store (see
  // epi_load_x)
  T xr[V], xi[V];
#pragma unroll
  for (int v = 0; v < V; ++v) epi_load_x(p, has_x, o + v, xr[v], xi[v]);
  // the folded step's decay rates of the row and the V columns, loaded with
  // them too (indices clamped, the values chosen at use)
  const int rl = e / BM;
  const int64_t row = int64_t(bi) * BM + rl;
  double fu = 0.0, fv[V];
#pragma unroll
  for (int v = 0; v < V; ++v) fv[v] = 0.0;
  if (p.fold_d && p.fold_n > 0) {
    const int64_t last = p.fold_n - 1;
    fu = p.fold_d[row < last ? row : last];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int64_t col = int64_t(bj) * BM + e % BM + v;
      fv[v] = p.fold_d[col < last ? col : last];
    }
  }
  vec sr = vec(T(0)), si = vec(T(0));
  for (int c0 = 0;;) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (c0 + g < p.split) {
        sr += lr[g];
        si += li[g];
      }
    }
    c0 += G;
    if (c0 >= p.split) break;
    load_group(c0);
  }
  const bool scaled = p.scale != nullptr;
  const double sc = scaled ? *p.scale : 1.0;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    T vr, vi;
    epi_combine(p, has_x, scaled, sc, sr[v], si[v], xr[v], xi[v], vr, vi);
    if (!p.fold_d) {
      p.c_re[o + v] = vr;
      p.c_im[o + v] = vi;
      continue;
    }
    // folded decoherence step (as fold_elem), mirror written directly
    const int cl = e % BM + v;
    if (bi == bj && cl > rl) continue;
    const int64_t col = int64_t(bj) * BM + cl;
    const double zr = double(vr), zi = double(vi);
    const double du = row < p.fold_n ? fu : 0.0;
    const double dv = col < p.fold_n ? fv[v] : 0.0;
    const double f = 1.0 - 0.5 * p.fold_dt * (du + dv);
    double xr = f * zr, xi = f * zi;
    if (row == col) {
      xi = 0.0;
      if (row < p.fold_n) p.zdiag[row] = zr;
    }
    p.c_re[o + v] = T(xr);
    p.c_im[o + v] = T(xi);
    if (row != col) {
      p.c_re[col * p.ld + row] = T(xr);
      p.c_im[col * p.ld + row] = T(-xi);
    }
  }
}

// x *= *scale over a state's planes (FP64 product, rounded to T)
template <typename T>
__global__ __launch_bounds__(256) void apply_scale_kernel(T *re, T *im, int64_t elems,
                                                          const double *scale) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= elems) return;
  const double s = *scale;
  re[i] = T(s * double(re[i]));
  im[i] = T(s * double(im[i]));
}

template <typename T>
hipError_t launch_apply_scale(T *re, T *im, int64_t elems, const double *scale, hipStream_t s) {
  if (elems <= 0) return hipSuccess;
  return launch_kernel(apply_scale_kernel<T>, dim3(unsigned((elems + 255) / 256)), dim3(256), 0, s,
                       re, im, elems, scale);
}
template hipError_t launch_apply_scale<float>(float *, float *, int64_t, const double *, hipStream_t);
template hipError_t launch_apply_scale<double>(double *, double *, int64_t, const double *,
                                               hipStream_t);

SplitPlan plan_tail_split(int tiles, int bm, int kt, int64_t ld, int cus, size_t cap_elems) {
  SplitPlan sp;
  const int all = tiles * (tiles + 1) / 2;
  if (cus <= 0 || all <= cus) return sp;
  const int tail = all % cus;
  if (tail == 0) return sp;
  int s = std::min<int>(cus / tail, int(ld / kt));
  while (s >= 2 && size_t(tail) * s * 2 * bm * bm > cap_elems) --s;
  if (s < 2) return sp;
  sp.full = all - tail;
  sp.split = s;
  return sp;
}

SplitPlan plan_small_split(int blocks, int bm, int kt, int64_t ld, int cus, size_t cap_elems) {
  SplitPlan sp;
  if (cus <= 0 || blocks <= 0 || 2 * blocks > cus) return sp;
  int s = std::min<int>(cus / blocks, int(ld / kt) / 2);
  while (s >= 2 && size_t(blocks) * s * 2 * bm * bm > cap_elems) --s;
  if (s < 2) return sp;
  sp.full = 0;
  sp.split = s;
  return sp;
}

template <typename T, bool LOWER>
static hipError_t split_reduce_tile(const CgemmArgs<T> &a, int tile, dim3 grid, hipStream_t s) {
  const dim3 block(64);
  if (tile == 128) return launch_kernel(split_reduce_kernel<T, 128, LOWER>, grid, block, 0, s, a);
  if (tile == 64) return launch_kernel(split_reduce_kernel<T, 64, LOWER>, grid, block, 0, s, a);
  if (tile == 32) return launch_kernel(split_reduce_kernel<T, 32, LOWER>, grid, block, 0, s, a);
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_split_reduce(const CgemmArgs<T> &a, int tile, bool lower, hipStream_t s) {
  if (a.split < 2) return hipSuccess;
  const int tiles = int(a.ld / tile);
  const int tail = (lower ? tiles * (tiles + 1) / 2 : tiles * tiles) - a.full;
  const int per_tile = tile * tile / (64 * int(16 / sizeof(T)));
  if (tail <= 0 || per_tile <= 0) return hipErrorInvalidValue;
  const dim3 grid(unsigned(tail * per_tile));
  return lower ? split_reduce_tile<T, true>(a, tile, grid, s)
               : split_reduce_tile<T, false>(a, tile, grid, s);
}
template hipError_t launch_split_reduce<float>(const CgemmArgs<float> &, int, bool, hipStream_t);
template hipError_t launch_split_reduce<double>(const CgemmArgs<double> &, int, bool, hipStream_t);

// ------------------------------------------------------------- launchers

template <typename Args, typename K>
static hipError_t launch(K kernel, const Args &a, int tile, bool lower, hipStream_t s) {
  const int tiles = int(a.ld / tile);
  int blocks = lower ? tiles * (tiles + 1) / 2 : tiles * tiles;
  if (blocks == 0) return hipSuccess;
  const bool split = a.split > 1;
  if (split) {
    if (!a.part || a.full < 0 || a.full >= blocks) return hipErrorInvalidValue;
    blocks = a.full + (blocks - a.full) * a.split;
  }
  hipError_t e = launch_kernel(kernel, dim3(blocks), dim3(kThreads), 0, s, a);
  if (e == hipSuccess && split) e = launch_split_reduce(a, tile, lower, s);
  return e;
}

#define QME_KERNEL_TABLE(NAME, ARGS)                                                          \
  template <int BM>                                                                           \
  static hipError_t NAME##_dispatch(const ARGS &a, int ops, bool lower, hipStream_t s) {      \
    switch (ops * 2 + (lower ? 1 : 0)) {                                                      \
      case 0: return launch(NAME<BM, 0, false>, a, BM, false, s);                             \
      case 1: return launch(NAME<BM, 0, true>, a, BM, true, s);                               \
      case 2: return launch(NAME<BM, 1, false>, a, BM, false, s);                             \
      case 3: return launch(NAME<BM, 1, true>, a, BM, true, s);                               \
      case 4: return launch(NAME<BM, 2, false>, a, BM, false, s);                             \
      case 5: return launch(NAME<BM, 2, true>, a, BM, true, s);                               \
      case 6: return launch(NAME<BM, 3, false>, a, BM, false, s);                             \
      case 7: return launch(NAME<BM, 3, true>, a, BM, true, s);                               \
      case 8: return launch(NAME<BM, 4, false>, a, BM, false, s);                             \
      case 9: return launch(NAME<BM, 4, true>, a, BM, true, s);                               \
      case 10: return launch(NAME<BM, 5, false>, a, BM, false, s);                            \
      case 11: return launch(NAME<BM, 5, true>, a, BM, true, s);                              \
      case 12: return launch(NAME<BM, 6, false>, a, BM, false, s);                            \
      case 13: return launch(NAME<BM, 6, true>, a, BM, true, s);                              \
      case 14: return launch(NAME<BM, 7, false>, a, BM, false, s);                            \
      case 15: return launch(NAME<BM, 7, true>, a, BM, true, s);                              \
    }                                                                                         \
    return hipErrorInvalidValue;                                                              \
  }

QME_KERNEL_TABLE(cgemm_f32_kernel, CgemmArgs<float>)
QME_KERNEL_TABLE(cgemm_f64_kernel, CgemmArgs<double>)
#undef QME_KERNEL_TABLE

static int ops_of(const GemmOps &o) {
  return (o.conj_a ? kConjA : 0) | (o.conj_b ? kConjB : 0) | (o.b_rows ? kBRow : 0);
}

template <int BM>
static hipError_t cgemm_f32_direct_dispatch(const CgemmArgs<float> &a, int ops, bool lower,
                                            hipStream_t s) {
  switch (ops * 2 + (lower ? 1 : 0)) {
    case 0: return launch(cgemm_f32_kernel<BM, 0, false, true>, a, BM, false, s);
    case 1: return launch(cgemm_f32_kernel<BM, 0, true, true>, a, BM, true, s);
    case 2: return launch(cgemm_f32_kernel<BM, 1, false, true>, a, BM, false, s);
    case 3: return launch(cgemm_f32_kernel<BM, 1, true, true>, a, BM, true, s);
    case 4: return launch(cgemm_f32_kernel<BM, 2, false, true>, a, BM, false, s);
    case 5: return launch(cgemm_f32_kernel<BM, 2, true, true>, a, BM, true, s);
    case 6: return launch(cgemm_f32_kernel<BM, 3, false, true>, a, BM, false, s);
    case 7: return launch(cgemm_f32_kernel<BM, 3, true, true>, a, BM, true, s);
  }
  return hipErrorInvalidValue;
}

// Whether a launch takes the direct-load tile body (see GemmOps::direct).
static bool use_direct(const CgemmArgs<float> &a, int tile, const GemmOps &o) {
  if (o.b_rows || o.direct == 0 || tile == 32) return false;
  if (o.direct > 0) return true;
  const int64_t tiles = a.ld / tile;
  int64_t blocks = o.lower ? tiles * (tiles + 1) / 2 : tiles * tiles;
  if (a.split > 1) blocks = a.full + (blocks - a.full) * a.split;
  return o.cus > 0 && blocks < 2 * int64_t(o.cus);
}

// Whether a tile's LDS holds the folded epilogue's staging (the condition
// the tile bodies test as kCanFold); a fold request elsewhere is an error,
// never a silent unfolded product.
template <int BM>
constexpr bool f32_folds() {
  return 2 * BM * (BM + 1) * sizeof(float) + 2 * BM * sizeof(double) <=
         (BM == 32 ? cgemm_s_smem<float, 32, kConjB>() : cgemm_f32_smem<BM, kConjB>()) * sizeof(float);
}
template <int BM>
constexpr bool f64_folds() {
  return 2 * BM * (BM + 1) + 2 * BM <= cgemm_f64_smem<BM, kConjB>();
}

static hipError_t cgemm_f32_panel_dispatch(const CgemmArgs<float> &a, int ops, bool lower,
                                           hipStream_t s) {
  switch (ops * 2 + (lower ? 1 : 0)) {
    case 0: return launch(cgemm_f32_panel_kernel<0, false>, a, 32, false, s);
    case 1: return launch(cgemm_f32_panel_kernel<0, true>, a, 32, true, s);
    case 2: return launch(cgemm_f32_panel_kernel<1, false>, a, 32, false, s);
    case 3: return launch(cgemm_f32_panel_kernel<1, true>, a, 32, true, s);
    case 4: return launch(cgemm_f32_panel_kernel<2, false>, a, 32, false, s);
    case 5: return launch(cgemm_f32_panel_kernel<2, true>, a, 32, true, s);
    case 6: return launch(cgemm_f32_panel_kernel<3, false>, a, 32, false, s);
    case 7: return launch(cgemm_f32_panel_kernel<3, true>, a, 32, true, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_cgemm_f32(const CgemmArgs<float> &args, int tile, const GemmOps &o, hipStream_t s) {
  if (args.ld % tile != 0) return hipErrorInvalidValue;
  // the trace inside the product: full 64- / 128-tile launches without a split
  // and whole-panel 32-tile ones
  const bool panel = tile == 32 && args.ld <= kPanelLd && !o.b_rows && args.split <= 1 && o.direct != 0;
  if (args.tr_aux && (o.lower || (tile == 32 && !panel) || args.split > 1 || args.scale || args.scale_set))
    return hipErrorInvalidValue;
  // progress-ranked wave priority for launches resident in one round (four
  // workgroups per CU at most; larger launches overlap their rounds anyway)
  CgemmArgs<float> a = args;
  {
    const int64_t tiles = a.ld / tile;
    int64_t blocks = o.lower ? tiles * (tiles + 1) / 2 : tiles * tiles;
    if (a.split > 1) blocks = a.full + (blocks - a.full) * a.split;
    a.rank_prio = o.cus > 0 && blocks <= 4 * int64_t(o.cus) ? 1 : 0;
  }
  if (a.fold_d && (!o.lower || o.b_rows ||
                   !(tile == 32 ? f32_folds<32>() : tile == 64 ? f32_folds<64>() : f32_folds<128>())))
    return hipErrorInvalidValue;
  const bool direct = use_direct(a, tile, o);
  if (tile == 128)
    return direct ? cgemm_f32_direct_dispatch<128>(a, ops_of(o), o.lower, s)
                  : cgemm_f32_kernel_dispatch<128>(a, ops_of(o), o.lower, s);
  if (tile == 64)
    return direct ? cgemm_f32_direct_dispatch<64>(a, ops_of(o), o.lower, s)
                  : cgemm_f32_kernel_dispatch<64>(a, ops_of(o), o.lower, s);
  if (tile == 32) {
    // small products: whole panels straight into LDS, unless register
    // staging is asked for (GemmOps::direct == 0)
    if (panel) return cgemm_f32_panel_dispatch(a, ops_of(o), o.lower, s);
    return cgemm_f32_kernel_dispatch<32>(a, ops_of(o), o.lower, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_cgemm_f64(const CgemmArgs<double> &a, int tile, const GemmOps &o, hipStream_t s) {
  if (a.ld % tile != 0) return hipErrorInvalidValue;
  if (a.fold_d && (!o.lower || o.b_rows || !(tile == 64 ? f64_folds<64>() : f64_folds<32>())))
    return hipErrorInvalidValue;
  if (tile == 64) return cgemm_f64_kernel_dispatch<64>(a, ops_of(o), o.lower, s);
  if (tile == 32) return cgemm_f64_kernel_dispatch<32>(a, ops_of(o), o.lower, s);
  return hipErrorInvalidValue;
}

}  // namespace qme
