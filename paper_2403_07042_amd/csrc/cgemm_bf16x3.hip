// Split-BF16x3 planar complex GEMM on CDNA4 matrix cores (gfx950).
//
//   C = alpha * opA(A) * opB(M^T) + beta * X     (FP32 in, FP32 out; "NT")
//
// Each FP32 value x is split, while its tile is staged into LDS, into three
// bf16 values x = hi + mid + lo + r with |r| <= 2^-24 |x| (round to nearest
// even at each stage).  A real product x*y is accumulated in FP32 from the
// six significant cross products
//   mid*mid, lo*hi, hi*lo, mid*hi, hi*mid, hi*hi      (smallest first);
// the dropped terms (mid*lo, lo*mid, lo*lo) are below 2^-24 |x y|.
// v_mfma_f32_32x32x16_bf16 does 16 k-terms per instruction, so the six
// products cost less than one FP32 MFMA sequence over the same k.
//
// Used for both products of a time step, in the same NT forms as the FP32
// kernel (A rows and M rows stream contiguous k; see cgemm.hip).
#include "cgemm_tile.hpp"
#include "dissipate_tile.hpp"   // trace_body: the folded steps' trace in the first product

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

namespace qme {

static constexpr int kThreads3 = 256;

typedef float float2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two values rounded to bf16 (nearest even) in one packed conversion;
// element 0 in the low half.
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  const float2v v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
__device__ __forceinline__ float bf16_lo(uint32_t u) { return __builtin_bit_cast(float, u << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t u) {
  return __builtin_bit_cast(float, u & 0xffff0000u);
}

// split3 of two values at once, as packed pairs (h, m, l): the same
// roundings as split3 element by element, one conversion per pair and stage.
__device__ __forceinline__ void split3_pair(float x0, float x1, uint32_t &h, uint32_t &m,
                                            uint32_t &l) {
  h = pack_bf16(x0, x1);
  const float r0 = x0 - bf16_lo(h), r1 = x1 - bf16_hi(h);
  m = pack_bf16(r0, r1);
  l = pack_bf16(r0 - bf16_lo(m), r1 - bf16_hi(m));
}

__device__ __forceinline__ void split3(float x, __bf16 &h, __bf16 &m, __bf16 &l) {
  h = __bf16(x);
  const float r1 = x - float(h);
  m = __bf16(r1);
  const float r2 = r1 - float(m);
  l = __bf16(r2);
}

// acc += x * y over the six significant split products; x[3], y[3] = hi, mid, lo
__device__ __forceinline__ floatx16 mac3(const bf16x8 *x, const bf16x8 *y, floatx16 acc) {
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[1], y[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[2], y[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[0], y[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[1], y[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[0], y[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[0], y[0], acc, 0, 0, 0);
  return acc;
}

// One workgroup per 64 x 64 output tile, 4 waves (2 x 2), each a 32 x 32
// block.  K tile 32 (two MFMA k-steps of 16).  LDS holds six bf16 planes
// (re/im x hi/mid/lo) per operand, single-buffered, rows unpadded with the
// k-chunks swizzled (48 KB: three workgroups per CU); the next K tile is
// prefetched into registers during the products.
// v_mfma_f32_32x32x16_bf16: A 32x16 (lane l: row l%32, k 8*(l/32)..+7),
// B 16x32 (lane l: k 8*(l/32)..+7, col l%32), D as for the FP32 32x32 MFMA.
// PRE: 0 both operands FP32 (split while staged), 1 first operand pre-split
// (a_split), 2 second operand pre-split (m_split).
// FOLD: the lower-triangle instantiation may apply the folded decoherence
// epilogue (CgemmArgs::fold_d), as the FP32 tiles do.
template <bool CONJA, bool CONJB, bool LOWER, int PRE, bool FOLD = false>
__global__ __launch_bounds__(kThreads3) void cgemm_bf16x3_kernel(CgemmArgs<float> p) {
  constexpr int BM = 64;
  constexpr int KT = 32;
  // LDS row (bf16): four 16-byte k-chunks, chunk c of row r at slot c ^ dma_swz(r)
  constexpr int LDK = KT;
  auto slot = [](int row, int c) { return 8 * (c ^ dma_swz(row)); };
  // one block for both operands: after the k loop the folded epilogue stages
  // its tile there (2 BM (BM + 1) floats and 2 BM doubles, 34 KB of 48 KB)
  __shared__ __align__(16) __bf16 lds[2][6][BM * LDK];
  __bf16 (*sA)[BM * LDK] = lds[0];
  __bf16 (*sB)[BM * LDK] = lds[1];

  const int tiles = int(p.ld / BM);
  int bi, bj, kb = 0, ke = int(p.ld / KT);
  float *part = nullptr;
  {
    int t = blockIdx.x;
    if (p.split > 1 && t >= p.full) {   // k-chunk of a split tile
      const int q = t - p.full, s = q % p.split, nk = int(p.ld / KT);
      t = p.full + q / p.split;
      kb = s * nk / p.split;
      ke = (s + 1) * nk / p.split;
      part = p.part + size_t(q) * 2 * BM * BM;
    }
    tile_coords(t, tiles, LOWER, bi, bj);
  }
  const int64_t ld = p.ld;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 31, h = lane >> 5;

  // loads: 64 rows x 32 k per plane = 512 float4, two per thread
  const int lr = tid >> 3, lk = (tid & 7) * 4;
  const float *src[4] = {p.a_re + (int64_t(bi) * BM + lr) * ld + lk,
                         p.a_im + (int64_t(bi) * BM + lr) * ld + lk,
                         p.m_re + (int64_t(bj) * BM + lr) * ld + lk,
                         p.m_im + (int64_t(bj) * BM + lr) * ld + lk};
  // a pre-split operand: 64 rows x 32 k per plane = 256 chunks of 8 bf16,
  // one per thread and plane
  const int pr = tid >> 2, pk = (tid & 3) * 8;
  const __bf16 *psrc = nullptr;
  if constexpr (PRE == 1)
    psrc = static_cast<const __bf16 *>(p.a_split) + (int64_t(bi) * BM + pr) * ld + pk;
  if constexpr (PRE == 2)
    psrc = static_cast<const __bf16 *>(p.m_split) + (int64_t(bj) * BM + pr) * ld + pk;
  const int64_t pstride = ld * ld;
  auto skip = [](int o) { return (PRE == 1 && o < 2) || (PRE == 2 && o >= 2); };
  floatx4 reg[4][2];
  bf16x8 preg[PRE ? 6 : 1];
  auto gload = [&](int k0) {
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      if (skip(o)) continue;
#pragma unroll
      for (int q = 0; q < 2; ++q)
        reg[o][q] = *reinterpret_cast<const floatx4 *>(src[o] + int64_t(q) * 32 * ld + k0);
    }
    if constexpr (PRE != 0) {
#pragma unroll
      for (int pl = 0; pl < 6; ++pl)
        preg[pl] = *reinterpret_cast<const bf16x8 *>(psrc + pl * pstride + k0);
    }
  };
  auto lstore = [&]() {
    if constexpr (PRE != 0) {
#pragma unroll
      for (int pl = 0; pl < 6; ++pl) {
        __bf16 *base = PRE == 1 ? &sA[pl][0] : &sB[pl][0];
        *reinterpret_cast<bf16x8 *>(base + pr * LDK + slot(pr, pk >> 3)) = preg[pl];
      }
    }
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      if (skip(o)) continue;
      __bf16 *base = (o < 2) ? &sA[(o & 1) * 3][0] : &sB[(o & 1) * 3][0];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        uint32_t vh[2], vm[2], vl[2];
        split3_pair(reg[o][q][0], reg[o][q][1], vh[0], vm[0], vl[0]);
        split3_pair(reg[o][q][2], reg[o][q][3], vh[1], vm[1], vl[1]);
        const int row = q * 32 + lr;
        const int off = row * LDK + slot(row, lk >> 3) + (lk & 7);
        *reinterpret_cast<uint2 *>(base + 0 * BM * LDK + off) = make_uint2(vh[0], vh[1]);
        *reinterpret_cast<uint2 *>(base + 1 * BM * LDK + off) = make_uint2(vm[0], vm[1]);
        *reinterpret_cast<uint2 *>(base + 2 * BM * LDK + off) = make_uint2(vl[0], vl[1]);
      }
    }
  };

  floatx16 cr, ci, crn, cin;   // crn / cin: the products of negative sign
#pragma unroll
  for (int r = 0; r < 16; ++r) { cr[r] = 0.0f; ci[r] = 0.0f; crn[r] = 0.0f; cin[r] = 0.0f; }

  gload(kb * KT);
  for (int kt = kb; kt < ke; ++kt) {
    __syncthreads();             // previous tile's fragments consumed
    lstore();
    __syncthreads();
    if (kt + 1 < ke) gload((kt + 1) * KT);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      bf16x8 ar[3], ai[3], br[3], bim[3];
      const int ra_ = wm * 32 + li, rb_ = wn * 32 + li;
      const int oa = ra_ * LDK + slot(ra_, 2 * s + h);
      const int ob = rb_ * LDK + slot(rb_, 2 * s + h);
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        ar[t] = *reinterpret_cast<const bf16x8 *>(&sA[t][oa]);
        ai[t] = *reinterpret_cast<const bf16x8 *>(&sA[3 + t][oa]);
        br[t] = *reinterpret_cast<const bf16x8 *>(&sB[t][ob]);
        bim[t] = *reinterpret_cast<const bf16x8 *>(&sB[3 + t][ob]);
      }
      // (Ar + i sA Ai)(Br + i sB Bi):
      //   Cr += Ar Br - sA sB Ai Bi,  Ci += sB Ar Bi + sA Ai Br
      // each product goes to the accumulator of its sign (no operand is
      // negated); the negative ones are subtracted once after the k loop
      cr = mac3(ar, br, cr);
      if constexpr (!CONJA) ci = mac3(ai, br, ci); else cin = mac3(ai, br, cin);
      if constexpr (CONJA != CONJB) cr = mac3(ai, bim, cr); else crn = mac3(ai, bim, crn);
      if constexpr (!CONJB) ci = mac3(ar, bim, ci); else cin = mac3(ar, bim, cin);
      // one k-step's fragments live at a time (hoisting the next step's
      // reads over these products costs 44 registers and a wave per SIMD)
      __builtin_amdgcn_sched_barrier(0);
    }
  }

#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if constexpr (CONJA == CONJB) cr[r] -= crn[r];
    if constexpr (CONJA || CONJB) ci[r] -= cin[r];
  }

  if (part) {   // raw accumulator of the chunk, tile-local row-major
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int o = (wm * 32 + 8 * (r >> 2) + 4 * h + (r & 3)) * BM + wn * 32 + li;
      part[o] = cr[r];
      part[BM * BM + o] = ci[r];
    }
    return;
  }
  if (p.scale || (FOLD && p.fold_d)) {
    // the FP64 scale or the folded decoherence step (folded steps): the FP32
    // tiles' epilogue (the 32 x 32 bf16 MFMA leaves its result in the FP32
    // 32 x 32 MFMA's layout); the fold stages its tile in the operand LDS
    // once every wave is done with it
    if (FOLD && p.fold_d) __syncthreads();
    const floatx16 acr[1][1] = {{cr}}, aci[1][1] = {{ci}};
    f32_tile_epilogue<BM, kConjB, FOLD, 1, 32>(p, bi, bj, reinterpret_cast<float *>(&lds[0][0][0]),
                                               acr, aci, nullptr);
    return;
  }
  const bool has_x = p.beta != 0.0f;
  const int64_t col = int64_t(bj) * BM + wn * 32 + li;
  float xr[16], xi[16];   // X loaded before any store (see epi_load_x)
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t row = int64_t(bi) * BM + wm * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
    epi_load_x(p, has_x, row * ld + col, xr[r], xi[r]);
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t row = int64_t(bi) * BM + wm * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
    const int64_t o = row * ld + col;
    float vr = p.alpha * cr[r], vi = p.alpha * ci[r];
    if (has_x) {
      vr += p.beta * xr[r];
      vi += p.beta * xi[r];
    }
    p.c_re[o] = vr;
    p.c_im[o] = vi;
  }
}

// Full-grid tile order of the wide first product (tr x tc tiles, block t
// dispatched to XCD t % 8): with tr % 4 == 0 and tc % 2 == 0 each XCD takes a
// (tr / 4) x (tc / 2) sub-grid walked column by column in groups of at most
// eight tile rows, so its workgroups share row and column panels in its L2;
// otherwise column-major groups of four tile rows.
__device__ __forceinline__ void wide_coords(int t, int tr, int tc, int &bi, int &bj) {
  if ((tr & 3) == 0 && (tc & 1) == 0) {
    const int x = t & 7, l = t >> 3;
    const int R = tr >> 2, C = tc >> 1;
    const int G = R < 8 ? R : 8;
    const int g = l / (G * C), in = l - g * (G * C);
    const int rows = min(G, R - g * G);
    bi = (x >> 1) * R + g * G + in % rows;
    bj = (x & 1) * C + in / rows;
    return;
  }
  const int gsz = 4 * tc, g = t / gsz, first = 4 * g;
  const int rows = min(4, tr - first), in = t - g * gsz;
  bi = first + in % rows;
  bj = in / rows;
}

// The first product of a time step, T = rho + dU rho in the NT form with M
// conjugated (dU pre-split as A), on 128 x 64 output tiles: 4 waves (2 x 2),
// each a 64 x 32 block of two 32 x 32 MFMA blocks that share the fragments
// of M, so a 16-k step reads 18 fragments from LDS for 48 MFMAs (the 64 x 64
// tile: 12 for 24).  LDS holds the six pre-split planes of 128 A rows and
// the six planes of 64 M rows split while staged (72 KB: two workgroups per
// CU, so a grid of twice the compute units runs in one round).  Per element
// the k order, the six products and the three accumulators are those of
// cgemm_bf16x3_kernel, and the epilogue is the FP32 tiles', so the two give
// bitwise-identical results.  With CgemmArgs::tr_aux (folded steps) every
// block first forms the previous step's trace as the trace pass does (block 0
// stores the scalars) and applies its factor as alpha = beta.
__global__ __launch_bounds__(kThreads3, 2) void cgemm_bf16x3_wide_kernel(CgemmArgs<float> p) {
  constexpr int BA = 128, BB = 64, KT = 32, LDK = KT;
  auto slot = [](int row, int c) { return 8 * (c ^ dma_swz(row)); };
  __shared__ __align__(16) __bf16 sA[6][BA * LDK];
  __shared__ __align__(16) __bf16 sB[6][BB * LDK];
  __shared__ double s_tr[3][kThreads3 / 64];
  bool scaled = p.scale != nullptr;
  double sc = 1.0;
  if (p.tr_aux) {
    DissArgs<float> da{nullptr, nullptr, nullptr, nullptr, p.ld, p.tr_n, p.tr_dt, nullptr,
                       p.tr_leak, nullptr, nullptr, 0, p.tr_aux, p.tr_aux, p.tr_w, p.tr_zdiag};
    da.slot_in = p.tr_slot_in;
    da.slot_out = p.tr_slot_out;
    sc = trace_body<float, kThreads3>(da, s_tr[0], s_tr[1], s_tr[2], blockIdx.x == 0);
    scaled = true;
  } else if (p.scale) {
    sc = *p.scale;
  }

  const int64_t ld = p.ld;
  int bi, bj;
  wide_coords(blockIdx.x, int(ld / BA), int(ld / BB), bi, bj);
  const int nk = int(ld / KT);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 31, h = lane >> 5;

  // A: 128 rows x 4 chunks of 8 bf16 per plane, two chunks per thread and
  // plane (rows pr and pr + 64); M: 64 rows x 32 k per FP32 plane, two
  // float4 per thread and plane (rows lr and lr + 32)
  const int pr = tid >> 2, pk = (tid & 3) * 8;
  const __bf16 *psrc = static_cast<const __bf16 *>(p.a_split) + (int64_t(bi) * BA + pr) * ld + pk;
  const int64_t pstride = ld * ld;
  const int lr = tid >> 3, lk = (tid & 7) * 4;
  const float *msrc[2] = {p.m_re + (int64_t(bj) * BB + lr) * ld + lk,
                          p.m_im + (int64_t(bj) * BB + lr) * ld + lk};
  bf16x8 preg[6][2];
  floatx4 reg[2][2];
  auto gload = [&](int k0) {
#pragma unroll
    for (int pl = 0; pl < 6; ++pl)
#pragma unroll
      for (int q = 0; q < 2; ++q)
        preg[pl][q] = *reinterpret_cast<const bf16x8 *>(psrc + pl * pstride + int64_t(q) * 64 * ld + k0);
#pragma unroll
    for (int o = 0; o < 2; ++o)
#pragma unroll
      for (int q = 0; q < 2; ++q)
        reg[o][q] = *reinterpret_cast<const floatx4 *>(msrc[o] + int64_t(q) * 32 * ld + k0);
  };
  auto lstore = [&]() {
#pragma unroll
    for (int pl = 0; pl < 6; ++pl)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int row = pr + 64 * q;
        *reinterpret_cast<bf16x8 *>(&sA[pl][row * LDK + slot(row, pk >> 3)]) = preg[pl][q];
      }
#pragma unroll
    for (int o = 0; o < 2; ++o) {
      __bf16 *base = &sB[o * 3][0];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        uint32_t vh[2], vm[2], vl[2];
        split3_pair(reg[o][q][0], reg[o][q][1], vh[0], vm[0], vl[0]);
        split3_pair(reg[o][q][2], reg[o][q][3], vh[1], vm[1], vl[1]);
        const int row = q * 32 + lr;
        const int off = row * LDK + slot(row, lk >> 3) + (lk & 7);
        *reinterpret_cast<uint2 *>(base + 0 * BB * LDK + off) = make_uint2(vh[0], vh[1]);
        *reinterpret_cast<uint2 *>(base + 1 * BB * LDK + off) = make_uint2(vm[0], vm[1]);
        *reinterpret_cast<uint2 *>(base + 2 * BB * LDK + off) = make_uint2(vl[0], vl[1]);
      }
    }
  };

  // (A + i Ai)(Br - i Bi): Cr += Ar Br + Ai Bi, Ci += Ai Br - Ar Bi, the
  // negative products in cin (subtracted once after the k loop)
  floatx16 cr[2], ci[2], cin[2];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) { cr[b][r] = 0.0f; ci[b][r] = 0.0f; cin[b][r] = 0.0f; }

  gload(0);
  for (int kt = 0; kt < nk; ++kt) {
    __syncthreads();             // previous tile's fragments consumed
    lstore();
    __syncthreads();
    if (kt + 1 < nk) gload((kt + 1) * KT);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      bf16x8 br[3], bim[3];
      const int rb_ = wn * 32 + li;
      const int ob = rb_ * LDK + slot(rb_, 2 * s + h);
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        br[t] = *reinterpret_cast<const bf16x8 *>(&sB[t][ob]);
        bim[t] = *reinterpret_cast<const bf16x8 *>(&sB[3 + t][ob]);
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        bf16x8 ar[3], ai[3];
        const int ra_ = wm * 64 + b * 32 + li;
        const int oa = ra_ * LDK + slot(ra_, 2 * s + h);
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          ar[t] = *reinterpret_cast<const bf16x8 *>(&sA[t][oa]);
          ai[t] = *reinterpret_cast<const bf16x8 *>(&sA[3 + t][oa]);
        }
        cr[b] = mac3(ar, br, cr[b]);
        ci[b] = mac3(ai, br, ci[b]);
        cr[b] = mac3(ai, bim, cr[b]);
        cin[b] = mac3(ar, bim, cin[b]);
        // one block's A fragments live at a time
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }

  const bool has_x = p.beta != 0.0f;
  const int64_t col = int64_t(bj) * BB + wn * 32 + li;
  float xr[2][16], xi[2][16];   // X loaded before any store (see epi_load_x)
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t row = int64_t(bi) * BA + wm * 64 + b * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
      epi_load_x(p, has_x, row * ld + col, xr[b][r], xi[b][r]);
    }
#pragma unroll
  for (int b = 0; b < 2; ++b) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t row = int64_t(bi) * BA + wm * 64 + b * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
      const int64_t o = row * ld + col;
      float vr, vi;
      epi_combine(p, has_x, scaled, sc, cr[b][r], ci[b][r] - cin[b][r], xr[b][r], xi[b][r], vr, vi);
      p.c_re[o] = vr;
      p.c_im[o] = vi;
    }
  }
}

template <typename K>
static hipError_t launch3(K kernel, const CgemmArgs<float> &a, bool lower, hipStream_t s) {
  const int tiles = int(a.ld / 64);
  int blocks = lower ? tiles * (tiles + 1) / 2 : tiles * tiles;
  if (blocks == 0) return hipSuccess;
  const bool split = a.split > 1;
  if (split) {
    if (!a.part || a.full < 0 || a.full >= blocks) return hipErrorInvalidValue;
    blocks = a.full + (blocks - a.full) * a.split;
  }
  hipError_t e = launch_kernel(kernel, dim3(blocks), dim3(kThreads3), 0, s, a);
  if (e == hipSuccess && split) e = launch_split_reduce(a, 64, lower, s);
  return e;
}

hipError_t launch_cgemm_bf16x3(const CgemmArgs<float> &a, const GemmOps &o, hipStream_t s) {
  if (a.ld % 64 != 0 || o.b_rows) return hipErrorInvalidValue;
  if (o.wide) {
    // 128 x 64 tiles: the step's first product only, unsplit, unfolded
    if (a.ld % 128 != 0 || !a.a_split || o.lower || o.conj_a || !o.conj_b || a.split > 1 ||
        a.fold_d || a.scale_set || (a.tr_aux && a.scale))
      return hipErrorInvalidValue;
    const int blocks = int((a.ld / 128) * (a.ld / 64));
    if (blocks == 0) return hipSuccess;
    return launch_kernel(cgemm_bf16x3_wide_kernel, dim3(blocks), dim3(kThreads3), 0, s, a);
  }
  // the folded epilogue exists for the step's lower-triangle product only,
  // the trace prologue for the 128 x 64 first product only
  if (a.fold_d && !(o.lower && a.m_split)) return hipErrorInvalidValue;
  if (a.tr_aux) return hipErrorInvalidValue;
  if (a.a_split && a.m_split) return hipErrorInvalidValue;
  if (a.a_split || a.m_split) {
    // the two forward products of a step: T = rho + dU rho^H-form (dU
    // pre-split as A) and rho_u = T + T conj(dU) (dU pre-split as M)
    if (o.conj_a || !o.conj_b) return hipErrorInvalidValue;
    if (a.a_split && !o.lower) return launch3(cgemm_bf16x3_kernel<false, true, false, 1>, a, false, s);
    if (a.m_split && o.lower) return launch3(cgemm_bf16x3_kernel<false, true, true, 2, true>, a, true, s);
    return hipErrorInvalidValue;
  }
  const int code = (o.conj_a ? 4 : 0) | (o.conj_b ? 2 : 0) | (o.lower ? 1 : 0);
  switch (code) {
    case 0: return launch3(cgemm_bf16x3_kernel<false, false, false, 0>, a, false, s);
    case 1: return launch3(cgemm_bf16x3_kernel<false, false, true, 0>, a, true, s);
    case 2: return launch3(cgemm_bf16x3_kernel<false, true, false, 0>, a, false, s);
    case 3: return launch3(cgemm_bf16x3_kernel<false, true, true, 0>, a, true, s);
    case 4: return launch3(cgemm_bf16x3_kernel<true, false, false, 0>, a, false, s);
    case 5: return launch3(cgemm_bf16x3_kernel<true, false, true, 0>, a, true, s);
    case 6: return launch3(cgemm_bf16x3_kernel<true, true, false, 0>, a, false, s);
    case 7: return launch3(cgemm_bf16x3_kernel<true, true, true, 0>, a, true, s);
  }
  return hipErrorInvalidValue;
}

__global__ __launch_bounds__(256) void split_bf16x3_kernel(const float *re, const float *im,
                                                          __bf16 *out, size_t elems) {
  const size_t i = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= elems) return;
  __bf16 h, m, l;
  split3(re[i], h, m, l);
  out[i] = h;
  out[elems + i] = m;
  out[2 * elems + i] = l;
  split3(im[i], h, m, l);
  out[3 * elems + i] = h;
  out[4 * elems + i] = m;
  out[5 * elems + i] = l;
}

hipError_t launch_split_bf16x3(const float *re, const float *im, void *out, size_t elems,
                               hipStream_t s) {
  if (elems == 0) return hipSuccess;
  hipLaunchKernelGGL(split_bf16x3_kernel, dim3(unsigned((elems + 255) / 256)), dim3(256), 0, s,
                     re, im, static_cast<__bf16 *>(out), elems);
  return hipGetLastError();
}

}  // namespace qme
