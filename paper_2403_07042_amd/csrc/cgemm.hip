// Planar complex GEMM on CDNA4 matrix cores (gfx950).
//
//   C = alpha * A * op(M) + beta * X,   op(M) = M^H or M^T,
//
// the two dense products of every time step ("unitary evolution" stage,
// Sec. IV.B / Table III):
//   T   = rho + dU rho      (A = dU, M = rho, rho Hermitian => rho = rho^H)
//   rho_u = T + T conj(dU)  (A = T,  M = dU,  dU symmetric => conj(dU) = dU^H)
// with dU = U - I so that the identity part of U is added exactly.
//
// Design (one workgroup per BM x BM output tile, 4 waves in a 2 x 2 grid):
//   * both operands are read by rows, k contiguous: float4 global loads,
//     staged through double-buffered LDS tiles [row][KT + pad];
//   * the k index inside a K tile is permuted per lane half so that each
//     lane fetches its 8 (FP32) or 4 (FP64) k values with two ds_read_b128;
//   * a complex multiply-add is four real MFMA products; the sign of the
//     imaginary cross terms is applied by negating one register fragment;
//   * 'lower' launches only the tiles on or below the diagonal (Hermitian
//     output), enumerated triangularly.
#include "device.hpp"

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef double doublex2 __attribute__((ext_vector_type(2)));

namespace qme {

static constexpr int kThreads = 256;

// Tile index -> (bi, bj).  Full grid: row-major tiles with the launch order
// remapped so that the blocks an XCD receives (block b goes to XCD b % 8)
// form compact groups of tile rows (L2 reuse of A rows and M rows).
__device__ __forceinline__ void tile_coords(int t, int tiles, bool lower, int &bi, int &bj) {
  if (lower) {
    int r = int((sqrtf(8.0f * float(t) + 1.0f) - 1.0f) * 0.5f);
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    while (r * (r + 1) / 2 > t) --r;
    bi = r;
    bj = t - r * (r + 1) / 2;
    return;
  }
  int nb = tiles * tiles;
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

// ----------------------------------------------------------------- FP32
// v_mfma_f32_32x32x2_f32: A 32x2 (lane l: row l%32, k-slot l/32), B 2x32
// (lane l: k-slot l/32, col l%32), D 32x32 in 16 registers (lane l: col l%32,
// register r: row 8*(r/4) + 4*(l/32) + r%4).

template <int BM, bool CONJ, bool LOWER>
__global__ __launch_bounds__(kThreads) void cgemm_f32_kernel(CgemmArgs<float> p) {
  constexpr int KT = 16;
  constexpr int LDK = KT + 4;          // padded LDS row (floats)
  constexpr int WM = BM / 2;           // wave tile
  constexpr int F = WM / 32;           // 32x32 blocks per wave side
  constexpr int PASSES = BM / 64;      // 64 rows per load pass (4 float4 per row)
  __shared__ float sA[2][2][BM * LDK];
  __shared__ float sM[2][2][BM * LDK];

  const int tiles = int(p.ld / BM);
  int bi, bj;
  tile_coords(blockIdx.x, tiles, LOWER, bi, bj);
  const int64_t ld = p.ld;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 31, h = lane >> 5;

  const int lr = tid >> 2, lk = (tid & 3) * 4;
  const float *ga_re = p.a_re + (int64_t(bi) * BM + lr) * ld + lk;
  const float *ga_im = p.a_im + (int64_t(bi) * BM + lr) * ld + lk;
  const float *gm_re = p.m_re + (int64_t(bj) * BM + lr) * ld + lk;
  const float *gm_im = p.m_im + (int64_t(bj) * BM + lr) * ld + lk;

  floatx4 ra[PASSES][2], rm[PASSES][2];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PASSES; ++q) {
      const int64_t off = int64_t(q) * 64 * ld + k0;
      ra[q][0] = *reinterpret_cast<const floatx4 *>(ga_re + off);
      ra[q][1] = *reinterpret_cast<const floatx4 *>(ga_im + off);
      rm[q][0] = *reinterpret_cast<const floatx4 *>(gm_re + off);
      rm[q][1] = *reinterpret_cast<const floatx4 *>(gm_im + off);
    }
  };
  auto lstore = [&](int st) {
#pragma unroll
    for (int q = 0; q < PASSES; ++q) {
      const int o = (q * 64 + lr) * LDK + lk;
      *reinterpret_cast<floatx4 *>(&sA[st][0][o]) = ra[q][0];
      *reinterpret_cast<floatx4 *>(&sA[st][1][o]) = ra[q][1];
      *reinterpret_cast<floatx4 *>(&sM[st][0][o]) = rm[q][0];
      *reinterpret_cast<floatx4 *>(&sM[st][1][o]) = rm[q][1];
    }
  };

  floatx16 cr[F][F], ci[F][F];
#pragma unroll
  for (int a = 0; a < F; ++a)
#pragma unroll
    for (int b = 0; b < F; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) { cr[a][b][r] = 0.0f; ci[a][b][r] = 0.0f; }

  const int nk = int(ld / KT);
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int st = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * KT);
    float ar[F][8], ai[F][8], mr[F][8], mi[F][8];
#pragma unroll
    for (int f = 0; f < F; ++f) {
      const int oa = (wm * WM + f * 32 + li) * LDK + h * 8;
      const int om = (wn * WM + f * 32 + li) * LDK + h * 8;
      floatx4 x0 = *reinterpret_cast<const floatx4 *>(&sA[st][0][oa]);
      floatx4 x1 = *reinterpret_cast<const floatx4 *>(&sA[st][0][oa + 4]);
      floatx4 y0 = *reinterpret_cast<const floatx4 *>(&sA[st][1][oa]);
      floatx4 y1 = *reinterpret_cast<const floatx4 *>(&sA[st][1][oa + 4]);
      floatx4 z0 = *reinterpret_cast<const floatx4 *>(&sM[st][0][om]);
      floatx4 z1 = *reinterpret_cast<const floatx4 *>(&sM[st][0][om + 4]);
      floatx4 w0 = *reinterpret_cast<const floatx4 *>(&sM[st][1][om]);
      floatx4 w1 = *reinterpret_cast<const floatx4 *>(&sM[st][1][om + 4]);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        ar[f][e] = x0[e]; ar[f][e + 4] = x1[e];
        ai[f][e] = y0[e]; ai[f][e + 4] = y1[e];
        mr[f][e] = z0[e]; mr[f][e + 4] = z1[e];
        mi[f][e] = w0[e]; mi[f][e + 4] = w1[e];
      }
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
#pragma unroll
      for (int a = 0; a < F; ++a) {
#pragma unroll
        for (int b = 0; b < F; ++b) {
          // op(M) = M^H: Cr += Ar Mr + Ai Mi, Ci += Ai Mr - Ar Mi
          // op(M) = M^T: Cr += Ar Mr - Ai Mi, Ci += Ai Mr + Ar Mi
          cr[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[a][s], mr[b][s], cr[a][b], 0, 0, 0);
          ci[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[a][s], mr[b][s], ci[a][b], 0, 0, 0);
          if (CONJ) {
            cr[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[a][s], mi[b][s], cr[a][b], 0, 0, 0);
            ci[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(-ar[a][s], mi[b][s], ci[a][b], 0, 0, 0);
          } else {
            cr[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai[a][s], mi[b][s], cr[a][b], 0, 0, 0);
            ci[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[a][s], mi[b][s], ci[a][b], 0, 0, 0);
          }
        }
      }
    }
    if (kt + 1 < nk) lstore(st ^ 1);
    __syncthreads();
  }

  // epilogue: C = alpha * acc + beta * X
  const bool has_x = p.beta != 0.0f;
#pragma unroll
  for (int a = 0; a < F; ++a) {
#pragma unroll
    for (int b = 0; b < F; ++b) {
      const int64_t col = int64_t(bj) * BM + wn * WM + b * 32 + li;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = int64_t(bi) * BM + wm * WM + a * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        const int64_t o = row * ld + col;
        float vr = p.alpha * cr[a][b][r], vi = p.alpha * ci[a][b][r];
        if (has_x) {
          vr += p.beta * p.x_re[o];
          vi += p.beta * p.x_im[o];
        }
        p.c_re[o] = vr;
        p.c_im[o] = vi;
      }
    }
  }
}

// ----------------------------------------------------------------- FP64
// v_mfma_f64_16x16x4_f64: A 16x4 (lane l: row l%16, k-slot l/16), B 4x16
// (lane l: k-slot l/16, col l%16), D 16x16 in 4 doubles (lane l: col l%16,
// register r: row l/16 + 4*r).

template <int BM, bool CONJ, bool LOWER>
__global__ __launch_bounds__(kThreads) void cgemm_f64_kernel(CgemmArgs<double> p) {
  constexpr int KT = 16;
  constexpr int LDK = KT + 2;          // padded LDS row (doubles)
  constexpr int WM = BM / 2;
  constexpr int F = WM / 16;           // 16x16 blocks per wave side
  constexpr int PASSES = BM / 32;      // 32 rows per pass (8 x doublex2 per row)
  __shared__ double sA[2][2][BM * LDK];
  __shared__ double sM[2][2][BM * LDK];

  const int tiles = int(p.ld / BM);
  int bi, bj;
  tile_coords(blockIdx.x, tiles, LOWER, bi, bj);
  const int64_t ld = p.ld;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, h = lane >> 4;

  const int lr = tid >> 3, lk = (tid & 7) * 2;
  const double *ga_re = p.a_re + (int64_t(bi) * BM + lr) * ld + lk;
  const double *ga_im = p.a_im + (int64_t(bi) * BM + lr) * ld + lk;
  const double *gm_re = p.m_re + (int64_t(bj) * BM + lr) * ld + lk;
  const double *gm_im = p.m_im + (int64_t(bj) * BM + lr) * ld + lk;

  doublex2 ra[PASSES][2], rm[PASSES][2];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PASSES; ++q) {
      const int64_t off = int64_t(q) * 32 * ld + k0;
      ra[q][0] = *reinterpret_cast<const doublex2 *>(ga_re + off);
      ra[q][1] = *reinterpret_cast<const doublex2 *>(ga_im + off);
      rm[q][0] = *reinterpret_cast<const doublex2 *>(gm_re + off);
      rm[q][1] = *reinterpret_cast<const doublex2 *>(gm_im + off);
    }
  };
  auto lstore = [&](int st) {
#pragma unroll
    for (int q = 0; q < PASSES; ++q) {
      const int o = (q * 32 + lr) * LDK + lk;
      *reinterpret_cast<doublex2 *>(&sA[st][0][o]) = ra[q][0];
      *reinterpret_cast<doublex2 *>(&sA[st][1][o]) = ra[q][1];
      *reinterpret_cast<doublex2 *>(&sM[st][0][o]) = rm[q][0];
      *reinterpret_cast<doublex2 *>(&sM[st][1][o]) = rm[q][1];
    }
  };

  doublex4 cr[F][F], ci[F][F];
#pragma unroll
  for (int a = 0; a < F; ++a)
#pragma unroll
    for (int b = 0; b < F; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) { cr[a][b][r] = 0.0; ci[a][b][r] = 0.0; }

  const int nk = int(ld / KT);
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int st = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * KT);
    double ar[F][4], ai[F][4], mr[F][4], mi[F][4];
#pragma unroll
    for (int f = 0; f < F; ++f) {
      const int oa = (wm * WM + f * 16 + li) * LDK + h * 4;
      const int om = (wn * WM + f * 16 + li) * LDK + h * 4;
      doublex2 x0 = *reinterpret_cast<const doublex2 *>(&sA[st][0][oa]);
      doublex2 x1 = *reinterpret_cast<const doublex2 *>(&sA[st][0][oa + 2]);
      doublex2 y0 = *reinterpret_cast<const doublex2 *>(&sA[st][1][oa]);
      doublex2 y1 = *reinterpret_cast<const doublex2 *>(&sA[st][1][oa + 2]);
      doublex2 z0 = *reinterpret_cast<const doublex2 *>(&sM[st][0][om]);
      doublex2 z1 = *reinterpret_cast<const doublex2 *>(&sM[st][0][om + 2]);
      doublex2 w0 = *reinterpret_cast<const doublex2 *>(&sM[st][1][om]);
      doublex2 w1 = *reinterpret_cast<const doublex2 *>(&sM[st][1][om + 2]);
      ar[f][0] = x0[0]; ar[f][1] = x0[1]; ar[f][2] = x1[0]; ar[f][3] = x1[1];
      ai[f][0] = y0[0]; ai[f][1] = y0[1]; ai[f][2] = y1[0]; ai[f][3] = y1[1];
      mr[f][0] = z0[0]; mr[f][1] = z0[1]; mr[f][2] = z1[0]; mr[f][3] = z1[1];
      mi[f][0] = w0[0]; mi[f][1] = w0[1]; mi[f][2] = w1[0]; mi[f][3] = w1[1];
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
      for (int a = 0; a < F; ++a) {
#pragma unroll
        for (int b = 0; b < F; ++b) {
          cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a][s], mr[b][s], cr[a][b], 0, 0, 0);
          ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a][s], mr[b][s], ci[a][b], 0, 0, 0);
          if (CONJ) {
            cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a][s], mi[b][s], cr[a][b], 0, 0, 0);
            ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ar[a][s], mi[b][s], ci[a][b], 0, 0, 0);
          } else {
            cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[a][s], mi[b][s], cr[a][b], 0, 0, 0);
            ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a][s], mi[b][s], ci[a][b], 0, 0, 0);
          }
        }
      }
    }
    if (kt + 1 < nk) lstore(st ^ 1);
    __syncthreads();
  }

  const bool has_x = p.beta != 0.0;
#pragma unroll
  for (int a = 0; a < F; ++a) {
#pragma unroll
    for (int b = 0; b < F; ++b) {
      const int64_t col = int64_t(bj) * BM + wn * WM + b * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = int64_t(bi) * BM + wm * WM + a * 16 + h + 4 * r;
        const int64_t o = row * ld + col;
        double vr = p.alpha * cr[a][b][r], vi = p.alpha * ci[a][b][r];
        if (has_x) {
          vr += p.beta * p.x_re[o];
          vi += p.beta * p.x_im[o];
        }
        p.c_re[o] = vr;
        p.c_im[o] = vi;
      }
    }
  }
}

// ------------------------------------------------------------- launchers

template <typename Args, typename K>
static hipError_t launch(K kernel, const Args &a, int tile, bool lower, hipStream_t s) {
  const int tiles = int(a.ld / tile);
  const int blocks = lower ? tiles * (tiles + 1) / 2 : tiles * tiles;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(kernel, dim3(blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_cgemm_f32(const CgemmArgs<float> &a, int tile, bool conj_m, bool lower,
                            hipStream_t s) {
  if (a.ld % tile != 0) return hipErrorInvalidValue;
#define QME_F32(BM)                                                                     \
  if (tile == BM) {                                                                     \
    if (conj_m) return lower ? launch(cgemm_f32_kernel<BM, true, true>, a, BM, true, s)  \
                             : launch(cgemm_f32_kernel<BM, true, false>, a, BM, false, s); \
    return lower ? launch(cgemm_f32_kernel<BM, false, true>, a, BM, true, s)             \
                 : launch(cgemm_f32_kernel<BM, false, false>, a, BM, false, s);          \
  }
  QME_F32(128)
  QME_F32(64)
#undef QME_F32
  return hipErrorInvalidValue;
}

hipError_t launch_cgemm_f64(const CgemmArgs<double> &a, int tile, bool conj_m, bool lower,
                            hipStream_t s) {
  if (a.ld % tile != 0) return hipErrorInvalidValue;
#define QME_F64(BM)                                                                     \
  if (tile == BM) {                                                                     \
    if (conj_m) return lower ? launch(cgemm_f64_kernel<BM, true, true>, a, BM, true, s)  \
                             : launch(cgemm_f64_kernel<BM, true, false>, a, BM, false, s); \
    return lower ? launch(cgemm_f64_kernel<BM, false, true>, a, BM, true, s)             \
                 : launch(cgemm_f64_kernel<BM, false, false>, a, BM, false, s);          \
  }
  QME_F64(64)
  QME_F64(32)
#undef QME_F64
  return hipErrorInvalidValue;
}

}  // namespace qme
