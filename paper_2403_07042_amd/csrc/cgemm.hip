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
//   * a complex multiply-add is four real MFMA products; conjugations and
//     the minus sign of Ai*Bi are applied by negating register fragments;
//   * LOWER launches only the tiles on or below the diagonal (Hermitian
//     output), enumerated triangularly.
#include "cgemm_tile.hpp"

namespace qme {

template <int BM, int OPS, bool LOWER>
__global__ __launch_bounds__(kThreads) void cgemm_f32_kernel(CgemmArgs<float> p) {
  __shared__ float smem[cgemm_f32_smem<BM, OPS>()];
  int bi, bj;
  tile_coords(blockIdx.x, int(p.ld / BM), LOWER, bi, bj);
  cgemm_f32_tile<BM, OPS>(p, bi, bj, smem);
}

template <int BM, int OPS, bool LOWER>
__global__ __launch_bounds__(kThreads) void cgemm_f64_kernel(CgemmArgs<double> p) {
  __shared__ double smem[cgemm_f64_smem<BM, OPS>()];
  int bi, bj;
  tile_coords(blockIdx.x, int(p.ld / BM), LOWER, bi, bj);
  cgemm_f64_tile<BM, OPS>(p, bi, bj, smem);
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

hipError_t launch_cgemm_f32(const CgemmArgs<float> &a, int tile, const GemmOps &o, hipStream_t s) {
  if (a.ld % tile != 0) return hipErrorInvalidValue;
  if (tile == 128) return cgemm_f32_kernel_dispatch<128>(a, ops_of(o), o.lower, s);
  if (tile == 64) return cgemm_f32_kernel_dispatch<64>(a, ops_of(o), o.lower, s);
  return hipErrorInvalidValue;
}

hipError_t launch_cgemm_f64(const CgemmArgs<double> &a, int tile, const GemmOps &o, hipStream_t s) {
  if (a.ld % tile != 0) return hipErrorInvalidValue;
  if (tile == 64) return cgemm_f64_kernel_dispatch<64>(a, ops_of(o), o.lower, s);
  if (tile == 32) return cgemm_f64_kernel_dispatch<32>(a, ops_of(o), o.lower, s);
  return hipErrorInvalidValue;
}

}  // namespace qme
