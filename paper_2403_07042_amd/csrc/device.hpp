// Device launchers shared by the context code (internal, not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qme {

// Planar complex GEMM  C = alpha * A * op(M) + beta * X  on N x N matrices
// stored row-major with leading dimension ld (padding rows/columns zero):
//   op(M) = M^H (conj_m) or M^T.
// Both A and M are read by rows, so both operands stream contiguous k.
// lower: compute only the tiles on or below the diagonal (for Hermitian C).
template <typename T>
struct CgemmArgs {
  const T *a_re, *a_im;
  const T *m_re, *m_im;
  const T *x_re, *x_im;   // may be null when beta == 0
  T *c_re, *c_im;
  int64_t ld;
  T alpha, beta;
};

hipError_t launch_cgemm_f32(const CgemmArgs<float> &a, int tile, bool conj_m, bool lower,
                            hipStream_t s);
hipError_t launch_cgemm_f64(const CgemmArgs<double> &a, int tile, bool conj_m, bool lower,
                            hipStream_t s);

// Fused decoherence step on the rotated state Z (lower triangle valid):
//   X = scale * Herm(Z + dt * D(Z)),  D(Z)[u,v] = sum_j cg_j[u] cg_j[v]
//   Z[pi_j[u], pi_j[v]] - (d[u] + d[v]) / 2 Z[u,v]
// written in full (both triangles).  aux[4] holds the scale.
template <typename T>
struct DissArgs {
  const T *z_re, *z_im;
  T *x_re, *x_im;
  int64_t ld, n;
  double dt;
  const double *d;       // [n]
  const double *leak;    // [n]
  const int32_t *pi;     // [n_gather * n]
  const double *cg;      // [n_gather * n]
  int n_gather;
  double *aux;           // state scalars (see qme_state_layout)
};

template <typename T>
hipError_t launch_trace(const DissArgs<T> &a, hipStream_t s);
template <typename T>
hipError_t launch_dissipate(const DissArgs<T> &a, hipStream_t s);
template <typename T>
hipError_t launch_diag(const T *x_re, int64_t ld, int64_t n, double *out, hipStream_t s);

}  // namespace qme
