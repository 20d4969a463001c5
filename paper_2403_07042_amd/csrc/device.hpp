// Device launchers shared by the context code (internal, not part of the ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace qme {

// The calling thread's index in its workgroup, for the tile bodies.  It is
// passed through an empty asm so that in a persistent kernel, which runs
// many bodies in one loop, the values derived from it (per-lane LDS and
// global offsets) are formed inside each body rather than hoisted out of the
// loop and kept live for every body at once (which needs more registers
// than any one body).
__device__ __forceinline__ int thread_index() {
  int t = int(threadIdx.x);
  asm volatile("" : "+v"(t));
  return t;
}

// Per-kernel timing of the step path (qme_profile_enable).  While a timer is
// armed on the calling thread, every kernel enqueued through launch_kernel
// takes a fresh start / stop event pair from it and is launched with
// hipExtLaunchKernel, which stamps the two events with that dispatch's own
// start and end: a duration is the kernel's execution alone, without the
// gaps between kernels or extra packets on the stream.
struct LaunchTimer {
  virtual hipError_t next_pair(hipEvent_t *start, hipEvent_t *stop) = 0;

 protected:
  ~LaunchTimer() = default;
};
LaunchTimer *&launch_timer();   // the calling thread's armed timer (nullptr: none)

template <typename F, typename... Args>
inline hipError_t launch_kernel(F kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t s,
                                Args... args) {
  if (LaunchTimer *t = launch_timer()) {
    hipEvent_t start = nullptr, stop = nullptr;
    const hipError_t e = t->next_pair(&start, &stop);
    if (e != hipSuccess) return e;
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, start, stop, 0, args...);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
  }
  return hipGetLastError();
}

// Planar complex GEMM  C = alpha * opA(A) * opB(B) + beta * X  on ld x ld
// row-major matrices (padding rows/columns zero).  The second operand is
// passed as m_re/m_im: with b_rows it is B itself (row-major [k][j]),
// otherwise it is M with B = M^T (B[k][j] = M[j][k]).  conj_a / conj_b
// conjugate A / B.  lower: only the tiles on or below the diagonal.
// direct (FP32 forms with M given by rows only): 1 uses the tile body that
// loads operands straight into LDS, 0 the register-staged one, -1 picks the
// direct body when the launch has fewer blocks than 2 per compute unit
// (`cus`), i.e. when resident workgroups cannot hide load latency by their
// number.  Both bodies give bitwise-identical results.
// FP32 32-tile products with ld up to this size load each tile's whole row
// panels into LDS at once (cgemm_s_panel) and are not split along k (unless
// GemmOps::direct == 0 asks for register staging).
// Measured on MI355X: faster at ld = 128 (N = 128 lattice 54.6k -> 64.8k
// steps/s) and 192 (N = 144: 46.0k -> 48.8k), slower at 256 (51.5k -> 47.3k:
// 128 KB of LDS leaves one workgroup per CU for the whole panel load).
constexpr int kPanelLd = 192;

struct GemmOps {
  bool conj_a = false, conj_b = false, b_rows = false, lower = false;
  int direct = 0, cus = 0;
  // BF16x3 first product of a step on 128 x 64 tiles (launch_cgemm_bf16x3)
  bool wide = false;
};

// Split launches (FP32, FP64 and BF16x3 products): when
// split > 1, tiles [full, all) are computed in `split` k-chunks each, into
// partial slots of 2 * tile^2 elements at `part` (re then im, tile-local
// row-major), and a reduce pass writes C = alpha * (sum of the chunks in
// order) + beta * X.
template <typename T>
struct CgemmArgs {
  const T *a_re, *a_im;
  const T *m_re, *m_im;
  const T *x_re, *x_im;   // may be null when beta == 0
  T *c_re, *c_im;
  int64_t ld;
  T alpha, beta;
  int32_t full = 0, split = 0;
  T *part = nullptr;
  // BF16x3 products only: the first operand (a_split) or the second
  // (m_split) given as six bf16 planes [re hi, re mid, re lo, im hi, im mid,
  // im lo] of ld x ld, split once instead of per tile
  const void *a_split = nullptr, *m_split = nullptr;
  // FP32 / FP64 products only.  scale: when set, alpha = beta = *scale,
  // applied in FP64 (the renormalisation of the previous step folded into
  // the first product).  fold_d: when set (lower-triangle products with
  // 64-tiles in FP32, 32- or 64-tiles in FP64), the epilogue applies the
  // decoherence step of a model without gather channels to
  // Z = alpha acc + beta X (rounded to T): C[u][v] = (1 - dt (d[u] + d[v]) / 2)
  // Z[u][v] for v <= u and its conjugate mirror for v > u, and writes
  // zdiag[u] = Z[u][u] (FP64) for u < fold_n.
  const double *scale = nullptr;
  const double *fold_d = nullptr;
  double fold_dt = 0.0;
  int64_t fold_n = 0;
  double *zdiag = nullptr;
  // Folded steps (FP32 64- and 128-tile and whole-panel 32-tile, and BF16x3
  // 128 x 64 first products, no split): the previous step's trace formed by
  // every block of the first product with the trace pass's arithmetic
  // (DissArgs: the stored diagonal of Z, trace and leak weights, the state's
  // scalars, the scalar slot pairs read and written); block 0 stores the
  // step's scalars, and the factor it gives is the product's alpha = beta
  // (in place of `scale`).
  const double *tr_zdiag = nullptr, *tr_w = nullptr, *tr_leak = nullptr;
  double *tr_aux = nullptr;
  int64_t tr_n = 0;
  double tr_dt = 0.0;
  int32_t tr_slot_in = 0, tr_slot_out = 0;
  // a factor given by value (scale_set): alpha = beta = scale_value in FP64,
  // as for `scale` (the kernels set it from the trace they form)
  double scale_value = 0.0;
  int32_t scale_set = 0;
  // FP32 register-staged tiles: the workgroups that are behind in their k
  // loop issue first (set by the launcher when the whole launch is resident
  // at once, so co-resident workgroups finish together)
  int32_t rank_prio = 0;
};

// Plan of a tail split for a lower-triangle product of `tiles` tile rows
// (tile edge bm) on a device with `cus` compute units, with room for
// `cap_elems` partial elements.  split = 0: no split.
struct SplitPlan {
  int32_t full = 0, split = 0;
};
SplitPlan plan_tail_split(int tiles, int bm, int kt, int64_t ld, int cus, size_t cap_elems);
// Plan of a split of every tile of a launch too small to occupy the device:
// `blocks` tiles (at most half as many as compute units) each cut along k
// into `split` chunks of at least two K tiles (full = 0), with room for
// `cap_elems` partial elements.  split = 0: no split.
SplitPlan plan_small_split(int blocks, int bm, int kt, int64_t ld, int cus, size_t cap_elems);
// Reduce pass of a split launch: tiles [full, all) of the launch's tile
// enumeration (lower triangle or full grid).
template <typename T>
hipError_t launch_split_reduce(const CgemmArgs<T> &a, int tile, bool lower, hipStream_t s);
// state planes (ld x ld each) *= *scale, in FP64 (the last step of a folded run)
template <typename T>
hipError_t launch_apply_scale(T *re, T *im, int64_t elems, const double *scale, hipStream_t s);

hipError_t launch_cgemm_f32(const CgemmArgs<float> &a, int tile, const GemmOps &o,
                            hipStream_t s);
hipError_t launch_cgemm_f64(const CgemmArgs<double> &a, int tile, const GemmOps &o,
                            hipStream_t s);
// Split-BF16x3 products on FP32 planes (tile 64, NT forms only).
hipError_t launch_cgemm_bf16x3(const CgemmArgs<float> &a, const GemmOps &o, hipStream_t s);
// The six bf16 planes of a complex FP32 matrix (elems per plane), with the
// split the BF16x3 products apply per tile.
hipError_t launch_split_bf16x3(const float *re, const float *im, void *out, size_t elems,
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
  const double *aux_in;  // scalars of the input state (sink)
  double *aux_out;       // scalars of the output state (see qme_state_layout)
  // trace weights: tr rho_d = sum_w trw[w] Z[w,w] with
  // trw[w] = 1 - dt d[w] + dt sum_{j,u: pi_j[u] = w} cg_j[u]^2
  const double *trw = nullptr;
  // when set, the diagonal of Z is read from this array (FP64, [n])
  const double *zdiag = nullptr;
  // decoherence operators that are not monomial (general-form models), in
  // sparse form: per channel q the rows of A on the basis (csr_ptr
  // [n_csr][n + 1] into csr_col / csr_val, unit rate) and its rate
  // csr_gamma[q]; (A Z A^dag)[u,v] = sum over rows u and v of
  // a_uk a_vl Z[k,l].  koff (CSR over rows, or nullptr): the off-diagonal
  // part of K = sum gamma A^dag A, whose -1/2 {K, Z} the pass adds (the
  // diagonal part is in d).  loff: n_loff off-diagonal entries (row, col,
  // value) of the lost probability's matrix: lost += sum value Re Z[col,row]
  // (non-zero only on a restricted basis).
  int n_csr = 0;
  const int64_t *csr_ptr = nullptr;
  const int32_t *csr_col = nullptr;
  const double *csr_val = nullptr;
  const double *csr_gamma = nullptr;
  const int64_t *koff_ptr = nullptr;
  const int32_t *koff_col = nullptr;
  const double *koff_val = nullptr;
  int64_t n_loff = 0;
  const int32_t *loff_row = nullptr;
  const int32_t *loff_col = nullptr;
  const double *loff_val = nullptr;
  // Scalar slots of the trace pass.  The sink and the step count are read
  // from slot pair slot_in and written to slot pair slot_out (pair 0:
  // scalars 0 and 3, as in qme_state_layout; pair 1: scalars 5 and 6).
  // When every block of the decoherence pass forms the trace itself (small
  // systems, launch_dissipate with fuse_trace) the state is updated in place
  // by many blocks at once, so the two pairs differ and alternate by step.
  int slot_in = 0, slot_out = 0;
  int fuse_trace = 0;
  // bit j: gather channel j maps every state to itself or out of the basis
  // (dephasing), so its term reads the element itself and needs no load
  uint32_t self_mask = 0;
};
// the scalar indices of the sink and the step count in slot pair `slot`
__host__ __device__ constexpr int sink_slot(int slot) { return slot ? 5 : 0; }
__host__ __device__ constexpr int steps_slot(int slot) { return slot ? 6 : 3; }

template <typename T>
hipError_t launch_trace(const DissArgs<T> &a, hipStream_t s);
// After a run of fused steps that ended in slot pair 1: the sink and step
// count moved back to pair 0 (one thread).
hipError_t launch_scalars_home(double *aux, hipStream_t s);
template <typename T>
hipError_t launch_dissipate(const DissArgs<T> &a, hipStream_t s);
template <typename T>
hipError_t launch_diag(const T *x_re, int64_t ld, int64_t n, double *out, hipStream_t s);

// Whole time steps of a system with n <= kSmallN in one single-workgroup
// launch (state and dU held in LDS; see small.hip).  re / im / aux: the
// state buffer (planes of ld x ld, FP64 scalars), updated in place.
constexpr int kSmallN = 32;
template <typename T>
struct SmallArgs {
  T *re, *im;
  double *aux;
  const T *u_re, *u_im;
  int64_t ld;
  int n;
  double dt;
  const double *d, *leak;
  const int32_t *pi;
  const double *cg;
  int n_gather;
  int64_t steps;
  const double *trw;       // trace weights (see DissArgs)
};
template <typename T>
hipError_t launch_small_steps(const SmallArgs<T> &a, hipStream_t s);

// Gather of a state onto a subset of its basis (state-space selection).
template <typename T>
struct CompactArgs {
  const T *from_re, *from_im;
  const double *aux_from;
  T *to_re, *to_im;
  double *aux_to;
  const int32_t *keep;     // [n_to] indices into the source basis
  int64_t n_from, ld_from, n_to, ld_to;
};
template <typename T>
hipError_t launch_compact(const CompactArgs<T> &a, hipStream_t s);

// The keep/delete decision of state-space selection on the device: the
// populations p_now[s] = Re rho[s][s] of a state, the states whose growth
// speed |p_now - p_prev| / interval is at least eps in increasing order, and
// their count (-1 when a population is not finite).  p_now may alias p_prev.
template <typename T>
struct DecideArgs {
  const T *re;
  int64_t ld, n;
  const double *p_prev;
  double *p_now;
  double interval, eps;
  int32_t *keep;
  int64_t *n_keep;
};
template <typename T>
hipError_t launch_select_decide(const DecideArgs<T> &a, hipStream_t s);

// One pure-state step of a closed model for nv vectors (planar, [nv][ld]):
// y_v = (x_v + dU x_v) / |x_v| (see pure.hip).  x and y must not overlap.
template <typename T>
struct PureArgs {
  const T *x_re, *x_im;
  T *y_re, *y_im;
  const T *u_re, *u_im;   // dU planes, ld x ld
  int64_t ld, n;
};
template <typename T>
hipError_t launch_pure_step(const PureArgs<T> &a, int nv, hipStream_t s);

// Adjoint of one step's decoherence, fused with the rate-gradient partials.
//   mu = lam + dt * sum_j gamma_j (A_j^dag lam A_j - 1/2 {A_j^dag A_j, lam})
// from the lower triangle of the Hermitian lam (written in full), and, with
// Z = rho_u of the same step,
//   e(u,v) = Re(Z[u,v] lam[v,u]) summed per row / column of each tile, and
//   sum_{u,v} c_a[u] c_a[v] Re(lam[v,u] Z[pi_a[u], pi_a[v]]) per block for
//   every channel a with arrivals inside the basis (unit rate).
template <typename T>
struct AdjArgs {
  const T *l_re, *l_im;
  T *mu_re, *mu_im;
  const T *z_re, *z_im;
  int64_t ld, n;
  double dt;
  const double *d;
  const int32_t *tau;    // [n_gather * n]
  const double *ca;      // [n_gather * n]
  int n_gather;
  const int32_t *upi;    // [n_arrival * n]
  const double *uc;      // [n_arrival * n]
  int n_arrival;
  double *rowbuf;        // [tiles * n]
  double *colbuf;        // [tiles * n]
  double *gbuf;          // [blocks * n_arrival]
  // sparse (non-monomial) channels: rows of A^T (csrt_ptr [n_csr][n + 1],
  // row k: the images u of preimage k with their unit-rate coefficients),
  // the rates, and K's off-diagonal part (nullptr: none), as in DissArgs:
  //   mu += dt (sum gamma A^T lam A - 1/2 {K_off, lam})
  int n_csr = 0;
  const int64_t *csrt_ptr = nullptr;
  const int32_t *csrt_col = nullptr;
  const double *csrt_val = nullptr;
  const double *csr_gamma = nullptr;
  const int64_t *koff_ptr = nullptr;
  const int32_t *koff_col = nullptr;
  const double *koff_val = nullptr;
};

// Rate-gradient partials of the sparse channels for one adjoint step: per
// channel q and lower-triangle tile of 64, the sum over the tile's elements
// (weight 2 off the diagonal) of Re(conj(lam[u,v]) E_q[u,v]) with
//   E_q = A_q Z A_q^T - 1/2 (K_q,off Z + Z K_q,off)      (unit rate)
// into part[q * blocks + tile]; the diagonal of K_q enters through
// launch_gamma_reduce like a monomial channel's.
template <typename T>
struct AdjSparseArgs {
  const T *l_re, *l_im;     // lam (lower triangle valid)
  const T *z_re, *z_im;     // Z = rho_u of the step (lower triangle valid)
  int64_t ld, n;
  int n_csr;
  const int64_t *csr_ptr;   // [n_csr][n + 1]: rows of A (images u)
  const int32_t *csr_col;
  const double *csr_val;
  const int64_t *kj_ptr;    // [n_csr][n + 1]: K_q off-diagonal, unit rate
  const int32_t *kj_col;
  const double *kj_val;
  double *part;             // [n_csr * blocks]
};
template <typename T>
hipError_t launch_adj_sparse_gamma(const AdjSparseArgs<T> &a, hipStream_t s);
// grad[channel[q]] += dt * sum_b part[q * blocks + b]  (b in order)
hipError_t launch_sparse_gamma_reduce(const double *part, int blocks, int n_csr,
                                      const int32_t *channel, double dt, double *grad,
                                      hipStream_t s);

constexpr int kAdjTile = 64;
constexpr int kMaxArrival = 16;

template <typename T>
hipError_t launch_adj_dissipate(const AdjArgs<T> &a, hipStream_t s);
// q[u] = sum of the row / column partials of e(u, .) (all tiles of u)
hipError_t launch_q_reduce(const double *rowbuf, const double *colbuf, int64_t n, double *q,
                           hipStream_t s);
// grad[j] += dt * (sum_b gbuf[b][arrival_of[j]] - sum_u ada[j][u] q[u])
hipError_t launch_gamma_reduce(const double *gbuf, int blocks, int n_arrival,
                               const int32_t *arrival_of, const double *ada, const double *q,
                               int64_t n, int n_jumps, double dt, double *grad, hipStream_t s);
// X = 0 except X[u][u] = o[u]
template <typename T>
hipError_t launch_set_diag(T *x_re, T *x_im, int64_t ld, int64_t n, const double *o,
                           hipStream_t s);

}  // namespace qme
