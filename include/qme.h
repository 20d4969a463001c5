/*
 * qme.h -- C ABI of the MI355X quantum-master-equation solver.
 *
 * The library time-steps the density matrix rho of a finite-dimensional
 * cavity-QED system (Jaynes-Cummings-Hubbard / Tavis-Cummings-Hubbard
 * lattices of cavities with two-level atoms) under the quantum master
 * equation of Sec. II, Eqs. 2-3 of Li, Miao, Ozhigov, "Supercomputer model of
 * finite-dimensional quantum electrodynamics applications" (hbar = 1):
 *
 *     d rho / dt = -i [H, rho] + sum_j gamma_j (A_j rho A_j^dag
 *                                 - 1/2 {A_j^dag A_j, rho}).
 *
 * The calls follow the paper's modelling scheme (Sec. II): fix the basis of
 * joint atom and photon states (qme_basis), build the Hamiltonian and the
 * decoherence operators (qme_hamiltonian), solve the equation by repeated
 * time steps (qme_step; the "Taylor approximation" stage builds the
 * propagator once, the "unitary evolution" stage applies it, Sec. IV.B,
 * Table III) and read out state probabilities (qme_observe; the quantities
 * plotted in Figs. 4-8).
 *
 * One time step k -> k+1 (propagator U = exp(-i H dt), built once):
 *     rho_u     = U rho_k U^dag
 *     rho_d     = rho_u + dt * sum_j gamma_j (A_j rho_u A_j^dag
 *                                   - 1/2 (A_j^dag A_j rho_u + rho_u A_j^dag A_j))
 *     sink     += dt * sum_j gamma_j [tr(A_j^dag A_j rho_u) - tr(A_j rho_u A_j^dag)]
 *     rho_{k+1} = Herm(rho_d) * (1 - sink) / tr Herm(rho_d)
 * where "sink" is the probability that decoherence moved out of a truncated
 * basis and Herm(X) is the Hermitian part of X.
 *
 * Conventions for every call:
 *   - Return a qme_status; nothing aborts, throws or exits across the ABI.
 *     On an error nothing the caller can observe has been modified and
 *     qme_last_error() describes the failure (thread-local text).
 *   - Arguments are validated before any device work is enqueued.
 *   - Pointers named *_dev are device pointers (HIP); all others are host.
 *     Input arrays are copied during the call; the caller keeps ownership.
 *   - hip_stream is a hipStream_t passed as void* (NULL = default stream).
 *     qme_step and qme_batch_step only enqueue work; calls that return host
 *     results (qme_observe, qme_get_state, qme_adjoint) synchronise the stream.
 *   - A context is used by one host thread / stream at a time.
 */
#ifndef QME_H
#define QME_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QME_OK = 0,
  QME_E_ARG = 1,          /* invalid argument (null pointer, bad index, NaN, ...) */
  QME_E_SIZE = 2,         /* buffer too small or problem too large */
  QME_E_DEVICE = 3,       /* a HIP runtime call failed */
  QME_E_NUMERIC = 4,      /* non-finite values or trace <= 0 in the state */
  QME_E_STATE = 5,        /* call not valid for this context / state */
  QME_E_UNSUPPORTED = 6   /* precision or option not available */
} qme_status;

/* Arithmetic of the two dense complex products of each step. */
typedef enum {
  QME_FP64 = 0,    /* FP64 storage, FP64 MFMA products */
  QME_FP32 = 1,    /* FP32 storage, FP32 MFMA products, FP64 dissipator/trace */
  QME_BF16X3 = 2   /* FP32 storage, each FP32 operand split into three bf16
                      planes, six bf16 MFMA cross products, FP32 accumulate */
} qme_precision;

/* Decoherence operators A_j (Sec. II, Eq. 3). */
typedef enum {
  QME_JUMP_PHOTON_LEAK = 0,   /* A = a_c, photon leaves cavity c */
  QME_JUMP_ATOM_DECAY = 1,    /* A = sigma_ck = |g><e| of atom k of cavity c */
  QME_JUMP_ATOM_DEPHASE = 2   /* A = sigma_ck^dag sigma_ck */
} qme_jump_kind;

/* Structure of the system.  Modes are ordered cavity by cavity: the photon
 * mode of cavity c (levels 0..photon_cap[c]), then its atoms[c] two-level
 * atoms.  The basis is every occupation tuple whose total excitation number
 * lies in [exc_min, exc_max] (exc_max < 0: no upper bound), in ascending
 * lexicographic order with mode 0 most significant (Kronecker order for a
 * full tensor product).  This is the working-subspace selection of Sec. II
 * (third point) and Sec. IV.B, Eqs. 10-11 (single-photon subspace). */
typedef struct {
  int32_t n_cavities;
  const int32_t *atoms;        /* [n_cavities], >= 0 */
  const int32_t *photon_cap;   /* [n_cavities], >= 0 */
  int32_t exc_min;
  int32_t exc_max;
} qme_system;

/* Photon hopping mu (a_a^dag a_b + a_b^dag a_a) between cavities a != b
 * (Sec. IV.B, Eq. 12, tunnelling strength zeta). */
typedef struct {
  int32_t a, b;
  double mu;
} qme_hop;

/* One decoherence channel: kind, cavity, atom index within the cavity
 * (ignored for photon leak), rate gamma >= 0. */
typedef struct {
  int32_t kind, cavity, atom;
  double gamma;
} qme_jump;

/* Hamiltonian (RWA, hbar = 1; Sec. IV.A Eq. 8b, Sec. IV.B Eq. 12):
 *   H = sum_c omega_c a_c^dag a_c + sum_atoms omega_a sigma^dag sigma
 *     + sum_atoms g (a_c^dag sigma + a_c sigma^dag)
 *     + sum_hops mu (a_a^dag a_b + a_b^dag a_a)
 * Atoms are numbered cavity-major. */
typedef struct {
  const double *omega_c;   /* [n_cavities] */
  const double *omega_a;   /* [total atoms] */
  const double *g;         /* [total atoms] */
  int32_t n_hops;
  const qme_hop *hops;     /* [n_hops] */
  int32_t n_jumps;
  const qme_jump *jumps;   /* [n_jumps] */
  double dt;               /* time step, > 0 */
} qme_params;

typedef struct qme_ctx qme_ctx;

/* ---------------------------------------------------------------- host only */

/* Enumerate the basis.  Writes N to *n_states.  If occ is non-NULL and
 * occ_rows >= N, also writes the occupation table, row-major N x n_modes
 * (n_modes = n_cavities + total atoms).  occ == NULL is a size query
 * (QME_OK); occ != NULL with occ_rows < N returns QME_E_SIZE (with *n_states
 * set).  QME_E_SIZE also when N would exceed 2^20. */
qme_status qme_basis(const qme_system *sys, int64_t *n_states, int32_t *occ,
                     int64_t occ_rows);

/* The Hamiltonian matrix restricted to the basis, as COO triplets sorted by
 * (row, col) with duplicates summed.  Two-call pattern as for qme_basis:
 * rows/cols/vals may be NULL for a size query; capacity < nnz gives
 * QME_E_SIZE with *nnz set. */
qme_status qme_hamiltonian_coo(const qme_system *sys, const qme_params *par,
                               int64_t *nnz, int32_t *rows, int32_t *cols,
                               double *vals, int64_t capacity);

/* The propagator increment dU = exp(-i H dt) - I in FP64, computed on the
 * host by the library's Taylor series (with scaling and squaring when
 * |H dt|_1 > 1/2).  du_re / du_im: row-major n x n, n must equal N. */
qme_status qme_propagator_host(const qme_system *sys, const qme_params *par,
                               double *du_re, double *du_im, int64_t n);

/* ------------------------------------------------------------- with a GPU */

/* Sec. II, first two points of the modelling scheme (the basis of joint
 * atom and photon states, then the Hamiltonian and the decoherence
 * operators), with
 * the Hamiltonian of Sec. IV.A Eq. 8b / Sec. IV.B Eq. 12 and the "Taylor
 * approximation" stage of Sec. IV.B, Table III (the propagator, built once).
 * Build a context on the current HIP device: basis, Hamiltonian, FP64
 * propagator (Taylor stage), decoherence tables, and the device copies of
 * the propagator in the arithmetic of `precision`.  Synchronous.
 * Errors: QME_E_ARG (invalid system or parameters, unknown precision),
 * QME_E_SIZE (basis larger than 2^20 states), QME_E_NUMERIC (propagator not
 * finite), QME_E_DEVICE (a HIP call failed); *out is NULL on error and owns
 * nothing.  The context owns its device tables until qme_destroy. */
qme_status qme_hamiltonian(const qme_system *sys, const qme_params *par,
                           int32_t precision, void *hip_stream, qme_ctx **out);

/* Layout of a device state buffer: two planes (real, imaginary) of ld x ld
 * elements each, row-major (ld >= n; rows and columns >= n are zero),
 * elements FP64 for QME_FP64 and FP32 otherwise, followed by 64 bytes of
 * FP64 scalars [sink, trace of the
 * last rotated state, lost-probability rate of the last step, steps taken,
 * last renormalisation factor, two library scratch scalars, 0]; the scratch
 * pair carries the sink and step count between the steps of one call and
 * holds no meaning afterwards.  The caller allocates state_bytes of device
 * memory (256-byte aligned) and owns it. */
qme_status qme_state_layout(const qme_ctx *ctx, int64_t *n, int64_t *ld,
                            int64_t *elem_bytes, size_t *state_bytes);

/* Device workspace qme_step needs (caller-allocated, 256-byte aligned):
 * four product planes of ld x ld elements, N FP64 values (the diagonal kept
 * by folded steps, qme_set_fold) and, for contexts whose
 * products are too small to occupy the device, the partial slots of their
 * k-split (qme_set_split; at most 12 planes, sized for every tile edge
 * qme_set_tiles accepts). */
qme_status qme_workspace_size(const qme_ctx *ctx, size_t *bytes);

/* Write a state: rho (host, row-major n x n FP64 planes, converted to the
 * context precision, padding zeroed) and the sink scalar.  Synchronous. */
qme_status qme_set_state(const qme_ctx *ctx, void *state_dev,
                         const double *rho_re, const double *rho_im,
                         double sink, void *hip_stream);

/* Read a state back (row-major n x n FP64 planes; either may be NULL) and
 * its sink (may be NULL).  Synchronous. */
qme_status qme_get_state(const qme_ctx *ctx, const void *state_dev,
                         double *rho_re, double *rho_im, double *sink,
                         void *hip_stream);

/* Sec. II, third point (solving the master equation of Eqs. 2-3 by
 * repeated time steps) and the "unitary evolution" stage of Sec. IV.B,
 * Table III (U rho U^dag applied every step).
 * Advance the state by n_steps >= 0 time steps on hip_stream.  The state
 * buffer holds rho_{k+n} afterwards (never a pending scale: folded steps
 * apply their last renormalisation before the call's work ends).
 * Asynchronous; the workspace must stay allocated until the stream reaches
 * this point.  Between its own kernels the call may keep intermediate
 * values in the state buffer, so the state must not be read by other work
 * on other streams until the stream reaches this point.
 * Failure injection for recovery tests: when the environment holds
 * QME_FAULT_AT_STEP=k at context creation, the call that would take the
 * context past its k-th step (counted over all qme_step calls) runs up to
 * that step and returns QME_E_DEVICE; the state then holds rho_k. */
qme_status qme_step(qme_ctx *ctx, void *state_dev, int64_t n_steps,
                    void *workspace_dev, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that forbid hipMalloc): qme_step with the step
 * workspace taken from a fixed device array of QME_NOALLOC_SCRATCH_BYTES
 * inside the library instead of a caller buffer.  Same kernels and
 * arithmetic as qme_step with the same knobs: results are bitwise those of
 * qme_step.  It calls no hipMalloc, hipFree or other allocating routine, and
 * runs eagerly (no graph replay; no profiling records).  Each device holds
 * one copy of the array, from library load until the process ends; its
 * address is looked up at context creation.  Calls on one device share the
 * array and keep the last call's contents (nothing in it needs to start at
 * zero), so calls that overlap on one device -- on several streams or
 * threads, or several contexts -- race; serialise them.
 * Errors: as qme_step; QME_E_SIZE when the context's workspace
 * (qme_workspace_size) exceeds QME_NOALLOC_SCRATCH_BYTES (for example FP64
 * at N = 2048); QME_E_STATE while failure injection is armed.
 * Asynchronous on hip_stream. */
#define QME_NOALLOC_SCRATCH_BYTES (80u * 1024u * 1024u)
qme_status qme_step_noalloc(qme_ctx *ctx, void *state_dev, int64_t n_steps, void *hip_stream);

/* The probabilities of basis states plotted in Figs. 4-8 (Sec. IV) and the
 * trace that the renormalisation of Sec. III.B keeps at 1 - sink.
 * Populations p_s = Re rho_ss (FP64, [N] or NULL), trace sum_s p_s and sink
 * (each may be NULL).  Synchronous.  Returns QME_E_NUMERIC when a population
 * is not finite or the trace is not positive (outputs still written). */
qme_status qme_observe(const qme_ctx *ctx, const void *state_dev,
                       double *populations, double *trace, double *sink,
                       void *hip_stream);

/* The objective of a parameter fit (Sec. II, fourth point): a weighted sum
 * of final populations, f = sum_s weights[s] Re rho_ss (weights: host [N],
 * finite, else QME_E_ARG), summed in FP64 in index order on the host from
 * the device diagonal, exactly as qme_adjoint forms its *value.  *value is
 * written; QME_E_NUMERIC when it is not finite.  Synchronous. */
qme_status qme_observe_weighted(const qme_ctx *ctx, const void *state_dev,
                                const double *weights, double *value, void *hip_stream);

/* Gradients of a final diagonal observable f = sum_s obs[s] Re rho_K[s,s]
 * (rho_K: the state after n_steps steps from state0) with respect to the
 * Hamiltonian couplings and the decoherence rates, by the adjoint of the
 * time step (the parameter fit of the paper's fourth modelling point,
 * Sec. II, needs them).  The forward pass keeps a checkpoint every
 * checkpoint_every steps and recomputes each segment backwards.  Outputs:
 * *value = f (may be NULL) and grad[qme_gradient_size] in the order g per
 * atom (cavity-major), mu per hop, gamma per jump; for a context made by
 * qme_hamiltonian_general the Hamiltonian parameters are H's symmetric
 * entries instead -- one per pair (r, c), r <= c, of the pattern of the
 * given triplets (duplicates merged), in (r, c) order, each moving H[r][c]
 * and H[c][r] together (zero for an entry a qme_subspace restriction
 * removed) -- then gamma per jump.  The Frechet derivative of
 * exp(-i H dt) is evaluated in FP64 (on the device; on the host when the
 * propagator needed squarings); the adjoint
 * products run in the context's storage arithmetic (FP32 for QME_BF16X3,
 * whose forward recomputation still uses the split-bf16 products).  state0 is
 * not modified.  workspace: device memory of at least
 * qme_adjoint_workspace_size bytes (256-byte aligned).  Synchronous. */
qme_status qme_adjoint(qme_ctx *ctx, const void *state0_dev, int64_t n_steps,
                       int32_t checkpoint_every, const double *obs, double *value,
                       double *grad, void *workspace_dev, size_t workspace_bytes,
                       void *hip_stream);

/* Number of entries qme_adjoint writes to grad for this context. */
qme_status qme_gradient_size(const qme_ctx *ctx, int64_t *n_params);

/* Device workspace qme_adjoint needs for these arguments. */
qme_status qme_adjoint_workspace_size(const qme_ctx *ctx, int64_t n_steps,
                                      int32_t checkpoint_every, size_t *bytes);

/* ---------------------------------------------------- general models */

/* One decoherence operator A_j of Sec. II, Eq. 3, as moves: A |source[e]>
 * has the component coef[e] |target[e]>, summed over its moves (moves with
 * the same source and target add up), so a state may have several images
 * and several preimages.  target -1: a component outside the basis (its
 * probability goes to the sink), orthogonal to every other component;
 * rate gamma >= 0.  Errors (QME_E_ARG): indices out of range, non-finite
 * coefficients or rates, NULL arrays with n_moves > 0. */
typedef struct {
  double gamma;
  int64_t n_moves;
  const int32_t *source;   /* [n_moves] */
  const int32_t *target;   /* [n_moves], -1 or a basis index */
  const double *coef;      /* [n_moves] */
} qme_general_jump;

/* A context for a model given directly as matrices, for systems beyond the
 * cavity / atom / hopping structure of qme_system -- for example the
 * hydrogen-bond model of Sec. IV.A (Eqs. 4-9), whose couplings are
 * conditional on other modes and include non-RWA terms.  H: real symmetric
 * n x n as COO triplets (duplicates summed; the summed matrix must equal its
 * transpose exactly, else QME_E_ARG); jumps: decoherence operators as
 * moves (see qme_general_jump).  The step, batching, selection
 * (qme_subspace), observation and gradients (qme_adjoint, with respect to
 * H's symmetric entries and the rates) work as for qme_hamiltonian.
 * Operators that give a state at most one move and a target at most one
 * source run in the gather form of the structured channels; the others
 * (several images or preimages, e.g. collective decay of several atoms)
 * in sparse form: per element of the decoherence pass a double sum over
 * the two rows of A, plus the off-diagonal part of A^dag A.  Synchronous. */
qme_status qme_hamiltonian_general(int64_t n, int64_t h_nnz, const int32_t *h_rows,
                                   const int32_t *h_cols, const double *h_vals, int32_t n_jumps,
                                   const qme_general_jump *jumps, double dt, int32_t precision,
                                   void *hip_stream, qme_ctx **out);

/* ------------------------------------------------ state-space selection */

/* State-space selection, Sec. III.B (the loop of Fig. 2 and Table I): after a
 * solve, compute each state's probability growth speed, remove the states
 * whose speed is below eps, renormalise, and continue on the states that
 * remain.  The growth speed of state s over an interval of length `interval`
 * is read as |p_now[s] - p_prev[s]| / interval (an absolute rate of change:
 * states whose probability neither grows nor decays do not take part in the
 * dynamics).  Writes the indices of the kept states (growth >= eps) into
 * keep[0..N) in ascending order and their count into *n_keep.  eps = 0 keeps
 * every state.  Host only; p_prev / p_now: the n populations of a basis
 * (qme_observe), n >= 1.
 * Errors: QME_E_ARG for interval <= 0, eps < 0 or non-finite values;
 * QME_E_STATE (with *n_keep = 0) when every state would be removed. */
qme_status qme_select_states(int64_t n, const double *p_prev, const double *p_now,
                             double interval, double eps, int32_t *keep, int64_t *n_keep);

/* The same keep/delete decision (Sec. III.B, growth speed against epsilon)
 * taken on the device, so a selection loop need not wait for the host after
 * every solve.  Reads the populations p_now[s] = Re rho[s][s] of state_dev
 * (a state of ctx), keeps s when |p_now[s] - p_prev[s]| / interval >= eps
 * (FP64, the operations of qme_select_states, so both keep the same
 * states), and writes the kept indices in increasing order to keep_dev and
 * their count to *n_keep_dev (-1 when a population is not finite; 0 when
 * every state would be removed).  p_prev_dev, p_now_dev: [n] FP64 device
 * vectors (p_now_dev may be p_prev_dev: updated in place); keep_dev: [n]
 * int32 device; n_keep_dev: one int64 on the device.  All caller-owned.
 * Errors: QME_E_ARG for NULL pointers, interval <= 0, eps < 0 or non-finite
 * arguments.  Asynchronous on hip_stream. */
qme_status qme_select_device(const qme_ctx *ctx, const void *state_dev, const double *p_prev_dev,
                             double *p_now_dev, double interval, double eps, int32_t *keep_dev,
                             int64_t *n_keep_dev, void *hip_stream);

/* Device area qme_select_run needs (caller-allocated, 256-byte aligned): a
 * state snapshot, two population vectors, two kept-index vectors and two
 * counts. */
qme_status qme_select_workspace_size(const qme_ctx *ctx, size_t *bytes);

/* The selection loop's solves without a host round trip between them
 * (Sec. III.B, Fig. 2): up to n_solves solves of steps_per_solve steps on
 * state_dev (workspace_dev as for qme_step), each followed by the decision
 * of qme_select_device with interval = steps_per_solve * dt.  Solve i + 1 is
 * queued from a snapshot of solve i's result before the host reads solve
 * i's count; when that count is below n (states to remove) the queued solve
 * is dropped and the state restored, so the run stops with the state of the
 * solve that decided.  fresh = 1 takes the populations the first solve
 * compares against from state_dev; fresh = 0 takes those the previous run
 * on this select area left (the populations of its last solve).  On return:
 * *solves_done = solves whose results stand; *n_keep = n when no decision
 * removed states, else the deciding solve's count with keep_host[0..n_keep)
 * ([n] int32 host, caller-owned) its kept states in increasing order.
 * Returns after the last decision is read (the stream is synchronised when
 * states are removed).  Errors: QME_E_ARG as for qme_step and for
 * n_solves < 0, steps_per_solve < 1, eps < 0 or not finite; QME_E_NUMERIC
 * when a population is not finite, QME_E_STATE when every state would be
 * removed (both with *solves_done and *n_keep set). */
qme_status qme_select_run(qme_ctx *ctx, void *state_dev, void *workspace_dev, void *select_ws_dev,
                          int64_t n_solves, int64_t steps_per_solve, double eps, int32_t fresh,
                          int64_t *solves_done, int64_t *n_keep, int32_t *keep_host,
                          void *hip_stream);

/* A context on the subset keep[0..n_keep) of ctx's basis (strictly
 * increasing indices, order kept), with ctx's parameters and precision: the
 * Hamiltonian restricted to the subset (P H P), decoherence operators whose
 * image leaves the subset counted in the sink as for the excitation window,
 * and a new propagator (Taylor stage).  Synchronous. */
qme_status qme_subspace(const qme_ctx *ctx, const int32_t *keep, int64_t n_keep,
                        void *hip_stream, qme_ctx **out);

/* Moves a state of `from` onto the subset context `to` (made by
 * qme_subspace from a context with from's basis):
 *   rho_to = P rho P * (1 - sink) / tr(P rho P),   sink_to = sink_from,
 * the renormalisation of Sec. III.B.  Scalar 2 of the new state (see
 * qme_state_layout) holds the probability the removed states had.  The two
 * buffers must differ.  Asynchronous on hip_stream. */
qme_status qme_compact_state(const qme_ctx *from, const void *state_from_dev,
                             const qme_ctx *to, void *state_to_dev, void *hip_stream);

/* ----------------------------------------------- pure states, closed models */

/* Sec. IV.B: the single photon on the plane of cavities is a closed system
 * (no leakage), so a pure start stays pure.  For a model with no
 * decoherence operator acting on its basis the step of qme_step maps
 * rho = psi psi^dag to psi' psi'^dag with psi' = U psi / |psi| (the
 * dissipator and the sink are zero, the symmetrisation leaves psi psi^dag
 * unchanged, the trace renormalisation divides by |psi|^2), so these calls
 * advance psi instead of rho: O(N^2) work per step instead of O(N^3).
 *
 * A pure state of n_vec vectors (1 <= n_vec <= QME_PURE_MAX_VECTORS) is
 * device memory owned by the caller: the real plane [n_vec][ld] then the
 * imaginary plane [n_vec][ld] in the context's storage precision (ld from
 * qme_state_layout, entries >= N zero).  The vectors evolve independently.
 * FP32 and FP64 contexts only (QME_E_UNSUPPORTED for QME_BF16X3). */
#define QME_PURE_MAX_VECTORS 4

/* Bytes of a pure state of n_vec vectors and of the workspace qme_pure_step
 * needs (each a multiple of 256; either pointer may be NULL). */
qme_status qme_pure_layout(const qme_ctx *ctx, int32_t n_vec, size_t *state_bytes,
                           size_t *workspace_bytes);

/* Write a pure state from host arrays psi_re / psi_im (n_vec x N, vector v
 * at [v * N], FP64), converted to the storage precision, padding zeroed.
 * QME_E_ARG for non-finite values or a zero vector.  Synchronous. */
qme_status qme_pure_set(const qme_ctx *ctx, void *state_dev, int32_t n_vec,
                        const double *psi_re, const double *psi_im, void *hip_stream);

/* Read a pure state into host arrays (n_vec x N, FP64; either may be NULL).
 * Synchronous. */
qme_status qme_pure_get(const qme_ctx *ctx, const void *state_dev, int32_t n_vec,
                        double *psi_re, double *psi_im, void *hip_stream);

/* Advance every vector by n_steps steps psi <- (psi + dU psi) / |psi|, with
 * dU = U - I the context's propagator and |psi| summed in FP64 from the
 * stored vector; the stored result is U applied to a unit vector.  One
 * launch per step.  state_dev and workspace_dev (qme_pure_layout bytes)
 * are 256-byte aligned and do not overlap.  QME_E_STATE when a decoherence
 * operator acts on the basis (the state would not stay pure).
 * Asynchronous on hip_stream. */
qme_status qme_pure_step(qme_ctx *ctx, void *state_dev, int32_t n_vec, int64_t n_steps,
                         void *workspace_dev, void *hip_stream);

/* ------------------------------------------------------- batched instances */

typedef struct qme_batch qme_batch;

/* Sec. II, third point (the time steps), for many independent instances at
 * once (a parameter sweep).
 * Bind `count` FP32 contexts and their device state buffers (one each,
 * layouts from qme_state_layout, 256-byte aligned) into a batch.  Each step
 * of the batch is one launch per phase (first product, lower-triangle
 * product, trace/sink pass, decoherence pass) covering the tiles of every
 * instance, largest instances first; a run of n steps is captured once into
 * a hipGraph and replayed.  Each instance's two products run in the tile
 * edges of its context (qme_set_tiles; 32 or 64, else QME_E_UNSUPPORTED),
 * read when the batch is created or configured.  Each instance advances
 * exactly as under qme_step with the same tiles, unfolded and unsplit (the
 * same tile arithmetic: bitwise-identical results).  The contexts and
 * states must outlive the batch. */
qme_status qme_batch_create(qme_ctx *const *ctxs, void *const *states_dev, int32_t count,
                            qme_batch **out);

/* Device workspace of a batch (the products' scratch planes of every
 * instance). */
qme_status qme_batch_workspace_size(const qme_batch *batch, size_t *bytes);

/* Whether runs are captured into (and replayed from) a hipGraph per
 * (n_steps, workspace), and whether larger instances come first in each
 * phase launch.  Rebuilds the batch's tables from the contexts' current
 * tiles (set them with qme_set_tiles, then call this) and drops earlier
 * captures.  Synchronises the device. */
qme_status qme_batch_config(qme_batch *batch, int32_t use_graph, int32_t largest_first);

/* Persistent form of the batched run (off by default): with enable = 1 a run
 * of n steps is ONE launch in which workgroups take (step, phase, instance,
 * tile) items in order from a global counter and each item waits only until
 * its own instance has finished the earlier phases (per-instance counters in
 * the batch workspace), so a small instance's next phase starts while large
 * instances are still in their last tiles.  Items are taken in order, so the
 * waits cannot deadlock whatever the number of resident workgroups; a wait
 * that exceeds a fixed bound ends the run and every instance's sink becomes
 * NaN (qme_observe then returns QME_E_NUMERIC).  Same tile arithmetic as the
 * phase launches: bitwise-identical results.  QME_E_SIZE from qme_batch_step
 * when a run is too long for the 32-bit counters (then split it).
 * Synchronises the device.
 * Switched off in this version: enable = 1 returns QME_E_UNSUPPORTED (the
 * launches did not finish on the device and the cause has not been
 * established); enable = 0 keeps the phase launches. */
qme_status qme_batch_persistent(qme_batch *batch, int32_t enable);

/* Advance every instance by n_steps on hip_stream (asynchronous). */
qme_status qme_batch_step(qme_batch *batch, int64_t n_steps, void *workspace_dev,
                          size_t workspace_bytes, void *hip_stream);

/* Release a batch (not its contexts or states). NULL is ignored. */
void qme_batch_destroy(qme_batch *batch);

/* The planar complex product used by every step and by the adjoint:
 *     C = alpha * opA(A) * opB(B) + beta * X
 * on ld x ld row-major planes in device memory (FP64 for QME_FP64, FP32 for
 * QME_FP32; x_re / x_im may be NULL when beta == 0).  opA(A) = conj(A) if
 * conj_a else A.  With b_rows != 0 the second operand (m_*) is B itself,
 * read row-major; otherwise it is M and B = M^T, i.e. the operand is read by
 * rows j.  opB = conj(B) if conj_b else B (so b_rows = 0, conj_b = 1 gives
 * M^H).  lower != 0 computes only the tile x tile blocks on or below the
 * diagonal.  tile: 128, 64 or 32 (FP32), 64 or 32 (FP64), 64 (QME_BF16X3: FP32
 * planes, split-bf16 products, b_rows must be 0); ld must be a multiple of
 * tile.  C must not overlap A or B; C may equal X (accumulation).
 * Asynchronous on hip_stream. */
qme_status qme_cgemm(int32_t precision, int64_t ld, const void *a_re_dev,
                     const void *a_im_dev, const void *m_re_dev, const void *m_im_dev,
                     const void *x_re_dev, const void *x_im_dev, void *c_re_dev,
                     void *c_im_dev, double alpha, double beta, int32_t conj_a,
                     int32_t conj_b, int32_t b_rows, int32_t lower, int32_t tile,
                     void *hip_stream);

/* Tile edge of the two products of each step (the autotuner's knob):
 * tile1 for T = rho + dU rho, tile2 for the lower-triangle product.
 * FP32 tiles: 128, 64 or 32; FP64 tiles: 64 or 32; BF16X3: tile2 64, tile1
 * 64 or 128 (128: the first product on 128 x 64 tiles, bitwise-identical
 * results; a split first product still takes 64-tiles).  Each must divide the
 * state's leading dimension ld (qme_state_layout), else QME_E_ARG.  Defaults:
 * FP64 32; FP32 32 when the full product in 64-tiles would give fewer than
 * four workgroups per compute unit, else 64; BF16X3 64, with tile1 128 when
 * ld is a multiple of 128 and the 128 x 64 tiles number at least twice the
 * compute units. */
qme_status qme_set_tiles(qme_ctx *ctx, int32_t tile1, int32_t tile2);

/* The tile edges the context's two products use now (defaults or
 * qme_set_tiles). */
qme_status qme_get_tiles(const qme_ctx *ctx, int32_t *tile1, int32_t *tile2);

/* Split of the products along k (on by default).  Tail split: when the
 * lower-triangle product's tile count exceeds a multiple of the device's
 * compute-unit count by a small remainder, the remainder tiles are computed
 * in k-chunks that fill the otherwise idle units, their partials in the
 * output state's planes, which the step overwrites afterwards.  Small-launch
 * split (every precision): a product with at most half as many tiles
 * as compute units has every tile computed in k-chunks of at least two K
 * tiles, their partials in the workspace's slots (qme_workspace_size).  A
 * reduce pass sums each tile's chunks in k order.  Results differ from the
 * unsplit products only by FP rounding (the k sum is regrouped) and are
 * deterministic for a given (ld, tile, device).  enable: 0 or 1, else
 * QME_E_ARG. */
qme_status qme_set_split(qme_ctx *ctx, int32_t enable);

/* Single-workgroup path (on by default): for FP32 and FP64 contexts with
 * N <= 32, qme_step runs all its steps in one launch of one workgroup per
 * 4096 steps, the state and dU held in LDS.  The arithmetic is the same step;
 * the products accumulate with scalar FMAs in k order instead of MFMA, so
 * results differ from the tiled path by rounding only.  With profiling on,
 * such a launch is counted under index 0 of qme_profile_read.  enable: 0 or
 * 1, else QME_E_ARG. */
qme_status qme_set_fused(qme_ctx *ctx, int32_t enable);

/* Folded steps (on by default).  For a model in which no decoherence
 * operator maps a basis state onto another basis state (every jump leaves
 * the basis, as the boundary leaks of the single-excitation lattice do), the
 * decoherence step is one factor per element, (1 - dt (d_u + d_v) / 2): the
 * lower-triangle product applies it in its epilogue and writes the state
 * (both triangles) directly, the trace pass reads the diagonal it stored,
 * and the renormalisation factor is applied by the next step's first
 * product (its scalars come from the state's scalars on the device) and,
 * after the last step of a qme_step call, by one pass over the state.  This
 * is the renormalisation "folded into the next product" and saves the
 * decoherence pass.  Applies to FP32 contexts whose lower-product tile is 64
 * or 32, and to FP64 and BF16X3 contexts; results differ from the unfolded
 * step by rounding only.  enable: 0 or 1, else QME_E_ARG. */
qme_status qme_set_fold(qme_ctx *ctx, int32_t enable);

/* Tile body of the FP32 products whose second operand is read by rows (all
 * products of qme_step and the first two of the adjoint step): mode 1 loads
 * the operand tiles from HBM straight into LDS (no register staging), 0
 * stages them through registers, -1 (default) takes the direct body for
 * launches with fewer than two blocks per compute unit, where the few
 * resident workgroups cannot hide the load latency by their number.  With a
 * mode other than 0, 32-tile products of a state with ld <= 192 load every K
 * tile of their row panels into LDS at once and are not split along k (mode
 * 0: staged per K tile, split as qme_set_split says).  The bodies accumulate
 * every output in the same order: results are bitwise identical (with the
 * split off).  Other values: QME_E_ARG. */
qme_status qme_set_direct_loads(qme_ctx *ctx, int32_t mode);

/* Graph replay of qme_step (off by default): with enable = 1, a call of
 * n_steps on a given (state, workspace) pair is captured once into a
 * hipGraph on a private stream and replayed onto the caller's stream with
 * one launch, which removes the host's per-kernel launch cost from
 * launch-bound sizes; results are bitwise those of the eager call.  Any knob
 * change (tiles, split, fold, fused, direct loads, this one) drops the
 * captures after synchronising the device; with profiling enabled the call
 * runs eagerly.  Calls that overlap on one context race (as eager ones do).
 * enable: 0 or 1, else QME_E_ARG. */
qme_status qme_set_graph(qme_ctx *ctx, int32_t enable);

/* Per-kernel timing of qme_step with HIP events recorded on the caller's
 * stream around every launch (the tracing facility used by the benchmark).
 * enable > 0 starts recording (and clears earlier records) on every
 * enable-th step counted from this call (1: every step; a larger stride
 * keeps the events' own cost out of the other steps); 0 stops it; negative:
 * QME_E_ARG. */
qme_status qme_profile_enable(qme_ctx *ctx, int32_t enable);

/* Synchronises on the recorded events and returns, per kernel kind, the
 * summed duration in milliseconds and the number of launches since the last
 * enable: kind 0 = first product (full), 1 = second product (lower tiles),
 * 2 = trace/sink pass, 3 = decoherence pass.  Arrays of 4 (either may be
 * NULL).  Recording stays enabled. */
qme_status qme_profile_read(qme_ctx *ctx, double *total_ms, int64_t *launches);

/* Release a context and its device tables. NULL is ignored. */
void qme_destroy(qme_ctx *ctx);

/* Text of the last error on this thread ("" if none). */
const char *qme_last_error(void);

/* Library version string. */
const char *qme_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QME_H */
