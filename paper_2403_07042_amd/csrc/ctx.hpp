// The opaque context behind qme_ctx (internal).
#pragma once

#include <cstdint>
#include <map>
#include <memory>
#include <tuple>
#include <vector>

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include "device.hpp"
#include "model.hpp"
#include "qme.h"

struct qme_ctx {
  qme::Model model;
  qme::Csr h;                         // Hamiltonian (host, FP64)
  qme::JumpTables jt;
  std::vector<double> du_re_host, du_im_host;   // dU = U - I, FP64, n x n
  int precision = QME_FP32;
  int64_t elem = 4;                   // storage bytes per real
  int64_t n = 0, ld = 0;
  int tile1 = 64, tile2 = 64;         // tiles of the two products of a step
  bool tail_split = true;             // qme_set_split
  bool fused = true;                  // qme_set_fused (single-workgroup path, n <= 32)
  bool fold = true;                   // qme_set_fold (decoherence folded into the products)
  int direct = -1;                    // qme_set_direct_loads (-1 auto, 0 off, 1 on)
  size_t split_elems = 0;             // partial slots of small-launch splits (elements)
  // qme_set_graph: a run of n steps captured once per (n, state, workspace)
  // into a hipGraph and replayed; any knob change drops the captures
  bool use_graph = false;
  std::map<std::tuple<int64_t, void *, void *>, hipGraphExec_t> graphs;
  std::vector<hipGraph_t> graph_defs;
  hipStream_t capture_stream = nullptr;
  void drop_graphs();
  int device = 0;
  int cus = 0;                        // compute units of the device
  void *scratch = nullptr;            // device address of the no-allocation workspace
  // device tables (owned)
  void *du_re = nullptr, *du_im = nullptr;   // dU planes, ld x ld, storage type
  void *du_split = nullptr;                  // BF16X3: dU as six bf16 planes (split once)
  double *d = nullptr, *leak = nullptr, *diag = nullptr;
  double *trw = nullptr;              // trace weights (DissArgs::trw)
  int32_t *pi = nullptr;
  double *cg = nullptr;
  // sparse (non-monomial) channels of general-form models (JumpTables)
  int64_t *csr_ptr = nullptr, *csrt_ptr = nullptr, *kj_ptr = nullptr, *koff_ptr = nullptr;
  int32_t *csr_col = nullptr, *csrt_col = nullptr, *kj_col = nullptr, *koff_col = nullptr;
  double *csr_val = nullptr, *csrt_val = nullptr, *kj_val = nullptr, *koff_val = nullptr;
  double *csr_gamma = nullptr;
  int32_t *csr_channel = nullptr;     // original jump index per sparse channel
  int32_t *loff_row = nullptr, *loff_col = nullptr;
  double *loff_val = nullptr;
  // the decoherence and trace passes' arguments for these tables
  template <typename T>
  void sparse_args(qme::DissArgs<T> &a) const {
    a.self_mask = self_mask;
    a.n_csr = jt.n_csr;
    a.csr_ptr = csr_ptr;
    a.csr_col = csr_col;
    a.csr_val = csr_val;
    a.csr_gamma = csr_gamma;
    a.koff_ptr = jt.koff_col.empty() ? nullptr : koff_ptr;
    a.koff_col = koff_col;
    a.koff_val = koff_val;
    a.n_loff = int64_t(jt.loff_val.size());
    a.loff_row = loff_row;
    a.loff_col = loff_col;
    a.loff_val = loff_val;
  }
  // adjoint tables (owned)
  int32_t *tau = nullptr;     // [n_gather x n]
  uint32_t self_mask = 0;     // DissArgs::self_mask of the gather channels
  double *ca = nullptr;
  int32_t *upi = nullptr;     // [n_arrival x n]
  double *uc = nullptr;
  double *ada = nullptr;      // [n_jumps x n]
  int32_t *arrival_of = nullptr;   // [n_jumps]
  int n_arrival = 0;
  // Hamiltonian (CSR, FP64) and the per-parameter term entries, for the
  // device-side Frechet finalisation of the adjoint
  int64_t *h_ptr = nullptr;
  int32_t *h_col = nullptr;
  double *h_val = nullptr;
  int32_t *t_row = nullptr, *t_col = nullptr;
  double *t_val = nullptr;
  std::vector<int64_t> term_offset;   // host: entries of term p are [off[p], off[p+1])
  int squarings = 0;                  // of the propagator build
  // failure injection for recovery tests: when QME_FAULT_AT_STEP=k is set in
  // the environment at context creation, qme_step stops after the context's
  // k-th step and returns QME_E_DEVICE (-1: off); steps_done counts the
  // steps qme_step has enqueued on this context
  int64_t fault_at = -1;
  int64_t steps_done = 0;
  // a context made by qme_subspace: the kept indices into its parent's basis
  int32_t *parent_keep = nullptr;     // device, [n]
  int64_t parent_n = 0, parent_ld = 0;
  double h_norm1 = 0.0;               // |H|_1

  // per-kernel timing (qme_profile_enable / qme_profile_read): on a sampled
  // step every launch takes a start / stop event pair that its own dispatch
  // stamps (qme::launch_kernel); each record groups the pairs of one kernel
  // kind of one step
  bool profiling = false;
  int profile_every = 1;               // record every profile_every-th step
  int64_t profile_step = 0;            // steps begun since enabling
  std::vector<void *> ev_start, ev_stop;   // hipEvent_t pools
  // qme_select_run: the decisions' counts in pinned host memory, one event
  // per slot (made on first use)
  int64_t *sel_count_host = nullptr;
  void *sel_ev[2] = {nullptr, nullptr};
  size_t pairs_used = 0, pairs_marked = 0;
  struct ProfileRecord {
    int kind;
    size_t first, last;                // pairs [first, last)
  };
  std::vector<ProfileRecord> records;
  struct Timer final : qme::LaunchTimer {
    qme_ctx *c = nullptr;
    hipError_t next_pair(hipEvent_t *start, hipEvent_t *stop) override;
  } timer;

  qme_ctx() = default;
  qme_ctx(const qme_ctx &) = delete;
  qme_ctx &operator=(const qme_ctx &) = delete;
  ~qme_ctx();   // frees the device tables
};

namespace qme {
// A roctx range over a scope (host side: the enqueue, or the whole call for
// synchronous entry points), shown by `rocprofv3 --marker-trace`.
struct TraceRange {
  explicit TraceRange(const char *name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange &) = delete;
  TraceRange &operator=(const TraceRange &) = delete;
};
int64_t round_up(int64_t x, int64_t m);
size_t plane_elems(const qme_ctx *c);
size_t state_bytes(const qme_ctx *c);
qme_status check_device(const qme_ctx *c);
// One time step from state `in` to state `out` (may alias) with the two
// workspace plane pairs y (product T) and z (rotated state, lower tiles).
template <typename T>
// split_area: the step workspace's partial slots for small-launch splits
// (nullptr: no such splits, as in the adjoint's recomputation).  parity >= 0:
// the trace is formed in the decoherence pass (fuse_trace_applies), reading
// the scalars from slot pair `parity` and writing them to the other one.
hipError_t step_once(qme_ctx *c, const void *in, void *out, void *y, void *z, hipStream_t s,
                     void *split_area = nullptr, int parity = -1);
bool uses_small_path(const qme_ctx *c);
bool uses_fold(const qme_ctx *c);
// Whether the unfolded step forms the trace inside the decoherence pass
// (every block reads the N diagonal values itself: small systems).
bool fuse_trace_applies(const qme_ctx *c);
}  // namespace qme
