// Batched time steps of many independent instances of uneven size.
//
// Every instance's step is the same four phases as the per-instance path
// (product T = rho + dU rho, lower-triangle product rho_u, FP64 trace/sink
// pass, decoherence pass; Sec. II Eqs. 2-3 and the "unitary evolution" stage
// of Sec. IV.B).  One launch per phase covers that phase's tiles of EVERY
// instance (instances ordered largest first; a block finds its instance and
// tile by a binary search over per-instance item offsets), so the grid stays
// full even when single instances are small.  Phases are ordered by the
// stream, never by waits between workgroups.  A run of n steps (4 n
// launches) is captured once into a hipGraph and replayed with one launch.
// Each instance's products run in the tile edges of its context (32 or 64,
// qme_set_tiles; the autotuner picks them per size), and the tile arithmetic
// is the per-instance kernels' own, so every instance advances bitwise as
// under qme_step with the same tiles (unfolded, unsplit).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "cgemm_tile.hpp"
#include "ctx.hpp"
#include "device.hpp"
#include "dissipate_tile.hpp"
#include "qme.h"

namespace qme {

struct BatchInstance {
  float *x_re, *x_im;
  double *aux;
  float *y_re, *y_im, *z_re, *z_im;
  const float *u_re, *u_im;
  const double *d, *leak, *cg, *trw;
  const int32_t *pi;
  int64_t n, ld;
  double dt;
  int32_t edge1, edge2;   // tile edges of the two products (32 or 64)
  int32_t tiles1, tiles2; // ld / edge
  int32_t n_gather;
  uint32_t items[4];   // per phase: tiles1^2, lower tiles2, 1, lower tiles (decoherence)
  DissArgs<float> sparse;   // the sparse-channel fields only (see DissArgs)
};

struct BatchPhase {
  const BatchInstance *inst;
  const int32_t *order;        // queue position -> instance
  const int64_t *off;          // [count + 1] item prefix of this phase per queue position
  int32_t count;
  // phases 2 and 3: scalar slot pairs of the step (DissArgs::slot_in /
  // slot_out) and, for phase 3, whether each block forms the trace itself
  int32_t slot_in = 0, slot_out = 0, fuse = 0;
};

static constexpr int kBatchThreads = 256;

__device__ __forceinline__ void tri_coords(int t, int &bi, int &bj) {
  int r = int((sqrtf(8.0f * float(t) + 1.0f) - 1.0f) * 0.5f);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  bi = r;
  bj = t - r * (r + 1) / 2;
}

constexpr int kGemmSmem = cgemm_f32_smem<64, kConjB>() > cgemm_s_smem<float, 32, kConjB>()
                              ? cgemm_f32_smem<64, kConjB>()
                              : cgemm_s_smem<float, 32, kConjB>();
template <int PHASE>
constexpr int phase_smem() {
  return PHASE <= 1 ? kGemmSmem
         : PHASE == 2 ? 3 * kBatchThreads * 2
                      : 2 * TD * (TD + 1) + int(sizeof(GatherLds) / sizeof(float)) + 2 +
                            3 * 2 * (kBatchThreads / 64);
}
constexpr int kPersistSmem =
    std::max(std::max(phase_smem<0>(), phase_smem<1>()), std::max(phase_smem<2>(), phase_smem<3>()));

// One item of a phase: tile `tile` of the instance at queue position `pos`.
// PHASE 3 with SPARSE: the decoherence body with the sparse channels' terms.
template <int PHASE, bool SPARSE>
__device__ __forceinline__ void batch_item(const BatchInstance &in, int tile, float *smem,
                                           int slot_in = 0, int slot_out = 0, bool fuse = false) {
  if constexpr (PHASE == 0) {
    const CgemmArgs<float> g{in.u_re, in.u_im, in.x_re, in.x_im, in.x_re, in.x_im,
                             in.y_re, in.y_im, in.ld, 1.0f, 1.0f};
    if (in.edge1 == 32)
      cgemm_s_tile<float, 32, kConjB>(g, tile / in.tiles1, tile % in.tiles1, smem);
    else
      cgemm_f32_tile<64, kConjB>(g, tile / in.tiles1, tile % in.tiles1, smem);
  } else if constexpr (PHASE == 1) {
    int bi, bj;
    tri_coords(tile, bi, bj);
    const CgemmArgs<float> g{in.y_re, in.y_im, in.u_re, in.u_im, in.y_re, in.y_im,
                             in.z_re, in.z_im, in.ld, 1.0f, 1.0f};
    if (in.edge2 == 32)
      cgemm_s_tile<float, 32, kConjB>(g, bi, bj, smem);
    else
      cgemm_f32_tile<64, kConjB>(g, bi, bj, smem);
  } else {
    DissArgs<float> da{in.z_re, in.z_im, in.x_re, in.x_im, in.ld, in.n, in.dt, in.d,
                       in.leak, in.pi, in.cg, in.n_gather, in.aux, in.aux, in.trw};
    da.self_mask = in.sparse.self_mask;
    da.n_csr = in.sparse.n_csr;
    da.csr_ptr = in.sparse.csr_ptr;
    da.csr_col = in.sparse.csr_col;
    da.csr_val = in.sparse.csr_val;
    da.csr_gamma = in.sparse.csr_gamma;
    da.koff_ptr = in.sparse.koff_ptr;
    da.koff_col = in.sparse.koff_col;
    da.koff_val = in.sparse.koff_val;
    da.n_loff = in.sparse.n_loff;
    da.loff_row = in.sparse.loff_row;
    da.loff_col = in.sparse.loff_col;
    da.loff_val = in.sparse.loff_val;
    da.slot_in = slot_in;
    da.slot_out = slot_out;
    if constexpr (PHASE == 2) {
      double *sd = reinterpret_cast<double *>(smem);
      trace_body<float, kBatchThreads>(da, sd, sd + kBatchThreads, sd + 2 * kBatchThreads);
    } else {
      float (*sr)[TD + 1] = reinterpret_cast<float (*)[TD + 1]>(smem);
      float (*si)[TD + 1] = reinterpret_cast<float (*)[TD + 1]>(smem + TD * (TD + 1));
      // 8-byte aligned start for the tables after the two staging arrays
      float *gp = smem + 2 * TD * (TD + 1);
      gp += (reinterpret_cast<uintptr_t>(gp) & 7) ? 1 : 0;
      double *st = reinterpret_cast<double *>(gp + sizeof(GatherLds) / sizeof(float));
      // the fused form: this block forms the instance's trace itself (the
      // first tile's block stores the step's scalars)
      const double scale = fuse ? trace_body<float, kBatchThreads>(da, st, st + kBatchThreads / 64,
                                                                   st + 2 * (kBatchThreads / 64),
                                                                   tile == 0)
                                : in.aux[4];
      dissipate_tile<float, SPARSE>(da, tile, [scale]() { return scale; }, sr, si,
                                    reinterpret_cast<GatherLds *>(gp));
    }
  }
}

// Queue position of item r of a phase (largest position with off[pos] <= r).
__device__ __forceinline__ int find_position(const int64_t *off, int count, int64_t r) {
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= r) lo = mid; else hi = mid;
  }
  return lo;
}

template <int PHASE, bool SPARSE = false>
__global__ __launch_bounds__(kBatchThreads) void batch_phase_kernel(BatchPhase p) {
  __shared__ float smem[phase_smem<PHASE>()];
  const int64_t r = blockIdx.x;
  const int lo = find_position(p.off, p.count, r);
  batch_item<PHASE, SPARSE>(p.inst[p.order[lo]], int(r - p.off[lo]), smem, p.slot_in, p.slot_out,
                            p.fuse != 0);
}

// After a run of fused steps that ended in slot pair 1, every instance's
// sink and step count move back to pair 0.
__global__ void batch_scalars_home_kernel(const BatchInstance *inst, int count) {
  const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double *aux = inst[i].aux;
  aux[sink_slot(0)] = aux[sink_slot(1)];
  aux[steps_slot(0)] = aux[steps_slot(1)];
}

// ------------------------------------------------------------ persistent form
// One launch runs every step of a run.  The items are (step, phase,
// instance, tile) in that order (instances largest first inside a phase);
// each workgroup takes the next item from a global counter, waits until the
// item's instance has finished every item of the earlier phases and steps
// (a per-instance completion counter), runs it, and counts it done.
//   * Progress: items are taken in order and an item waits only on items of
//     smaller index, so the earliest unfinished item has all its
//     predecessors taken -- hence finished -- and proceeds: no deadlock,
//     whatever the number of resident workgroups.
//   * Visibility across XCDs (each has its own L2): after the workgroup
//     barrier that ends an item, one thread increments the counter with an
//     agent-scope release (it writes the L2's dirty lines back first).  The
//     wait polls with relaxed agent-scope loads, which read the counter past
//     the caches without invalidating them, and acquires once, when the
//     count is reached; every wave then acquires after the barrier that ends
//     the wait.  (An acquire on every poll would invalidate the caches of
//     the compute unit on every iteration of every waiting workgroup and
//     starve the items that are running.)
//   * Termination: a wait gives up after spin_limit polls or wait_ticks of
//     the 100 MHz real-time counter (far above any real wait), sets the
//     abort flag and leaves; every workgroup checks the flag before taking
//     an item and every 64 polls, so the launch ends.  A closing pass then
//     marks every instance's sink NaN (qme_observe reports
//     QME_E_NUMERIC).
struct PersistArgs {
  const BatchInstance *inst;
  const int32_t *order;
  const int64_t *phase_off;   // [4][count + 1]
  int32_t count;
  int64_t phase_items[4];
  int64_t per_step, total;
  uint32_t *done;             // [count], per queue position
  unsigned long long *next;
  uint32_t *abort_flag;
  uint32_t spin_limit;
  uint64_t wait_ticks;        // bound of one wait on the 100 MHz real-time counter
};

// (four waves per SIMD, the phase kernels' own occupancy: the bound keeps the
// four inlined bodies within the register budget of one of them)
template <bool SPARSE>
__global__ __launch_bounds__(kBatchThreads, 4) void batch_persistent_kernel(PersistArgs a) {
  __shared__ float smem[kPersistSmem];
  __shared__ int s_item;
  __shared__ int s_go;
  for (;;) {
    if (threadIdx.x == 0) {
      int g = -1;
      if (__hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
        const unsigned long long t =
            __hip_atomic_fetch_add(a.next, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (t < (unsigned long long)a.total) g = int(t);
      }
      s_item = g;
    }
    __syncthreads();
    // the item is the same for the whole workgroup: keep it (and everything
    // derived from it) in scalar registers
    const int g = __builtin_amdgcn_readfirstlane(s_item);
    if (g < 0) return;
    const int64_t k = g / a.per_step;
    int64_t r = g - k * a.per_step;
    int ph = 0;
    while (r >= a.phase_items[ph]) r -= a.phase_items[ph++];
    const int64_t *off = a.phase_off + ph * (a.count + 1);
    const int pos = find_position(off, a.count, r);
    const BatchInstance &in = a.inst[a.order[pos]];
    const int tile = int(r - off[pos]);
    __syncthreads();   // every wave has read s_item before it is written again
    if (threadIdx.x == 0) {
      uint32_t per_inst = 0, before = 0;
      for (int q = 0; q < 4; ++q) {
        per_inst += in.items[q];
        if (q < ph) before += in.items[q];
      }
      const uint32_t need = uint32_t(k) * per_inst + before;
      uint32_t spins = 0;
      int go = 1;
      if (__hip_atomic_load(a.done + pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        while (__hip_atomic_load(a.done + pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          ++spins;
          if ((spins & 63u) == 0u) {
            if (spins > a.spin_limit || __builtin_amdgcn_s_memrealtime() - t0 > a.wait_ticks) {
              __hip_atomic_store(a.abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              go = 0;
              break;
            }
            if (__hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
              go = 0;
              break;
            }
          }
          __builtin_amdgcn_s_sleep(8);
        }
      }
      if (go) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      s_go = go;
    }
    __syncthreads();
    if (!__builtin_amdgcn_readfirstlane(s_go)) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    switch (ph) {
      case 0: batch_item<0, SPARSE>(in, tile, smem); break;
      case 1: batch_item<1, SPARSE>(in, tile, smem); break;
      case 2: batch_item<2, SPARSE>(in, tile, smem); break;
      default: batch_item<3, SPARSE>(in, tile, smem); break;
    }
    __syncthreads();   // every wave's writes done; LDS free for the next item
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(a.done + pos, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Counters of a persistent run set to zero (a kernel, not a memset, so the
// run can sit in a captured graph).
__global__ void persist_reset_kernel(uint32_t *done, int count, unsigned long long *next,
                                     uint32_t *abort_flag) {
  const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) done[i] = 0u;
  if (i == 0) {
    *next = 0ull;
    *abort_flag = 0u;
  }
}

// After a persistent run: if it gave up, every instance's sink becomes NaN.
__global__ void persist_finish_kernel(const BatchInstance *inst, int count,
                                      const uint32_t *abort_flag) {
  const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count && *abort_flag != 0u) inst[i].aux[0] = __builtin_nan("");
}

}  // namespace qme

using namespace qme;

struct qme_batch {
  std::vector<qme_ctx *> ctxs;
  std::vector<void *> states;
  int device = 0;
  int32_t count = 0;
  bool use_graph = true;
  bool lpt = true;
  bool sparse = false;              // some instance has sparse decoherence channels
  bool persistent = false;          // qme_batch_persistent
  bool fuse = false;                // every instance small: the trace formed in the decoherence phase
  int resident = 0;                 // workgroups of the persistent kernel that fit the device
  size_t ctr_off = 0;               // workspace offset of the persistent run's counters
  // device tables (owned)
  BatchInstance *inst = nullptr;
  int32_t *order = nullptr;
  int64_t *phase_off = nullptr;   // [4][count + 1]
  int64_t phase_items[4] = {0, 0, 0, 0};
  size_t ws_bytes = 0;
  std::vector<size_t> ws_off;      // per instance: Y planes offset (Z follows)
  hipStream_t capture_stream = nullptr;
  std::map<std::pair<int64_t, void *>, hipGraphExec_t> graphs;
  std::vector<hipGraph_t> graph_defs;
  void *last_ws = nullptr;

  void drop_graphs() {
    for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
    for (hipGraph_t g : graph_defs) (void)hipGraphDestroy(g);
    graph_defs.clear();
  }
  void drop_tables() {
    for (void *p : {(void *)inst, (void *)order, (void *)phase_off})
      if (p) (void)hipFree(p);
    inst = nullptr;
    order = nullptr;
    phase_off = nullptr;
    last_ws = nullptr;
  }
  ~qme_batch() {
    drop_graphs();
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    drop_tables();
  }
};

#define B_OK(call)                                                               \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) {                                                      \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));              \
      return QME_E_DEVICE;                                                       \
    }                                                                            \
  } while (0)

static size_t a256(size_t x) { return (x + 255) / 256 * 256; }

static qme_status build_tables(qme_batch *b) {
  const int nb = b->count;
  b->sparse = false;
  // The trace formed by every block of the decoherence phase saves the trace
  // phase's launch but repeats an instance's diagonal sums in each of its
  // blocks: kept while the phase is one round of blocks (up to four per CU),
  // where the launch costs more (measured on the 256-instance sweep, 11840
  // blocks: a separate trace phase 1135 -> 1176 batched steps/s).
  b->fuse = true;
  int64_t blocks3 = 0;
  int cus = 0;
  for (qme_ctx *c : b->ctxs) {
    b->fuse = b->fuse && fuse_trace_applies(c);
    const int64_t td = (c->n + TD - 1) / TD;
    blocks3 += td * (td + 1) / 2;
    cus = std::max(cus, c->cus);
  }
  if (blocks3 > 4 * int64_t(std::max(cus, 1))) b->fuse = false;
  std::vector<int32_t> ord(nb);
  std::iota(ord.begin(), ord.end(), 0);
  if (b->lpt)
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int x, int y) { return b->ctxs[x]->n > b->ctxs[y]->n; });
  std::vector<BatchInstance> tab(nb);
  b->ws_off.assign(nb, 0);
  size_t off = 0;
  for (int i = 0; i < nb; ++i) {
    qme_ctx *c = b->ctxs[i];
    const size_t pe = plane_elems(c);
    BatchInstance &t = tab[i];
    t.x_re = static_cast<float *>(b->states[i]);
    t.x_im = t.x_re + pe;
    t.aux = reinterpret_cast<double *>(t.x_im + pe);
    b->ws_off[i] = off;
    off += a256(4 * pe * sizeof(float));
    t.y_re = t.y_im = t.z_re = t.z_im = nullptr;   // bound per workspace
    t.u_re = static_cast<const float *>(c->du_re);
    t.u_im = static_cast<const float *>(c->du_im);
    t.d = c->d;
    t.leak = c->leak;
    t.trw = c->trw;
    t.cg = c->cg;
    t.pi = c->pi;
    t.n = c->n;
    t.ld = c->ld;
    t.dt = c->model.dt;
    t.edge1 = c->tile1;
    t.edge2 = c->tile2;
    t.tiles1 = int32_t(c->ld / c->tile1);
    t.tiles2 = int32_t(c->ld / c->tile2);
    t.n_gather = c->jt.n_gather;
    t.sparse = DissArgs<float>{};
    c->sparse_args(t.sparse);
    if (t.sparse.n_csr > 0 || t.sparse.koff_ptr) b->sparse = true;
    const int td = int((c->n + TD - 1) / TD);
    t.items[0] = uint32_t(t.tiles1) * uint32_t(t.tiles1);
    t.items[1] = uint32_t(t.tiles2) * uint32_t(t.tiles2 + 1) / 2;
    t.items[2] = 1;
    t.items[3] = uint32_t(td) * uint32_t(td + 1) / 2;
  }
  // counters of the persistent form: per-instance completion counts, the
  // item counter and the abort flag
  b->ctr_off = off;
  off += a256(sizeof(uint32_t) * size_t(nb)) + 256;
  b->ws_bytes = off;
  std::vector<int64_t> po(4 * (nb + 1), 0);
  for (int ph = 0; ph < 4; ++ph) {
    int64_t acc = 0;
    for (int k = 0; k < nb; ++k) {
      po[ph * (nb + 1) + k] = acc;
      acc += tab[ord[k]].items[ph];
    }
    po[ph * (nb + 1) + nb] = acc;
    b->phase_items[ph] = acc;
  }
  B_OK(hipMalloc(&b->inst, sizeof(BatchInstance) * nb));
  B_OK(hipMalloc(&b->order, sizeof(int32_t) * nb));
  B_OK(hipMalloc(&b->phase_off, sizeof(int64_t) * po.size()));
  B_OK(hipMemcpy(b->inst, tab.data(), sizeof(BatchInstance) * nb, hipMemcpyHostToDevice));
  B_OK(hipMemcpy(b->order, ord.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice));
  B_OK(hipMemcpy(b->phase_off, po.data(), sizeof(int64_t) * po.size(), hipMemcpyHostToDevice));
  return QME_OK;
}

// Points the instance table at a workspace (Y / Z planes); synchronous.
static qme_status bind_workspace(qme_batch *b, char *ws) {
  if (ws == b->last_ws) return QME_OK;
  B_OK(hipDeviceSynchronize());   // an earlier launch may still read the table
  std::vector<BatchInstance> tab(b->count);
  B_OK(hipMemcpy(tab.data(), b->inst, sizeof(BatchInstance) * b->count, hipMemcpyDeviceToHost));
  for (int i = 0; i < b->count; ++i) {
    const size_t pe = plane_elems(b->ctxs[i]);
    float *y = reinterpret_cast<float *>(ws + b->ws_off[i]);
    tab[i].y_re = y;
    tab[i].y_im = y + pe;
    tab[i].z_re = y + 2 * pe;
    tab[i].z_im = y + 3 * pe;
  }
  B_OK(hipMemcpy(b->inst, tab.data(), sizeof(BatchInstance) * b->count, hipMemcpyHostToDevice));
  b->last_ws = ws;
  return QME_OK;
}

static hipError_t enqueue_persistent(qme_batch *b, int64_t n_steps, hipStream_t s) {
  char *ws = static_cast<char *>(b->last_ws);
  PersistArgs a{};
  a.inst = b->inst;
  a.order = b->order;
  a.phase_off = b->phase_off;
  a.count = b->count;
  a.per_step = 0;
  for (int ph = 0; ph < 4; ++ph) {
    a.phase_items[ph] = b->phase_items[ph];
    a.per_step += b->phase_items[ph];
  }
  a.total = a.per_step * n_steps;
  a.done = reinterpret_cast<uint32_t *>(ws + b->ctr_off);
  a.next = reinterpret_cast<unsigned long long *>(ws + b->ctr_off + a256(sizeof(uint32_t) * size_t(b->count)));
  a.abort_flag = reinterpret_cast<uint32_t *>(a.next + 1);
  a.spin_limit = 1u << 22;
  a.wait_ticks = 100000000ull;   // 1 s
  const int rb = (b->count + 255) / 256;
  hipLaunchKernelGGL(persist_reset_kernel, dim3(rb), dim3(256), 0, s, a.done, b->count, a.next,
                     a.abort_flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned grid = unsigned(std::min<int64_t>(a.total, int64_t(b->resident)));
  if (b->sparse)
    hipLaunchKernelGGL(batch_persistent_kernel<true>, dim3(grid), dim3(kBatchThreads), 0, s, a);
  else
    hipLaunchKernelGGL(batch_persistent_kernel<false>, dim3(grid), dim3(kBatchThreads), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(persist_finish_kernel, dim3(rb), dim3(256), 0, s, b->inst, b->count,
                     a.abort_flag);
  return hipGetLastError();
}

static hipError_t enqueue(qme_batch *b, int64_t n_steps, hipStream_t s) {
  if (b->persistent) return enqueue_persistent(b, n_steps, s);
  for (int64_t k = 0; k < n_steps; ++k) {
    const int parity = b->fuse ? int(k & 1) : 0;
    for (int ph = 0; ph < 4; ++ph) {
      if (ph == 2 && b->fuse) continue;   // formed by the decoherence phase's blocks
      BatchPhase p{b->inst, b->order, b->phase_off + ph * (b->count + 1), b->count};
      if (b->fuse) {
        p.slot_in = parity;
        p.slot_out = 1 - parity;
        p.fuse = 1;
      }
      const dim3 grid(unsigned(b->phase_items[ph])), block(kBatchThreads);
      switch (ph) {
        case 0: hipLaunchKernelGGL(batch_phase_kernel<0>, grid, block, 0, s, p); break;
        case 1: hipLaunchKernelGGL(batch_phase_kernel<1>, grid, block, 0, s, p); break;
        case 2: hipLaunchKernelGGL(batch_phase_kernel<2>, grid, block, 0, s, p); break;
        default:
          if (b->sparse)
            hipLaunchKernelGGL((batch_phase_kernel<3, true>), grid, block, 0, s, p);
          else
            hipLaunchKernelGGL((batch_phase_kernel<3, false>), grid, block, 0, s, p);
          break;
      }
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  if (b->fuse && (n_steps & 1)) {
    hipLaunchKernelGGL(batch_scalars_home_kernel, dim3((b->count + 255) / 256), dim3(256), 0, s,
                       b->inst, b->count);
    return hipGetLastError();
  }
  return hipSuccess;
}

extern "C" qme_status qme_batch_create(qme_ctx *const *ctxs, void *const *states, int32_t count,
                                       qme_batch **out) {
  try {
    set_error("");
    if (!ctxs || !states || !out || count < 1) { set_error("bad arguments"); return QME_E_ARG; }
    *out = nullptr;
    auto b = std::make_unique<qme_batch>();
    b->count = count;
    for (int i = 0; i < count; ++i) {
      qme_ctx *c = ctxs[i];
      if (!c || !states[i]) { set_error("NULL context or state"); return QME_E_ARG; }
      if (c->precision != QME_FP32 || c->ld % 64 != 0) {
        set_error("batched steps need FP32 contexts (leading dimension a multiple of 64)");
        return QME_E_UNSUPPORTED;
      }
      if ((c->tile1 != 32 && c->tile1 != 64) || (c->tile2 != 32 && c->tile2 != 64)) {
        set_error("batched products take 32- or 64-tiles (qme_set_tiles on the context)");
        return QME_E_UNSUPPORTED;
      }
      if (reinterpret_cast<uintptr_t>(states[i]) & 255) { set_error("states must be 256-byte aligned"); return QME_E_ARG; }
      if (i > 0 && c->device != ctxs[0]->device) { set_error("contexts on different devices"); return QME_E_ARG; }
      b->ctxs.push_back(c);
      b->states.push_back(states[i]);
    }
    b->device = ctxs[0]->device;
    qme_status st = check_device(ctxs[0]);
    if (st != QME_OK) return st;
    st = build_tables(b.get());
    if (st != QME_OK) return st;
    {
      // workgroups of the persistent kernel that fit the device at once (the
      // persistent grid; more would only queue behind them)
      int per_cu = 0, per_cu_sparse = 0;
      B_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void *>(batch_persistent_kernel<false>), kBatchThreads, 0));
      B_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu_sparse, reinterpret_cast<const void *>(batch_persistent_kernel<true>), kBatchThreads, 0));
      b->resident = std::max(1, std::min(per_cu, per_cu_sparse)) * std::max(1, ctxs[0]->cus);
    }
    *out = b.release();
    return QME_OK;
  } catch (const std::exception &e) {
    set_error(std::string("internal error: ") + e.what());
    return QME_E_STATE;
  }
}

extern "C" qme_status qme_batch_workspace_size(const qme_batch *b, size_t *bytes) {
  set_error("");
  if (!b || !bytes) { set_error("NULL argument"); return QME_E_ARG; }
  *bytes = b->ws_bytes;
  return QME_OK;
}

extern "C" qme_status qme_batch_config(qme_batch *b, int32_t use_graph, int32_t largest_first) {
  set_error("");
  if (!b) { set_error("NULL batch"); return QME_E_ARG; }
  qme_status st = check_device(b->ctxs[0]);
  if (st != QME_OK) return st;
  B_OK(hipDeviceSynchronize());   // no launch may still use the old graphs or tables
  for (qme_ctx *c : b->ctxs)
    if ((c->tile1 != 32 && c->tile1 != 64) || (c->tile2 != 32 && c->tile2 != 64)) {
      set_error("batched products take 32- or 64-tiles (qme_set_tiles on the context)");
      return QME_E_UNSUPPORTED;
    }
  b->drop_graphs();
  b->use_graph = use_graph != 0;
  // the tables follow the instance order and each context's current tiles
  b->lpt = largest_first != 0;
  b->drop_tables();
  return build_tables(b);
}

extern "C" qme_status qme_batch_persistent(qme_batch *b, int32_t enable) {
  set_error("");
  if (!b) { set_error("NULL batch"); return QME_E_ARG; }
  if (enable != 0 && enable != 1) { set_error("enable must be 0 or 1"); return QME_E_ARG; }
  if (enable == 1) {
    // switched off: its launches did not finish on the device and the cause
    // has not been established
    set_error("the persistent batched launch is switched off (its launches did not finish on "
              "the device; cause not established)");
    return QME_E_UNSUPPORTED;
  }
  qme_status st = check_device(b->ctxs[0]);
  if (st != QME_OK) return st;
  B_OK(hipDeviceSynchronize());   // no launch may still use the old graphs
  b->drop_graphs();
  b->persistent = enable != 0;
  return QME_OK;
}

extern "C" qme_status qme_batch_step(qme_batch *b, int64_t n_steps, void *ws, size_t ws_bytes,
                                     void *hip_stream) {
  try {
    TraceRange range("qme_batch_step");
    set_error("");
    if (!b || !ws) { set_error("NULL argument"); return QME_E_ARG; }
    if (n_steps < 0) { set_error("n_steps < 0"); return QME_E_ARG; }
    if (ws_bytes < b->ws_bytes) { set_error("batch workspace too small"); return QME_E_SIZE; }
    if (reinterpret_cast<uintptr_t>(ws) & 255) { set_error("workspace must be 256-byte aligned"); return QME_E_ARG; }
    qme_status st = check_device(b->ctxs[0]);
    if (st != QME_OK) return st;
    if (n_steps == 0) return QME_OK;
    if (b->persistent) {
      // per-instance completion counts are 32-bit
      int64_t per_inst_max = 0;
      for (int i = 0; i < b->count; ++i) {
        const qme_ctx *c = b->ctxs[i];
        const int64_t t1 = c->ld / c->tile1, t2 = c->ld / c->tile2, td = (c->n + TD - 1) / TD;
        per_inst_max = std::max<int64_t>(per_inst_max, t1 * t1 + t2 * (t2 + 1) / 2 + 1 + td * (td + 1) / 2);
      }
      int64_t per_step = 0;
      for (int ph = 0; ph < 4; ++ph) per_step += b->phase_items[ph];
      if (n_steps > (int64_t(INT32_MAX) - 1) / std::max<int64_t>(1, per_inst_max) ||
          n_steps > (int64_t(INT32_MAX) - 1) / std::max<int64_t>(1, per_step)) {
        set_error("persistent batch run too long for one launch; split it into shorter runs");
        return QME_E_SIZE;
      }
    }
    st = bind_workspace(b, static_cast<char *>(ws));
    if (st != QME_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (!b->use_graph) {
      B_OK(enqueue(b, n_steps, s));
      return QME_OK;
    }
    auto key = std::make_pair(n_steps, ws);
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
      if (!b->capture_stream) B_OK(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      B_OK(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = enqueue(b, n_steps, b->capture_stream);
      hipError_t e2 = hipStreamEndCapture(b->capture_stream, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        set_error(std::string("graph capture failed: ") + hipGetErrorString(e != hipSuccess ? e : e2));
        return QME_E_DEVICE;
      }
      hipGraphExec_t ex = nullptr;
      B_OK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
      b->graph_defs.push_back(g);
      it = b->graphs.emplace(key, ex).first;
    }
    B_OK(hipGraphLaunch(it->second, s));
    return QME_OK;
  } catch (const std::exception &e) {
    set_error(std::string("internal error: ") + e.what());
    return QME_E_STATE;
  }
}

extern "C" void qme_batch_destroy(qme_batch *b) { delete b; }
