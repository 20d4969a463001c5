// Device-side entry points of the C ABI: context build (tables and the
// propagator on the device), state layout and transfer, the time-step driver
// and the observables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "ctx.hpp"
#include "device.hpp"
#include "model.hpp"
#include "qme.h"

using namespace qme;

#define QME_GUARD_BEGIN try {
#define QME_GUARD_END                                      \
  }                                                        \
  catch (const std::bad_alloc &) {                         \
    set_error("out of host memory");                       \
    return QME_E_SIZE;                                     \
  }                                                        \
  catch (const std::exception &e) {                        \
    set_error(std::string("internal error: ") + e.what()); \
    return QME_E_STATE;                                    \
  }

#define HIP_OK(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));               \
      return QME_E_DEVICE;                                                        \
    }                                                                             \
  } while (0)

// Step workspace of qme_step_noalloc, for callers that cannot allocate
// device memory: one copy per device, held until the process ends.  Host
// code never passes `scratch` itself to a kernel or a copy (on the host the
// name is a stand-in, not a device address): it uses the address
// hipGetSymbolAddress returned on that device (scratch_address).
static __device__ __align__(256) unsigned char scratch[QME_NOALLOC_SCRATCH_BYTES];

namespace qme {

// The device address of `scratch` on `device`, looked up once per device
// with that device current (context creation) and kept.
static qme_status scratch_address(int device, void **out) {
  static std::mutex mu;
  static std::vector<void *> addr;   // per device ordinal; nullptr: not looked up yet
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0) {
    set_error("invalid device");
    return QME_E_DEVICE;
  }
  if (size_t(device) >= addr.size()) addr.resize(size_t(device) + 1, nullptr);
  if (!addr[size_t(device)]) {
    int cur = -1;
    HIP_OK(hipGetDevice(&cur));
    if (cur != device) {
      set_error("scratch_address: device is not current");
      return QME_E_DEVICE;
    }
    void *p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("hipGetSymbolAddress returned no address for the step scratch");
      return QME_E_DEVICE;
    }
    addr[size_t(device)] = p;
  }
  *out = addr[size_t(device)];
  return QME_OK;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

void pick_tiles(qme_ctx *c) {
  // Measured on MI355X at N = 2048: 64 x 64 FP32 tiles (4 workgroups per CU)
  // beat 128 x 128 (one wave per SIMD) on both products, and 32 x 32 FP64
  // tiles beat 64 x 64.  The padded leading dimension is a multiple of the
  // tile; qme_set_tiles may pick a larger tile when it divides ld.
  // FP32 systems whose full product in 64-tiles would leave fewer than four
  // workgroups per compute unit take 32-tiles: four times as many
  // workgroups, which beat the larger tiles' operand reuse up to N = 1152
  // and lose to it at N = 2048 (ld stays a multiple of 64, so every FP32
  // tile edge divides it).
  const int64_t rows64 = round_up(c->n, 64) / 64;
  if (c->precision == QME_FP64) {
    c->tile1 = c->tile2 = 32;
  } else if (c->precision == QME_FP32 && rows64 * rows64 < 4 * int64_t(c->cus)) {
    c->tile1 = c->tile2 = 32;
  } else {
    c->tile1 = c->tile2 = 64;
  }
  c->ld = round_up(c->n, c->precision == QME_FP64 ? std::max(c->tile1, c->tile2) : 64);
  // BF16x3: the first product on 128 x 64 tiles (two workgroups per CU) when
  // they fill at least one round of the device: at N = 2048, 512 such tiles
  // in one round took 243 us against 281 us for the 64-tiles' 1024 in a round
  // of three per CU and a second one
  if (c->precision == QME_BF16X3 && c->ld % 128 == 0 &&
      2 * (c->ld / 128) * (c->ld / 128) >= 2 * int64_t(c->cus))
    c->tile1 = 128;
}

size_t plane_elems(const qme_ctx *c) { return size_t(c->ld) * size_t(c->ld); }

size_t state_bytes(const qme_ctx *c) { return 2 * plane_elems(c) * c->elem + 64; }

qme_status check_device(const qme_ctx *c) {
  int dev = -1;
  HIP_OK(hipGetDevice(&dev));
  if (dev != c->device) HIP_OK(hipSetDevice(c->device));
  return QME_OK;
}

LaunchTimer *&launch_timer() {
  static thread_local LaunchTimer *armed = nullptr;
  return armed;
}

// Profiling marks of the step path: kind < 0 begins a step and arms the
// context's timer on this thread when the step is one of the sampled ones
// (every launch then takes an event pair); kind >= 0 ends a kernel kind:
// the pairs taken since the previous mark become one record of that kind.
static hipError_t mark(qme_ctx *c, hipStream_t, int kind) {
  if (!c->profiling) return hipSuccess;
  if (kind < 0) {
    const bool sampled = c->profile_step++ % c->profile_every == 0;
    c->timer.c = c;
    launch_timer() = sampled ? &c->timer : nullptr;
    c->pairs_marked = c->pairs_used;
    return hipSuccess;
  }
  if (c->pairs_used > c->pairs_marked)
    c->records.push_back({kind, c->pairs_marked, c->pairs_used});
  c->pairs_marked = c->pairs_used;
  return hipSuccess;
}

// Disarms the launch timer when a step driver returns.
struct TimerScope {
  TimerScope() = default;
  TimerScope(const TimerScope &) = delete;
  TimerScope &operator=(const TimerScope &) = delete;
  ~TimerScope() { launch_timer() = nullptr; }
};

// Products whose launches cannot occupy the device are split along k (all
// their tiles, in every precision); the partials need their own slots.
// Room for the largest plan over the tile edges the context may be set to,
// at most 12 planes.
// K tile (elements of k per iteration) of a product tile body
static int k_tile(const qme_ctx *c, int tile) {
  if (c->precision == QME_BF16X3) return 32;
  return c->precision == QME_FP32 && tile == 32 ? 32 : 16;
}

static bool small_split_applies(const qme_ctx *c) { return c->tail_split; }

// BF16x3 contexts with tile1 = 128 run the step's first product on 128 x 64
// tiles (launch_cgemm_bf16x3, GemmOps::wide) unless its launch is split; the
// split plan is that of the 64-tiles, which the split launch then takes.
static int plan_tile1(const qme_ctx *c) { return c->precision == QME_BF16X3 ? 64 : c->tile1; }
template <typename T>
static bool wide_first(const qme_ctx *c, const CgemmArgs<T> &g1) {
  return c->precision == QME_BF16X3 && c->tile1 == 128 && g1.split <= 1;
}

static size_t small_split_elems(const qme_ctx *c) {
  const std::vector<int> edges = c->precision == QME_FP64   ? std::vector<int>{32, 64}
                                 : c->precision == QME_FP32 ? std::vector<int>{32, 64, 128}
                                                            : std::vector<int>{64};
  size_t need = 0;
  for (int bm : edges) {
    if (c->ld % bm != 0) continue;
    const int t = int(c->ld / bm);
    for (int blocks : {t * t, t * (t + 1) / 2}) {
      const SplitPlan sp = plan_small_split(blocks, bm, k_tile(c, bm), c->ld, c->cus, SIZE_MAX);
      need = std::max(need, size_t(blocks) * sp.split * 2 * bm * bm);
    }
  }
  return std::min(need, 12 * plane_elems(c));
}

// The split of one product: every tile when the launch is small and the
// partial slots exist, else (lower-triangle products) the tail beyond the
// last full wave of compute units, its partials in `tail_part` (room for
// `tail_cap` elements).
template <typename T>
static void plan_product(const qme_ctx *c, CgemmArgs<T> &g, int tile, bool lower, T *area,
                         T *tail_part, size_t tail_cap) {
  if (!c->tail_split) return;
  // FP32 32-tile products this small load whole panels instead (cgemm_s_panel)
  // unless register staging is asked for
  if (c->precision == QME_FP32 && tile == 32 && c->ld <= kPanelLd && c->direct != 0) return;
  const int t = int(c->ld / tile);
  const int blocks = lower ? t * (t + 1) / 2 : t * t;
  if (area && small_split_applies(c)) {
    const SplitPlan sp = plan_small_split(blocks, tile, k_tile(c, tile), c->ld, c->cus, c->split_elems);
    if (sp.split > 1) {
      g.full = sp.full;
      g.split = sp.split;
      g.part = area;
      return;
    }
  }
  if (!lower) return;
  const SplitPlan sp = plan_tail_split(t, tile, k_tile(c, tile), c->ld, c->cus, tail_cap);
  g.full = sp.full;
  g.split = sp.split;
  g.part = tail_part;
}

template <typename T>
hipError_t step_once(qme_ctx *c, const void *in, void *out, void *y, void *z, hipStream_t s,
                     void *split_area, int parity) {
  const size_t pe = plane_elems(c);
  const T *x_re = static_cast<const T *>(in), *x_im = x_re + pe;
  const double *aux_in = reinterpret_cast<const double *>(x_im + pe);
  T *o_re = static_cast<T *>(out), *o_im = o_re + pe;
  double *aux_out = reinterpret_cast<double *>(o_im + pe);
  T *y_re = static_cast<T *>(y), *y_im = y_re + pe;
  T *z_re = static_cast<T *>(z), *z_im = z_re + pe;
  const T *u_re = static_cast<const T *>(c->du_re), *u_im = static_cast<const T *>(c->du_im);

  CgemmArgs<T> g1{u_re, u_im, x_re, x_im, x_re, x_im, y_re, y_im, c->ld, T(1), T(1)};
  CgemmArgs<T> g2{y_re, y_im, u_re, u_im, y_re, y_im, z_re, z_im, c->ld, T(1), T(1)};
  DissArgs<T> da{z_re, z_im, o_re, o_im, c->ld, c->n, c->model.dt, c->d, c->leak,
                 c->pi, c->cg, c->jt.n_gather, aux_in, aux_out, c->trw};
  c->sparse_args(da);
  if (parity >= 0) {
    da.fuse_trace = 1;
    da.slot_in = parity;
    da.slot_out = 1 - parity;
  }
  GemmOps o1, o2;
  o1.conj_b = o2.conj_b = true;
  o2.lower = true;
  o1.direct = o2.direct = c->direct;
  o1.cus = o2.cus = c->cus;
  // split launches: small ones into the workspace's partial slots (when the
  // caller has them); the lower product's tail into the output planes, dead
  // until the decoherence pass
  T *area = static_cast<T *>(split_area);
  plan_product<T>(c, g1, plan_tile1(c), false, area, nullptr, 0);
  plan_product<T>(c, g2, c->tile2, true, area, o_re, 2 * pe);
  o1.wide = wide_first(c, g1);
  hipError_t e = mark(c, s, -1);
  if constexpr (sizeof(T) == 4) {
    if (c->precision == QME_BF16X3) {
      // dU pre-split (six bf16 planes, split once per context) for both
      // products: the first reads it as A, the lower-triangle one as M
      g1.a_split = c->du_split;
      g2.m_split = c->du_split;
      if (e == hipSuccess) e = launch_cgemm_bf16x3(g1, o1, s);
      if (e == hipSuccess) e = mark(c, s, 0);
      if (e == hipSuccess) e = launch_cgemm_bf16x3(g2, o2, s);
    } else {
      if (e == hipSuccess) e = launch_cgemm_f32(g1, c->tile1, o1, s);
      if (e == hipSuccess) e = mark(c, s, 0);
      if (e == hipSuccess) e = launch_cgemm_f32(g2, c->tile2, o2, s);
    }
  } else {
    if (e == hipSuccess) e = launch_cgemm_f64(g1, c->tile1, o1, s);
    if (e == hipSuccess) e = mark(c, s, 0);
    if (e == hipSuccess) e = launch_cgemm_f64(g2, c->tile2, o2, s);
  }
  if (e == hipSuccess) e = mark(c, s, 1);
  if (e == hipSuccess && !da.fuse_trace) e = launch_trace<T>(da, s);
  if (e == hipSuccess) e = mark(c, s, 2);
  if (e == hipSuccess) e = launch_dissipate<T>(da, s);
  if (e == hipSuccess) e = mark(c, s, 3);
  return e;
}

template hipError_t step_once<float>(qme_ctx *, const void *, void *, void *, void *, hipStream_t,
                                     void *, int);
template hipError_t step_once<double>(qme_ctx *, const void *, void *, void *, void *, hipStream_t,
                                      void *, int);

// Systems up to this size form the trace in the decoherence pass (each of
// its blocks reads the N diagonal values of the rotated state once more).
static constexpr int64_t kFuseTraceMaxN = 1024;

bool fuse_trace_applies(const qme_ctx *c) {
  return c->n <= kFuseTraceMaxN && !uses_small_path(c) && !uses_fold(c);
}

// The single-workgroup path applies to FP32 / FP64 contexts with n <= kSmallN
// whose decoherence operators are all monomial.
bool uses_small_path(const qme_ctx *c) {
  return c->fused && c->n <= kSmallN && c->precision != QME_BF16X3 && c->jt.n_csr == 0;
}

// The folded step applies when no decoherence operator maps a basis state
// onto another (no gather channels: the decoherence step is a factor per
// element), in FP32 with 64-tiles for the lower product or in FP64.
bool uses_fold(const qme_ctx *c) {
  if (!c->fold || c->jt.n_gather != 0 || c->jt.n_csr != 0) return false;
  if (c->precision == QME_FP32) return c->tile2 == 64 || c->tile2 == 32;
  return c->precision == QME_FP64 || c->precision == QME_BF16X3;
}

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// The step workspace: 4 product planes, the diagonal of Z (N FP64), the
// partial slots of small-launch splits.
template <typename T>
static T *split_area_of(const qme_ctx *c, void *ws) {
  if (c->split_elems == 0) return nullptr;
  return reinterpret_cast<T *>(static_cast<char *>(ws) + align256(4 * plane_elems(c) * sizeof(T)) +
                               align256(sizeof(double) * size_t(c->n)));
}

// Folded steps: the lower-triangle product writes the decoherence step of
// its tiles (unscaled, both triangles) straight into the state and the
// diagonal of Z into the workspace; the trace pass reads that diagonal and
// stores the renormalisation factor, which the next step's first product
// applies (alpha = beta = factor); after the last step one pass applies it.
template <typename T>
static hipError_t fold_steps(qme_ctx *c, void *state, int64_t n_steps, void *ws, hipStream_t s) {
  const size_t pe = plane_elems(c);
  T *x_re = static_cast<T *>(state), *x_im = x_re + pe;
  double *aux = reinterpret_cast<double *>(x_im + pe);
  T *y_re = static_cast<T *>(ws), *y_im = y_re + pe;
  T *z_re = y_im + pe;                      // chunk partials of the split tail
  double *zdiag = reinterpret_cast<double *>(static_cast<char *>(ws) +
                                             align256(4 * pe * sizeof(T)));
  T *area = split_area_of<T>(c, ws);
  const T *u_re = static_cast<const T *>(c->du_re), *u_im = static_cast<const T *>(c->du_im);
  const double dt = c->model.dt;
  // FP32 first products in 64- or 128-tiles or whole 32-tile panels and
  // BF16x3 ones in 128 x 64 tiles, without a split, form the previous step's
  // trace themselves (every block sums the stored diagonal,
  // block 0 stores the scalars), so the trace pass runs once per call, after
  // the last step; the sink and step count alternate between the scalar
  // pairs by step parity (as for the unfolded steps)
  bool fused_tr = false;
  if constexpr (sizeof(T) == 4) {
    if (c->precision == QME_FP32 && c->tile1 != 32) {
      CgemmArgs<T> probe{u_re, u_im, x_re, x_im, x_re, x_im, y_re, y_im, c->ld, T(1), T(1)};
      plan_product<T>(c, probe, c->tile1, false, area, nullptr, 0);
      fused_tr = probe.split <= 1;
    }
    // (and FP32 32-tile first products that load whole panels)
    if (c->precision == QME_FP32 && c->tile1 == 32 && c->ld <= kPanelLd && c->direct != 0)
      fused_tr = true;
    // (and BF16x3 first products on 128 x 64 tiles)
    if (c->precision == QME_BF16X3) {
      CgemmArgs<T> probe{u_re, u_im, x_re, x_im, x_re, x_im, y_re, y_im, c->ld, T(1), T(1)};
      plan_product<T>(c, probe, plan_tile1(c), false, area, nullptr, 0);
      fused_tr = wide_first(c, probe);
    }
  }
  for (int64_t k = 0; k < n_steps; ++k) {
    CgemmArgs<T> g1{u_re, u_im, x_re, x_im, x_re, x_im, y_re, y_im, c->ld, T(1), T(1)};
    if (k > 0 && fused_tr) {
      g1.tr_zdiag = zdiag;
      g1.tr_w = c->trw;
      g1.tr_leak = c->leak;
      g1.tr_aux = aux;
      g1.tr_n = c->n;
      g1.tr_dt = dt;
      g1.tr_slot_in = int32_t((k - 1) & 1);
      g1.tr_slot_out = int32_t(k & 1);
    } else if (k > 0) {
      g1.scale = aux + 4;
    }
    CgemmArgs<T> g2{y_re, y_im, u_re, u_im, y_re, y_im, x_re, x_im, c->ld, T(1), T(1)};
    g2.fold_d = c->d;
    g2.fold_dt = dt;
    g2.fold_n = c->n;
    g2.zdiag = zdiag;
    plan_product<T>(c, g1, plan_tile1(c), false, area, nullptr, 0);
    plan_product<T>(c, g2, c->tile2, true, area, z_re, 2 * pe);
    DissArgs<T> da{nullptr, nullptr, x_re, x_im, c->ld, c->n, dt, c->d, c->leak,
                   c->pi, c->cg, 0, aux, aux, c->trw, zdiag};
    if (fused_tr) {
      da.slot_in = int(k & 1);
      da.slot_out = int((k + 1) & 1);
    }
    GemmOps o1, o2;
    o1.conj_b = o2.conj_b = true;
    o2.lower = true;
    o1.direct = o2.direct = c->direct;
    o1.cus = o2.cus = c->cus;
    if (c->precision == QME_BF16X3) {
      // dU pre-split for both products, as in step_once
      g1.a_split = c->du_split;
      g2.m_split = c->du_split;
      o1.wide = wide_first(c, g1);
    }
    auto gemm = [&](const CgemmArgs<T> &g, int tile, const GemmOps &o) {
      if constexpr (sizeof(T) == 4) {
        if (c->precision == QME_BF16X3) return launch_cgemm_bf16x3(g, o, s);
        return launch_cgemm_f32(g, tile, o, s);
      } else {
        return launch_cgemm_f64(g, tile, o, s);
      }
    };
    hipError_t e = mark(c, s, -1);
    if (e == hipSuccess) e = gemm(g1, c->tile1, o1);
    if (e == hipSuccess) e = mark(c, s, 0);
    if (e == hipSuccess) e = gemm(g2, c->tile2, o2);
    if (e == hipSuccess) e = mark(c, s, 1);
    // with fused_tr the next step's first product forms this trace
    if (e == hipSuccess && (!fused_tr || k == n_steps - 1)) e = launch_trace<T>(da, s);
    if (e == hipSuccess) e = mark(c, s, 2);
    if (e != hipSuccess) return e;
  }
  launch_timer() = nullptr;   // the closing passes are no step's kernels
  if (fused_tr && (n_steps & 1)) {
    const hipError_t e = launch_scalars_home(aux, s);
    if (e != hipSuccess) return e;
  }
  return n_steps > 0 ? launch_apply_scale<T>(x_re, x_im, int64_t(pe), aux + 4, s) : hipSuccess;
}

template <typename T>
static qme_status step_impl(qme_ctx *c, void *state, int64_t n_steps, void *ws,
                            hipStream_t s) {
  const TimerScope timer_scope;
  const size_t pe = plane_elems(c);
  if (!uses_small_path(c) && uses_fold(c)) {
    hipError_t e = fold_steps<T>(c, state, n_steps, ws, s);
    if (e != hipSuccess) {
      set_error(std::string("kernel launch failed: ") + hipGetErrorString(e));
      return QME_E_DEVICE;
    }
    return QME_OK;
  }
  if (uses_small_path(c)) {
    if (n_steps == 0) return QME_OK;
    T *re = static_cast<T *>(state);
    SmallArgs<T> a{re, re + pe, reinterpret_cast<double *>(re + 2 * pe),
                   static_cast<const T *>(c->du_re), static_cast<const T *>(c->du_im),
                   c->ld, int(c->n), c->model.dt, c->d, c->leak, c->pi, c->cg,
                   c->jt.n_gather, n_steps, c->trw};
    hipError_t e = mark(c, s, -1);
    if (e == hipSuccess) e = launch_small_steps<T>(a, s);
    if (e == hipSuccess) e = mark(c, s, 0);
    if (e != hipSuccess) {
      set_error(std::string("kernel launch failed: ") + hipGetErrorString(e));
      return QME_E_DEVICE;
    }
    return QME_OK;
  }
  T *y = static_cast<T *>(ws);
  T *z = y + 2 * pe;
  // small systems: the trace formed in the decoherence pass, the sink and
  // step count alternating between two slot pairs (back to pair 0 at the end)
  const bool fuse = fuse_trace_applies(c);
  for (int64_t k = 0; k < n_steps; ++k) {
    hipError_t e = step_once<T>(c, state, state, y, z, s, split_area_of<T>(c, ws),
                                fuse ? int(k & 1) : -1);
    if (e != hipSuccess) {
      set_error(std::string("kernel launch failed: ") + hipGetErrorString(e));
      return QME_E_DEVICE;
    }
  }
  if (fuse && (n_steps & 1)) {
    launch_timer() = nullptr;   // not a step's kernel
    const hipError_t e = launch_scalars_home(
        reinterpret_cast<double *>(static_cast<char *>(state) + 2 * pe * sizeof(T)), s);
    if (e != hipSuccess) {
      set_error(std::string("kernel launch failed: ") + hipGetErrorString(e));
      return QME_E_DEVICE;
    }
  }
  return QME_OK;
}

// Everything of a context after its basis is fixed: Hamiltonian, FP64
// propagator, decoherence tables and the device copies.
static qme_status finish_context(qme_ctx *c, int32_t precision, void *hip_stream) {
  std::string err;
  c->precision = precision;
  c->elem = precision == QME_FP64 ? 8 : 4;
  c->n = c->model.n;
  if (const char *f = std::getenv("QME_FAULT_AT_STEP")) {
    char *end = nullptr;
    const long long k = std::strtoll(f, &end, 10);
    if (end != f && *end == '\0' && k >= 0) c->fault_at = k;
  }
  std::vector<int32_t> r, cc;
  std::vector<double> v;
  hamiltonian_coo(c->model, r, cc, v);
  c->h = to_csr(c->n, r, cc, v);
  if (!propagator_increment(c->model, c->h, c->du_re_host, c->du_im_host, err, nullptr,
                            &c->squarings)) {
    set_error(err);
    return QME_E_NUMERIC;
  }
  c->jt = jump_tables(c->model);

  HIP_OK(hipGetDevice(&c->device));
  HIP_OK(hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, c->device));
  {
    const qme_status st = scratch_address(c->device, &c->scratch);
    if (st != QME_OK) return st;
  }
  pick_tiles(c);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const size_t pe = plane_elems(c);
  c->split_elems = small_split_elems(c);
  // propagator planes, padded with zeros, in the storage type
  std::vector<char> buf(pe * c->elem);
  for (int plane = 0; plane < 2; ++plane) {
    const std::vector<double> &src = plane ? c->du_im_host : c->du_re_host;
    std::memset(buf.data(), 0, buf.size());
    for (int64_t i = 0; i < c->n; ++i)
      for (int64_t j = 0; j < c->n; ++j) {
        double x = src[size_t(i) * c->n + j];
        size_t o = size_t(i) * c->ld + j;
        if (c->elem == 8) reinterpret_cast<double *>(buf.data())[o] = x;
        else reinterpret_cast<float *>(buf.data())[o] = float(x);
      }
    void **dst = plane ? &c->du_im : &c->du_re;
    HIP_OK(hipMalloc(dst, buf.size()));
    HIP_OK(hipMemcpyAsync(*dst, buf.data(), buf.size(), hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
  }
  if (c->precision == QME_BF16X3) {
    HIP_OK(hipMalloc(&c->du_split, 6 * pe * sizeof(uint16_t)));
    HIP_OK(launch_split_bf16x3(static_cast<const float *>(c->du_re),
                               static_cast<const float *>(c->du_im), c->du_split, pe, s));
    HIP_OK(hipStreamSynchronize(s));
  }
  const int64_t n = c->n;
  HIP_OK(hipMalloc(&c->d, sizeof(double) * n));
  HIP_OK(hipMalloc(&c->leak, sizeof(double) * n));
  HIP_OK(hipMalloc(&c->diag, sizeof(double) * (n + 8)));
  HIP_OK(hipMemcpy(c->d, c->jt.d.data(), sizeof(double) * n, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(c->leak, c->jt.leak.data(), sizeof(double) * n, hipMemcpyHostToDevice));
  {
    // trace weights: every jump term c_j[u]^2 Z[w,w] (w = pi_j[u]) counted
    // at the state w it reads
    const double dt = c->model.dt;
    std::vector<double> trw(static_cast<size_t>(n), 0.0);
    // (sparse channels: the probability a state sends into the basis)
    for (int64_t w = 0; w < n; ++w)
      trw[size_t(w)] = 1.0 - dt * c->jt.d[size_t(w)] + dt * c->jt.arrive[size_t(w)];
    for (int j = 0; j < c->jt.n_gather; ++j)
      for (int64_t u = 0; u < n; ++u) {
        const int32_t w = c->jt.pi[size_t(j) * n + u];
        if (w >= 0) {
          const double cg = c->jt.cg[size_t(j) * n + u];
          trw[size_t(w)] += dt * cg * cg;
        }
      }
    HIP_OK(hipMalloc(&c->trw, sizeof(double) * n));
    HIP_OK(hipMemcpy(c->trw, trw.data(), sizeof(double) * n, hipMemcpyHostToDevice));
  }
  // gather channels that map every state to itself (or out of the basis)
  c->self_mask = 0;
  for (int j = 0; j < c->jt.n_gather && j < 32; ++j) {
    bool self = true;
    for (int64_t u = 0; u < n && self; ++u) {
      const int32_t w = c->jt.pi[size_t(j) * n + u];
      self = w < 0 || w == u;
    }
    if (self) c->self_mask |= 1u << j;
  }
  const size_t ng = size_t(std::max(1, c->jt.n_gather)) * n;
  HIP_OK(hipMalloc(&c->pi, sizeof(int32_t) * ng));
  HIP_OK(hipMalloc(&c->cg, sizeof(double) * ng));
  if (c->jt.n_gather > 0) {
    HIP_OK(hipMemcpy(c->pi, c->jt.pi.data(), sizeof(int32_t) * c->jt.pi.size(), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->cg, c->jt.cg.data(), sizeof(double) * c->jt.cg.size(), hipMemcpyHostToDevice));
  }
  // sparse channels (general-form models whose operators are not monomial)
  {
    const JumpTables &t = c->jt;
    auto up = [&](auto **dst, const auto &v) -> qme_status {
      using E = typename std::decay_t<decltype(v)>::value_type;
      const size_t cnt = std::max<size_t>(1, v.size());
      HIP_OK(hipMalloc(reinterpret_cast<void **>(dst), sizeof(E) * cnt));
      if (!v.empty()) HIP_OK(hipMemcpy(*dst, v.data(), sizeof(E) * v.size(), hipMemcpyHostToDevice));
      return QME_OK;
    };
    std::vector<double> gam;
    for (int32_t j : t.csr_channel) gam.push_back(c->model.jumps[size_t(j)].gamma);
    qme_status st = QME_OK;
    if (st == QME_OK) st = up(&c->csr_ptr, t.csr_ptr);
    if (st == QME_OK) st = up(&c->csr_col, t.csr_col);
    if (st == QME_OK) st = up(&c->csr_val, t.csr_val);
    if (st == QME_OK) st = up(&c->csrt_ptr, t.csrt_ptr);
    if (st == QME_OK) st = up(&c->csrt_col, t.csrt_col);
    if (st == QME_OK) st = up(&c->csrt_val, t.csrt_val);
    if (st == QME_OK) st = up(&c->kj_ptr, t.kj_ptr);
    if (st == QME_OK) st = up(&c->kj_col, t.kj_col);
    if (st == QME_OK) st = up(&c->kj_val, t.kj_val);
    if (st == QME_OK) st = up(&c->koff_ptr, t.koff_ptr);
    if (st == QME_OK) st = up(&c->koff_col, t.koff_col);
    if (st == QME_OK) st = up(&c->koff_val, t.koff_val);
    if (st == QME_OK) st = up(&c->loff_row, t.loff_row);
    if (st == QME_OK) st = up(&c->loff_col, t.loff_col);
    if (st == QME_OK) st = up(&c->loff_val, t.loff_val);
    if (st == QME_OK) st = up(&c->csr_gamma, gam);
    if (st == QME_OK) st = up(&c->csr_channel, t.csr_channel);
    if (st != QME_OK) return st;
  }
  // adjoint tables
  const int nj = int(c->model.jumps.size());
  c->n_arrival = int(c->jt.arrival_channel.size());
  const size_t ntau = size_t(std::max(1, c->jt.n_gather)) * n;
  HIP_OK(hipMalloc(&c->tau, sizeof(int32_t) * ntau));
  HIP_OK(hipMalloc(&c->ca, sizeof(double) * ntau));
  if (c->jt.n_gather > 0) {
    HIP_OK(hipMemcpy(c->tau, c->jt.tau.data(), sizeof(int32_t) * c->jt.tau.size(), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->ca, c->jt.ca.data(), sizeof(double) * c->jt.ca.size(), hipMemcpyHostToDevice));
  }
  const size_t nup = size_t(std::max(1, c->n_arrival)) * n;
  HIP_OK(hipMalloc(&c->upi, sizeof(int32_t) * nup));
  HIP_OK(hipMalloc(&c->uc, sizeof(double) * nup));
  {
    std::vector<int32_t> upi;
    std::vector<double> uc;
    for (int32_t j : c->jt.arrival_channel) {
      upi.insert(upi.end(), c->jt.unit_pi.begin() + size_t(j) * n, c->jt.unit_pi.begin() + size_t(j + 1) * n);
      uc.insert(uc.end(), c->jt.unit_c.begin() + size_t(j) * n, c->jt.unit_c.begin() + size_t(j + 1) * n);
    }
    if (!upi.empty()) {
      HIP_OK(hipMemcpy(c->upi, upi.data(), sizeof(int32_t) * upi.size(), hipMemcpyHostToDevice));
      HIP_OK(hipMemcpy(c->uc, uc.data(), sizeof(double) * uc.size(), hipMemcpyHostToDevice));
    }
  }
  HIP_OK(hipMalloc(&c->ada, sizeof(double) * size_t(std::max(1, nj)) * n));
  HIP_OK(hipMalloc(&c->arrival_of, sizeof(int32_t) * size_t(std::max(1, nj))));
  if (nj > 0) {
    HIP_OK(hipMemcpy(c->ada, c->jt.unit_ada.data(), sizeof(double) * c->jt.unit_ada.size(), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->arrival_of, c->jt.arrival_of.data(), sizeof(int32_t) * nj, hipMemcpyHostToDevice));
  }
  // Hamiltonian CSR and the parameter terms (device Frechet finalisation)
  for (int64_t i = 0; i < n; ++i) {
    double rs = 0.0;
    for (int64_t q = c->h.ptr[i]; q < c->h.ptr[i + 1]; ++q) rs += std::fabs(c->h.val[q]);
    c->h_norm1 = std::max(c->h_norm1, rs);
  }
  const size_t nnz = std::max<size_t>(1, c->h.val.size());
  HIP_OK(hipMalloc(&c->h_ptr, sizeof(int64_t) * (n + 1)));
  HIP_OK(hipMalloc(&c->h_col, sizeof(int32_t) * nnz));
  HIP_OK(hipMalloc(&c->h_val, sizeof(double) * nnz));
  HIP_OK(hipMemcpy(c->h_ptr, c->h.ptr.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice));
  if (!c->h.val.empty()) {
    HIP_OK(hipMemcpy(c->h_col, c->h.col.data(), sizeof(int32_t) * c->h.col.size(), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->h_val, c->h.val.data(), sizeof(double) * c->h.val.size(), hipMemcpyHostToDevice));
  }
  {
    const std::vector<TermCoo> terms = hamiltonian_terms(c->model);
    std::vector<int32_t> tr, tc;
    std::vector<double> tv;
    c->term_offset.assign(1, 0);
    for (const TermCoo &t : terms) {
      tr.insert(tr.end(), t.row.begin(), t.row.end());
      tc.insert(tc.end(), t.col.begin(), t.col.end());
      tv.insert(tv.end(), t.val.begin(), t.val.end());
      c->term_offset.push_back(int64_t(tv.size()));
    }
    const size_t ne = std::max<size_t>(1, tv.size());
    HIP_OK(hipMalloc(&c->t_row, sizeof(int32_t) * ne));
    HIP_OK(hipMalloc(&c->t_col, sizeof(int32_t) * ne));
    HIP_OK(hipMalloc(&c->t_val, sizeof(double) * ne));
    if (!tv.empty()) {
      HIP_OK(hipMemcpy(c->t_row, tr.data(), sizeof(int32_t) * tr.size(), hipMemcpyHostToDevice));
      HIP_OK(hipMemcpy(c->t_col, tc.data(), sizeof(int32_t) * tc.size(), hipMemcpyHostToDevice));
      HIP_OK(hipMemcpy(c->t_val, tv.data(), sizeof(double) * tv.size(), hipMemcpyHostToDevice));
    }
  }
  return QME_OK;
}

}  // namespace qme

extern "C" qme_status qme_hamiltonian(const qme_system *sys, const qme_params *par,
                                      int32_t precision, void *hip_stream, qme_ctx **out) {
  QME_GUARD_BEGIN
  set_error("");
  if (!out) { set_error("out is NULL"); return QME_E_ARG; }
  *out = nullptr;
  if (!par) { set_error("params is NULL"); return QME_E_ARG; }
  if (precision != QME_FP64 && precision != QME_FP32 && precision != QME_BF16X3) {
    set_error("unknown precision");
    return QME_E_ARG;
  }
  auto c = std::make_unique<qme_ctx>();
  std::string err;
  if (!build_model(sys, par, c->model, err)) { set_error(err); return QME_E_ARG; }
  if (!enumerate_basis(c->model, err)) { set_error(err); return QME_E_SIZE; }
  qme_status st = finish_context(c.get(), precision, hip_stream);
  if (st != QME_OK) return st;
  *out = c.release();
  return QME_OK;
  QME_GUARD_END
}

extern "C" qme_status qme_hamiltonian_general(int64_t n, int64_t h_nnz, const int32_t *h_rows,
                                              const int32_t *h_cols, const double *h_vals,
                                              int32_t n_jumps, const qme_general_jump *jumps,
                                              double dt, int32_t precision, void *hip_stream,
                                              qme_ctx **out) {
  QME_GUARD_BEGIN
  set_error("");
  if (!out) { set_error("out is NULL"); return QME_E_ARG; }
  *out = nullptr;
  if (precision != QME_FP64 && precision != QME_FP32 && precision != QME_BF16X3) {
    set_error("unknown precision");
    return QME_E_ARG;
  }
  auto c = std::make_unique<qme_ctx>();
  std::string err;
  bool unsupported = false;
  if (!build_general_model(n, h_nnz, h_rows, h_cols, h_vals, n_jumps, jumps, dt, c->model, err,
                           unsupported)) {
    set_error(err);
    return unsupported ? QME_E_UNSUPPORTED : QME_E_ARG;
  }
  qme_status st = finish_context(c.get(), precision, hip_stream);
  if (st != QME_OK) return st;
  *out = c.release();
  return QME_OK;
  QME_GUARD_END
}

extern "C" qme_status qme_select_states(int64_t n, const double *p_prev, const double *p_now,
                                        double interval, double eps, int32_t *keep,
                                        int64_t *n_keep) {
  QME_GUARD_BEGIN
  set_error("");
  if (!p_prev || !p_now || !keep || !n_keep) { set_error("NULL argument"); return QME_E_ARG; }
  if (n < 1 || n > (int64_t(1) << 31) - 1) { set_error("n must be in [1, 2^31)"); return QME_E_ARG; }
  if (!(interval > 0.0) || !std::isfinite(interval)) { set_error("interval must be > 0"); return QME_E_ARG; }
  if (!(eps >= 0.0) || !std::isfinite(eps)) { set_error("eps must be finite and >= 0"); return QME_E_ARG; }
  int64_t k = 0;
  for (int64_t s = 0; s < n; ++s) {
    if (!std::isfinite(p_prev[s]) || !std::isfinite(p_now[s])) {
      set_error("populations are not finite");
      return QME_E_ARG;
    }
    if (std::fabs(p_now[s] - p_prev[s]) / interval >= eps) keep[k++] = int32_t(s);
  }
  *n_keep = k;
  if (k == 0) { set_error("every state would be removed"); return QME_E_STATE; }
  return QME_OK;
  QME_GUARD_END
}

extern "C" qme_status qme_select_device(const qme_ctx *c, const void *state, const double *p_prev,
                                        double *p_now, double interval, double eps, int32_t *keep,
                                        int64_t *n_keep, void *hip_stream) {
  QME_GUARD_BEGIN
  TraceRange range("qme_select_device");
  set_error("");
  if (!c || !state || !p_prev || !p_now || !keep || !n_keep) {
    set_error("NULL argument");
    return QME_E_ARG;
  }
  if (!(interval > 0.0) || !std::isfinite(interval)) { set_error("interval must be > 0"); return QME_E_ARG; }
  if (!(eps >= 0.0) || !std::isfinite(eps)) { set_error("eps must be finite and >= 0"); return QME_E_ARG; }
  qme_status st = check_device(c);
  if (st != QME_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e;
  if (c->elem == 8) {
    DecideArgs<double> a{static_cast<const double *>(state), c->ld, c->n, p_prev, p_now,
                         interval, eps, keep, n_keep};
    e = launch_select_decide<double>(a, s);
  } else {
    DecideArgs<float> a{static_cast<const float *>(state), c->ld, c->n, p_prev, p_now,
                        interval, eps, keep, n_keep};
    e = launch_select_decide<float>(a, s);
  }
  if (e != hipSuccess) { set_error(std::string("kernel launch failed: ") + hipGetErrorString(e)); return QME_E_DEVICE; }
  return QME_OK;
  QME_GUARD_END
}

// The selection run's device area: a snapshot of the state, two population
// vectors, two kept-index vectors, two counts (slots alternate by solve).
struct SelectArea {
  void *snap;
  double *p[2];
  int32_t *keep[2];
  int64_t *count;
};
static SelectArea select_area(const qme_ctx *c, void *base) {
  char *b = static_cast<char *>(base);
  SelectArea a;
  a.snap = b;
  b += align256(state_bytes(c));
  a.p[0] = reinterpret_cast<double *>(b);
  a.p[1] = a.p[0] + c->n;
  b += align256(2 * sizeof(double) * size_t(c->n));
  a.keep[0] = reinterpret_cast<int32_t *>(b);
  a.keep[1] = a.keep[0] + c->n;
  b += align256(2 * sizeof(int32_t) * size_t(c->n));
  a.count = reinterpret_cast<int64_t *>(b);
  return a;
}

extern "C" qme_status qme_select_workspace_size(const qme_ctx *c, size_t *bytes) {
  set_error("");
  if (!c || !bytes) { set_error("NULL argument"); return QME_E_ARG; }
  *bytes = align256(state_bytes(c)) + align256(2 * sizeof(double) * size_t(c->n)) +
           align256(2 * sizeof(int32_t) * size_t(c->n)) + 2 * sizeof(int64_t);
  return QME_OK;
}

template <typename T>
static hipError_t decide_on(const qme_ctx *c, const void *state, const double *prev, double *now,
                            double interval, double eps, int32_t *keep, int64_t *count,
                            hipStream_t s) {
  DecideArgs<T> a{static_cast<const T *>(state), c->ld, c->n, prev, now, interval, eps, keep, count};
  return launch_select_decide<T>(a, s);
}

extern "C" qme_status qme_select_run(qme_ctx *c, void *state, void *ws, void *sel_ws,
                                     int64_t n_solves, int64_t steps_per_solve, double eps,
                                     int32_t fresh, int64_t *solves_done, int64_t *n_keep,
                                     int32_t *keep_host, void *hip_stream) {
  QME_GUARD_BEGIN
  TraceRange range("qme_select_run");
  set_error("");
  if (!c || !state || !ws || !sel_ws || !solves_done || !n_keep || !keep_host) {
    set_error("NULL argument");
    return QME_E_ARG;
  }
  if (n_solves < 0 || steps_per_solve < 1) {
    set_error("n_solves must be >= 0 and steps_per_solve >= 1");
    return QME_E_ARG;
  }
  if (!(eps >= 0.0) || !std::isfinite(eps)) { set_error("eps must be finite and >= 0"); return QME_E_ARG; }
  if ((reinterpret_cast<uintptr_t>(state) | reinterpret_cast<uintptr_t>(ws) |
       reinterpret_cast<uintptr_t>(sel_ws)) & 255) {
    set_error("state and workspaces must be 256-byte aligned");
    return QME_E_ARG;
  }
  qme_status st = check_device(c);
  if (st != QME_OK) return st;
  *solves_done = 0;
  *n_keep = c->n;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (!c->sel_count_host)
    HIP_OK(hipHostMalloc(reinterpret_cast<void **>(&c->sel_count_host), 2 * sizeof(int64_t)));
  for (void *&e : c->sel_ev)
    if (!e) HIP_OK(hipEventCreateWithFlags(reinterpret_cast<hipEvent_t *>(&e), hipEventDisableTiming));
  const SelectArea a = select_area(c, sel_ws);
  const bool f64 = c->elem == 8;
  auto decide = [&](const double *prev, double *now, double interval, double e, int slot) {
    return f64 ? decide_on<double>(c, state, prev, now, interval, e, a.keep[slot], a.count + slot, s)
               : decide_on<float>(c, state, prev, now, interval, e, a.keep[slot], a.count + slot, s);
  };
  if (fresh) HIP_OK(decide(a.p[0], a.p[0], 1.0, 0.0, 0));   // populations of the entry state
  if (n_solves == 0) return QME_OK;
  const double interval = double(steps_per_solve) * c->model.dt;
  const size_t sbytes = state_bytes(c);
  auto issue = [&](int slot) -> qme_status {
    const qme_status r = f64 ? step_impl<double>(c, state, steps_per_solve, ws, s)
                             : step_impl<float>(c, state, steps_per_solve, ws, s);
    if (r != QME_OK) return r;
    HIP_OK(decide(a.p[slot], a.p[1 - slot], interval, eps, slot));
    HIP_OK(hipMemcpyAsync(c->sel_count_host + slot, a.count + slot, sizeof(int64_t),
                          hipMemcpyDeviceToHost, s));
    HIP_OK(hipEventRecord(static_cast<hipEvent_t>(c->sel_ev[slot]), s));
    return QME_OK;
  };
  // solve i compares p[i % 2] with the populations it writes to p[(i + 1) % 2];
  // solve i + 1 is queued (from a snapshot of the state) before the host reads
  // solve i's count
  int slot = 0;
  st = issue(slot);
  if (st != QME_OK) return st;
  int64_t done = 1;
  for (;;) {
    const int cur = slot;
    const bool ahead = done < n_solves;
    if (ahead) {
      HIP_OK(hipMemcpyAsync(a.snap, state, sbytes, hipMemcpyDeviceToDevice, s));
      slot ^= 1;
      st = issue(slot);
      if (st != QME_OK) return st;
    }
    HIP_OK(hipEventSynchronize(static_cast<hipEvent_t>(c->sel_ev[cur])));
    const int64_t cnt = c->sel_count_host[cur];
    if (cnt != c->n) {
      // the solve queued ahead is dropped: the state returns to solve `done`'s
      if (ahead) HIP_OK(hipMemcpyAsync(state, a.snap, sbytes, hipMemcpyDeviceToDevice, s));
      if (cnt > 0)
        HIP_OK(hipMemcpyAsync(keep_host, a.keep[cur], sizeof(int32_t) * size_t(cnt),
                              hipMemcpyDeviceToHost, s));
      HIP_OK(hipStreamSynchronize(s));
      *solves_done = done;
      *n_keep = cnt;
      if (cnt < 0) { set_error("populations are not finite"); return QME_E_NUMERIC; }
      if (cnt == 0) { set_error("every state would be removed"); return QME_E_STATE; }
      return QME_OK;
    }
    if (!ahead) break;
    ++done;
  }
  // the last solve (slot `slot`) wrote its populations to p[1 - slot]: back
  // to p[0] for a following run
  if (slot == 0)
    HIP_OK(hipMemcpyAsync(a.p[0], a.p[1], sizeof(double) * size_t(c->n), hipMemcpyDeviceToDevice, s));
  *solves_done = done;
  return QME_OK;
  QME_GUARD_END
}

extern "C" qme_status qme_subspace(const qme_ctx *parent, const int32_t *keep, int64_t n_keep,
                                   void *hip_stream, qme_ctx **out) {
  QME_GUARD_BEGIN
  set_error("");
  if (!out) { set_error("out is NULL"); return QME_E_ARG; }
  *out = nullptr;
  if (!parent || !keep) { set_error("NULL argument"); return QME_E_ARG; }
  qme_status st = check_device(parent);
  if (st != QME_OK) return st;
  auto c = std::make_unique<qme_ctx>();
  c->model = parent->model;
  std::string err;
  if (!restrict_basis(c->model, keep, n_keep, err)) { set_error(err); return QME_E_ARG; }
  st = finish_context(c.get(), parent->precision, hip_stream);
  if (st != QME_OK) return st;
  c->tail_split = parent->tail_split;
  c->fused = parent->fused;
  c->parent_n = parent->n;
  c->parent_ld = parent->ld;
  HIP_OK(hipMalloc(&c->parent_keep, sizeof(int32_t) * size_t(n_keep)));
  HIP_OK(hipMemcpy(c->parent_keep, keep, sizeof(int32_t) * size_t(n_keep), hipMemcpyHostToDevice));
  *out = c.release();
  return QME_OK;
  QME_GUARD_END
}

extern "C" qme_status qme_compact_state(const qme_ctx *from, const void *state_from,
                                        const qme_ctx *to, void *state_to, void *hip_stream) {
  QME_GUARD_BEGIN
  set_error("");
  if (!from || !to || !state_from || !state_to) { set_error("NULL argument"); return QME_E_ARG; }
  if (!to->parent_keep || to->parent_n != from->n || to->parent_ld != from->ld ||
      to->precision != from->precision) {
    set_error("'to' was not made by qme_subspace from a context with the basis of 'from'");
    return QME_E_STATE;
  }
  if (state_from == state_to) { set_error("the two states must be different buffers"); return QME_E_ARG; }
  qme_status st = check_device(to);
  if (st != QME_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const size_t pf = plane_elems(from), pt = plane_elems(to);
  hipError_t e;
  if (from->elem == 8) {
    const double *fr = static_cast<const double *>(state_from);
    double *tr = static_cast<double *>(state_to);
    CompactArgs<double> a{fr, fr + pf, reinterpret_cast<const double *>(fr + 2 * pf),
                          tr, tr + pt, reinterpret_cast<double *>(tr + 2 * pt), to->parent_keep,
                          from->n, from->ld, to->n, to->ld};
    e = launch_compact<double>(a, s);
  } else {
    const float *fr = static_cast<const float *>(state_from);
    float *tr = static_cast<float *>(state_to);
    CompactArgs<float> a{fr, fr + pf, reinterpret_cast<const double *>(fr + 2 * pf),
                         tr, tr + pt, reinterpret_cast<double *>(tr + 2 * pt), to->parent_keep,
                         from->n, from->ld, to->n, to->ld};
    e = launch_compact<float>(a, s);
  }
  if (e != hipSuccess) { set_error(std::string("kernel launch failed: ") + hipGetErrorString(e)); return QME_E_DEVICE; }
  return QME_OK;
  QME_GUARD_END
}

extern "C" qme_status qme_state_layout(const qme_ctx *c, int64_t *n, int64_t *ld,
                                       int64_t *elem_bytes, size_t *bytes) {
  set_error("");
  if (!c) { set_error("ctx is NULL"); return QME_E_ARG; }
  if (n) *n = c->n;
  if (ld) *ld = c->ld;
  if (elem_bytes) *elem_bytes = c->elem;
  if (bytes) *bytes = state_bytes(c);
  return QME_OK;
}

extern "C" qme_status qme_workspace_size(const qme_ctx *c, size_t *bytes) {
  set_error("");
  if (!c || !bytes) { set_error("NULL argument"); return QME_E_ARG; }
  // the step's product planes, the diagonal of Z for folded steps and the
  // partial slots of products split along k
  *bytes = align256(4 * plane_elems(c) * c->elem) + align256(sizeof(double) * size_t(c->n)) +
           align256(c->split_elems * c->elem);
  return QME_OK;
}

extern "C" qme_status qme_set_state(const qme_ctx *c, void *state, const double *rho_re,
                                    const double *rho_im, double sink, void *hip_stream) {
  QME_GUARD_BEGIN
  set_error("");
  if (!c || !state || !rho_re || !rho_im) { set_error("NULL argument"); return QME_E_ARG; }
  if (!std::isfinite(sink)) { set_error("sink is not finite"); return QME_E_ARG; }
  qme_status st = check_device(c);
  if (st != QME_OK) return st;
  const size_t pe = plane_elems(c);
  std::vector<char> buf(state_bytes(c), 0);
  for (int64_t i = 0; i < c->n; ++i)
    for (int64_t j = 0; j < c->n; ++j) {
      size_t src = size_t(i) * c->n + j, o = size_t(i) * c->ld + j;
      double xr = rho_re[src], xi = rho_im[src];
      if (!std::isfinite(xr) || !std::isfinite(xi)) { set_error("rho is not finite"); return QME_E_ARG; }
      if (c->elem == 8) {
        reinterpret_cast<double *>(buf.data())[o] = xr;
        reinterpret_cast<double *>(buf.data())[pe + o] = xi;
      } else {
        reinterpret_cast<float *>(buf.data())[o] = float(xr);
        reinterpret_cast<float *>(buf.data())[pe + o] = float(xi);
      }
    }
  double *aux = reinterpret_cast<double *>(buf.data() + 2 * pe * c->elem);
  aux[0] = sink;
  aux[4] = 1.0;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  HIP_OK(hipMemcpyAsync(state, buf.data(), buf.size(), hipMemcpyHostToDevice, s));
  HIP_OK(hipStreamSynchronize(s));
  return QME_OK;
  QME_GUARD_END
}

extern "C" qme_status qme_get_state(const qme_ctx *c, const void *state, double *rho_re,
                                    double *rho_im, double *sink, void *hip_stream) {
  QME_GUARD_BEGIN
  set_error("");
  if (!c || !state) { set_error("NULL argument"); return QME_E_ARG; }
  qme_status st = check_device(c);
  if (st != QME_OK) return st;
  const size_t pe = plane_elems(c);
  std::vector<char> buf(state_bytes(c));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  HIP_OK(hipMemcpyAsync(buf.data(), state, buf.size(), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  for (int64_t i = 0; i < c->n; ++i)
    for (int64_t j = 0; j < c->n; ++j) {
      size_t dst = size_t(i) * c->n + j, o = size_t(i) * c->ld + j;
      double xr, xi;
      if (c->elem == 8) {
        xr = reinterpret_cast<double *>(buf.data())[o];
        xi = reinterpret_cast<double *>(buf.data())[pe + o];
      } else {
        xr = reinterpret_cast<float *>(buf.data())[o];
        xi = reinterpret_cast<float *>(buf.data())[pe + o];
      }
      if (rho_re) rho_re[dst] = xr;
      if (rho_im) rho_im[dst] = xi;
    }
  if (sink) *sink = reinterpret_cast<double *>(buf.data() + 2 * pe * c->elem)[0];
  return QME_OK;
  QME_GUARD_END
}

extern "C" qme_status qme_step(qme_ctx *c, void *state, int64_t n_steps, void *ws,
                               void *hip_stream) {
  QME_GUARD_BEGIN
  TraceRange range("qme_step");
  set_error("");
  if (!c || !state || !ws) { set_error("NULL argument"); return QME_E_ARG; }
  if (n_steps < 0) { set_error("n_steps < 0"); return QME_E_ARG; }
  if ((reinterpret_cast<uintptr_t>(state) | reinterpret_cast<uintptr_t>(ws)) & 255) {
    set_error("state and workspace must be 256-byte aligned");
    return QME_E_ARG;
  }
  qme_status st = check_device(c);
  if (st != QME_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  auto run = [&](hipStream_t on) {
    return c->elem == 8 ? step_impl<double>(c, state, n_steps, ws, on)
                        : step_impl<float>(c, state, n_steps, ws, on);
  };
  if (c->fault_at >= 0 && c->steps_done + n_steps > c->fault_at) {
    // injected failure: run up to the fault step, then report a device error
    n_steps = std::max<int64_t>(0, c->fault_at - c->steps_done);
    const qme_status r = n_steps > 0 ? run(s) : QME_OK;
    c->steps_done += n_steps;
    if (r != QME_OK) return r;
    set_error("injected fault (QME_FAULT_AT_STEP) after step " + std::to_string(c->fault_at));
    return QME_E_DEVICE;
  }
  c->steps_done += n_steps;
  if (!c->use_graph || c->profiling || n_steps == 0) return run(s);
  const auto key = std::make_tuple(n_steps, state, ws);
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    // capture the run's launches once, on a private default-priority stream
    if (!c->capture_stream) HIP_OK(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
    HIP_OK(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
    const qme_status r = run(c->capture_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->capture_stream, &g);
    if (r != QME_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      if (r != QME_OK) return r;
      set_error(std::string("graph capture failed: ") + hipGetErrorString(e));
      return QME_E_DEVICE;
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(g);
      set_error(std::string("graph instantiation failed: ") + hipGetErrorString(ei));
      return QME_E_DEVICE;
    }
    c->graph_defs.push_back(g);
    it = c->graphs.emplace(key, ex).first;
  }
  HIP_OK(hipGraphLaunch(it->second, s));
  return QME_OK;
  QME_GUARD_END
}

extern "C" qme_status qme_step_noalloc(qme_ctx *c, void *state, int64_t n_steps,
                                       void *hip_stream) {
  QME_GUARD_BEGIN
  TraceRange range("qme_step_noalloc");
  set_error("");
  if (!c || !state) { set_error("NULL argument"); return QME_E_ARG; }
  if (n_steps < 0) { set_error("n_steps < 0"); return QME_E_ARG; }
  if (reinterpret_cast<uintptr_t>(state) & 255) {
    set_error("state must be 256-byte aligned");
    return QME_E_ARG;
  }
  size_t need = 0;
  qme_status st = qme_workspace_size(c, &need);
  if (st != QME_OK) return st;
  if (need > size_t(QME_NOALLOC_SCRATCH_BYTES)) {
    set_error("qme_step_noalloc: the step workspace of this context (" + std::to_string(need) +
              " bytes) exceeds the library's fixed scratch of " +
              std::to_string(size_t(QME_NOALLOC_SCRATCH_BYTES)) + " bytes; use qme_step");
    return QME_E_SIZE;
  }
  st = check_device(c);
  if (st != QME_OK) return st;
  if (!c->scratch) { set_error("no scratch address for this context's device"); return QME_E_DEVICE; }
  if (c->fault_at >= 0 && c->steps_done + n_steps > c->fault_at) {
    set_error("qme_step_noalloc: failure injection (QME_FAULT_AT_STEP) is served by qme_step");
    return QME_E_STATE;
  }
  // eager launches only (a graph capture or profiling events would allocate)
  const bool was_profiling = c->profiling;
  c->profiling = false;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const qme_status r = c->elem == 8 ? step_impl<double>(c, state, n_steps, c->scratch, s)
                                    : step_impl<float>(c, state, n_steps, c->scratch, s);
  c->profiling = was_profiling;
  if (r == QME_OK) c->steps_done += n_steps;
  return r;
  QME_GUARD_END
}

extern "C" qme_status qme_set_graph(qme_ctx *c, int32_t enable) {
  set_error("");
  if (!c) { set_error("ctx is NULL"); return QME_E_ARG; }
  if (enable != 0 && enable != 1) { set_error("enable must be 0 or 1"); return QME_E_ARG; }
  c->drop_graphs();
  c->use_graph = enable != 0;
  return QME_OK;
}

extern "C" qme_status qme_observe(const qme_ctx *c, const void *state, double *pops,
                                  double *trace, double *sink, void *hip_stream) {
  QME_GUARD_BEGIN
  set_error("");
  if (!c || !state) { set_error("NULL argument"); return QME_E_ARG; }
  qme_status st = check_device(c);
  if (st != QME_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const size_t pe = plane_elems(c);
  hipError_t e;
  if (c->elem == 8) e = launch_diag<double>(static_cast<const double *>(state), c->ld, c->n, c->diag, s);
  else e = launch_diag<float>(static_cast<const float *>(state), c->ld, c->n, c->diag, s);
  if (e != hipSuccess) { set_error(hipGetErrorString(e)); return QME_E_DEVICE; }
  std::vector<double> host(c->n + 8);
  const char *auxp = static_cast<const char *>(state) + 2 * pe * c->elem;
  HIP_OK(hipMemcpyAsync(host.data(), c->diag, sizeof(double) * c->n, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(host.data() + c->n, auxp, 64, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  double tr = 0.0;
  bool finite = true;
  for (int64_t u = 0; u < c->n; ++u) {
    tr += host[u];
    finite = finite && std::isfinite(host[u]);
  }
  if (pops) std::memcpy(pops, host.data(), sizeof(double) * c->n);
  if (trace) *trace = tr;
  if (sink) *sink = host[c->n];
  if (!finite || !std::isfinite(host[c->n]) || !(tr > 0.0)) {
    set_error("state is not finite or its trace is not positive");
    return QME_E_NUMERIC;
  }
  return QME_OK;
  QME_GUARD_END
}

extern "C" qme_status qme_observe_weighted(const qme_ctx *c, const void *state,
                                           const double *weights, double *value,
                                           void *hip_stream) {
  QME_GUARD_BEGIN
  set_error("");
  if (!c || !state || !weights || !value) { set_error("NULL argument"); return QME_E_ARG; }
  for (int64_t u = 0; u < c->n; ++u)
    if (!std::isfinite(weights[u])) { set_error("weights are not finite"); return QME_E_ARG; }
  qme_status st = check_device(c);
  if (st != QME_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e;
  if (c->elem == 8) e = launch_diag<double>(static_cast<const double *>(state), c->ld, c->n, c->diag, s);
  else e = launch_diag<float>(static_cast<const float *>(state), c->ld, c->n, c->diag, s);
  if (e != hipSuccess) { set_error(hipGetErrorString(e)); return QME_E_DEVICE; }
  std::vector<double> pops(c->n);
  HIP_OK(hipMemcpyAsync(pops.data(), c->diag, sizeof(double) * c->n, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  // the same FP64 sum, in index order, as the objective qme_adjoint returns
  double f = 0.0;
  for (int64_t u = 0; u < c->n; ++u) f += weights[u] * pops[u];
  *value = f;
  if (!std::isfinite(f)) { set_error("the weighted population is not finite"); return QME_E_NUMERIC; }
  return QME_OK;
  QME_GUARD_END
}

extern "C" qme_status qme_cgemm(int32_t precision, int64_t ld, const void *a_re,
                                const void *a_im, const void *m_re, const void *m_im,
                                const void *x_re, const void *x_im, void *c_re, void *c_im,
                                double alpha, double beta, int32_t conj_a, int32_t conj_b,
                                int32_t b_rows, int32_t lower, int32_t tile, void *hip_stream) {
  QME_GUARD_BEGIN
  set_error("");
  if (!a_re || !a_im || !m_re || !m_im || !c_re || !c_im) { set_error("NULL operand"); return QME_E_ARG; }
  if (beta != 0.0 && (!x_re || !x_im)) { set_error("beta != 0 needs X"); return QME_E_ARG; }
  if (ld <= 0 || tile <= 0 || ld % tile != 0) { set_error("ld must be a positive multiple of tile"); return QME_E_ARG; }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e;
  GemmOps o;
  o.conj_a = conj_a != 0;
  o.conj_b = conj_b != 0;
  o.b_rows = b_rows != 0;
  o.lower = lower != 0;
  {   // tile body chosen by launch size, as in the steps
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess) {
      o.direct = -1;
      o.cus = cus;
    }
  }
  if (precision == QME_FP32) {
    if (tile != 128 && tile != 64 && tile != 32) { set_error("FP32 tile must be 128, 64 or 32"); return QME_E_ARG; }
    CgemmArgs<float> g{static_cast<const float *>(a_re), static_cast<const float *>(a_im),
                       static_cast<const float *>(m_re), static_cast<const float *>(m_im),
                       static_cast<const float *>(x_re), static_cast<const float *>(x_im),
                       static_cast<float *>(c_re), static_cast<float *>(c_im), ld,
                       float(alpha), float(beta)};
    e = launch_cgemm_f32(g, tile, o, s);
  } else if (precision == QME_FP64) {
    if (tile != 64 && tile != 32) { set_error("FP64 tile must be 64 or 32"); return QME_E_ARG; }
    CgemmArgs<double> g{static_cast<const double *>(a_re), static_cast<const double *>(a_im),
                        static_cast<const double *>(m_re), static_cast<const double *>(m_im),
                        static_cast<const double *>(x_re), static_cast<const double *>(x_im),
                        static_cast<double *>(c_re), static_cast<double *>(c_im), ld, alpha, beta};
    e = launch_cgemm_f64(g, tile, o, s);
  } else if (precision == QME_BF16X3) {
    if (tile != 64 || o.b_rows) { set_error("BF16X3 products use tile 64 and the M^T / M^H forms"); return QME_E_ARG; }
    CgemmArgs<float> g{static_cast<const float *>(a_re), static_cast<const float *>(a_im),
                       static_cast<const float *>(m_re), static_cast<const float *>(m_im),
                       static_cast<const float *>(x_re), static_cast<const float *>(x_im),
                       static_cast<float *>(c_re), static_cast<float *>(c_im), ld,
                       float(alpha), float(beta)};
    e = launch_cgemm_bf16x3(g, o, s);
  } else {
    set_error("unknown precision");
    return QME_E_ARG;
  }
  if (e != hipSuccess) { set_error(std::string("launch failed: ") + hipGetErrorString(e)); return QME_E_DEVICE; }
  return QME_OK;
  QME_GUARD_END
}

extern "C" qme_status qme_set_fold(qme_ctx *c, int32_t enable) {
  set_error("");
  if (!c) { set_error("ctx is NULL"); return QME_E_ARG; }
  if (enable != 0 && enable != 1) { set_error("enable must be 0 or 1"); return QME_E_ARG; }
  c->drop_graphs();
  c->fold = enable != 0;
  return QME_OK;
}

extern "C" qme_status qme_set_direct_loads(qme_ctx *c, int32_t mode) {
  set_error("");
  if (!c) { set_error("ctx is NULL"); return QME_E_ARG; }
  if (mode < -1 || mode > 1) { set_error("mode must be -1, 0 or 1"); return QME_E_ARG; }
  c->drop_graphs();
  c->direct = mode;
  return QME_OK;
}

extern "C" qme_status qme_set_fused(qme_ctx *c, int32_t enable) {
  set_error("");
  if (!c) { set_error("ctx is NULL"); return QME_E_ARG; }
  if (enable != 0 && enable != 1) { set_error("enable must be 0 or 1"); return QME_E_ARG; }
  c->drop_graphs();
  c->fused = enable != 0;
  return QME_OK;
}

extern "C" qme_status qme_set_split(qme_ctx *c, int32_t enable) {
  set_error("");
  if (!c) { set_error("ctx is NULL"); return QME_E_ARG; }
  if (enable != 0 && enable != 1) { set_error("enable must be 0 or 1"); return QME_E_ARG; }
  c->drop_graphs();
  c->tail_split = enable != 0;
  return QME_OK;
}

extern "C" qme_status qme_set_tiles(qme_ctx *c, int32_t tile1, int32_t tile2) {
  set_error("");
  if (!c) { set_error("ctx is NULL"); return QME_E_ARG; }
  auto ok = [&](int t) {
    bool valid = c->precision == QME_FP64   ? (t == 64 || t == 32)
                 : c->precision == QME_FP32 ? (t == 128 || t == 64 || t == 32)
                                            : t == 64;
    return valid && c->ld % t == 0;
  };
  // BF16x3: the first product also on 128 x 64 tiles
  const bool wide = c->precision == QME_BF16X3 && tile1 == 128 && c->ld % 128 == 0 && tile2 == 64;
  if (!(ok(tile1) || wide) || !ok(tile2)) {
    set_error("tile not supported for this precision or does not divide ld");
    return QME_E_ARG;
  }
  c->drop_graphs();
  c->tile1 = tile1;
  c->tile2 = tile2;
  return QME_OK;
}

extern "C" qme_status qme_gradient_size(const qme_ctx *c, int64_t *n_params) {
  set_error("");
  if (!c || !n_params) { set_error("NULL argument"); return QME_E_ARG; }
  *n_params = int64_t(c->term_offset.size()) - 1 + int64_t(c->model.jumps.size());
  return QME_OK;
}

extern "C" qme_status qme_get_tiles(const qme_ctx *c, int32_t *tile1, int32_t *tile2) {
  set_error("");
  if (!c || !tile1 || !tile2) { set_error("NULL argument"); return QME_E_ARG; }
  *tile1 = c->tile1;
  *tile2 = c->tile2;
  return QME_OK;
}

extern "C" qme_status qme_profile_enable(qme_ctx *c, int32_t enable) {
  set_error("");
  if (!c) { set_error("ctx is NULL"); return QME_E_ARG; }
  if (enable < 0) { set_error("enable must be >= 0"); return QME_E_ARG; }
  c->profiling = enable != 0;
  c->profile_every = enable > 0 ? enable : 1;
  c->profile_step = 0;
  c->pairs_used = c->pairs_marked = 0;
  c->records.clear();
  return QME_OK;
}

hipError_t qme_ctx::Timer::next_pair(hipEvent_t *start, hipEvent_t *stop) {
  if (c->pairs_used == c->ev_start.size()) {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&b);
    if (e != hipSuccess) {
      (void)hipEventDestroy(a);
      return e;
    }
    c->ev_start.push_back(a);
    c->ev_stop.push_back(b);
  }
  *start = static_cast<hipEvent_t>(c->ev_start[c->pairs_used]);
  *stop = static_cast<hipEvent_t>(c->ev_stop[c->pairs_used]);
  ++c->pairs_used;
  return hipSuccess;
}

extern "C" qme_status qme_profile_read(qme_ctx *c, double *total_ms, int64_t *launches) {
  QME_GUARD_BEGIN
  set_error("");
  if (!c) { set_error("ctx is NULL"); return QME_E_ARG; }
  double ms[4] = {0, 0, 0, 0};
  int64_t cnt[4] = {0, 0, 0, 0};
  if (c->pairs_used > 0)
    HIP_OK(hipEventSynchronize(static_cast<hipEvent_t>(c->ev_stop[c->pairs_used - 1])));
  for (const qme_ctx::ProfileRecord &r : c->records) {
    if (r.kind < 0 || r.kind > 3) continue;
    for (size_t i = r.first; i < r.last; ++i) {
      float t = 0.0f;
      HIP_OK(hipEventElapsedTime(&t, static_cast<hipEvent_t>(c->ev_start[i]),
                                 static_cast<hipEvent_t>(c->ev_stop[i])));
      ms[r.kind] += t;
    }
    cnt[r.kind] += 1;
  }
  for (int k = 0; k < 4; ++k) {
    if (total_ms) total_ms[k] = ms[k];
    if (launches) launches[k] = cnt[k];
  }
  return QME_OK;
  QME_GUARD_END
}

void qme_ctx::drop_graphs() {
  if (graphs.empty() && graph_defs.empty()) return;
  (void)hipDeviceSynchronize();   // no replay may still run
  for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
  graphs.clear();
  for (hipGraph_t g : graph_defs) (void)hipGraphDestroy(g);
  graph_defs.clear();
}

qme_ctx::~qme_ctx() {
  if (launch_timer() == &timer) launch_timer() = nullptr;
  drop_graphs();
  if (capture_stream) (void)hipStreamDestroy(capture_stream);
  for (void *e : sel_ev)
    if (e) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
  if (sel_count_host) (void)hipHostFree(sel_count_host);
  for (void *e : ev_start) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
  for (void *e : ev_stop) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
  for (void *p : {(void *)csr_ptr, (void *)csrt_ptr, (void *)kj_ptr, (void *)koff_ptr,
                  (void *)csr_col, (void *)csrt_col, (void *)kj_col, (void *)koff_col,
                  (void *)csr_val, (void *)csrt_val, (void *)kj_val, (void *)koff_val,
                  (void *)csr_gamma, (void *)csr_channel, (void *)loff_row, (void *)loff_col,
                  (void *)loff_val})
    if (p) (void)hipFree(p);
  for (void *p : {du_re, du_im, du_split, (void *)parent_keep, (void *)d, (void *)leak, (void *)trw, (void *)diag, (void *)pi, (void *)cg,
                  (void *)tau, (void *)ca, (void *)upi, (void *)uc, (void *)ada, (void *)arrival_of,
                  (void *)h_ptr, (void *)h_col, (void *)h_val, (void *)t_row, (void *)t_col,
                  (void *)t_val})
    if (p) (void)hipFree(p);
}

extern "C" void qme_destroy(qme_ctx *c) { delete c; }
