"""Python front end of the solver: marshals a workload description into the
C ABI structures and wraps a context.  PyTorch provides device memory and the
stream; every step of the method runs in libqme.so."""
from __future__ import annotations

import ctypes
from ctypes import POINTER, byref, c_double, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

from . import _lib as L


class Marshal:
    """C structures for one workload dict (keeps the arrays alive)."""

    def __init__(self, wl: dict):
        atoms = list(wl["atoms"])
        nc = len(atoms)
        self._atoms = (c_int32 * nc)(*atoms)
        self._caps = (c_int32 * nc)(*wl["photon_cap"])
        self.system = L.System(nc, self._atoms, self._caps, int(wl.get("exc_min", 0)),
                               int(wl.get("exc_max", -1)))
        na = int(sum(atoms))
        self._oc = (c_double * nc)(*wl["omega_c"])
        self._oa = (c_double * max(na, 1))(*(wl["omega_a"] or [0.0]))
        self._g = (c_double * max(na, 1))(*(wl["g"] or [0.0]))
        hops = wl.get("hops", [])
        jumps = wl.get("jumps", [])
        self._hops = (L.Hop * max(len(hops), 1))(*[L.Hop(int(a), int(b), float(m)) for a, b, m in hops])
        self._jumps = (L.Jump * max(len(jumps), 1))(
            *[L.Jump(int(k), int(c), int(a), float(gm)) for k, c, a, gm in jumps])
        self.params = L.Params(self._oc, self._oa, self._g, len(hops), self._hops,
                               len(jumps), self._jumps, float(wl["dt"]))


class MarshalGeneral:
    """C arrays of a general-form workload: {"general": True, "n": N,
    "h": (rows, cols, vals), "jumps": [(gamma, source, target, coef), ...],
    "dt": dt} (keeps the arrays alive)."""

    def __init__(self, wl: dict):
        rows, cols, vals = wl["h"]
        self.n = int(wl["n"])
        self.rows = np.ascontiguousarray(rows, dtype=np.int32)
        self.cols = np.ascontiguousarray(cols, dtype=np.int32)
        self.vals = np.ascontiguousarray(vals, dtype=np.float64)
        self._keep = []
        js = []
        for gamma, src, dst, coef in wl["jumps"]:
            src = np.ascontiguousarray(src, dtype=np.int32)
            dst = np.ascontiguousarray(dst, dtype=np.int32)
            coef = np.ascontiguousarray(coef, dtype=np.float64)
            self._keep += [src, dst, coef]
            js.append(L.GeneralJump(float(gamma), int(src.size),
                                    src.ctypes.data_as(POINTER(c_int32)),
                                    dst.ctypes.data_as(POINTER(c_int32)),
                                    coef.ctypes.data_as(POINTER(c_double))))
        self.jumps = (L.GeneralJump * max(len(js), 1))(*js)
        self.n_jumps = len(js)
        self.dt = float(wl["dt"])

    def create(self, lib, precision: int, stream, out):
        return lib.qme_hamiltonian_general(
            self.n, int(self.vals.size), self.rows.ctypes.data_as(POINTER(c_int32)),
            self.cols.ctypes.data_as(POINTER(c_int32)), _dptr(self.vals), self.n_jumps,
            self.jumps, self.dt, precision, stream, out)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_double))


def basis(wl: dict) -> np.ndarray:
    """Occupation table (N x n_modes, int32) of the workload's basis."""
    lib = L.load()
    m = Marshal(wl)
    n = c_int64(0)
    L.check(lib.qme_basis(byref(m.system), byref(n), None, 0))
    n_modes = len(wl["atoms"]) + int(sum(wl["atoms"]))
    occ = np.zeros((n.value, n_modes), dtype=np.int32)
    L.check(lib.qme_basis(byref(m.system), byref(n), occ.ctypes.data_as(POINTER(c_int32)),
                          n.value))
    return occ


def hamiltonian_coo(wl: dict):
    """(rows, cols, vals) of H in the basis."""
    lib = L.load()
    m = Marshal(wl)
    nnz = c_int64(0)
    L.check(lib.qme_hamiltonian_coo(byref(m.system), byref(m.params), byref(nnz), None,
                                    None, None, 0))
    r = np.zeros(nnz.value, np.int32)
    c = np.zeros(nnz.value, np.int32)
    v = np.zeros(nnz.value, np.float64)
    L.check(lib.qme_hamiltonian_coo(byref(m.system), byref(m.params), byref(nnz),
                                    r.ctypes.data_as(POINTER(c_int32)),
                                    c.ctypes.data_as(POINTER(c_int32)), _dptr(v), nnz.value))
    return r, c, v


def propagator_increment(wl: dict, n: int) -> np.ndarray:
    """dU = exp(-i H dt) - I computed by the library's FP64 Taylor stage."""
    lib = L.load()
    m = Marshal(wl)
    re = np.zeros((n, n))
    im = np.zeros((n, n))
    L.check(lib.qme_propagator_host(byref(m.system), byref(m.params), _dptr(re), _dptr(im), n))
    return re + 1j * im


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("a HIP device is required")
    return torch


class Solver:
    """One context on the current HIP device plus a torch-owned state buffer
    and workspace."""

    def __init__(self, wl: dict, precision: str = "fp32", stream=None, _ctx=None):
        torch = _torch()
        self.torch = torch
        self.lib = L.load()
        self.wl = wl
        self.general = bool(wl.get("general", False))
        self._m = MarshalGeneral(wl) if self.general else Marshal(wl)
        self.precision = precision
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        if _ctx is None:
            ctx = c_void_p()
            if self.general:
                L.check(self._m.create(self.lib, L.PRECISIONS[precision], self._sptr(), byref(ctx)))
            else:
                L.check(self.lib.qme_hamiltonian(byref(self._m.system), byref(self._m.params),
                                                 L.PRECISIONS[precision], self._sptr(), byref(ctx)))
        else:
            ctx = _ctx
        self.ctx = ctx
        n, ld, eb, sb = c_int64(), c_int64(), c_int64(), c_size_t()
        L.check(self.lib.qme_state_layout(ctx, byref(n), byref(ld), byref(eb), byref(sb)))
        self.n, self.ld, self.elem, self.state_bytes = n.value, ld.value, eb.value, sb.value
        ws = c_size_t()
        L.check(self.lib.qme_workspace_size(ctx, byref(ws)))
        self.workspace_bytes = ws.value
        dev = torch.device("cuda", torch.cuda.current_device())
        self.state = torch.zeros(self.state_bytes, dtype=torch.uint8, device=dev)
        self.workspace = torch.zeros(max(self.workspace_bytes, 256), dtype=torch.uint8, device=dev)

    def _sptr(self):
        return c_void_p(self.stream.cuda_stream)

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            self.lib.qme_destroy(self.ctx)
            self.ctx = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_state(self):
        """A fresh zeroed device state buffer of this context's layout."""
        return self.torch.zeros(self.state_bytes, dtype=self.torch.uint8, device=self.state.device)

    def set_rho(self, rho: np.ndarray, sink: float = 0.0, state=None):
        rho = np.asarray(rho, dtype=np.complex128)
        if rho.shape != (self.n, self.n):
            raise ValueError("rho has the wrong shape")
        re = np.ascontiguousarray(rho.real)
        im = np.ascontiguousarray(rho.imag)
        st = self.state if state is None else state
        L.check(self.lib.qme_set_state(self.ctx, c_void_p(st.data_ptr()), _dptr(re), _dptr(im),
                                       float(sink), self._sptr()))

    def get_rho(self, state=None):
        st = self.state if state is None else state
        re = np.zeros((self.n, self.n))
        im = np.zeros((self.n, self.n))
        sink = c_double()
        L.check(self.lib.qme_get_state(self.ctx, c_void_p(st.data_ptr()), _dptr(re), _dptr(im),
                                       byref(sink), self._sptr()))
        return re + 1j * im, sink.value

    def step(self, n_steps: int, state=None):
        st = self.state if state is None else state
        L.check(self.lib.qme_step(self.ctx, c_void_p(st.data_ptr()), int(n_steps),
                                  c_void_p(self.workspace.data_ptr()), self._sptr()))

    def step_noalloc(self, n_steps: int, state=None):
        """qme_step_noalloc: the same steps with the library's fixed device
        scratch as the workspace (no allocation; calls on one device must
        not overlap)."""
        st = self.state if state is None else state
        L.check(self.lib.qme_step_noalloc(self.ctx, c_void_p(st.data_ptr()), int(n_steps),
                                          self._sptr()))

    def observe(self, state=None):
        st = self.state if state is None else state
        pops = np.zeros(self.n)
        tr, sink = c_double(), c_double()
        L.check(self.lib.qme_observe(self.ctx, c_void_p(st.data_ptr()), _dptr(pops),
                                     byref(tr), byref(sink), self._sptr()))
        return pops, tr.value, sink.value

    def observe_weighted(self, weights, state=None) -> float:
        """f = sum_s weights[s] Re rho_ss in FP64 (qme_observe_weighted: the
        objective qme_adjoint differentiates, summed the same way)."""
        st = self.state if state is None else state
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
        if w.shape != (self.n,):
            raise ValueError("weights must have one entry per basis state")
        val = c_double()
        L.check(self.lib.qme_observe_weighted(self.ctx, c_void_p(st.data_ptr()), _dptr(w),
                                              byref(val), self._sptr()))
        return val.value

    def adjoint(self, n_steps: int, obs, checkpoint_every: int = 32, state=None):
        """(f, grad) for f = sum_s obs[s] Re rho_K[s,s] after n_steps from the
        given state (default: this solver's state, left unchanged); grad is
        ordered g per atom, mu per hop, gamma per jump (general-form models:
        H's symmetric entries in (r, c) order, r <= c, then gamma per jump)."""
        st = self.state if state is None else state
        obs = np.ascontiguousarray(np.asarray(obs, dtype=np.float64))
        if obs.shape != (self.n,):
            raise ValueError("obs must have one weight per basis state")
        ws = c_size_t()
        L.check(self.lib.qme_adjoint_workspace_size(self.ctx, int(n_steps), int(checkpoint_every),
                                                    byref(ws)))
        buf = self.torch.empty(max(ws.value, 256), dtype=self.torch.uint8, device=st.device)
        np_c = c_int64()
        L.check(self.lib.qme_gradient_size(self.ctx, byref(np_c)))
        n_par = np_c.value
        grad = np.zeros(max(n_par, 1))
        val = c_double()
        L.check(self.lib.qme_adjoint(self.ctx, c_void_p(st.data_ptr()), int(n_steps),
                                     int(checkpoint_every), _dptr(obs), byref(val), _dptr(grad),
                                     c_void_p(buf.data_ptr()), ws.value, self._sptr()))
        del buf
        return val.value, grad[:n_par]

    # ------------------------------------------- pure states (closed models)
    def set_psi(self, psi):
        """Pure state(s) for a closed model: psi of shape [N] or [n_vec, N]
        (complex); allocates the pure-state buffer and its workspace."""
        psi = np.asarray(psi, dtype=np.complex128)
        vecs = psi.reshape(1, -1) if psi.ndim == 1 else psi
        if vecs.ndim != 2 or vecs.shape[1] != self.n:
            raise ValueError("psi must have N entries per vector")
        self.psi_shape = psi.shape
        self.n_vec = int(vecs.shape[0])
        sb, wb = c_size_t(), c_size_t()
        L.check(self.lib.qme_pure_layout(self.ctx, self.n_vec, byref(sb), byref(wb)))
        dev = self.state.device
        self.psi = self.torch.zeros(sb.value, dtype=self.torch.uint8, device=dev)
        self.psi_workspace = self.torch.zeros(wb.value, dtype=self.torch.uint8, device=dev)
        re = np.ascontiguousarray(vecs.real)
        im = np.ascontiguousarray(vecs.imag)
        L.check(self.lib.qme_pure_set(self.ctx, c_void_p(self.psi.data_ptr()), self.n_vec,
                                      _dptr(re), _dptr(im), self._sptr()))

    def step_pure(self, n_steps: int):
        """n_steps steps psi <- U psi / |psi| of every vector (qme_pure_step)."""
        L.check(self.lib.qme_pure_step(self.ctx, c_void_p(self.psi.data_ptr()), self.n_vec,
                                       int(n_steps), c_void_p(self.psi_workspace.data_ptr()),
                                       self._sptr()))

    def get_psi(self):
        """The pure state(s), in the shape given to set_psi."""
        re = np.zeros((self.n_vec, self.n))
        im = np.zeros((self.n_vec, self.n))
        L.check(self.lib.qme_pure_get(self.ctx, c_void_p(self.psi.data_ptr()), self.n_vec,
                                      _dptr(re), _dptr(im), self._sptr()))
        return (re + 1j * im).reshape(self.psi_shape)

    # ------------------------------------------------ state-space selection
    def subspace(self, keep) -> "Solver":
        """A solver on the subset `keep` (ascending indices into this basis);
        its state is zero until compact_into or set_rho fills it."""
        keep = np.ascontiguousarray(keep, dtype=np.int32)
        ctx = c_void_p()
        L.check(self.lib.qme_subspace(self.ctx, keep.ctypes.data_as(POINTER(c_int32)),
                                      int(keep.size), self._sptr(), byref(ctx)))
        return Solver(self.wl, self.precision, self.stream, _ctx=ctx)

    def compact_into(self, sub: "Solver", state=None):
        """Renormalised P rho P of this solver's state into sub's state."""
        st = self.state if state is None else state
        L.check(self.lib.qme_compact_state(self.ctx, c_void_p(st.data_ptr()), sub.ctx,
                                           c_void_p(sub.state.data_ptr()), self._sptr()))

    def select_device(self, p_prev, p_now, interval: float, eps: float, keep, n_keep, state=None):
        """qme_select_device: the keep/delete decision on the device.  p_prev,
        p_now: float64 device tensors of at least n entries (may be one
        tensor); keep: int32 device tensor of at least n entries; n_keep:
        int64 device tensor (its first entry receives the count, -1 for a
        non-finite population).  Asynchronous on the solver's stream."""
        torch = self.torch
        for t, dt_, size in ((p_prev, torch.float64, self.n), (p_now, torch.float64, self.n),
                             (keep, torch.int32, self.n), (n_keep, torch.int64, 1)):
            if (not isinstance(t, torch.Tensor) or t.dtype != dt_ or not t.is_cuda
                    or not t.is_contiguous() or t.numel() < size):
                raise ValueError("select_device needs contiguous device tensors of the documented "
                                 "dtypes and sizes")
        st = self.state if state is None else state
        L.check(self.lib.qme_select_device(self.ctx, c_void_p(st.data_ptr()),
                                           c_void_p(p_prev.data_ptr()), c_void_p(p_now.data_ptr()),
                                           float(interval), float(eps), c_void_p(keep.data_ptr()),
                                           c_void_p(n_keep.data_ptr()), self._sptr()))

    def set_tiles(self, tile1: int, tile2: int):
        L.check(self.lib.qme_set_tiles(self.ctx, int(tile1), int(tile2)))

    @property
    def tiles(self):
        """(tile1, tile2): the tile edges of the two products."""
        a, b = c_int32(), c_int32()
        L.check(self.lib.qme_get_tiles(self.ctx, byref(a), byref(b)))
        return a.value, b.value

    @property
    def tile1(self):
        return self.tiles[0]

    @property
    def tile2(self):
        return self.tiles[1]

    def set_split(self, enable: bool):
        """k-splits of the products on (default) or off: the tail of the
        lower-triangle product, and every tile of a launch too small for the
        device (FP32 / FP64)."""
        L.check(self.lib.qme_set_split(self.ctx, int(bool(enable))))

    def set_fold(self, enable: bool):
        """Folded steps (decoherence in the lower product's epilogue,
        renormalisation in the next product) on (default) or off."""
        L.check(self.lib.qme_set_fold(self.ctx, int(bool(enable))))

    def set_direct_loads(self, mode: int):
        """FP32 product tile body: 1 direct HBM-to-LDS loads, 0 register
        staging, -1 (default) direct for launches with fewer than two
        blocks per compute unit.  Bitwise-neutral."""
        L.check(self.lib.qme_set_direct_loads(self.ctx, int(mode)))

    def set_graph(self, enable: bool):
        """Replay qme_step runs from captured hipGraphs (off by default)."""
        L.check(self.lib.qme_set_graph(self.ctx, int(bool(enable))))

    def set_fused(self, enable: bool):
        """Single-workgroup path for N <= 32 (FP32 / FP64) on (default) or off."""
        L.check(self.lib.qme_set_fused(self.ctx, int(bool(enable))))

    # ---------------------------------------------------------- profiling
    KINDS = ("product_full", "product_lower", "trace", "dissipate")

    def profile(self, enable=True):
        """Per-kernel event timing: True / 1 on every step, an int k > 1 on
        every k-th step, False / 0 off."""
        L.check(self.lib.qme_profile_enable(self.ctx, int(enable)))

    def profile_read(self):
        """{kind: (total_ms, launches)} since profiling was enabled."""
        ms = (c_double * 4)()
        cnt = (c_int64 * 4)()
        L.check(self.lib.qme_profile_read(self.ctx, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.KINDS)}


class Batch:
    """Many FP32 solvers stepped together: one launch per phase covers every
    instance's tiles; a run of steps is replayed from one captured hipGraph."""

    def __init__(self, solvers):
        self.solvers = list(solvers)
        if not self.solvers:
            raise ValueError("empty batch")
        self.lib = L.load()
        self.torch = self.solvers[0].torch
        n = len(self.solvers)
        ctxs = (c_void_p * n)(*[s.ctx.value for s in self.solvers])
        states = (c_void_p * n)(*[s.state.data_ptr() for s in self.solvers])
        b = c_void_p()
        L.check(self.lib.qme_batch_create(ctxs, states, n, byref(b)))
        self.handle = b
        ws = c_size_t()
        L.check(self.lib.qme_batch_workspace_size(b, byref(ws)))
        self.workspace_bytes = ws.value
        self.workspace = self.torch.zeros(max(ws.value, 256), dtype=self.torch.uint8,
                                          device=self.solvers[0].state.device)
        self.stream = self.solvers[0].stream

    def config(self, use_graph=True, largest_first=True):
        L.check(self.lib.qme_batch_config(self.handle, int(use_graph), int(largest_first)))

    def persistent(self, enable=True):
        """One launch per run (qme_batch_persistent) on or off."""
        L.check(self.lib.qme_batch_persistent(self.handle, int(bool(enable))))

    def step(self, n_steps: int):
        L.check(self.lib.qme_batch_step(self.handle, int(n_steps),
                                        c_void_p(self.workspace.data_ptr()),
                                        self.workspace_bytes, c_void_p(self.stream.cuda_stream)))

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self.lib.qme_batch_destroy(self.handle)
            self.handle = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def select_states(p_prev, p_now, interval: float, eps: float) -> np.ndarray:
    """Indices of the states whose probability growth speed
    |p_now - p_prev| / interval is at least eps (qme_select_states)."""
    lib = L.load()
    p_prev = np.ascontiguousarray(p_prev, dtype=np.float64)
    p_now = np.ascontiguousarray(p_now, dtype=np.float64)
    if p_prev.shape != p_now.shape or p_prev.ndim != 1:
        raise ValueError("p_prev and p_now must be vectors of one length")
    keep = np.zeros(p_now.size, dtype=np.int32)
    n_keep = c_int64(0)
    L.check(lib.qme_select_states(int(p_now.size), _dptr(p_prev), _dptr(p_now), float(interval),
                                  float(eps), keep.ctypes.data_as(POINTER(c_int32)), byref(n_keep)))
    return keep[:n_keep.value].copy()


def evolve_with_selection(sol: Solver, n_steps: int, eps: float, every: int = 1,
                          device: bool = False):
    """The selection loop of Sec. III.B on a solver whose state is set: solve
    `every` steps, compare each state's growth speed over them with eps, move
    the state onto the kept states (renormalised), repeat until n_steps.  The
    next comparison starts from the renormalised state.  Returns (solver,
    kept, sizes): the solver on the final basis (the input solver if nothing
    was removed; solvers made on the way are closed except the last, which
    the caller owns), the indices of its states in the input basis, and the
    basis size after each solve.

    device=True takes each decision on the device (qme_select_device) and
    runs one solve ahead of it: the next solve is queued from a snapshot of
    the state before the host reads the decision, and is dropped (the state
    restored from the snapshot) when the decision removes states.  The same
    decisions, subsets and states as the host loop, without a host round
    trip between solves."""
    if device:
        return _evolve_with_selection_device(sol, n_steps, eps, every)
    kept = np.arange(sol.n, dtype=np.int64)
    sizes = []
    owned = False
    p_prev, _, _ = sol.observe()
    done = 0
    while done < n_steps:
        k = min(every, n_steps - done)
        sol.step(k)
        done += k
        p_now, _, _ = sol.observe()
        keep = select_states(p_prev, p_now, k * float(sol.wl["dt"]), eps)
        if keep.size < sol.n:
            sub = sol.subspace(keep)
            sol.compact_into(sub)
            p_now, _, _ = sub.observe()          # synchronises the stream
            if owned:
                sol.close()
            sol, owned = sub, True
            kept = kept[keep]
        p_prev = p_now
        sizes.append(sol.n)
    return sol, kept, sizes


def _evolve_with_selection_device(sol: Solver, n_steps: int, eps: float, every: int):
    torch = sol.torch
    kept = np.arange(sol.n, dtype=np.int64)
    sizes = []
    owned = False
    if n_steps <= 0:
        return sol, kept, sizes
    lib = sol.lib
    done_steps = 0
    fresh = 1
    area = None
    while done_steps < n_steps:
        if area is None:
            nbytes = c_size_t()
            L.check(lib.qme_select_workspace_size(sol.ctx, byref(nbytes)))
            area = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=sol.state.device)
            keep = np.zeros(sol.n, dtype=np.int32)
        k = min(every, n_steps - done_steps)
        solves = (n_steps - done_steps) // k
        done, n_keep = c_int64(0), c_int64(0)
        L.check(lib.qme_select_run(sol.ctx, c_void_p(sol.state.data_ptr()),
                                   c_void_p(sol.workspace.data_ptr()), c_void_p(area.data_ptr()),
                                   int(solves), int(k), float(eps), int(fresh), byref(done),
                                   byref(n_keep), keep.ctypes.data_as(POINTER(c_int32)),
                                   sol._sptr()))
        done_steps += done.value * k
        fresh = 0
        if n_keep.value == sol.n:
            sizes += [sol.n] * done.value
            continue
        sizes += [sol.n] * (done.value - 1)
        idx = keep[:n_keep.value].copy()
        sub = sol.subspace(idx)
        sol.compact_into(sub)
        if owned:
            sol.close()
        sol, owned = sub, True
        kept = kept[idx]
        sizes.append(sol.n)
        fresh, area = 1, None
    return sol, kept, sizes
