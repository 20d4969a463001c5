"""State-space selection on the device (qme_select_states, qme_subspace,
qme_compact_state, driven by evolve_with_selection) against the oracle's
selection loop: identical kept sets and basis-size histories (integer
results, bit-exact), states within the precision's tolerance.  Every case
checks on the oracle side that no growth speed lies near epsilon, so both
sides take each keep/delete decision the same way."""
import numpy as np
import pytest

import workloads as W
from oracle import evolve as ev
from oracle import selection as sel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2403_07042_amd")
from paper_2403_07042_amd import _lib as L  # noqa: E402

TOL = {"fp64": 1e-11, "fp32": 1e-5}


def oracle_margin(wl, rho0, steps, eps, every):
    """Smallest |log10(speed / eps)| over every solve of the oracle loop."""
    sysm = ev.System(wl)
    rho, sink = rho0.astype(np.complex128), 0.0
    worst = np.inf
    done = 0
    while done < steps:
        k = min(every, steps - done)
        p0 = np.real(np.diag(rho)).copy()
        for _ in range(k):
            rho, sink = ev.step(rho, sink, sysm.u, sysm.jumps, sysm.dt)
        done += k
        speed = sel.growth_speed(p0, np.real(np.diag(rho)), k * sysm.dt)
        pos = speed[speed > 0]
        if pos.size:
            worst = min(worst, float(np.abs(np.log10(pos / eps)).min()))
        keep = np.nonzero(speed >= eps)[0]
        if keep.size < sysm.n:
            block = rho[np.ix_(keep, keep)]
            rho = block * ((1.0 - sink) / np.trace(block).real)
            sysm = ev.System(wl, occ=sysm.occ[keep])
    return worst


CASES = {
    "damped_jc": (lambda: W.jc_single(), 2000, 1e-20, 100),
    "lattice_9x9": (lambda: W.photon_lattice(9, 9, gamma=0.0), 200, 1e-20, 1),
    "tch_2x2_lossy_cut": (lambda: W.tch_2x2(steps=50), 50, 1e-4, 5),
}


# The lossy cut starts from a Haar state, so its growth speeds spread
# continuously and some lie within FP32 resolution of eps: FP64 only.
PAIRS = [("fp64", c) for c in sorted(CASES)] + [("fp32", "damped_jc"), ("fp32", "lattice_9x9")]


@pytest.mark.parametrize("precision,case", PAIRS)
def test_selection_loop_matches_oracle(case, precision):
    make, steps, eps, every = CASES[case]
    wl = make()
    occ = P.basis(wl)
    rho0 = W.initial_rho(wl, occ)
    margin = oracle_margin(wl, rho0, steps, eps, every)
    need = 1e-6 if precision == "fp64" else 1e-2      # decades between any speed and eps
    if margin < need:
        pytest.skip(f"a growth speed lies within 10^{margin:.1e} of eps")
    ref_rho, ref_sink, ref_kept, ref_sizes = sel.select_evolve(wl, rho0, steps, eps, every)
    sol = P.Solver(wl, precision)
    sol.set_rho(rho0)
    print(f"selection {case} {precision}: {steps} steps eps={eps} every={every}", flush=True)
    out, kept, sizes = P.evolve_with_selection(sol, steps, eps, every)
    rho, sink = out.get_rho()
    if out is not sol:
        out.close()
    sol.close()
    assert sizes == ref_sizes
    assert np.array_equal(kept, ref_kept)
    assert np.abs(rho - ref_rho).max() < TOL[precision]
    assert abs(sink - ref_sink) < (1e-12 if precision == "fp64" else 1e-6)


def test_eps_zero_changes_nothing():
    wl = W.tch_2x2(steps=20)
    rho0 = W.initial_rho(wl, P.basis(wl))
    a = P.Solver(wl, "fp32")
    a.set_rho(rho0)
    out, kept, sizes = P.evolve_with_selection(a, 20, 0.0, 1)
    assert out is a and sizes == [a.n] * 20 and np.array_equal(kept, np.arange(a.n))
    b = P.Solver(wl, "fp32")
    b.set_rho(rho0)
    b.step(20)
    assert np.array_equal(a.get_rho()[0], b.get_rho()[0])
    a.close()
    b.close()


def test_lattice_2048_first_solve_keeps_radius_two_ball_and_matches_oracle():
    """The full-size 32 x 32 lattice (N = 2048): after one FP32 step with
    eps = 1e-20 the basis is the 18-state ball of radius 2 around the start
    (the oracle's decision), then 1000 steps run on it."""
    wl = W.photon_lattice(gamma=0.0)
    occ = P.basis(wl)
    rho0 = W.initial_rho(wl, occ)
    r1, _, k1, _ = sel.select_evolve(wl, rho0, 1, 1e-20)
    assert k1.size == 18
    sol = P.Solver(wl, "fp32")
    sol.set_rho(rho0)
    print("selection lattice 2048 fp32: first solve", flush=True)
    out, kept, sizes = P.evolve_with_selection(sol, 1, 1e-20, 1)
    assert np.array_equal(kept, k1) and sizes == [18]
    rho, _ = out.get_rho()
    assert np.abs(rho - r1).max() < 1e-6
    out.step(999)
    rho, _ = out.get_rho()
    sysm = ev.System(wl, occ=occ[k1])
    ref, _ = ev.evolve(sysm, r1, 999)
    assert np.abs(rho - ref).max() < 1e-5
    out.close()
    sol.close()


def test_compact_state_argument_errors():
    wl = W.tch_2x2(steps=5)
    a = P.Solver(wl, "fp32")
    a.set_rho(W.initial_rho(wl, P.basis(wl)))
    b = P.Solver(wl, "fp32")
    sub = a.subspace(np.arange(0, a.n, 2))
    with pytest.raises(L.QmeError) as e:
        b.compact_into(a)                         # a was not made by qme_subspace
    assert "QME_E_STATE" in str(e.value)
    lib = L.load()
    st = lib.qme_compact_state(a.ctx, L.c_void_p(a.state.data_ptr()), sub.ctx,
                               L.c_void_p(a.state.data_ptr()), None)
    assert st == L.QME_E_ARG                      # same buffer
    sub64 = P.Solver(wl, "fp64").subspace(np.arange(4))
    with pytest.raises(L.QmeError):
        a.compact_into(sub64)                     # precision differs
    for bad in ([], [3, 2], [0, a.n]):
        with pytest.raises(L.QmeError):
            a.subspace(np.array(bad, dtype=np.int32))
    a.compact_into(sub)
    rho, _ = sub.get_rho()
    assert abs(np.trace(rho).real - 1.0) < 1e-6
    for s in (a, b, sub, sub64):
        s.close()


def diagonal_model(n):
    """A general-form model of n states with a diagonal Hamiltonian and no
    decoherence: a state's populations are exactly what set_rho put there."""
    idx = np.arange(n, dtype=np.int32)
    return {"general": True, "name": f"diag_{n}", "n": n,
            "h": (idx, idx, np.linspace(0.0, 1.0, n)), "jumps": [], "dt": 0.01, "steps": 1}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [1, 5, 1023, 1024, 1025, 2500])
def test_device_decision_matches_host_decision(n, precision):
    """qme_select_device against qme_select_states on the same populations:
    the same kept indices in the same order and the same count, across the
    kernel's 1024-state chunks; speeds exactly at eps are kept on both sides;
    the populations written are the state's diagonal."""
    rng = np.random.default_rng(100 + n)
    sol = P.Solver(diagonal_model(n), precision)
    p_now = rng.random(n) / n
    p_prev = p_now + rng.choice([0.0, 1e-9, -1e-9, 3e-7], size=n)
    p_prev[::7] = p_now[::7]                             # zero speed: removed unless eps = 0
    sol.set_rho(np.diag(p_now).astype(np.complex128))
    stored = np.real(np.diag(sol.get_rho()[0])).copy()  # the stored (possibly FP32) diagonal
    interval, eps = 0.5, 2e-9                            # 1e-9 / 0.5 = eps exactly: kept
    dev = sol.state.device
    prev = torch.tensor(p_prev, dtype=torch.float64, device=dev)
    now = torch.zeros(n, dtype=torch.float64, device=dev)
    keep = torch.full((n,), -7, dtype=torch.int32, device=dev)
    nk = torch.zeros(1, dtype=torch.int64, device=dev)
    print(f"device decision n={n} {precision}", flush=True)
    sol.select_device(prev, now, interval, eps, keep, nk)
    torch.cuda.synchronize()
    ref = P.select_states(p_prev, stored, interval, eps) if np.any(
        np.abs(stored - p_prev) / interval >= eps) else np.zeros(0, np.int32)
    assert int(nk.item()) == ref.size
    assert np.array_equal(keep[:ref.size].cpu().numpy(), ref)
    assert np.array_equal(now.cpu().numpy(), stored)
    # in place (p_now aliases p_prev), eps = 0 keeps every state
    sol.select_device(prev, prev, interval, 0.0, keep, nk)
    torch.cuda.synchronize()
    assert int(nk.item()) == n and np.array_equal(keep.cpu().numpy(), np.arange(n))
    assert np.array_equal(prev.cpu().numpy(), stored)
    # a non-finite population: count -1
    bad = torch.tensor(p_prev, dtype=torch.float64, device=dev)
    bad[n // 2] = float("nan")
    sol.select_device(bad, now, interval, eps, keep, nk)
    torch.cuda.synchronize()
    assert int(nk.item()) == -1
    with pytest.raises(L.QmeError):
        sol.select_device(prev, now, 0.0, eps, keep, nk)      # interval must be > 0
    with pytest.raises(ValueError):
        sol.select_device(prev[: n - 1] if n > 1 else prev.float(), now, interval, eps, keep, nk)
    sol.close()


DEVICE_LOOP_CASES = [("fp64", "damped_jc"), ("fp64", "lattice_9x9"), ("fp64", "tch_2x2_lossy_cut"),
                     ("fp32", "lattice_9x9"), ("fp32", "damped_jc")]


@pytest.mark.parametrize("precision,case", DEVICE_LOOP_CASES)
def test_device_selection_loop_matches_host_loop(case, precision):
    """The loop that decides on the device and queues the next solve ahead
    gives the host loop's sizes, kept states, final state and sink bit for
    bit, and leaves the input solver's state where the host loop leaves it."""
    make, steps, eps, every = CASES[case]
    wl = make()
    rho0 = W.initial_rho(wl, P.basis(wl))
    res = {}
    for device in (False, True):
        sol = P.Solver(wl, precision)
        sol.set_rho(rho0)
        print(f"selection loop {case} {precision} device={device}", flush=True)
        out, kept, sizes = P.evolve_with_selection(sol, steps, eps, every, device=device)
        rho, sink = out.get_rho()
        res[device] = (rho, sink, kept, sizes, sol.get_rho()[0])
        if out is not sol:
            out.close()
        sol.close()
    (a, sa, ka, za, ia), (b, sb, kb, zb, ib) = res[False], res[True]
    assert za == zb and np.array_equal(ka, kb)
    assert np.array_equal(a, b) and sa == sb
    assert np.array_equal(ia, ib)
    assert len(za) == -(-steps // every)


def test_device_selection_loop_lattice_2048():
    """N = 2048, FP32, compared after every step: the first solve keeps the
    18-state ball, then the loop runs on it; device and host loops agree
    bitwise."""
    wl = W.photon_lattice(gamma=0.0)
    rho0 = W.initial_rho(wl, P.basis(wl))
    res = {}
    for device in (False, True):
        sol = P.Solver(wl, "fp32")
        sol.set_rho(rho0)
        print(f"selection loop lattice 2048 device={device}", flush=True)
        out, kept, sizes = P.evolve_with_selection(sol, 40, 1e-20, 1, device=device)
        res[device] = (out.get_rho(), kept, sizes)
        if out is not sol:
            out.close()
        sol.close()
    (ra, ka, za), (rb, kb, zb) = res[False], res[True]
    assert za == zb and za[0] == 18 and np.array_equal(ka, kb)
    assert np.array_equal(ra[0], rb[0]) and ra[1] == rb[1]


def test_device_selection_loop_ragged_runs_and_errors():
    """A step count that is not a multiple of the solve length (a run of
    whole solves, then one of the remainder continuing from the populations
    the first left) agrees with the host loop bitwise; qme_select_run
    rejects bad arguments."""
    wl = W.jc_single()
    rho0 = W.initial_rho(wl, P.basis(wl))
    res = {}
    for device in (False, True):
        sol = P.Solver(wl, "fp64")
        sol.set_fused(False)                  # the tiled step path as well
        sol.set_rho(rho0)
        print(f"selection ragged device={device}", flush=True)
        out, kept, sizes = P.evolve_with_selection(sol, 2050, 1e-20, 100, device=device)
        res[device] = (out.get_rho(), kept, sizes)
        if out is not sol:
            out.close()
        sol.close()
    (ra, ka, za), (rb, kb, zb) = res[False], res[True]
    assert za == zb and len(za) == 21 and np.array_equal(ka, kb)
    assert np.array_equal(ra[0], rb[0]) and ra[1] == rb[1]
    sol = P.Solver(wl, "fp32")
    sol.set_rho(rho0)
    lib = L.load()
    nbytes = L.c_size_t()
    L.check(lib.qme_select_workspace_size(sol.ctx, L.ctypes.byref(nbytes)))
    area = torch.empty(nbytes.value, dtype=torch.uint8, device=sol.state.device)
    keep = np.zeros(sol.n, dtype=np.int32)
    done, nk = L.c_int64(0), L.c_int64(0)
    args = lambda solves, k, eps: (sol.ctx, L.c_void_p(sol.state.data_ptr()),  # noqa: E731
                                   L.c_void_p(sol.workspace.data_ptr()), L.c_void_p(area.data_ptr()),
                                   solves, k, eps, 1, L.ctypes.byref(done), L.ctypes.byref(nk),
                                   keep.ctypes.data_as(L.POINTER(L.c_int32)), None)
    assert lib.qme_select_run(*args(-1, 1, 0.0)) == L.QME_E_ARG
    assert lib.qme_select_run(*args(1, 0, 0.0)) == L.QME_E_ARG
    assert lib.qme_select_run(*args(1, 1, -1.0)) == L.QME_E_ARG
    assert lib.qme_select_run(*args(1, 1, float("nan"))) == L.QME_E_ARG
    assert lib.qme_select_run(*args(0, 1, 0.0)) == L.QME_OK and done.value == 0
    # eps = 0 keeps everything: 5 solves, state as 5 plain steps
    assert lib.qme_select_run(*args(5, 2, 0.0)) == L.QME_OK
    assert done.value == 5 and nk.value == sol.n
    ref = P.Solver(wl, "fp32")
    ref.set_rho(rho0)
    ref.step(10)
    assert np.array_equal(sol.get_rho()[0], ref.get_rho()[0])
    ref.close()
    sol.close()
