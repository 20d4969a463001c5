"""Parity of the full GPU time step (both MFMA products, decoherence,
symmetrisation, renormalisation, sink) with the CPU oracle on the same seeded
inputs, element by element, plus the invariants the method guarantees."""
import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as cf
from oracle import evolve as ev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2403_07042_amd")

# tolerance on max_ab |rho_gpu - rho_oracle| (complex modulus)
TOL = {"fp64": 1e-11, "fp32": 1e-5, "bf16x3": 1e-4}
TRACE_TOL = {"fp64": 1e-12, "fp32": 1e-6, "bf16x3": 1e-6}


def gpu_run(wl, precision, checkpoints):
    """Run the workload on the GPU; returns {k: (rho, sink, trace)}."""
    sol = P.Solver(wl, precision)
    occ = P.basis(wl)
    sol.set_rho(W.initial_rho(wl, occ))
    out, done = {}, 0
    for k in sorted(checkpoints):
        print(f"{wl.get('name', 'wl')} {precision} -> step {k}", flush=True)
        sol.step(k - done)
        done = k
        rho, sink = sol.get_rho()
        _, trace, sink2 = sol.observe()
        assert sink == sink2
        out[k] = (rho, sink, trace)
    sol.close()
    return out


def folded_trace_fused(sol, precision):
    """Whether folded steps form the trace inside the next first product:
    FP32 64- or 128-tile first products, FP32 32-tile ones that load whole
    panels (ld <= 192) and BF16x3 128 x 64 ones, not cut along k (a
    small-launch split applies below two tiles per compute unit; a BF16x3
    split takes the 64-tiles)."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    if precision == "bf16x3":
        return sol.tile1 == 128 and 2 * (sol.ld // 64) ** 2 > cus
    if precision != "fp32":
        return False
    if sol.tile1 == 32:
        return sol.ld <= 192         # whole-panel 32-tile products
    return 2 * (sol.ld // sol.tile1) ** 2 > cus


def oracle_run(wl, checkpoints):
    s = ev.System(wl)
    rho, sink = W.initial_rho(wl, s.occ), 0.0
    out, done = {}, 0
    for k in sorted(checkpoints):
        rho, sink = ev.evolve(s, rho, k - done, sink0=sink)
        done = k
        out[k] = (rho.copy(), sink)
    return out


def compare(wl, precision, checkpoints, tol=None, ref=None):
    ref = ref or oracle_run(wl, checkpoints)
    got = gpu_run(wl, precision, checkpoints)
    tol = tol or TOL[precision]
    for k in checkpoints:
        rho, sink, trace = got[k]
        rref, sref = ref[k]
        err = np.abs(rho - rref).max()
        assert err < tol, (k, err)
        assert np.array_equal(rho, rho.conj().T)          # exactly Hermitian
        assert np.all(np.imag(np.diag(rho)) == 0.0)
        assert abs(sink - sref) < TRACE_TOL[precision]
        assert abs(trace - (1.0 - sink)) < TRACE_TOL[precision]
    return got


def small_open_system(window=(0, -1)):
    return {
        "name": "small_open", "atoms": [1, 2], "photon_cap": [2, 1],
        "exc_min": window[0], "exc_max": window[1],
        "omega_c": [1.0, 1.1], "omega_a": [0.9, 1.0, 1.05], "g": [0.2, 0.15, 0.1],
        "hops": [(0, 1, 0.07)],
        "jumps": [(W.PHOTON_LEAK, 0, -1, 0.05), (W.PHOTON_LEAK, 1, -1, 0.02),
                  (W.ATOM_DECAY, 1, 1, 0.04), (W.ATOM_DEPHASE, 0, 0, 0.03),
                  (W.ATOM_DEPHASE, 1, 0, 0.01)],
        "dt": 0.05, "steps": 300, "init": {"kind": "haar", "seed": 11},
    }


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("window", [(0, -1), (1, 2)])
def test_small_open_system_all_jump_kinds(precision, window):
    compare(small_open_system(window), precision, [1, 7, 300])


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_jaynes_cummings_n8(precision):
    wl = W.jc_single()
    got = compare(wl, precision, [1, 1000, 10000])
    # closed form of the damped Jaynes-Cummings model at t = 100 (first-order
    # splitting error ~3e-6, see the oracle pins)
    rho = got[10000][0]
    p1, p2, _ = cf.damped_jc(0.01, 0.001, 100.0)
    assert abs(rho[2, 2].real - p1) < 5e-6 and abs(rho[1, 1].real - p2) < 5e-6


def n32_system():
    """Two cavities (photon caps 3 and 1, one atom each), full tensor product:
    N = 32, the largest size of the single-workgroup path; every jump kind."""
    return {
        "name": "n32", "atoms": [1, 1], "photon_cap": [3, 1], "exc_min": 0, "exc_max": -1,
        "omega_c": [1.0, 0.95], "omega_a": [1.0, 1.02], "g": [0.12, 0.08],
        "hops": [(0, 1, 0.05)],
        "jumps": [(W.PHOTON_LEAK, 0, -1, 0.03), (W.ATOM_DECAY, 1, 0, 0.02),
                  (W.ATOM_DEPHASE, 0, 0, 0.01)],
        "dt": 0.05, "steps": 1000, "init": {"kind": "haar", "seed": 13},
    }


def n33_system():
    """One cavity with photon cap 32, no atoms: N = 33, just past the
    single-workgroup path."""
    return {
        "name": "n33", "atoms": [0], "photon_cap": [32], "exc_min": 0, "exc_max": -1,
        "omega_c": [1.0], "omega_a": [], "g": [], "hops": [],
        "jumps": [(W.PHOTON_LEAK, 0, -1, 0.01)],
        "dt": 0.05, "steps": 100, "init": {"kind": "haar", "seed": 17},
    }


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_n32_all_jump_kinds_against_oracle(precision):
    compare(n32_system(), precision, [1, 10, 1000])


@pytest.mark.parametrize("make", [W.jc_single, n32_system, lambda: small_open_system((1, 2))])
@pytest.mark.parametrize("precision,steps,tol", [("fp64", 5000, 1e-12), ("fp32", 1000, 1e-5)])
def test_single_workgroup_path_matches_tiled(make, precision, steps, tol):
    """N <= 32: all steps in one single-workgroup launch (per 4096 steps)
    against the tiled four-launch step; 5000 FP64 steps span two launches."""
    wl = make()
    occ = P.basis(wl)
    rho0 = W.initial_rho(wl, occ)
    sol = P.Solver(wl, precision)
    out = {}
    for fused in (True, False):
        sol.set_fused(fused)
        sol.set_rho(rho0, sink=0.125)
        print(f"{wl['name']} {precision} fused={fused} {steps} steps", flush=True)
        sol.step(steps)
        rho, sink = sol.get_rho()
        pops, trace, _ = sol.observe()
        out[fused] = (rho, sink, trace)
    sol.close()
    (a, sa, ta), (b, sb, tb) = out[True], out[False]
    assert np.abs(a - b).max() < tol
    assert abs(sa - sb) < TRACE_TOL[precision] and abs(ta - tb) < TRACE_TOL[precision]
    assert np.array_equal(a, a.conj().T)          # exactly Hermitian on both paths
    assert sa >= 0.125                             # the sink is carried (grows where jumps leave the basis)


def test_single_workgroup_dispatch_rule():
    """N <= 32 in FP32 / FP64 takes the single launch (only index 0 of the
    per-kind launch counts moves); N = 33, BF16X3, and the knob off take the
    unfolded step, whose trace a system this small forms inside the
    decoherence pass (three launches, none of kind 2)."""
    def launches(wl, precision, fused=True):
        sol = P.Solver(wl, precision)
        sol.set_fused(fused)
        sol.set_rho(W.initial_rho(wl, P.basis(wl)))
        sol.profile(True)
        sol.step(3)
        torch.cuda.synchronize()
        counts = [c for _, c in sol.profile_read().values()]
        sol.close()
        return counts
    assert launches(n32_system(), "fp64") == [1, 0, 0, 0]
    assert launches(n32_system(), "fp32") == [1, 0, 0, 0]
    assert launches(n32_system(), "fp32", fused=False) == [3, 3, 0, 3]
    assert launches(n32_system(), "bf16x3") == [3, 3, 0, 3]
    assert launches(n33_system(), "fp64") == [3, 3, 0, 3]


def _scalars(sol):
    """The state's eight FP64 scalars (after the two planes)."""
    off = 2 * sol.ld * sol.ld * sol.elem
    return sol.state[off:off + 64].cpu().numpy().view(np.float64).copy()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("make", [W.tch_2x2, lambda: W.photon_lattice(12, 12)])
def test_fused_trace_scalars_across_calls(make, precision, graph):
    """A small unfolded system forms its trace in the decoherence pass and
    keeps the sink and step count in two alternating scalar pairs; whatever
    the split of steps over calls (odd and even counts) the state, the sink
    and the step count equal those of one call, bit for bit.  The sink
    starts at 1/8 (the lattice's boundary adds to it)."""
    wl = make()
    rho0 = W.initial_rho(wl, P.basis(wl))
    out = []
    for split in ([7], [1, 2, 4], [3, 3, 1], [2, 5]):
        sol = P.Solver(wl, precision)
        sol.set_fold(False)
        sol.set_graph(graph)
        sol.set_rho(rho0, sink=0.125)
        sol.profile(not graph)          # profiling runs eagerly
        for k in split:
            sol.step(k)                 # graph: [3, 3, 1] replays the 3-step capture
        torch.cuda.synchronize()
        counts = [c for _, c in sol.profile_read().values()]
        rho, sink = sol.get_rho()
        aux = _scalars(sol)
        sol.close()
        if not graph:
            assert counts == [7, 7, 0, 7]
        assert aux[3] == 7.0 and aux[0] == sink and sink >= 0.125
        out.append((rho, aux[:5]))
    for rho, aux in out[1:]:
        assert np.array_equal(rho, out[0][0])
        assert np.array_equal(aux, out[0][1])


@pytest.mark.parametrize("precision,tiles", [("fp32", (64, 64)), ("fp32", (128, 64)),
                                             ("fp32", (32, 64)), ("bf16x3", (64, 64)),
                                             ("bf16x3", (128, 64))])
def test_folded_trace_in_first_product_scalars(precision, tiles):
    """Folded steps at N = 2048: with FP32 64- or 128-tile first products
    and BF16x3 128 x 64 ones every block of the next first product forms the
    previous step's trace (one trace launch per call, the sink and step
    count alternating between the scalar pairs); FP32 32-tile and BF16x3
    64-tile first products keep the trace pass.  Over any
    split of 7 steps into calls the step count is 7, the sink agrees with one
    call's to rounding and the trace is 1 - sink."""
    folded_trace_scalars(dict(W.photon_lattice(gamma=0.05), init={"kind": "haar", "seed": 11}),
                         precision, tiles)


def test_whole_panel_folded_trace_scalars():
    """The same at N = 128 with FP32 32-tiles, whose first products load
    whole panels and form the previous step's trace while the loads are in
    flight."""
    folded_trace_scalars(dict(W.photon_lattice(8, 8, gamma=0.05), init={"kind": "haar", "seed": 11}),
                         "fp32", (32, 32))


def folded_trace_scalars(wl, precision, tiles):
    rho0 = W.initial_rho(wl, P.basis(wl))
    ref = None
    for split in ([7], [1, 2, 4], [3, 3, 1], [2, 5], [1, 1, 1, 1, 1, 1, 1]):
        sol = P.Solver(wl, precision)
        sol.set_tiles(*tiles)
        sol.set_rho(rho0, sink=0.125)
        sol.profile(True)
        print(f"folded trace {precision} tiles={tiles} split={split}", flush=True)
        for k in split:
            sol.step(k)
        torch.cuda.synchronize()
        counts = [c for _, c in sol.profile_read().values()]
        rho, sink = sol.get_rho()
        _, trace, _ = sol.observe()
        aux = _scalars(sol)
        fused = folded_trace_fused(sol, precision)
        sol.close()
        assert counts[0] == 7 and counts[1] == 7 and counts[3] == 0
        assert counts[2] == (len(split) if fused else 7)
        assert aux[3] == 7.0 and aux[0] == sink and sink > 0.125
        assert abs(trace - (1.0 - sink)) < 1e-6
        if ref is None:
            ref = (rho, sink)
        else:
            assert abs(sink - ref[1]) < 1e-9
            assert np.abs(rho - ref[0]).max() < 1e-6 * np.abs(ref[0]).max()


@pytest.mark.parametrize("make", [lambda: W.photon_lattice(32, 16, gamma=0.05),
                                  lambda: W.photon_lattice(gamma=0.05)])
@pytest.mark.parametrize("fold", [True, False])
def test_bf16x3_wide_first_product_bitwise(make, fold):
    """BF16x3 first products on 128 x 64 tiles (tile1 = 128) against the
    64 x 64 tiles: the same k order, products and epilogue per element, so
    the states and scalars after 3 + 4 steps are bitwise identical, folded
    (the renormalisation in the first product; on 128 x 64 tiles its trace
    formed there too) and unfolded, at
    N = 1024 and N = 2048 (leaking lattices, Haar start, sink 0.125).  The
    default takes 128 x 64 tiles where there are at least twice as many of
    them as compute units (N = 2048 on 256 compute units)."""
    wl = dict(make(), init={"kind": "haar", "seed": 5})
    rho0 = W.initial_rho(wl, P.basis(wl))
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = {}
    for tiles in ((64, 64), (128, 64)):
        sol = P.Solver(wl, "bf16x3")
        if tiles == (64, 64):
            wide = sol.ld % 128 == 0 and 2 * (sol.ld // 128) ** 2 >= 2 * cus
            assert sol.tiles == ((128, 64) if wide else (64, 64))
        sol.set_tiles(*tiles)
        sol.set_fold(fold)
        sol.set_rho(rho0, sink=0.125)
        print(f"bf16x3 wide N={sol.n} tiles={tiles} fold={fold}", flush=True)
        sol.step(3)
        sol.step(4)
        torch.cuda.synchronize()
        rho, sink = sol.get_rho()
        out[tiles] = (rho, sink, _scalars(sol))
        sol.close()
    a, b = out[(64, 64)], out[(128, 64)]
    assert np.array_equal(a[0], b[0])
    assert a[1] == b[1]
    # sink, population sums, lost rate, step count, factor (slots 5 and 6 are
    # scratch: the folded 128 x 64 steps alternate the sink there)
    assert np.array_equal(a[2][:5], b[2][:5])
    assert a[1] > 0.125 and np.array_equal(a[0], a[0].conj().T)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_tch_n144(precision):
    wl = W.tch_2x2()
    compare(wl, precision, [1, 1000, 5000])


def test_lattice_small_with_sink():
    wl = W.photon_lattice(6, 5, mu=0.2, g=0.15, gamma=0.05, dt=0.1, start=(0, 2))
    got = compare(wl, "fp32", [10, 200])
    assert got[200][1] > 1e-3        # population really left through the boundary
    compare(wl, "fp64", [10, 200])
    compare(wl, "bf16x3", [10, 200])  # folded BF16x3 steps with a real sink


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_lattice_2048_closed_form(precision):
    """Full-size 32 x 32 lattice (N = 2048), 1000 steps, against the
    sine-mode closed form; the boundary leak moves less than 1e-20 of
    probability by t = 10 for a photon started at the centre."""
    wl = W.photon_lattice()
    occ = P.basis(wl)
    got = gpu_run(wl, precision, [1, 1000])
    for k in (1, 1000):
        ref = cf.lattice_rho(occ, 1, 32, 32, 0.01, 0.01, 1.0, k * wl["dt"], wl["centre_site"])
        rho, sink, trace = got[k]
        assert np.abs(rho - ref).max() < TOL[precision]
        assert abs(trace - 1.0) < 1e-6 and sink < 1e-15


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_lattice_2048_long_run(precision):
    """The full-size lattice over 10^4 steps (t = 100, ten times the
    benchmark run) against the closed form, at the 1000-step tolerances:
    rounding does not accumulate past them (measured 6.5e-7 FP32, 7.0e-7
    BF16x3)."""
    wl = W.photon_lattice()
    occ = P.basis(wl)
    print(f"lattice 2048 {precision}: 10000 steps", flush=True)
    got = gpu_run(wl, precision, [10000])
    ref = cf.lattice_rho(occ, 1, 32, 32, 0.01, 0.01, 1.0, 10000 * wl["dt"], wl["centre_site"])
    rho, sink, trace = got[10000]
    assert np.abs(rho - ref).max() < TOL[precision]
    assert abs(trace - (1.0 - sink)) < TRACE_TOL[precision]


def test_lattice_2048_fp64_against_oracle_steps():
    wl = W.photon_lattice()
    compare(wl, "fp64", [1, 3])


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("bf16x3", 1e-5)])
def test_tail_split_of_the_lower_product(precision, tol):
    """N = 2048: the lower-triangle product has 528 tiles of 64 (2080 of 32
    in FP64), 16 (32) more than a multiple of the 256 compute units, so its
    tail tiles run in k-chunks summed by a reduce pass.  From a dense pure
    state, split and unsplit steps differ only by the regrouped k sums."""
    wl = dict(W.photon_lattice(), init={"kind": "haar", "seed": 7})
    occ = P.basis(wl)
    rho0 = W.initial_rho(wl, occ)
    sol = P.Solver(wl, precision)
    outs = {}
    for split in (False, True):
        sol.set_split(split)
        sol.set_rho(rho0)
        print(f"tail split {precision} split={split}", flush=True)
        sol.step(3)
        outs[split] = sol.get_rho()
    sol.close()
    (a, sa), (b, sb) = outs[False], outs[True]
    assert not np.array_equal(a, b)          # the split really ran
    assert np.abs(a - b).max() < tol * np.abs(a).max()
    assert abs(sa - sb) < 1e-12


@pytest.mark.parametrize("precision,tol,tiles", [("fp32", 1e-5, (64, 64)), ("bf16x3", 1e-5, (64, 64)),
                                                ("fp64", 1e-12, (64, 64))])
def test_tail_split_in_two_reduce_groups(precision, tol, tiles):
    """N = 2862 lattice (ld = 2880, 45 tile rows of 64, folded steps): the
    lower-triangle product has 1035 tiles, 11 past the last full wave of 256
    compute units, cut into 23 k-chunks each, so the reduce pass sums its
    chunks in two groups (16, then the rest) and applies the folded
    decoherence step and mirror.  Split and unsplit steps from a dense pure
    state differ only by the regrouped k sums."""
    wl = dict(W.photon_lattice(27, 53, gamma=0.05), init={"kind": "haar", "seed": 9})
    occ = P.basis(wl)
    rho0 = W.initial_rho(wl, occ)
    sol = P.Solver(wl, precision)
    sol.set_tiles(*tiles)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    t = sol.ld // 64
    tail = (t * (t + 1) // 2) % cus
    kt = 32 if precision == "bf16x3" else 16
    chunks = min(cus // tail, sol.ld // kt) if tail else 0
    if chunks <= 16:
        sol.close()
        pytest.skip(f"{cus} compute units: {chunks} chunks per tail tile, one reduce group")
    outs = {}
    for split in (False, True):
        sol.set_split(split)
        sol.set_rho(rho0)
        print(f"two-group tail split N={sol.n} {precision} chunks={chunks} split={split}", flush=True)
        sol.step(2)
        sol.step(1)
        rho, sink = sol.get_rho()
        _, trace, _ = sol.observe()
        outs[split] = (rho, sink, trace)
    sol.close()
    (a, sa, ta), (b, sb, tb) = outs[False], outs[True]
    assert not np.array_equal(a, b)          # the split really ran
    assert np.abs(a - b).max() < tol * np.abs(a).max()
    assert abs(sa - sb) < 1e-12
    assert np.array_equal(b, b.conj().T)     # the mirror written by the reduce pass
    assert abs(tb - (1.0 - sb)) < TRACE_TOL[precision]


@pytest.mark.parametrize("precision,tol,tiles", [("fp64", 1e-12, None), ("fp32", 1e-5, None),
                                                ("fp64", 1e-12, (64, 64)),
                                                ("bf16x3", 1e-5, None)])
def test_folded_steps_match_unfolded(precision, tol, tiles):
    """N = 2048 lattice (every decoherence operator leaves the basis, so the
    decoherence step is a factor per element): folded steps (decoherence in
    the lower product's epilogue, renormalisation in the next first product,
    one closing pass per call) against the four-kernel step, from a dense
    state, over several qme_step calls; exact Hermiticity and the trace."""
    wl = dict(W.photon_lattice(gamma=0.05), init={"kind": "haar", "seed": 9})
    occ = P.basis(wl)
    rho0 = W.initial_rho(wl, occ)
    sol = P.Solver(wl, precision)
    if tiles:
        sol.set_tiles(*tiles)
    out = {}
    for fold in (True, False):
        sol.set_fold(fold)
        sol.set_rho(rho0)
        print(f"fold={fold} {precision}", flush=True)
        sol.profile(True)
        sol.step(3)
        sol.step(20)
        sol.step(1)
        torch.cuda.synchronize()
        counts = [c for _, c in sol.profile_read().values()]
        sol.profile(False)
        rho, sink = sol.get_rho()
        pops, trace, _ = sol.observe()
        out[fold] = (rho, sink, trace, counts)
    # FP32 64-tile first products form the previous step's trace: one trace
    # launch per qme_step call
    fused_trace = folded_trace_fused(sol, precision)
    sol.close()
    (a, sa, ta, ca), (b, sb, tb, cb) = out[True], out[False]
    assert ca == [24, 24, 3 if fused_trace else 24, 0] and cb == [24, 24, 24, 24]
    assert np.abs(a - b).max() < tol * np.abs(b).max()
    assert abs(sa - sb) < TRACE_TOL[precision] and sa > 1e-6       # real sink
    assert abs(ta - (1.0 - sa)) < TRACE_TOL[precision]
    assert np.array_equal(a, a.conj().T)


def test_state_roundtrip_and_zero_steps():
    wl = W.tch_2x2()
    sol = P.Solver(wl, "fp64")
    rho0 = W.initial_rho(wl, P.basis(wl))
    sol.set_rho(rho0, sink=0.25)
    sol.step(0)
    rho, sink = sol.get_rho()
    assert np.array_equal(rho, rho0) and sink == 0.25
    sol.close()


def _golden(name):
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", f"{name}.json")
    return json.load(open(path))


def _golden_blocks(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", f"{name}.npz")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


_CHAIN3_LIVE = {}


def chain3_live_oracle():
    """The N = 1728 chain's oracle states after 1 and 10 steps, computed here
    (a few seconds of host BLAS), whole."""
    if not _CHAIN3_LIVE:
        wl = W.tch_chain3()
        print("oracle: N = 1728 chain, steps 1 and 10", flush=True)
        _CHAIN3_LIVE.update(oracle_run(wl, [1, 10]))
    return _CHAIN3_LIVE


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp64"])
def test_tch_chain3_n1728_against_oracle(precision):
    """Full-size TCH chain (3 cavities x 1 atom, cap 5, N = 1728; dephasing and
    leaks), 2000 steps, against the oracle: the whole state after 1 and 10
    steps (oracle computed live), whole 64 x 64 blocks of every tile class
    (diagonal, interior, the k-split tail of a 64-tile lower-triangle product,
    the far corner, upper-triangle mirrors) after 1000 and 2000 steps, and the
    diagonal plus a seeded sample of entries at steps 1, 10, 1000 and 2000
    (the last two stored by tests/golden/make_golden.py)."""
    gold = _golden("tch_chain3")
    blocks = _golden_blocks("tch_chain3_blocks")
    wl = W.tch_chain3()
    assert gold["n"] == 1728 and int(blocks["n"]) == 1728
    pairs = np.array(gold["pairs"])
    tol = TOL[precision]
    ks = sorted(int(k) for k in gold["records"])
    got = gpu_run(wl, precision, ks)
    live = chain3_live_oracle()
    for k, (rref, sref) in live.items():
        rho, sink, trace = got[k]
        err = np.abs(rho - rref).max()
        print(f"chain3 {precision} step {k}: whole state max|drho| = {err:.3e}", flush=True)
        assert err < tol, (k, err)
        assert abs(sink - sref) < TRACE_TOL[precision]
        assert np.array_equal(rho, rho.conj().T)
    bs = int(blocks["block"])
    for i, k in enumerate(blocks["steps"]):
        rho, sink, trace = got[int(k)]
        for b, (r, c) in enumerate(blocks["block_rc"]):
            sub = rho[r * bs:(r + 1) * bs, c * bs:(c + 1) * bs]
            err = np.abs(sub - blocks["blocks"][b, i]).max()
            assert err < tol, (int(k), (int(r), int(c)), err)
        assert abs(sink - blocks["sink"][i]) < TRACE_TOL[precision]
        assert abs(trace - blocks["trace"][i]) < TRACE_TOL[precision]
    for k in ks:
        rec = gold["records"][str(k)]
        rho, sink, trace = got[k]
        assert np.abs(np.real(np.diag(rho)) - np.array(rec["diag"])).max() < tol
        sample = rho[pairs[:, 0], pairs[:, 1]]
        ref = np.array(rec["sample_re"]) + 1j * np.array(rec["sample_im"])
        assert np.abs(sample - ref).max() < tol
        assert abs(sink - rec["sink"]) < TRACE_TOL[precision]
        assert abs(trace - rec["trace"]) < TRACE_TOL[precision]


_LATTICE_ORACLE = {}


def leaking_lattice(side):
    """side x side lattice, one atom per site, boundary leak 0.05 (strong
    enough that the sink is macroscopic), Haar-random start (the state is
    dense, so every tile of both products and every row / column factor of
    the folded epilogue carries weight)."""
    return dict(W.photon_lattice(side, side, gamma=0.05), init={"kind": "haar", "seed": 21})


@pytest.mark.parametrize("side,steps", [(16, 50), (32, 5)])
@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp64"])
def test_leaking_lattice_folded_against_oracle(side, steps, precision):
    """Multi-tile leaking lattices (N = 512 over 50 steps, N = 2048 over 5
    steps) on the default path, which folds the decoherence step into the
    lower-triangle product's epilogue (no decoherence pass runs), against the
    oracle element by element, with the sink."""
    wl = leaking_lattice(side)
    key = (side, steps)
    if key not in _LATTICE_ORACLE:
        print(f"oracle: {side} x {side} leaking lattice, {steps} steps", flush=True)
        _LATTICE_ORACLE[key] = oracle_run(wl, [steps])[steps]
    rref, sref = _LATTICE_ORACLE[key]
    sol = P.Solver(wl, precision)
    sol.set_rho(W.initial_rho(wl, P.basis(wl)))
    sol.profile(True)
    print(f"lattice {side}x{side} {precision}: {steps} steps", flush=True)
    sol.step(steps)
    torch.cuda.synchronize()
    counts = [c for _, c in sol.profile_read().values()]
    sol.profile(False)
    # FP32 64-tile first products form the previous step's trace themselves:
    # one trace launch per call
    fused_trace = folded_trace_fused(sol, precision)
    rho, sink = sol.get_rho()
    _, trace, _ = sol.observe()
    sol.close()
    # folded: no decoherence pass
    assert counts == [steps, steps, 1 if fused_trace else steps, 0]
    err = np.abs(rho - rref).max()
    print(f"lattice {side}x{side} {precision}: max|drho| = {err:.3e}, sink {sink:.6e}", flush=True)
    assert err < TOL[precision]
    assert sref > 1e-4                                  # a real sink
    assert abs(sink - sref) < (1e-12 if precision == "fp64" else 1e-6)
    assert abs(trace - (1.0 - sink)) < TRACE_TOL[precision]
    assert np.array_equal(rho, rho.conj().T)


def test_profile_sampling_stride():
    """qme_profile_enable(k): events on every k-th step only, counted from
    the enabling call across qme_step calls."""
    wl = W.photon_lattice(16, 16)
    sol = P.Solver(wl, "fp32")
    sol.set_rho(W.initial_rho(wl, P.basis(wl)))
    sol.profile(4)
    sol.step(5)
    sol.step(7)                     # steps 0, 4, 8 are sampled
    counts = [c for _, c in sol.profile_read().values()]
    assert counts[:3] == [3, 3, 3]
    sol.profile(1)
    sol.step(2)
    counts = [c for _, c in sol.profile_read().values()]
    assert counts[:3] == [2, 2, 2]
    with pytest.raises(Exception):
        sol.profile(-1)
    sol.profile(False)
    sol.close()


def small_split_expected(ld, tile, precision, cus):
    """Whether the small-launch split must cut a product of this tiling: at
    most half as many tiles as compute units, and at least two chunks of two
    K tiles (K tile: 32 for BF16x3 and FP32 32-tiles, else 16).  Returns
    (first product split, lower-triangle product split)."""
    if precision == "bf16x3":
        tile = 64                    # a split BF16x3 product runs on 64-tiles
    if precision == "fp32" and tile == 32 and ld <= 192:
        return False, False          # whole-panel products, never split
    t = ld // tile
    kt = 32 if precision == "bf16x3" or (precision == "fp32" and tile == 32) else 16

    def applies(blocks):
        return 2 * blocks <= cus and min(cus // blocks, (ld // kt) // 2) >= 2
    return applies(t * t), applies(t * (t + 1) // 2)


@pytest.mark.parametrize("make,precision,tol", [
    (W.tch_2x2, "fp32", 1e-5),                                   # N = 144: 9 + 6 tiles
    (W.tch_2x2, "fp64", 1e-12),
    (lambda: W.photon_lattice(16, 16, gamma=0.05), "fp32", 1e-5),   # N = 512, folded steps
    (lambda: W.photon_lattice(16, 16, gamma=0.05), "fp64", 1e-12),
    (W.tch_2x2, "bf16x3", 1e-5),
    (lambda: W.photon_lattice(16, 16, gamma=0.05), "bf16x3", 1e-5),
])
def test_small_launch_split(make, precision, tol):
    """Products too small to occupy the device are cut along k: the split
    step against the unsplit one and (N = 144) the oracle, over several
    qme_step calls, with 64- and 128-tiles (FP32), 32- and 64-tiles (FP64) or
    64-tiles and a 128 x 64 first product (BF16x3, whose split launch takes
    the 64-tiles).  Where the split rule applies to a tiling, the split
    result must differ from the unsplit one (the k sums are regrouped), so a
    split that silently did not run fails."""
    wl = dict(make(), init={"kind": "haar", "seed": 11})
    occ = P.basis(wl)
    rho0 = W.initial_rho(wl, occ)
    sol = P.Solver(wl, precision)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    tiles = {"fp32": [(64, 64), (128, 128), (32, 32)], "fp64": [(32, 32), (64, 64)],
             "bf16x3": [(64, 64), (128, 64)]}[precision]
    outs = {}
    ran = []
    for t in tiles:
        if sol.ld % t[0]:
            continue
        sol.set_tiles(*t)
        if any(small_split_expected(sol.ld, t[0], precision, cus)):
            ran.append(t)
        for split in (True, False):
            print(f"N={sol.n} {precision} tiles={t} split={split}", flush=True)
            sol.set_split(split)
            sol.set_rho(rho0)
            sol.step(7)
            sol.step(13)
            rho, sink = sol.get_rho()
            _, trace, _ = sol.observe()
            outs[(t, split)] = (rho, sink, trace)
    sol.close()
    assert ran                                   # every case has a tiling the split applies to
    for t in ran:
        assert not np.array_equal(outs[(t, True)][0], outs[(t, False)][0]), t
    ref_rho = outs[(tiles[0], False)][0]
    scale = np.abs(ref_rho).max()
    for key, (rho, sink, trace) in outs.items():
        assert np.abs(rho - ref_rho).max() < tol * scale, key
        assert abs(trace - (1.0 - sink)) < TRACE_TOL[precision], key
        assert np.array_equal(rho, rho.conj().T), key
    if sol.n == 144:
        s = ev.System(wl)
        ref, _ = ev.evolve(s, rho0, 20)
        for key, (rho, _, _) in outs.items():
            assert np.abs(rho - ref).max() < tol, key
