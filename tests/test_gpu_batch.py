"""Batched steps of uneven instances (one launch per phase over every
instance's tiles, replayed from a captured hipGraph): every instance must
equal its own unfolded qme_step run bitwise (same tile arithmetic), with and without
the graph and for both instance orders; graph replays interleaved with eager
work; oracle parity; argument errors."""
import numpy as np
import pytest

import workloads as W
from oracle import evolve as ev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2403_07042_amd")
from paper_2403_07042_amd import _lib as L  # noqa: E402


def mixed_instances():
    sweep = W.batch_sweep(per_size=2, sizes=(64, 128, 256))
    extra = W.photon_lattice(6, 5, mu=0.2, g=0.15, gamma=0.05, dt=0.1, start=(0, 2))  # N = 60, padded
    tch = W.tch_2x2(steps=30)                                                            # N = 144, padded
    return sweep + [extra, tch]


def make_solvers(wls):
    sols = []
    for wl in wls:
        s = P.Solver(wl, "fp32")
        s.set_rho(W.initial_rho(wl, P.basis(wl)))
        sols.append(s)
    return sols


def solo_rho(wl, steps, tiles=None):
    """The instance alone under qme_step, as the batch runs it: unfolded,
    unsplit, with the tiles of its context in the batch (default: the
    context's default tiles)."""
    s = P.Solver(wl, "fp32")
    s.set_fold(False)            # the batched step does not fold its decoherence pass
    s.set_split(False)           # nor split its products along k
    if tiles:
        s.set_tiles(*tiles)
    s.set_rho(W.initial_rho(wl, P.basis(wl)))
    s.step(steps)
    rho, sink = s.get_rho()
    s.close()
    return rho, sink


@pytest.mark.parametrize("graph,largest", [(False, True), (False, False), (True, True)])
def test_batch_equals_solo_bitwise(graph, largest):
    wls = mixed_instances()
    sols = make_solvers(wls)
    b = P.Batch(sols)
    b.config(use_graph=graph, largest_first=largest)
    print(f"batch of {len(wls)} instances, graph={graph} largest_first={largest}", flush=True)
    b.step(30)
    torch.cuda.synchronize()
    for wl, s in zip(wls, sols):
        rho, sink = s.get_rho()
        ref, ref_sink = solo_rho(wl, 30)
        assert np.array_equal(rho, ref), wl["name"]
        assert sink == ref_sink
    b.close()
    for s in sols:
        s.close()


def test_batch_per_instance_tiles_bitwise():
    """Instances whose contexts take different tile edges (32 or 64 for each
    product) in one batch: each equals its solo run with the same tiles
    bitwise; then the tiles of every context change and a reconfigured batch
    follows them."""
    wls = mixed_instances()
    sols = make_solvers(wls)
    choices = [(32, 32), (64, 64), (32, 64), (64, 32)]
    assign = [choices[i % 4] for i in range(len(sols))]
    for s, t in zip(sols, assign):
        s.set_tiles(*t)
    b = P.Batch(sols)
    b.config(use_graph=True, largest_first=True)
    print(f"batch of {len(wls)} instances, mixed tiles", flush=True)
    b.step(12)
    torch.cuda.synchronize()
    for wl, s, t in zip(wls, sols, assign):
        rho, sink = s.get_rho()
        ref, ref_sink = solo_rho(wl, 12, t)
        assert np.array_equal(rho, ref), (wl["name"], t)
        assert sink == ref_sink
    # swap the tiles of every context; the tables follow after config()
    assign = [choices[(i + 1) % 4] for i in range(len(sols))]
    for wl, s, t in zip(wls, sols, assign):
        s.set_tiles(*t)
        s.set_rho(W.initial_rho(wl, P.basis(wl)))
    b.config(use_graph=False, largest_first=True)
    b.step(12)
    torch.cuda.synchronize()
    for wl, s, t in zip(wls, sols, assign):
        rho, _ = s.get_rho()
        ref, _ = solo_rho(wl, 12, t)
        assert np.array_equal(rho, ref), (wl["name"], t)
    s128 = sols[0]
    s128.set_tiles(*((128, 128) if s128.ld % 128 == 0 else (64, 64)))
    if s128.tiles == (128, 128):
        with pytest.raises(L.QmeError) as e:
            b.config()
        assert e.value.status == L.QME_E_UNSUPPORTED
    b.close()
    for s in sols:
        s.close()


def test_graph_replays_with_eager_work_between():
    wls = mixed_instances()
    sols = make_solvers(wls)
    b = P.Batch(sols)
    b.config(use_graph=True)
    other = P.Solver(W.jc_single(), "fp32")
    other.set_rho(W.initial_rho(W.jc_single(), P.basis(W.jc_single())))
    for rep in range(3):
        b.step(10)
        other.step(5)                       # eager work on the same stream
        torch.cuda.synchronize()
        for wl, s in zip(wls, sols):
            rho, _ = s.get_rho()
            ref, _ = solo_rho(wl, 10 * (rep + 1))
            assert np.array_equal(rho, ref), (rep, wl["name"])
    b.close()
    other.close()
    for s in sols:
        s.close()


def test_batch_against_oracle():
    """One instance of every size of the sweep (N = 64, 128, 256, 512) in one
    batch, 200 steps, against the oracle element by element."""
    wls = [W.batch_sweep(per_size=1, sizes=(n,))[0] for n in (64, 128, 256, 512)]
    sols = make_solvers(wls)
    b = P.Batch(sols)
    b.step(200)
    torch.cuda.synchronize()
    for wl, s in zip(wls, sols):
        sysm = ev.System(wl)
        ref, ref_sink = ev.evolve(sysm, W.initial_rho(wl, sysm.occ), 200)
        rho, sink = s.get_rho()
        assert np.abs(rho - ref).max() < 1e-5, wl["name"]
        assert abs(sink - ref_sink) < 1e-6
    b.close()
    for s in sols:
        s.close()


def test_batch_argument_errors():
    wl = W.tch_2x2()
    s64 = P.Solver(wl, "fp64")
    s64.set_rho(W.initial_rho(wl, P.basis(wl)))
    with pytest.raises(L.QmeError) as e:
        P.Batch([s64])
    assert e.value.status == L.QME_E_UNSUPPORTED
    s32 = P.Solver(wl, "fp32")
    b = P.Batch([s32])
    import ctypes
    st = L.load().qme_batch_step(b.handle, 1, ctypes.c_void_p(b.workspace.data_ptr()), 16,
                                 ctypes.c_void_p(0))
    assert st == L.QME_E_SIZE
    assert L.load().qme_batch_step(b.handle, -1, ctypes.c_void_p(b.workspace.data_ptr()),
                                   b.workspace_bytes, ctypes.c_void_p(0)) == L.QME_E_ARG
    b.close()
    s32.close()
    s64.close()


def test_full_sweep_256_instances():
    """The batched sweep workload at full size: 256 instances (64 each of
    N = 64, 128, 256, 512), 500 steps in one launch; 16 instances of every
    size equal their solo runs bitwise, and one instance of every size
    matches the oracle element by element after the 500 steps."""
    wls = W.batch_sweep()
    sols = make_solvers(wls)
    b = P.Batch(sols)
    print("full sweep: 256 instances x 500 steps", flush=True)
    b.step(500)
    torch.cuda.synchronize()
    picks = {}
    for i, wl in enumerate(wls):
        picks.setdefault(wl["expected_n"], []).append(i)
    for n, idx in sorted(picks.items()):
        print(f"full sweep: 16 solo runs of N = {n}", flush=True)
        for i in idx[:16]:
            rho, sink = sols[i].get_rho()
            ref, ref_sink = solo_rho(wls[i], 500)
            assert np.array_equal(rho, ref), (n, i)
            assert sink == ref_sink
    for n, idx in sorted(picks.items()):
        i = idx[0]
        print(f"full sweep: oracle, N = {n}, 500 steps", flush=True)
        sysm = ev.System(wls[i])
        ref, ref_sink = ev.evolve(sysm, W.initial_rho(wls[i], sysm.occ), 500)
        rho, sink = sols[i].get_rho()
        assert np.abs(rho - ref).max() < 1e-5, n
        assert abs(sink - ref_sink) < 1e-6, n
    b.close()
    for s in sols:
        s.close()


PERSISTENT_OFF = ("the persistent batched launch is switched off: its launches did not "
                  "finish on the device (a first run and the run of the fix, which moved the "
                  "per-poll acquire out of the wait loop), and the cause is not established")


@pytest.mark.skip(reason=PERSISTENT_OFF)
@pytest.mark.parametrize("graph", [False, True])
def test_persistent_batch_equals_phase_launches_bitwise(graph):
    """qme_batch_persistent: one launch per run (work taken in order from a
    counter, per-instance waits) equals the phase launches bitwise -- the same
    tile arithmetic -- over two runs in a row, and each instance its solo run."""
    wls = mixed_instances()
    out = {}
    for persistent in (False, True):
        sols = make_solvers(wls)
        b = P.Batch(sols)
        b.config(use_graph=graph, largest_first=True)
        b.persistent(persistent)
        print(f"batch of {len(wls)}, persistent={persistent}, graph={graph}: 7 + 5 steps", flush=True)
        b.step(7)
        b.step(5)
        torch.cuda.synchronize()
        out[persistent] = [s.get_rho() for s in sols]
        b.close()
        for s in sols:
            s.close()
    for wl, (ra, sa), (rb, sb) in zip(wls, out[False], out[True]):
        assert np.isfinite(sb)                        # no wait gave up
        assert np.array_equal(ra, rb) and sa == sb, wl["name"]
    ref, ref_sink = solo_rho(wls[0], 12)
    assert np.array_equal(out[True][0][0], ref)


@pytest.mark.skip(reason=PERSISTENT_OFF)
def test_persistent_full_sweep():
    """The 256-instance sweep in one persistent launch of 100 steps: 8
    instances of every size bitwise against solo runs, one of every size
    against the oracle."""
    wls = W.batch_sweep()
    sols = make_solvers(wls)
    b = P.Batch(sols)
    b.config(use_graph=True, largest_first=True)
    b.persistent(True)
    print("persistent sweep: 256 instances x 100 steps", flush=True)
    b.step(100)
    torch.cuda.synchronize()
    picks = {}
    for i, wl in enumerate(wls):
        picks.setdefault(wl["expected_n"], []).append(i)
    for n, idx in sorted(picks.items()):
        for i in idx[:8]:
            rho, sink = sols[i].get_rho()
            ref, ref_sink = solo_rho(wls[i], 100)
            assert np.array_equal(rho, ref), (n, i)
        i = idx[0]
        sysm = ev.System(wls[i])
        ref, ref_sink = ev.evolve(sysm, W.initial_rho(wls[i], sysm.occ), 100)
        rho, sink = sols[i].get_rho()
        assert np.abs(rho - ref).max() < 1e-5 and abs(sink - ref_sink) < 1e-6
    b.close()
    for s in sols:
        s.close()


def test_persistent_batch_is_switched_off():
    """Asking for the persistent launch is refused (QME_E_UNSUPPORTED); the
    phase launches stay in use (no kernel of the persistent form runs)."""
    wls = mixed_instances()[:2]
    sols = make_solvers(wls)
    b = P.Batch(sols)
    with pytest.raises(L.QmeError) as e:
        b.persistent(True)
    assert e.value.status == L.QME_E_UNSUPPORTED
    b.persistent(False)
    b.step(3)
    torch.cuda.synchronize()
    for wl, s in zip(wls, sols):
        ref, _ = solo_rho(wl, 3)
        assert np.array_equal(s.get_rho()[0], ref)
    b.close()
    for s in sols:
        s.close()
