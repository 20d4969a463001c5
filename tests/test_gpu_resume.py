"""Checkpoint / resume: a run interrupted after k steps, its state read to
the host (qme_get_state: rho and sink, a complete checkpoint) and written
into a fresh context (qme_set_state), continues bitwise as the same run on
one context with a call boundary at step k, in every precision and on every
step path (folded steps, the four-kernel step with gather channels, the
single-workgroup path for N <= 32, small-launch splits).  A call boundary
changes rounding only for folded steps: inside a call each step's
renormalisation factor is applied by the next product in FP64, at the end of
a call one pass rounds it into the stored state; the unfolded paths are
bitwise independent of how a run is split into calls."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2403_07042_amd")

CASES = {
    "lattice_16x16_folded": lambda: W.photon_lattice(16, 16, gamma=0.05),
    "tch_2x2_gather": W.tch_2x2,
    "jc_single_small_path": W.jc_single,
}


@pytest.mark.parametrize("precision", ["fp32", "fp64", "bf16x3"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_resume_from_host_checkpoint_is_bitwise(case, precision):
    wl = CASES[case]()
    occ = P.basis(wl)
    rho0 = W.initial_rho(wl, occ)
    total, cut = 100, 37
    print(f"resume {case} {precision}: {cut} + {total - cut} steps", flush=True)
    tol = {"fp32": 1e-5, "fp64": 1e-12, "bf16x3": 1e-4}[precision]
    a = P.Solver(wl, precision)
    a.set_rho(rho0)
    a.step(total)
    one_call, one_sink = a.get_rho()
    a.set_rho(rho0)
    a.step(cut)
    a.step(total - cut)
    ref, ref_sink = a.get_rho()
    a.close()
    assert np.abs(ref - one_call).max() < tol and abs(ref_sink - one_sink) < tol
    b = P.Solver(wl, precision)
    b.set_rho(rho0)
    b.step(cut)
    chk, chk_sink = b.get_rho()
    b.close()                                   # the interrupted run ends here
    c = P.Solver(wl, precision)
    c.set_rho(chk, chk_sink)
    c.step(total - cut)
    got, got_sink = c.get_rho()
    c.close()
    assert np.array_equal(got, ref)
    assert got_sink == ref_sink
    assert np.abs(ref - rho0).max() > 1e-6


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_split_calls_equal_one_call(precision):
    """Unfolded steps: step(1); step(20); step(29) on one context equals
    step(50) bitwise."""
    wl = W.photon_lattice(16, 16, gamma=0.05)
    rho0 = W.initial_rho(wl, P.basis(wl))
    sol = P.Solver(wl, precision)
    sol.set_fold(False)
    sol.set_rho(rho0)
    sol.step(50)
    ref = sol.get_rho()
    sol.set_rho(rho0)
    for k in (1, 20, 29):
        sol.step(k)
    got = sol.get_rho()
    sol.close()
    assert np.array_equal(got[0], ref[0]) and got[1] == ref[1]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_injected_fault_then_resume(monkeypatch, precision):
    """QME_FAULT_AT_STEP=40: the 100-step call stops after step 40 with
    QME_E_DEVICE; the state left behind is the checkpoint, and a fresh
    context resumed from it matches an uninterrupted run with a call
    boundary at step 40, bitwise."""
    from paper_2403_07042_amd import _lib as L
    wl = W.tch_2x2()
    rho0 = W.initial_rho(wl, P.basis(wl))
    monkeypatch.setenv("QME_FAULT_AT_STEP", "40")
    faulty = P.Solver(wl, precision)
    monkeypatch.delenv("QME_FAULT_AT_STEP")
    faulty.set_rho(rho0)
    faulty.step(25)                                  # below the fault step: runs
    with pytest.raises(L.QmeError) as e:
        faulty.step(75)
    assert "QME_E_DEVICE" in str(e.value) and "injected" in str(e.value)
    chk, chk_sink = faulty.get_rho()
    with pytest.raises(L.QmeError):
        faulty.step(1)                               # stays failed past the fault step
    faulty.close()
    ref = P.Solver(wl, precision)
    ref.set_rho(rho0)
    ref.step(25)
    ref.step(15)
    mid, mid_sink = ref.get_rho()
    ref.step(60)
    want, want_sink = ref.get_rho()
    ref.close()
    assert np.array_equal(chk, mid) and chk_sink == mid_sink
    res = P.Solver(wl, precision)
    res.set_rho(chk, chk_sink)
    res.step(60)
    got, got_sink = res.get_rho()
    res.close()
    assert np.array_equal(got, want) and got_sink == want_sink
