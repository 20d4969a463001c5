"""qme_step_noalloc (the step with the library's fixed device scratch as its
workspace, for callers that cannot allocate) against qme_step on the same
context and input: bitwise-equal states and sinks, over two calls in a row
with the second on a smaller system (the scratch keeps the first call's
contents), in every precision; and the size limit."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2403_07042_amd")
from paper_2403_07042_amd import _lib as L  # noqa: E402


def run_both(wl, precision, steps):
    occ = P.basis(wl)
    rho0 = W.initial_rho(wl, occ)
    sol = P.Solver(wl, precision)
    sol.set_rho(rho0)
    print(f"{wl['name']} {precision}: qme_step x {steps}", flush=True)
    sol.step(steps)
    ref = sol.get_rho()
    sol.set_rho(rho0)
    print(f"{wl['name']} {precision}: qme_step_noalloc x {steps}", flush=True)
    sol.step_noalloc(steps)
    got = sol.get_rho()
    sol.close()
    return ref, got


def haar(wl, seed):
    return dict(wl, init={"kind": "haar", "seed": seed})


@pytest.mark.parametrize("precision,first,second", [
    # N = 512 folded lattice (k-split products), then the N = 144 TCH model
    ("fp32", lambda: haar(W.photon_lattice(16, 16, gamma=0.05), 31), lambda: W.tch_2x2()),
    # N = 2048 lattice (the largest workspace here), then N = 144
    ("bf16x3", lambda: haar(W.photon_lattice(32, 32, gamma=0.05), 32), lambda: W.tch_2x2()),
    # N = 1152 FP64, then the N = 144 model with gather channels (decoherence pass)
    ("fp64", lambda: haar(W.photon_lattice(24, 24, gamma=0.05), 33), lambda: W.tch_2x2()),
])
def test_noalloc_step_matches_step(precision, first, second):
    for wl, steps in ((first(), 6), (second(), 9)):
        (a, sa), (b, sb) = run_both(wl, precision, steps)
        assert np.array_equal(a, b), wl["name"]
        assert sa == sb


def test_noalloc_rejects_too_large_workspace():
    """FP64 at N = 2048 needs a 128 MiB step workspace, above the scratch."""
    wl = W.photon_lattice()
    sol = P.Solver(wl, "fp64")
    assert sol.workspace_bytes > (80 << 20)
    sol.set_rho(W.initial_rho(wl, P.basis(wl)))
    with pytest.raises(L.QmeError) as e:
        sol.step_noalloc(1)
    assert e.value.status == L.QME_E_SIZE
    sol.close()
