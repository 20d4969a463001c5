"""Graph replay of qme_step (qme_set_graph): every replay is bitwise the eager
run's step, with eager work and synchronisation between replays, and a knob
change drops the captures (the next replay follows the new knob)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2403_07042_amd")


@pytest.mark.parametrize("make,precision", [
    (W.tch_2x2, "fp32"),                                          # N = 144, split products
    (W.tch_2x2, "fp64"),
    (lambda: W.photon_lattice(16, 16, gamma=0.05), "fp32"),       # N = 512, folded steps
    (lambda: W.photon_lattice(4, 4), "fp64"),                     # N = 32, single workgroup
])
def test_graph_replays_match_eager(make, precision):
    wl = dict(make(), init={"kind": "haar", "seed": 5})
    rho0 = W.initial_rho(wl, P.basis(wl))
    sol = P.Solver(wl, precision)

    def run():
        sol.set_split(True)
        sol.set_rho(rho0)
        out = []
        for _ in range(3):
            sol.step(10)
            out.append(sol.get_rho())
            sol.observe()                        # eager work and a sync between replays
        sol.set_split(False)                     # drops the captures
        for _ in range(2):
            sol.step(10)
            out.append(sol.get_rho())
        return out

    print(f"N={sol.n} {precision} eager", flush=True)
    ref = run()
    sol.set_graph(True)
    print(f"N={sol.n} {precision} graph", flush=True)
    got = run()
    sol.set_graph(False)
    sol.close()
    for (a, sa), (b, sb) in zip(got, ref):
        assert np.array_equal(a, b) and sa == sb
    assert np.abs(ref[-1][0] - rho0).max() > 1e-6


def test_graph_knob_validation():
    sol = P.Solver(W.photon_lattice(4, 4), "fp32")
    assert sol.lib.qme_set_graph(sol.ctx, 2) != 0          # QME_E_ARG
    sol.close()
