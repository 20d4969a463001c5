"""The FP32 products' two tile bodies (operands staged through registers, or
loaded from HBM straight into LDS) accumulate every output in the same order,
so steps and adjoint gradients must agree bitwise whichever body runs; the
automatic choice must agree with both."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2403_07042_amd")


@pytest.mark.parametrize("length,tiles,fold,split", [
    (16, (64, 64), True, True),      # N = 512: folded steps
    (16, (64, 64), False, True),     # N = 512: four-kernel steps
    (16, (128, 128), False, True),   # 128-tiles
    (24, (64, 64), True, True),      # N = 1152, ragged tile rows of the triangle
    (24, (64, 64), True, False),     # tail split off
    (32, (64, 64), True, True),      # N = 2048: the split tail of the lower product
])
def test_tile_bodies_bitwise_equal(length, tiles, fold, split):
    wl = dict(W.photon_lattice(length, length, gamma=0.05), init={"kind": "haar", "seed": 3})
    occ = P.basis(wl)
    rho0 = W.initial_rho(wl, occ)
    sol = P.Solver(wl, "fp32")
    sol.set_tiles(*tiles)
    sol.set_fold(fold)
    sol.set_split(split)
    out = {}
    for mode in (0, 1, -1):
        print(f"N={sol.n} tiles={tiles} fold={fold} split={split} direct={mode}", flush=True)
        sol.set_direct_loads(mode)
        sol.set_rho(rho0)
        sol.step(7)
        sol.step(5)
        out[mode] = sol.get_rho()
    sol.close()
    for mode in (1, -1):
        assert np.array_equal(out[mode][0], out[0][0])
        assert out[mode][1] == out[0][1]
    assert np.abs(out[0][0] - rho0).max() > 1e-6          # the state moved


@pytest.mark.parametrize("make,fold", [
    (lambda: W.photon_lattice(8, 8, gamma=0.05), True),    # N = 128: folded steps
    (lambda: W.photon_lattice(8, 8, gamma=0.05), False),
    (W.tch_2x2, False),                                    # N = 144, ld = 192, gather channels
    (lambda: W.photon_lattice(12, 8, gamma=0.05), True),   # N = 192
])
def test_whole_panel_body_bitwise_equal(make, fold):
    """FP32 32-tile products with ld <= 192 load every K tile of their row
    panels into LDS at once (direct modes 1 and -1) or stage them K tile by
    K tile (mode 0, split off): the same accumulation, bitwise."""
    wl = dict(make(), init={"kind": "haar", "seed": 5})
    occ = P.basis(wl)
    rho0 = W.initial_rho(wl, occ)
    sol = P.Solver(wl, "fp32")
    sol.set_tiles(32, 32)
    sol.set_fold(fold)
    sol.set_split(False)
    assert sol.ld <= 192
    out = {}
    for mode in (0, 1, -1):
        print(f"whole panels N={sol.n} fold={fold} direct={mode}", flush=True)
        sol.set_direct_loads(mode)
        sol.set_rho(rho0, sink=0.0625)
        sol.step(9)
        sol.step(4)
        out[mode] = sol.get_rho()
    sol.close()
    for mode in (1, -1):
        assert np.array_equal(out[mode][0], out[0][0])
        assert out[mode][1] == out[0][1]
    assert np.abs(out[0][0] - rho0).max() > 1e-6


def test_adjoint_bitwise_equal():
    wl = dict(W.photon_lattice(16, 16, gamma=0.05), init={"kind": "haar", "seed": 4})
    occ = P.basis(wl)
    sol = P.Solver(wl, "fp32")
    sol.set_rho(W.initial_rho(wl, occ))
    obs = np.zeros(sol.n)
    obs[sol.n // 2] = 1.0
    res = []
    for mode in (0, 1):
        print(f"adjoint direct={mode}", flush=True)
        sol.set_direct_loads(mode)
        res.append(sol.adjoint(12, obs, checkpoint_every=5))
    sol.close()
    (f0, g0), (f1, g1) = res
    assert f0 == f1 and np.array_equal(np.asarray(g0), np.asarray(g1))
    assert np.abs(g0).max() > 0


def test_direct_loads_mode_validation():
    sol = P.Solver(W.photon_lattice(4, 4), "fp32")
    with pytest.raises(Exception):
        sol.set_direct_loads(2)
    sol.set_direct_loads(-1)
    sol.close()
