"""The autotuner on the device: it picks a valid tile pair and split setting,
caches them, and every tile pair gives bitwise-identical steps when no tail
split applies (tile size does not change the accumulation order)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2403_07042_amd")
from paper_2403_07042_amd import autotune as A  # noqa: E402


@pytest.mark.parametrize("precision", ["fp32", "fp64", "bf16x3"])
def test_tile_choice_is_bitwise_neutral_and_tuner_picks_valid(precision, tmp_path):
    wl = W.photon_lattice(16, 16)          # N = 512
    occ = P.basis(wl)
    rho0 = W.initial_rho(wl, occ)
    sol = P.Solver(wl, precision)
    sol.set_fold(False)          # folding depends on the lower tile; compare tiles alone
    sol.set_split(False)         # so do the k-splits of small launches
    outs = []
    # one matrix-core shape: FP32 64/128-tiles (32x32 MFMA), FP64 32/64
    # (16x16), BF16x3 64 x 64 and 128 x 64 first-product tiles
    same_shape = [t for t in A.candidates(precision, sol.ld)
                  if precision != "fp32" or 32 not in t]
    for tiles in same_shape:
        sol.set_tiles(*tiles)
        sol.set_rho(rho0)
        sol.step(20)
        outs.append(sol.get_rho()[0])
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    path = str(tmp_path / "tune.json")
    sol.set_rho(rho0)
    best = A.tune_solver(sol, steps=2, trials=2, path=path)
    assert best[:2] in A.candidates(precision, sol.ld) and best[2] in (True, False)
    rho, _ = sol.get_rho()
    assert np.array_equal(rho, rho0)      # tuning ran on a scratch state
    key = A.solver_key(A._arch(torch), precision, sol.n, sol.ld)
    entry = A.load_cache(path)[key]
    assert tuple(entry["tiles"]) == best[:2] and entry["split"] == best[2]
    assert A.tune_solver(sol, path=path) == best          # served from the cache
    sol.close()


def test_batch_tuner(tmp_path):
    """The batch tuner picks tile edges per instance size (all instances of
    one N share them), graph replay and order; the choice is cached and
    re-applied; the tuned batch still equals its solo runs bitwise."""
    wls = W.batch_sweep(per_size=4, sizes=(64, 256))
    sols = []
    for wl in wls:
        s = P.Solver(wl, "fp32")
        s.set_rho(W.initial_rho(wl, P.basis(wl)))
        sols.append(s)
    b = P.Batch(sols)
    path = str(tmp_path / "tune.json")
    best, results = A.tune_batch(b, steps=2, trials=2, use_cache=True, path=path)
    use_graph, largest, per_n = best
    assert set(per_n) == {64, 256} and all(t in A.BATCH_TILES for t in per_n.values())
    for s in sols:
        assert s.tiles == per_n[s.n]
    assert len([k for k in results if k[0] == "tiles"]) == 8
    again, _ = A.tune_batch(b, use_cache=True, path=path)       # from the cache
    assert again == best
    for wl, s in zip(wls, sols):
        s.set_rho(W.initial_rho(wl, P.basis(wl)))
    b.step(10)
    torch.cuda.synchronize()
    for wl, s in zip(wls, sols):
        solo = P.Solver(wl, "fp32")
        solo.set_fold(False)
        solo.set_split(False)
        solo.set_tiles(*per_n[s.n])
        solo.set_rho(W.initial_rho(wl, P.basis(wl)))
        solo.step(10)
        assert np.array_equal(s.get_rho()[0], solo.get_rho()[0]), wl["name"]
        solo.close()
    b.close()
    for s in sols:
        s.close()
