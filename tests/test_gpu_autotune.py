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


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_tile_choice_is_bitwise_neutral_and_tuner_picks_valid(precision, tmp_path):
    wl = W.photon_lattice(16, 16)          # N = 512
    occ = P.basis(wl)
    rho0 = W.initial_rho(wl, occ)
    sol = P.Solver(wl, precision)
    sol.set_fold(False)          # folding depends on the lower tile; compare tiles alone
    sol.set_split(False)         # so do the k-splits of small launches
    outs = []
    # one matrix-core shape: FP32 64/128-tiles (32x32 MFMA), FP64 32/64 (16x16)
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


def test_batch_tuner():
    wls = W.batch_sweep(per_size=4, sizes=(64, 256))
    sols = []
    for wl in wls:
        s = P.Solver(wl, "fp32")
        s.set_rho(W.initial_rho(wl, P.basis(wl)))
        sols.append(s)
    b = P.Batch(sols)
    best, results = A.tune_batch(b, steps=2, trials=2)
    assert best in results and len(results) == 3
    b.close()
    for s in sols:
        s.close()
