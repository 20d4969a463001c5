"""The paper's own 2D photon-motion workload at full size (Sec. IV.B): an
81 x 51 plane of cavities, one photon, N = 4131 (not a multiple of the tile:
ld = 4160, ragged last tile row, tail-split lower product).  Closed system,
so the sine-mode closed form gives the exact state; the symmetric start
(40, 0) keeps P(i, j) = P(80 - i, j) at all times, the asymmetric start
(20, 0) does not."""
import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as cf

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2403_07042_amd")


def plane_populations(pops, occ):
    """P(i, j) on the 81 x 51 plane from the basis populations."""
    grid = np.zeros(81 * 51)
    site = np.argmax(occ, axis=1)              # the one occupied photon mode
    grid[site] = pops
    return grid.reshape(81, 51)


@pytest.mark.parametrize("precision,checkpoints,tol",
                         [("fp32", (1, 400, 1000), 1e-5), ("fp64", (1, 100), 1e-11)])
@pytest.mark.parametrize("start", [(40, 0), (20, 0)])
def test_photon_plane_4131_against_closed_form(start, precision, checkpoints, tol):
    wl = W.photon_plane(start=start)
    occ = P.basis(wl)
    assert occ.shape[0] == 4131
    sol = P.Solver(wl, precision)
    assert sol.ld == (4160 if precision == "fp32" else 4160)
    sol.set_rho(W.initial_rho(wl, occ))
    done = 0
    for k in checkpoints:
        print(f"plane {start} {precision}: step {k}", flush=True)
        sol.step(k - done)
        done = k
        rho, sink = sol.get_rho()
        ref = cf.lattice_rho(occ, 0, 81, 51, wl["hops"][0][2], 0.0, wl["omega_c"][0],
                             k * wl["dt"], wl["centre_site"])
        assert np.abs(rho - ref).max() < tol, k
        assert sink == 0.0
        grid = plane_populations(np.real(np.diag(rho)), occ)
        mirror = np.abs(grid - grid[::-1, :]).max()
        if start == (40, 0):
            assert mirror < 10 * tol
        elif k >= 100:
            assert mirror > 1e-3                # the asymmetric start really is asymmetric
    sol.close()
