"""Pins of the oracle's pure-state step for closed models (Sec. IV.B: the
photon plane without leakage) against facts that do not come from it: the
sine-mode closed form of the lattice, the Jaynes-Cummings Rabi formula, and
the density-matrix step of the same closed model (itself pinned elsewhere).
A time-reversed propagator (U^dag for U) keeps every population of a real
start but conjugates rho; the comparisons of whole density matrices below
catch it, as they catch a missing or wrong normalisation."""
import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as cf
from oracle import evolve as ev


@pytest.mark.parametrize("atoms_per_site,shape", [(0, (6, 5)), (1, (5, 4))])
def test_pure_lattice_matches_sine_mode_closed_form(atoms_per_site, shape):
    length, height = shape
    wl = W.photon_lattice(length, height, mu=0.3, g=0.2, gamma=0.0, dt=0.05,
                          atoms_per_site=atoms_per_site, start=(2, 1))
    s = ev.System(wl)
    psi0 = W.initial_psi(wl, s.occ)
    k = 150
    psi = ev.evolve_pure(s, psi0, k)
    ref = cf.lattice_rho(s.occ, atoms_per_site, length, height, 0.3, 0.2, 1.0,
                         k * wl["dt"], wl["centre_site"])
    assert np.abs(np.outer(psi, psi.conj()) - ref).max() < 1e-12
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-14


@pytest.mark.parametrize("n", [1, 2, 3])
def test_pure_rabi_closed_form(n):
    wl = W.jc_single(gamma=0.0)
    s = ev.System(wl)
    psi0 = np.zeros(s.n, complex)
    psi0[2 * n] = 1.0
    k = 10000
    psi = ev.evolve_pure(s, psi0, k)
    assert abs(abs(psi[2 * n]) ** 2 - cf.rabi(0.01, n, k * wl["dt"])) < 1e-11


def test_pure_equals_density_step_of_closed_model():
    wl = dict(W.tch_2x2(), jumps=[])
    s = ev.System(wl)
    psi0 = W.initial_psi(wl, s.occ)          # Haar-random complex start
    rho, sink = ev.evolve(s, np.outer(psi0, psi0.conj()), 200)
    psi = ev.evolve_pure(s, psi0, 200)
    assert sink == 0.0
    assert np.abs(np.outer(psi, psi.conj()) - rho).max() < 1e-13


def test_pure_step_renormalises():
    """A propagator scaled by 1.01 (not unitary) still yields unit vectors,
    equal to the unitary run: the normalisation divides the scale out."""
    wl = dict(W.tch_2x2(), jumps=[])
    s = ev.System(wl)
    psi0 = W.initial_psi(wl, s.occ)
    a, b = psi0.copy(), psi0.copy()
    for _ in range(50):
        a = ev.step_pure(a, 1.01 * s.u)
        b = ev.step_pure(b, s.u)
    assert abs(np.linalg.norm(a) - 1.0) < 1e-14
    assert np.abs(a - b).max() < 1e-13


def test_closed_model_detection():
    assert ev.is_closed(ev.System(dict(W.tch_2x2(), jumps=[])).jumps)
    assert not ev.is_closed(ev.System(W.tch_2x2()).jumps)
    lat = W.photon_lattice(4, 4, gamma=0.001)
    assert not ev.is_closed(ev.System(lat).jumps)           # leaks out of the basis only
    assert ev.is_closed(ev.System(W.photon_lattice(4, 4, gamma=0.0)).jumps)
    zero_rate = dict(W.tch_2x2(), jumps=[(0, 0, -1, 0.0)])
    assert ev.is_closed(ev.System(zero_rate).jumps)
    with pytest.raises(ValueError):
        ev.evolve_pure(ev.System(W.tch_2x2()), np.ones(144) / 12.0, 1)
