"""Pins of the oracle's state-space selection loop (Sec. III.B) against
facts it does not compute itself: the special case epsilon = 0 (plain
evolution), the excitation-number selection rule of the closed
Jaynes-Cummings model with its Rabi closed form, the damped closed form, the
perturbative reach of one step on the lattice (a breadth-first search over
the Hamiltonian's coupling graph), and the trace / Hermiticity / positivity
invariants after a deletion.  CPU only."""
import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as cf
from oracle import evolve as ev
from oracle import model as md
from oracle import selection as sel


def test_growth_speed_is_absolute_rate():
    g = sel.growth_speed([0.5, 0.2, 0.0], [0.4, 0.3, 0.0], 0.5)
    assert np.allclose(g, [0.2, 0.2, 0.0])


def test_eps_zero_equals_plain_evolution():
    wl = dict(W.tch_2x2(steps=20))
    s = ev.System(wl)
    rho0 = W.initial_rho(wl, s.occ)
    rho, sink = ev.evolve(s, rho0, 20)
    rho_s, sink_s, kept, sizes = sel.select_evolve(wl, rho0, 20, eps=0.0)
    assert np.array_equal(kept, np.arange(s.n)) and sizes == [s.n] * 20
    assert np.array_equal(rho_s, rho) and sink_s == sink


def test_closed_jc_keeps_one_excitation_manifold_and_follows_rabi():
    """Without decoherence H conserves the excitation number: from |1, g>
    every other manifold keeps probability ~0, so any epsilon between that
    round-off level and the manifold's own rate removes exactly them, and the
    kept pair then oscillates as cos^2(g t)."""
    wl = W.jc_single(gamma=0.0)
    occ = md.basis(wl["atoms"], wl["photon_cap"])
    rho0 = W.initial_rho(wl, occ)
    steps, g, dt = 2000, wl["g"][0], wl["dt"]
    rho, sink, kept, sizes = sel.select_evolve(wl, rho0, steps, eps=1e-20)
    one = np.nonzero(md.excitation_number(occ) == 1)[0]
    assert np.array_equal(kept, one) and sizes[0] == 2 and sizes[-1] == 2
    p1g = rho[list(kept).index(int(np.nonzero((occ[:, 0] == 1) & (occ[:, 1] == 0))[0][0])),
              list(kept).index(int(np.nonzero((occ[:, 0] == 1) & (occ[:, 1] == 0))[0][0]))].real
    assert abs(p1g - cf.rabi(g, 1, steps * dt)) < 1e-12
    assert sink == 0.0 and abs(np.trace(rho).real - 1.0) < 1e-14


def test_damped_jc_selection_matches_closed_form_and_full_run():
    """With the photon leak the vacuum |0, g> is fed at rate gamma p_{1,g},
    so the excitation <= 1 states stay and the two-excitation states go; the
    deleted states never held probability, so the reduced run equals the
    full one and the damped closed form (first-order splitting error)."""
    wl = W.jc_single()
    s = ev.System(wl)
    rho0 = W.initial_rho(wl, s.occ)
    steps = 10000
    rho, sink, kept, _ = sel.select_evolve(wl, rho0, steps, eps=1e-20, every=100)
    assert np.array_equal(kept, np.nonzero(md.excitation_number(s.occ) <= 1)[0])
    full, full_sink = ev.evolve(s, rho0, steps)
    assert np.abs(rho - full[np.ix_(kept, kept)]).max() < 1e-12
    assert abs(sink - full_sink) < 1e-14
    i1g = list(kept).index(int(np.nonzero((s.occ[:, 0] == 1) & (s.occ[:, 1] == 0))[0][0]))
    i0e = list(kept).index(int(np.nonzero((s.occ[:, 0] == 0) & (s.occ[:, 1] == 1))[0][0]))
    p1, p2, _ = cf.damped_jc(wl["g"][0], wl["jumps"][0][3], steps * wl["dt"])
    assert abs(rho[i1g, i1g].real - p1) < 5e-6 and abs(rho[i0e, i0e].real - p2) < 5e-6


def _graph_ball(h, start, radius):
    """States within `radius` applications of H from `start` (breadth-first
    search over the non-zero off-diagonal pattern of H)."""
    adj = (np.abs(h) > 0) & ~np.eye(h.shape[0], dtype=bool)
    seen = {int(start)}
    frontier = [int(start)]
    for _ in range(radius):
        nxt = []
        for u in frontier:
            for v in np.nonzero(adj[u])[0]:
                if int(v) not in seen:
                    seen.add(int(v))
                    nxt.append(int(v))
        frontier = nxt
    return np.array(sorted(seen))


def test_lattice_first_step_keeps_the_radius_two_ball():
    """One step of length dt moves amplitude (mu dt)^m / m! onto states m
    hops away (and g dt for the atom): on a 9 x 9 lattice with mu dt = g dt =
    1e-4 a state at distance m gets probability ~1e-8 m, i.e. growth speeds
    ~1e-6, 1e-14 and 1e-22 for m = 1, 2, 3, so epsilon = 1e-20 keeps exactly
    the radius-2 ball of the coupling graph around the start."""
    wl = W.photon_lattice(9, 9, gamma=0.0)
    s = ev.System(wl)
    rho0 = W.initial_rho(wl, s.occ)
    start = int(np.argmax(np.real(np.diag(rho0))))
    rho, sink, kept, sizes = sel.select_evolve(wl, rho0, 1, eps=1e-20)
    ball = _graph_ball(s.h, start, 2)
    assert np.array_equal(kept, ball)
    assert ball.size == 13 + 5              # photon at distance <= 2, atom at <= 1
    assert abs(np.trace(rho).real - 1.0) < 1e-14


def test_deletion_renormalises_and_keeps_invariants():
    """A large epsilon deletes states that hold probability: the reduced
    state is Hermitian, positive semidefinite and has trace 1 - sink."""
    wl = dict(W.tch_2x2(steps=50))
    s = ev.System(wl)
    rho0 = W.initial_rho(wl, s.occ)
    # about half of the Haar state's 144 states move slower than 1e-4 over
    # the first 5 steps, and they hold ~40 % of the probability
    rho, sink, kept, sizes = sel.select_evolve(wl, rho0, 50, eps=1e-4, every=5)
    assert sizes[0] < s.n and sizes[-1] >= 1
    assert all(a >= b for a, b in zip(sizes, sizes[1:]))
    assert np.abs(rho - rho.conj().T).max() < 1e-15
    assert abs(np.trace(rho).real - (1.0 - sink)) < 1e-13
    # P rho P of a positive matrix is positive; what remains is the explicit
    # Euler dissipator's known excursion, below k (dt sum_j gamma_j |A_j^dag A_j|)^2
    rates = sum(gm for *_, gm in wl["jumps"])
    bound = 50 * (wl["dt"] * rates * max(wl["photon_cap"])) ** 2
    assert np.linalg.eigvalsh(0.5 * (rho + rho.conj().T)).min() > -bound


def test_basis_size_shrinks_with_eps():
    """The trend of Table I: larger epsilon, smaller selected basis."""
    wl = W.photon_lattice(8, 8, gamma=0.0, steps=30)
    s = ev.System(wl)
    rho0 = W.initial_rho(wl, s.occ)
    final = []
    for eps in (0.0, 1e-30, 1e-20, 1e-10):
        _, _, kept, _ = sel.select_evolve(wl, rho0, 30, eps=eps, every=10)
        final.append(kept.size)
    assert final[0] == s.n
    assert all(a >= b for a, b in zip(final, final[1:])) and final[-1] < final[1]
