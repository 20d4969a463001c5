"""Pins of the CPU oracle against facts that do not come from the oracle:
values the paper prints, closed forms, textbook constructions (Kronecker
products, scipy's expm / expm_frechet), brute force on tiny inputs and exact
invariants.  Each test names what a plausible mistake would break."""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import closed_forms as cf
from oracle import evolve as ev
from oracle import gradients as gr
from oracle import model as md

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def small_wl(atoms, caps, exc=(0, -1), g=0.013, mus=(), jumps=(), dt=0.05,
             omega_c=None, omega_a=None):
    n_at = sum(atoms)
    return {
        "atoms": list(atoms), "photon_cap": list(caps),
        "exc_min": exc[0], "exc_max": exc[1],
        "omega_c": list(omega_c) if omega_c else [1.0] * len(atoms),
        "omega_a": list(omega_a) if omega_a else [1.0] * n_at,
        "g": [g * (1 + 0.1 * k) for k in range(n_at)],
        "hops": list(mus), "jumps": list(jumps), "dt": dt, "steps": 10,
        "init": {"kind": "haar", "seed": 7},
    }


# ---------------------------------------------------------------- basis


def test_basis_dimensions_printed_in_paper():
    gold = json.load(open(os.path.join(GOLD, "paper_dimensions.json")))
    # six / twelve two-level modes (Eqs. 6 and 9): cavities of cap 1, 1 atom
    assert md.basis([1] * 3, [1] * 3).shape[0] == gold["hb_one_bond"]["value"]
    assert md.basis([1] * 6, [1] * 6).shape[0] == gold["hb_two_bonds"]["value"]
    # single-photon window of the 81 x 51 plane (Eq. 11)
    length, height = gold["photon_plane_length"]["value"], gold["photon_plane_height"]["value"]
    occ = md.basis([0] * (length * height), [1] * (length * height), 1, 1)
    assert occ.shape[0] == gold["photon_plane_single_photon_dim"]["value"] == length * height


def test_basis_dimensions_of_workloads():
    assert md.basis([1], [3]).shape[0] == 8
    assert md.basis([2, 2], [2, 2]).shape[0] == 144
    assert md.basis([1, 1, 1], [5, 5, 5]).shape[0] == 1728
    assert md.basis([1] * 1024, [1] * 1024, 1, 1).shape[0] == 2048
    for n, atoms in W.BATCH_STRUCTURES.items():
        assert md.basis(atoms, [3] * len(atoms)).shape[0] == n


@pytest.mark.parametrize("atoms,caps,exc", [
    ([1], [3], (0, -1)), ([2, 1], [2, 1], (0, -1)), ([1, 0, 2], [1, 2, 1], (1, 3)),
    ([0, 0, 0, 0], [2, 1, 3, 1], (2, 2)), ([2, 2], [2, 2], (0, 2)), ([1, 1], [3, 3], (4, -1)),
])
def test_basis_matches_brute_force(atoms, caps, exc):
    levels = []
    for c, m in enumerate(atoms):
        levels.append(range(caps[c] + 1))
        levels.extend([range(2)] * m)
    lo, hi = exc
    want = [t for t in itertools.product(*levels)
            if sum(t) >= lo and (hi < 0 or sum(t) <= hi)]   # product order = lexicographic
    got = [tuple(r) for r in md.basis(atoms, caps, lo, hi)]
    assert got == want


def test_basis_full_product_is_kronecker_order():
    occ = md.basis([1, 2], [2, 1])
    dims = [3, 2, 2, 2, 2]
    strides = np.cumprod([1] + dims[::-1][:-1])[::-1]
    assert np.array_equal(occ @ strides, np.arange(occ.shape[0]))


# ------------------------------------------------------------ Hamiltonian


def _kron_ops(dims):
    """Truncated ladder matrices embedded in the tensor product."""
    def embed(op, k):
        out = np.eye(1)
        for i, d in enumerate(dims):
            out = np.kron(out, op if i == k else np.eye(d))
        return out
    return embed


def test_hamiltonian_matches_kronecker_construction():
    atoms, caps = [2, 1], [2, 3]
    wl = small_wl(atoms, caps, mus=[(0, 1, 0.021)], omega_c=[1.1, 0.9],
                  omega_a=[1.0, 1.2, 0.8])
    occ = md.basis(atoms, caps)
    dims, kinds = [], []
    for c, m in enumerate(atoms):
        dims.append(caps[c] + 1); kinds.append(("photon", c))
        for _ in range(m):
            dims.append(2); kinds.append(("atom", c))
    embed = _kron_ops(dims)
    h = np.zeros((occ.shape[0],) * 2)
    pmode = {c: i for i, (k, c) in enumerate(kinds) if k == "photon"}
    amodes = [i for i, (k, c) in enumerate(kinds) if k == "atom"]
    lower = {i: np.diag(np.sqrt(np.arange(1, d)), 1) for i, d in enumerate(dims)}
    for c, p in pmode.items():
        a = embed(lower[p], p)
        h += wl["omega_c"][c] * a.T @ a
    for k, m in enumerate(amodes):
        s = embed(lower[m], m)
        a = embed(lower[pmode[kinds[m][1]]], pmode[kinds[m][1]])
        h += wl["omega_a"][k] * s.T @ s + wl["g"][k] * (a.T @ s + a @ s.T)
    a0, a1 = embed(lower[pmode[0]], pmode[0]), embed(lower[pmode[1]], pmode[1])
    h += 0.021 * (a0.T @ a1 + a1.T @ a0)
    assert np.array_equal(md.hamiltonian(wl, occ), h) or np.abs(md.hamiltonian(wl, occ) - h).max() < 1e-15


def test_hamiltonian_window_is_restriction_of_full():
    atoms, caps = [1, 1, 1], [2, 2, 2]
    wl = small_wl(atoms, caps, mus=[(0, 1, 0.01), (1, 2, 0.02)])
    full = md.basis(atoms, caps)
    h_full = md.hamiltonian(wl, full)
    for lo, hi in [(1, 1), (2, 3), (0, 2)]:
        wl_w = dict(wl, exc_min=lo, exc_max=hi)
        occ = md.basis(atoms, caps, lo, hi)
        keep = [i for i, r in enumerate(full) if lo <= r.sum() <= hi]
        assert np.array_equal(md.hamiltonian(wl_w, occ), h_full[np.ix_(keep, keep)])


def test_hamiltonian_symmetric_and_conserves_excitations():
    wl = W.tch_2x2()
    occ = md.basis(wl["atoms"], wl["photon_cap"])
    h = md.hamiltonian(wl, occ)
    assert np.array_equal(h, h.T)
    nexc = np.diag(md.excitation_number(occ).astype(float))
    assert np.abs(h @ nexc - nexc @ h).max() == 0.0


def test_hamiltonian_elements_sqrt_n():
    wl = W.jc_single(g=0.3)
    occ = md.basis([1], [3])
    h = md.hamiltonian(wl, occ)
    # |n, g> (index 2n) <-> |n-1, e> (index 2n-1), element g sqrt(n)
    for n in (1, 2, 3):
        assert h[2 * n, 2 * n - 1] == pytest.approx(0.3 * np.sqrt(n), abs=1e-15)
        assert h[2 * n, 2 * n] == pytest.approx(n)
    hop = small_wl([0, 0], [3, 3], mus=[(0, 1, 0.5)])
    occ2 = md.basis([0, 0], [3, 3])
    h2 = md.hamiltonian(hop, occ2)
    # |2,1> -> |1,2>: mu sqrt(2) sqrt(2)
    i, j = 2 * 4 + 1, 1 * 4 + 2
    assert h2[j, i] == pytest.approx(0.5 * 2.0, abs=1e-15)


# ------------------------------------------------------------ propagator


def test_propagator_vs_scipy_expm_and_unitary():
    wl = W.tch_2x2()
    s = ev.System(wl)
    ref = sla.expm(-1j * s.h * s.dt)
    assert np.abs(s.u - ref).max() < 1e-13
    assert np.abs(s.u.conj().T @ s.u - np.eye(s.n)).max() < 1e-13
    assert np.abs(s.u - s.u.T).max() < 1e-13


# --------------------------------------------------------- closed forms


@pytest.mark.parametrize("n", [1, 2, 3])
def test_rabi_closed_form(n):
    wl = W.jc_single(gamma=0.0, steps=10000)
    s = ev.System(wl)
    rho0 = np.zeros((8, 8), complex)
    rho0[2 * n, 2 * n] = 1.0
    rho, _ = ev.evolve(s, rho0, 10000)
    t = 10000 * wl["dt"]
    assert abs(rho[2 * n, 2 * n].real - cf.rabi(0.01, n, t)) < 1e-11
    if n == 1:
        assert abs(rho[2, 2].real - np.cos(1.0) ** 2) < 1e-11


def test_damped_jc_closed_form():
    """Workload 1 against the damped Jaynes-Cummings solution.  The splitting
    (rotate, then an Euler dissipator step) is first order in dt: the error
    halves with dt, and the Richardson combination 2 P(dt/2) - P(dt) meets the
    closed form far more tightly than either run."""
    p_ref = np.array(cf.damped_jc(0.01, 0.001, 100.0))
    runs = {}
    for dt in (0.01, 0.005):
        wl = W.jc_single(dt=dt)
        s = ev.System(wl)
        rho, sink = ev.evolve(s, W.initial_rho(wl, s.occ), int(round(100.0 / dt)))
        runs[dt] = np.real(np.array([rho[2, 2], rho[1, 1], rho[0, 0]]))
        assert sink == 0.0 and abs(rho.trace().real - 1) < 1e-13
    err1 = runs[0.01] - p_ref
    err2 = runs[0.005] - p_ref
    assert np.abs(err1).max() < 5e-6
    assert np.all(np.abs(err1 / err2 - 2.0) < 0.01)
    assert np.abs(2 * runs[0.005] - runs[0.01] - p_ref).max() < 1e-9


def test_bare_cavity_leak_exact_decay():
    gamma, dt = 0.02, 0.05
    wl = small_wl([0], [6], jumps=[(W.PHOTON_LEAK, 0, -1, gamma)], dt=dt)
    s = ev.System(wl)
    rho0 = np.zeros((7, 7), complex)
    rho0[4, 4] = 0.5; rho0[2, 2] = 0.5; rho0[2, 4] = rho0[4, 2] = 0.5
    nvec = np.arange(7)
    rho = rho0
    for k in range(1, 201):
        rho, _ = ev.step(rho, 0.0, s.u, s.jumps, dt)
        if k % 50 == 0:
            mean = float(nvec @ np.real(np.diag(rho)))
            assert abs(mean - cf.bare_leak_mean(3.0, gamma, dt, k)) < 1e-13


def test_dephasing_exact_factor():
    gamma, dt = 0.03, 0.1
    wl = small_wl([1], [1], g=0.0, jumps=[(W.ATOM_DEPHASE, 0, 0, gamma)], dt=dt)
    wl["g"] = [0.0]
    s = ev.System(wl)
    rho0 = np.zeros((4, 4), complex)
    rho0[0, 0] = rho0[1, 1] = rho0[0, 1] = rho0[1, 0] = 0.5   # (|0,g> + |0,e>)/sqrt2
    rho = rho0
    for k in range(1, 101):
        rho, _ = ev.step(rho, 0.0, s.u, s.jumps, dt)
    assert abs(abs(rho[1, 0]) - 0.5 * cf.dephasing_factor(gamma, dt, 100)) < 1e-14
    assert abs(rho[1, 1].real - 0.5) < 1e-14


def test_atom_decay_matches_superoperator_and_rate():
    gamma, dt = 0.05, 0.02
    wl = small_wl([1], [1], g=0.0, jumps=[(W.ATOM_DECAY, 0, 0, gamma)], dt=dt)
    wl["g"] = [0.0]
    s = ev.System(wl)
    rho = np.zeros((4, 4), complex); rho[1, 1] = 1.0
    for k in range(50):
        rho, _ = ev.step(rho, 0.0, s.u, s.jumps, dt)
    assert abs(rho[1, 1].real - (1 - gamma * dt) ** 50) < 1e-14


# ------------------------------------------------- brute-force step map


@pytest.mark.parametrize("window", [(0, -1), (1, 2)])
def test_step_map_equals_superoperator(window):
    wl = small_wl([1, 1], [1, 2], exc=window, mus=[(0, 1, 0.07)], dt=0.3,
                  jumps=[(W.PHOTON_LEAK, 0, -1, 0.05), (W.PHOTON_LEAK, 1, -1, 0.02),
                         (W.ATOM_DECAY, 1, 0, 0.04), (W.ATOM_DEPHASE, 0, 0, 0.03)])
    wl["g"] = [0.11, 0.09]
    s = ev.System(wl)
    rho0 = W.initial_rho(wl, s.occ)
    m = ev.superoperator(s)
    v = rho0.reshape(-1)
    rho, sink = rho0, 0.0
    for k in range(60):
        v = m @ v
        rho, sink = ev.step(rho, sink, s.u, s.jumps, s.dt)
    assert np.abs(rho - v.reshape(s.n, s.n)).max() < 1e-12
    assert abs(np.trace(v.reshape(s.n, s.n)).real - (1 - sink)) < 1e-12
    if window == (0, -1):
        assert abs(sink) < 1e-15


def test_sink_equals_explicit_vacuum():
    length, height = 4, 3
    base = W.photon_lattice(length, height, mu=0.2, g=0.15, gamma=0.05, dt=0.1,
                            start=(0, 1))
    s_block = ev.System(base)
    s_vac = ev.System(dict(base, exc_min=0, exc_max=1))
    assert s_vac.n == s_block.n + 1
    rho_b = W.initial_rho(base, s_block.occ)
    rho_v = W.initial_rho(base, s_vac.occ)
    rho_b, sink = ev.evolve(s_block, rho_b, 300)
    rho_v, sink_v = ev.evolve(s_vac, rho_v, 300)
    assert sink > 1e-2 and abs(sink_v) < 1e-15
    # the vacuum is index 0 of the larger basis (all levels 0 sorts first)
    assert abs(rho_v[0, 0].real - sink) < 1e-13
    assert np.abs(rho_v[1:, 1:] - rho_b).max() < 1e-13


def test_invariants_hermitian_trace_positive():
    wl = W.tch_2x2()
    s = ev.System(wl)
    rho = W.initial_rho(wl, s.occ)
    rho, sink = ev.evolve(s, rho, 500)
    assert np.abs(rho - rho.conj().T).max() == 0.0
    assert abs(rho.trace().real - (1 - sink)) < 1e-14
    # the Euler dissipator step equals a completely positive map minus
    # (dt^2/4) sum gamma^2 A^dag A rho A^dag A, so eigenvalues may dip below zero
    # by at most k (dt sum_j gamma_j |A_j^dag A_j|)^2 after k steps
    bound = 500 * (wl["dt"] * sum(j[3] for j in wl["jumps"]) * 2) ** 2
    assert np.linalg.eigvalsh(rho).min() > -bound


def test_block_structure_preserved_without_decoherence():
    wl = dict(W.tch_2x2(), jumps=[])
    s = ev.System(wl)
    rho0 = W.initial_rho(wl, s.occ)
    nexc = md.excitation_number(s.occ)
    rho, _ = ev.evolve(s, rho0, 200)
    # U commutes with the excitation number: each sector's block evolves alone
    for e in np.unique(nexc):
        idx = np.nonzero(nexc == e)[0]
        blk0 = rho0[np.ix_(idx, idx)]
        assert abs(np.trace(rho[np.ix_(idx, idx)]).real - np.trace(blk0).real) < 1e-13


# --------------------------------------------------------------- lattice


@pytest.mark.parametrize("atoms_per_site,shape", [(0, (6, 5)), (1, (5, 4))])
def test_lattice_matches_sine_mode_closed_form(atoms_per_site, shape):
    length, height = shape
    wl = W.photon_lattice(length, height, mu=0.3, g=0.2, gamma=0.0, dt=0.05,
                          atoms_per_site=atoms_per_site, start=(2, 1))
    s = ev.System(wl)
    rho0 = W.initial_rho(wl, s.occ)
    k = 150
    rho, _ = ev.evolve(s, rho0, k)
    ref = cf.lattice_rho(s.occ, atoms_per_site, length, height, 0.3, 0.2, 1.0,
                         k * wl["dt"], wl["centre_site"])
    assert np.abs(rho - ref).max() < 1e-12


def test_lattice_transpose_symmetry_of_centre_start():
    wl = W.photon_lattice(6, 6, mu=0.4, g=0.2, gamma=0.0, dt=0.05, start=(3, 3))
    s = ev.System(wl)
    rho, _ = ev.evolve(s, W.initial_rho(wl, s.occ), 200)
    pops = np.real(np.diag(rho))
    grid = np.zeros((6, 6))
    for idx in range(s.n):
        m = int(np.nonzero(s.occ[idx])[0][0])
        if m % 2 == 0:
            site = m // 2
            grid[site // 6, site % 6] = pops[idx]
    assert np.abs(grid - grid.T).max() < 1e-13
    assert grid.sum() > 0.1


# ------------------------------------------------------------- gradients


def test_frechet_matches_scipy():
    wl = W.tch_2x2()
    s = ev.System(wl)
    rng = np.random.default_rng(3)
    dh = rng.standard_normal((s.n, s.n)); dh = dh + dh.T
    mine = gr.frechet_exp_minus_i_h_dt(s.h, s.dt, dh)
    _, ref = sla.expm_frechet(-1j * s.dt * s.h, -1j * s.dt * dh)
    assert np.abs(mine - ref).max() < 1e-13


def test_tangent_linear_matches_central_differences():
    wl = small_wl([1, 1], [2, 2], mus=[(0, 1, 0.04)], dt=0.1,
                  jumps=[(W.PHOTON_LEAK, 0, -1, 0.03), (W.PHOTON_LEAK, 1, -1, 0.01),
                         (W.ATOM_DEPHASE, 1, 0, 0.02)])
    wl["g"] = [0.09, 0.06]
    s = ev.System(wl)
    rho0 = W.initial_rho(wl, s.occ)
    obs = md.photon_number(wl, s.occ).astype(float)
    f, grad = gr.gradient(s, rho0, 40, obs)
    fd = np.array([gr.finite_difference(wl, rho0, 40, obs, np.eye(len(grad))[i], 1e-5)
                   for i in range(len(grad))])
    assert np.linalg.norm(grad - fd) / np.linalg.norm(grad) < 1e-7


def test_tangent_linear_matches_lattice_closed_form_gradient():
    length, height = 4, 4
    wl = W.photon_lattice(length, height, mu=0.3, g=0.25, gamma=0.0, dt=0.05,
                          start=(1, 2))
    s = ev.System(wl)
    rho0 = W.initial_rho(wl, s.occ)
    k = 60
    obs = np.zeros(s.n)
    site = wl["centre_site"]
    obs[int(np.nonzero(s.occ[:, 2 * site] == 1)[0][0])] = 1.0
    pop, dmu, dg = cf.lattice_population_grad(length, height, 0.3, 0.25, 1.0,
                                              k * wl["dt"], site, site)
    f, tmu = gr.tangent(s, rho0, k, obs, gr.tied_direction(wl, "mu"))
    _, tg = gr.tangent(s, rho0, k, obs, gr.tied_direction(wl, "g"))
    assert abs(f - pop) < 1e-12
    assert abs(tmu - dmu) < 1e-10 * max(1.0, abs(dmu))
    assert abs(tg - dg) < 1e-10 * max(1.0, abs(dg))


def test_closed_form_gradient_matches_its_own_differences():
    args = (6, 5, 0.3, 0.25, 1.0, 3.0, 7, 7)
    pop, dmu, dg = cf.lattice_population_grad(*args)
    h = 1e-6
    pm = cf.lattice_population_grad(6, 5, 0.3 + h, 0.25, 1.0, 3.0, 7, 7)[0]
    pmm = cf.lattice_population_grad(6, 5, 0.3 - h, 0.25, 1.0, 3.0, 7, 7)[0]
    pg = cf.lattice_population_grad(6, 5, 0.3, 0.25 + h, 1.0, 3.0, 7, 7)[0]
    pgm = cf.lattice_population_grad(6, 5, 0.3, 0.25 - h, 1.0, 3.0, 7, 7)[0]
    assert abs((pm - pmm) / (2 * h) - dmu) < 1e-8
    assert abs((pg - pgm) / (2 * h) - dg) < 1e-8
