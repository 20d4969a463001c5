"""Pins of the oracle's general-form system and of the hydrogen-bond model
builder (Sec. IV.A): a structured model exported to matrices evolves exactly
as the structured oracle; the two-bond model is the Kronecker sum of two
one-bond models (bond independence, basis order); the conditional and
non-rotating-wave couplings sit where the model says; the sizes are the
paper's 64 and 4096.  CPU only."""
import numpy as np
import scipy.sparse as sp

import workloads as W
from workloads import hydrogen_bond as hb
from oracle import evolve as ev
from general_models import export_general


import functools


@functools.lru_cache(maxsize=None)
def model(n_bonds):
    return hb.hb_model(n_bonds)


def sparse_h(wl):
    r, c, v = wl["h"]
    return sp.coo_matrix((v, (r, c)), shape=(wl["n"], wl["n"])).tocsr()


def dense_h(wl):
    return sparse_h(wl).toarray()


def jump_mats(wl):
    out = []
    for gamma, src, dst, coef in wl["jumps"]:
        src, dst, coef = np.asarray(src), np.asarray(dst), np.asarray(coef, float)
        ok = dst >= 0
        out.append(sp.csr_matrix((coef[ok], (dst[ok], src[ok])), shape=(wl["n"], wl["n"])))
    return out


def same(a, b):
    d = (a - b).tocsr()
    d.eliminate_zeros()
    return d.nnz == 0


def test_exported_structured_model_evolves_identically():
    for wl in (W.tch_2x2(steps=30), W.jc_single(steps=30), W.photon_lattice(6, 5, gamma=0.05)):
        s = ev.System(wl)
        g = ev.GeneralSystem(export_general(wl))
        assert np.array_equal(g.h, s.h)
        for (ga, a, ada), (gb, b, bdb) in zip(g.jumps, s.jumps):
            assert ga == gb and np.array_equal(a.toarray(), b.toarray())
            assert np.allclose(ada.toarray(), bdb.toarray(), rtol=0, atol=1e-15)
        rho0 = W.initial_rho(wl, s.occ)
        r1, k1 = ev.evolve(s, rho0, 30)
        r2, k2 = ev.evolve(g, rho0, 30)
        assert np.abs(r1 - r2).max() < 1e-14 and abs(k1 - k2) < 1e-15


def test_hb_sizes_symmetry_and_no_sink():
    one, two = model(1), model(2)
    assert one["n"] == 64 and two["n"] == 4096          # the paper's sizes
    for wl in (one, two):
        h = sparse_h(wl)
        assert same(h, h.T)
        for gamma, src, dst, coef in wl["jumps"]:
            assert min(dst) >= 0                       # leaks stay inside the qubit basis


def test_hb_two_bonds_is_kronecker_sum_of_one_bond():
    one, two = model(1), model(2)
    h1 = sparse_h(one)
    eye = sp.identity(64, format="csr")
    assert same(sparse_h(two), sp.kron(h1, eye) + sp.kron(eye, h1))
    a1 = jump_mats(one)
    a2 = jump_mats(two)
    for k in range(3):
        assert same(a2[k], sp.kron(a1[k], eye))       # bond 0
        assert same(a2[3 + k], sp.kron(eye, a1[k]))   # bond 1


def test_hb_conditional_and_non_rwa_couplings():
    wl = hb.hb_model(1, g=0.1)
    h = dense_h(wl)
    idx = lambda m, l, n, p, e, d: hb._index([[m, l, n, p, e, d]])
    # distance moves only with the electron excited and no bond; it changes
    # the excitation number (no rotating-wave partner)
    assert h[idx(0, 1, 0, 0, 1, 0), idx(0, 1, 0, 0, 1, 1)] == 0.1
    assert h[idx(0, 1, 0, 0, 0, 0), idx(0, 1, 0, 0, 0, 1)] == 0.0
    assert h[idx(0, 0, 0, 0, 1, 0), idx(0, 0, 0, 0, 1, 1)] == 0.0
    # the electron absorbs the photon only when the bond exists (l = 0)
    assert h[idx(0, 0, 0, 1, 0, 1), idx(0, 0, 0, 0, 1, 1)] == 0.1
    assert h[idx(0, 1, 0, 1, 0, 1), idx(0, 1, 0, 0, 1, 1)] == 0.0
    # the proton tunnels with the omega_tun phonon when far, omega_hyd when close
    assert h[idx(1, 0, 0, 0, 0, 1), idx(0, 1, 0, 0, 0, 1)] == 0.1
    assert h[idx(1, 0, 0, 0, 0, 0), idx(0, 1, 0, 0, 0, 0)] == 0.0
    assert h[idx(0, 0, 1, 0, 0, 0), idx(0, 1, 0, 0, 0, 0)] == 0.1
    assert h[idx(0, 0, 1, 0, 1, 0), idx(0, 1, 0, 0, 1, 0)] == 0.0      # not with e = 1
    exc = np.array([sum(hb._bits(s, 1)[0]) for s in range(64)])
    off = np.nonzero(h - np.diag(np.diag(h)))
    assert np.any(exc[off[0]] != exc[off[1]])          # non-RWA terms present


def test_hb_oracle_invariants():
    wl = hb.hb_model(1, steps=2000)
    s = ev.GeneralSystem(wl)
    rho, sink = ev.evolve(s, hb.initial_rho(wl), 2000)
    assert abs(sink) < 1e-15 and abs(np.trace(rho).real - 1.0) < 1e-13   # every leak stays inside
    assert np.abs(rho - rho.conj().T).max() == 0.0
    bound = 2000 * (wl["dt"] * 0.03) ** 2
    assert np.linalg.eigvalsh(rho).min() > -bound
    probs = hb.bond_probabilities(wl, np.real(np.diag(rho)))
    assert abs(probs.sum() - 1.0) < 1e-13 and 0.0 < probs[1] < 1.0


# ------------------------------------------------ non-monomial operators
# Sec. II, Eq. 3 with operators that give a state several images and
# several preimages: collective decay A = sigma_0 + sigma_1 of two atoms.

from workloads import collective as CO  # noqa: E402


def _proj(rho, vec):
    return float(np.real(vec.conj() @ rho @ vec))


def test_collective_decay_superradiant_and_dark_states():
    """Two atoms with collective decay: the symmetric one-excitation state
    decays at twice the single-atom rate, P_S(k) = (1 - 2 gamma dt)^k exactly
    under the discrete map (A|S> = sqrt 2 |gg>, A^dag A |S> = 2 |S>); the
    antisymmetric state is dark (A|A> = 0) and does not move; from |ee> the
    populations follow the three-level cascade ee -> S -> gg at rate
    2 gamma, stepped here as scalars.  Independent decay of the two atoms
    (two monomial operators) would give rate gamma and a decaying |A>."""
    gamma, dt, k = 0.05, 0.01, 200
    s_vec = np.array([0, 1, 1, 0]) / np.sqrt(2.0)
    a_vec = np.array([0, -1, 1, 0]) / np.sqrt(2.0)
    gg = np.array([1, 0, 0, 0.0])
    ee = np.array([0, 0, 0, 1.0])
    f = 1.0 - 2.0 * gamma * dt
    wl, rho0 = CO.dicke_pair(gamma=gamma, dt=dt, start="symmetric")
    rho, sink = ev.evolve(ev.GeneralSystem(wl), rho0, k)
    assert abs(_proj(rho, s_vec) - f ** k) < 1e-13
    assert abs(_proj(rho, gg) - (1.0 - f ** k)) < 1e-13 and abs(sink) < 1e-15
    wl, rho0 = CO.dicke_pair(gamma=gamma, dt=dt, start="antisymmetric")
    rho, _ = ev.evolve(ev.GeneralSystem(wl), rho0, k)
    assert np.abs(rho - rho0).max() < 1e-13
    wl, rho0 = CO.dicke_pair(gamma=gamma, dt=dt, start="excited")
    rho, _ = ev.evolve(ev.GeneralSystem(wl), rho0, k)
    p_ee, p_s, p_gg = 1.0, 0.0, 0.0
    for _ in range(k):
        p_ee, p_s, p_gg = f * p_ee, f * p_s + 2 * gamma * dt * p_ee, p_gg + 2 * gamma * dt * p_s
    assert abs(_proj(rho, ee) - p_ee) < 1e-13
    assert abs(_proj(rho, s_vec) - p_s) < 1e-13
    assert abs(_proj(rho, gg) - p_gg) < 1e-13
    assert abs(_proj(rho, a_vec)) < 1e-13


def _dense_operator(n, src, dst, coef):
    """A with one private row per move leaving the basis (as dense)."""
    n_out = sum(1 for d in dst if d < 0)
    a = np.zeros((n + n_out, n))
    o = n
    for s, d, c in zip(src, dst, coef):
        if d >= 0:
            a[d, s] += c
        else:
            a[o, s] += c
            o += 1
    return a


def test_general_operators_match_kronecker_superoperator():
    """Random real operators with several images and preimages per state
    (and components leaving the basis) on N = 5 against the step map built
    here from dense Kronecker products: vec rho_{k+1} = (I + dt L_D)(U kron
    conj U) vec rho_k with U = expm(-i H dt) (scipy, not the oracle's
    eigendecomposition) and L_D from the dense operators.  The oracle's
    renormalisation is the identity in exact arithmetic, so M^k vec rho_0
    equals its state after k steps and 1 - its trace equals the sink."""
    import scipy.linalg as sla
    rng = np.random.default_rng(20240311 + 40)
    n, dt, steps = 5, 0.05, 40
    h = rng.standard_normal((n, n))
    h = h + h.T
    r, c = np.nonzero(np.ones((n, n)))
    jumps = []
    for _ in range(2):
        m = 9
        src = list(rng.integers(0, n, m))
        dst = list(rng.integers(-1, n, m))
        coef = list(rng.uniform(0.2, 1.0, m))
        jumps.append((float(rng.uniform(0.1, 0.5)), src, dst, coef))
    wl = {"general": True, "name": "random_general", "n": n,
          "h": (r.astype(np.int32), c.astype(np.int32), h[r, c]), "jumps": jumps, "dt": dt}
    psi = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    psi /= np.linalg.norm(psi)
    rho0 = np.outer(psi, psi.conj())
    u = sla.expm(-1j * h * dt)
    eye = np.eye(n)
    lsup = np.zeros((n * n, n * n), dtype=np.complex128)
    for gamma, src, dst, coef in jumps:
        a_full = _dense_operator(n, src, dst, coef)
        k_mat = a_full.T @ a_full
        a_in = a_full[:n]
        lsup += gamma * (np.kron(a_in, a_in) - 0.5 * (np.kron(k_mat, eye) + np.kron(eye, k_mat.T)))
    step = (np.eye(n * n) + dt * lsup) @ np.kron(u, u.conj())
    vec = rho0.reshape(-1)
    for _ in range(steps):
        vec = step @ vec
    ref = vec.reshape(n, n)
    rho, sink = ev.evolve(ev.GeneralSystem(wl), rho0, steps)
    assert any(len(set(d for s2, d in zip(s, dd) if s2 == x and d >= 0)) > 1
               for _, s, dd, _ in jumps for x in set(s))          # several images somewhere
    assert np.abs(rho - ref).max() < 1e-13
    assert sink > 1e-3 and abs(sink - (1.0 - np.trace(ref).real)) < 1e-13


def test_restricted_operator_books_cross_terms_in_the_sink():
    """Two kept states that decay onto the same removed state: restricting the
    basis forms A^dag A before the projection, so the sink takes the
    coherent cross term 2 c1 c2 Re rho_12 as well.  A removed state that H
    does not couple to the others and that A does not leave is exactly the
    sink: the full evolution's block on the kept states and its population
    of the removed state equal the restricted run's state and sink."""
    rng = np.random.default_rng(20240311 + 41)
    n, dt, steps = 4, 0.05, 60
    h = np.zeros((n, n))
    blk = rng.standard_normal((3, 3))
    h[:3, :3] = blk + blk.T
    h[3, 3] = 0.7
    r, c = np.nonzero(h)
    jumps = [(0.3, [1, 2, 0], [3, 3, 1], [0.8, 0.6, 0.5])]
    wl = {"general": True, "name": "shared_removed_target", "n": n,
          "h": (r.astype(np.int32), c.astype(np.int32), h[r, c]), "jumps": jumps, "dt": dt}
    psi = np.zeros(n, dtype=np.complex128)
    psi[:3] = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    psi /= np.linalg.norm(psi)
    rho0 = np.outer(psi, psi.conj())
    full, _ = ev.evolve(ev.GeneralSystem(wl), rho0, steps)
    part = ev.GeneralSystem(wl, keep=np.array([0, 1, 2]))
    rho, sink = ev.evolve(part, rho0[:3, :3], steps)
    assert np.abs(rho - full[:3, :3]).max() < 1e-13
    assert abs(sink - full[3, 3].real) < 1e-13
    # the cross term matters here: without it the sink would differ
    k_diag_only = ev.GeneralSystem(wl, keep=np.array([0, 1, 2]))
    k_diag_only.jumps = [(g, a, sp.diags(k.diagonal()).tocsr()) for g, a, k in k_diag_only.jumps]
    _, sink_wrong = ev.evolve(k_diag_only, rho0[:3, :3], steps)
    assert abs(sink_wrong - sink) > 1e-4


# ------------------------------------------------ general-model gradients

from oracle import gradients as GR  # noqa: E402


def _collective_general(atoms=(1, 2), cap=1):
    st, ch = CO.tch_collective(atoms=atoms, cap=cap, g=0.2, mu=0.1, gamma_collective=0.1,
                               gamma_leak=0.05, dt=0.05)
    s = ev.System(st)
    jumps = [(g, *m(s.occ)) for g, m in ch]
    r, c = np.nonzero(s.h)
    return st, s, CO.general_workload(st, s.n, (r, c, s.h[r, c]), jumps)


def test_general_model_tangent_gradient_matches_finite_differences():
    """Gradients of a general-form model (parameters: H's symmetric entries,
    then the rates) with collective decay: the tangent-linear pass against
    central differences of the whole evolution along random directions."""
    st, s, wl = _collective_general()
    g = ev.GeneralSystem(wl)
    rho0 = W.initial_rho(st, s.occ)
    obs = np.random.default_rng(20240311 + 42).uniform(0.0, 1.0, g.n)
    rng = np.random.default_rng(20240311 + 43)
    for _ in range(2):
        d = rng.standard_normal(GR.n_params(wl))
        _, df = GR.tangent(g, rho0, 30, obs, d)
        fd = GR.finite_difference(wl, rho0, 30, obs, d, 1e-5)
        assert abs(df - fd) < 1e-7 * max(1.0, abs(fd))


def test_general_parameters_chain_to_structured_ones():
    """A structured model exported to matrices: its g and mu gradients are the
    general gradient contracted with dH/dg and dH/dmu on the symmetric
    entries (chain rule), and its rate gradients are equal."""
    wl = dict(W.tch_2x2(steps=20), jumps=[(W.PHOTON_LEAK, 0, -1, 0.05),
                                          (W.ATOM_DECAY, 1, 0, 0.03)])
    wl["g"] = [0.2, 0.15, 0.1, 0.12]
    s = ev.System(wl)
    gen = export_general(wl)
    g = ev.GeneralSystem(gen)
    rho0 = W.initial_rho(wl, s.occ)
    obs = np.real(np.diag(rho0)) + 0.5
    _, grad_s = GR.gradient(s, rho0, 20, obs)
    pattern = GR.general_pattern(gen)
    n_h = len(pattern)
    rng = np.random.default_rng(20240311 + 44)
    for _ in range(2):
        d_s = rng.standard_normal(GR.n_params(wl))
        # the structured direction as a direction in the general parameters
        dirs = GR.parameter_directions(s)
        dh = sum(w * item for w, (kind, item) in zip(d_s, dirs) if kind == "h")
        d_g = np.zeros(GR.n_params(gen))
        for i, (r, c) in enumerate(pattern):
            d_g[i] = dh[r, c]
        d_g[n_h:] = d_s[len(d_s) - len(wl["jumps"]):]
        _, df_g = GR.tangent(g, rho0, 20, obs, d_g)
        assert abs(df_g - grad_s @ d_s) < 1e-11 * max(1.0, abs(df_g))
