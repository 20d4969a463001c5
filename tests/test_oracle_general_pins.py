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
