"""CPU checks of the C ABI: the library loads and exports every declared
symbol, and the host-side logic (basis, Hamiltonian, FP64 Taylor propagator,
decoherence validation) matches the oracle.  No GPU compute is called."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import evolve as ev
from oracle import model as md

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qme.h")

P = pytest.importorskip("paper_2403_07042_amd")
from paper_2403_07042_amd import _lib as L  # noqa: E402


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qme_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
        assert name in L.SIGNATURES, f"binding lacks {name}"


def test_version_and_error_text():
    lib = L.load()
    assert b"gfx950" in lib.qme_version()
    assert lib.qme_last_error() is not None


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_basis_bit_exact_against_oracle(k):
    wl = W.workload(k)
    ref = md.basis(wl["atoms"], wl["photon_cap"], wl["exc_min"], wl["exc_max"])
    assert np.array_equal(P.basis(wl), ref)


@pytest.mark.parametrize("atoms,caps,exc", [
    ([1, 0, 2], [1, 2, 1], (1, 3)), ([0, 0, 0, 0], [2, 1, 3, 1], (2, 2)),
    ([2, 2], [2, 2], (0, 2)), ([1, 1], [3, 3], (4, -1)), ([3], [0], (0, -1)),
])
def test_basis_windows_against_oracle(atoms, caps, exc):
    wl = {"atoms": atoms, "photon_cap": caps, "exc_min": exc[0], "exc_max": exc[1]}
    ref = md.basis(atoms, caps, *exc)
    got = P.basis(dict(wl, omega_c=[1.0] * len(atoms), omega_a=[1.0] * sum(atoms),
                       g=[0.0] * sum(atoms), dt=0.1))
    assert np.array_equal(got, ref)


def test_paper_lattice_dimension():
    # 81 x 51 plane, single-photon subspace (Sec. IV.B, Eq. 11)
    wl = W.photon_lattice(81, 51, atoms_per_site=0)
    assert P.basis(wl).shape[0] == 4131


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_hamiltonian_matches_oracle(k):
    wl = W.workload(k)
    occ = md.basis(wl["atoms"], wl["photon_cap"], wl["exc_min"], wl["exc_max"])
    ref = md.hamiltonian(wl, occ)
    r, c, v = P.hamiltonian_coo(wl)
    h = np.zeros_like(ref)
    h[r, c] = v
    assert np.abs(h - ref).max() < 1e-14
    assert np.all(np.diff(r.astype(np.int64) * len(ref) + c) > 0)   # sorted, no duplicates


@pytest.mark.parametrize("k,dt", [(1, None), (2, None), (1, 3.0), (2, 2.5)])
def test_taylor_propagator_matches_eigendecomposition(k, dt):
    wl = W.workload(k)
    if dt is not None:
        wl = dict(wl, dt=dt)   # |H dt| > 1/2: exercises scaling and squaring
    s = ev.System(wl)
    du = P.propagator_increment(wl, s.n)
    assert np.abs(du + np.eye(s.n) - s.u).max() < 1e-13
    assert np.array_equal(du, du.T)


def test_propagator_of_config3_and_lattice():
    for wl in (W.tch_chain3(), W.photon_lattice(8, 8)):
        s = ev.System(wl)
        du = P.propagator_increment(wl, s.n)
        assert np.abs(du + np.eye(s.n) - s.u).max() < 1e-13


def bad(wl, **kw):
    w = dict(wl)
    w.update(kw)
    return w


@pytest.mark.parametrize("mutate", [
    dict(exc_min=3, exc_max=2), dict(exc_min=-1), dict(photon_cap=[-1]),
    dict(dt=0.0), dict(dt=float("nan")), dict(g=[float("nan")]),
    dict(jumps=[(0, 5, -1, 0.1)]), dict(jumps=[(1, 0, 3, 0.1)]), dict(jumps=[(0, 0, -1, -0.1)]),
    dict(jumps=[(7, 0, -1, 0.1)]), dict(hops=[(0, 0, 0.1)]),
])
def test_invalid_arguments_rejected(mutate):
    wl = bad(W.jc_single(), **mutate)
    with pytest.raises(L.QmeError) as e:
        P.hamiltonian_coo(wl)
    assert e.value.status in (L.QME_E_ARG, L.QME_E_SIZE)
    assert L.load().qme_last_error()


def test_too_large_basis_rejected():
    wl = {"atoms": [0] * 40, "photon_cap": [1] * 40, "exc_min": 0, "exc_max": -1}
    with pytest.raises(L.QmeError) as e:
        P.basis(dict(wl, omega_c=[1.0] * 40, omega_a=[], g=[], dt=0.1))
    assert e.value.status == L.QME_E_SIZE


def test_size_query_two_call_pattern():
    lib = L.load()
    m = P.api.Marshal(W.tch_2x2())
    n = ctypes.c_int64(0)
    assert lib.qme_basis(ctypes.byref(m.system), ctypes.byref(n), None, 0) == L.QME_OK
    assert n.value == 144
    small = np.zeros((10, 6), np.int32)
    st = lib.qme_basis(ctypes.byref(m.system), ctypes.byref(n),
                       small.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 10)
    assert st == L.QME_E_SIZE and n.value == 144


def test_select_states_matches_oracle_decisions():
    """qme_select_states keeps exactly the states whose growth speed
    |p_now - p_prev| / interval is >= eps, as the oracle decides it (same
    FP64 expression), including a speed exactly at eps."""
    import numpy as np
    from oracle import selection as sel
    rng = np.random.default_rng(20240311 + 41)
    p_prev = rng.random(1000) * 1e-3
    p_now = p_prev + rng.standard_normal(1000) * 1e-6
    p_now[7] = p_prev[7]                       # zero speed
    interval = 0.05
    speed = sel.growth_speed(p_prev, p_now, interval)
    for eps in (0.0, 1e-6, float(np.median(speed)), float(speed[123])):
        keep = P.select_states(p_prev, p_now, interval, eps)
        assert np.array_equal(keep, np.nonzero(speed >= eps)[0])
    assert 123 in P.select_states(p_prev, p_now, interval, float(speed[123]))
    assert P.select_states(p_prev, p_now, interval, 0.0).size == 1000


def test_select_states_errors():
    import numpy as np
    p = np.array([0.5, 0.5])
    q = np.array([0.4, 0.6])
    for args in [(p, q, 0.0, 0.1), (p, q, -1.0, 0.1), (p, q, 0.1, -1e-9),
                 (p, np.array([0.4, np.nan]), 0.1, 0.1), (p, q, 0.1, float("inf"))]:
        with pytest.raises(L.QmeError) as e:
            P.select_states(*args)
        assert "QME_E_ARG" in str(e.value)
    with pytest.raises(L.QmeError) as e:
        P.select_states(p, p, 0.1, 1e-3)         # nothing moves: every state removed
    assert "QME_E_STATE" in str(e.value)


def test_knob_setters_reject_null_context():
    lib = L.load()
    for name, arg in (("qme_set_fold", 1), ("qme_set_split", 1), ("qme_set_fused", 1),
                      ("qme_set_direct_loads", -1), ("qme_set_graph", 1)):
        assert getattr(lib, name)(None, arg) == L.QME_E_ARG, name


def test_pure_state_calls_reject_null_context():
    """The pure-state calls validate before touching the device."""
    from ctypes import byref, c_size_t
    lib = L.load()
    sb, wb = c_size_t(), c_size_t()
    assert lib.qme_pure_layout(None, 1, byref(sb), byref(wb)) == L.QME_E_ARG
    assert lib.qme_pure_step(None, None, 1, 1, None, None) == L.QME_E_ARG
    assert lib.qme_pure_set(None, None, 1, None, None, None) == L.QME_E_ARG
    assert lib.qme_pure_get(None, None, 1, None, None, None) == L.QME_E_ARG
