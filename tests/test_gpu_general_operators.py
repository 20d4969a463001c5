"""Decoherence operators that are not monomial (Sec. II, Eq. 3 with operators
giving a state several images and several preimages), on general-form
contexts: collective atomic decay against its closed forms (superradiant
symmetric state, dark antisymmetric state), Tavis-Cummings-Hubbard models
with collective decay against the oracle in every precision (N = 144 and,
over several tiles, N = 1024), a restricted basis whose removed states are
shared targets (the cross terms of the sink), and batches of such contexts
against their solo runs."""
import numpy as np
import pytest

import workloads as W
from workloads import collective as CO
from oracle import evolve as ev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2403_07042_amd")

TOL = {"fp64": 1e-11, "fp32": 1e-5, "bf16x3": 1e-4}
SINK_TOL = {"fp64": 1e-12, "fp32": 1e-6, "bf16x3": 1e-6}


def collective_pair(structured, channels):
    """(library workload, oracle workload): the same operators (moves over the
    basis), each side with its own Hamiltonian -- the library's
    qme_hamiltonian_coo and the oracle's matrix."""
    s = ev.System(structured)
    occ = P.basis(structured)
    assert np.array_equal(occ, s.occ)
    jumps = [(g, *moves(occ)) for g, moves in channels]
    # each side's own Hamiltonian, its non-zero entries (the same pattern, so
    # the general gradient parameters correspond)
    r, c, v = P.hamiltonian_coo(structured)
    nz = v != 0.0
    lib = CO.general_workload(structured, s.n, (r[nz], c[nz], v[nz]), jumps)
    h = s.h
    r, c = np.nonzero(h)
    orc = CO.general_workload(structured, s.n, (r, c, h[r, c]), jumps)
    assert set(zip(lib["h"][0].tolist(), lib["h"][1].tolist())) == set(zip(r.tolist(), c.tolist()))
    return lib, orc, W.initial_rho(structured, occ)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_dicke_pair_superradiant_and_dark(precision):
    gamma, dt, k = 0.05, 0.01, 200
    f = 1.0 - 2.0 * gamma * dt
    s_vec = np.array([0, 1, 1, 0]) / np.sqrt(2.0)
    for start in ("symmetric", "antisymmetric"):
        wl, rho0 = CO.dicke_pair(gamma=gamma, dt=dt, start=start)
        sol = P.Solver(wl, precision)
        sol.set_rho(rho0)
        print(f"dicke pair {start} {precision}: {k} steps", flush=True)
        sol.step(k)
        rho, sink = sol.get_rho()
        sol.close()
        tol = 1e-12 if precision == "fp64" else 1e-6
        if start == "symmetric":
            assert abs(np.real(s_vec @ rho @ s_vec) - f ** k) < tol
            assert abs(rho[0, 0].real - (1.0 - f ** k)) < tol
        else:
            assert np.abs(rho - rho0).max() < tol
        assert abs(sink) < 1e-15


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_tch_collective_decay_n144_against_oracle(precision):
    structured, channels = CO.tch_collective(atoms=(2, 2), cap=2, gamma_collective=0.02,
                                             gamma_leak=0.01)
    lib, orc, rho0 = collective_pair(structured, channels)
    s = ev.GeneralSystem(orc)
    sol = P.Solver(lib, precision)
    assert sol.n == 144
    sol.set_rho(rho0)
    rho_ref, sink_ref, done = rho0, 0.0, 0
    for k in (1, 50, 500):
        rho_ref, sink_ref = ev.evolve(s, rho_ref, k - done, sink0=sink_ref)
        print(f"tch collective 144 {precision}: step {k}", flush=True)
        sol.step(k - done)
        done = k
        rho, sink = sol.get_rho()
        _, trace, _ = sol.observe()
        assert np.abs(rho - rho_ref).max() < TOL[precision], k
        assert abs(sink - sink_ref) < SINK_TOL[precision]
        assert abs(trace - (1.0 - sink)) < SINK_TOL[precision]
        assert np.array_equal(rho, rho.conj().T)
    sol.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_tch_collective_decay_n1024_against_oracle(precision):
    """Two cavities of three atoms each, photon cap 3: N = 1024 (several tiles
    of both products and of the decoherence pass); states with two or three
    excited atoms in a cavity have two or three images."""
    structured, channels = CO.tch_collective(atoms=(3, 3), cap=3, g=0.02, gamma_collective=0.02,
                                             gamma_leak=0.01, dt=0.02)
    lib, orc, rho0 = collective_pair(structured, channels)
    print("tch collective 1024: oracle", flush=True)
    ref, ref_sink = ev.evolve(ev.GeneralSystem(orc), rho0, 20)
    sol = P.Solver(lib, precision)
    assert sol.n == 1024
    sol.set_rho(rho0)
    print(f"tch collective 1024 {precision}: 20 steps", flush=True)
    sol.step(20)
    rho, sink = sol.get_rho()
    sol.close()
    assert np.abs(rho - ref).max() < TOL[precision]
    assert abs(sink - ref_sink) < SINK_TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_collective_decay_on_a_restricted_basis(precision):
    """qme_subspace removes states onto which two kept states decay together:
    A^dag A is formed before the projection, so the sink takes the cross
    terms; against the oracle's restricted system."""
    structured, channels = CO.tch_collective(atoms=(2, 2), cap=2, gamma_collective=0.05,
                                             gamma_leak=0.01)
    lib, orc, rho0 = collective_pair(structured, channels)
    occ = P.basis(structured)
    # remove every state with no atom excited in cavity 0 and no photon there:
    # both single-excitation atom states of that cavity decay onto them
    removed = (occ[:, 1] == 0) & (occ[:, 2] == 0) & (occ[:, 0] == 0)
    keep = np.nonzero(~removed)[0].astype(np.int32)
    part = ev.GeneralSystem(orc, keep=keep)
    rho_k0 = rho0[np.ix_(keep, keep)]
    rho_k0 = rho_k0 / np.trace(rho_k0).real
    ref, ref_sink = ev.evolve(part, rho_k0, 40)
    sol = P.Solver(lib, precision)
    sub = sol.subspace(keep)
    sub.set_rho(rho_k0)
    print(f"restricted collective {precision}: 40 steps", flush=True)
    sub.step(40)
    rho, sink = sub.get_rho()
    sub.close()
    sol.close()
    assert ref_sink > 1e-4
    assert np.abs(rho - ref).max() < TOL[precision]
    assert abs(sink - ref_sink) < SINK_TOL[precision]


def test_batch_of_collective_contexts_equals_solo():
    wls = []
    for atoms, cap in (((2, 2), 2), ((1, 2), 3), ((2, 1), 2)):
        structured, channels = CO.tch_collective(atoms=atoms, cap=cap, gamma_collective=0.02)
        lib, _, rho0 = collective_pair(structured, channels)
        wls.append((lib, rho0))
    sols = []
    for lib, rho0 in wls:
        s = P.Solver(lib, "fp32")
        s.set_rho(rho0)
        sols.append(s)
    b = P.Batch(sols)
    b.step(25)
    torch.cuda.synchronize()
    for (lib, rho0), s in zip(wls, sols):
        solo = P.Solver(lib, "fp32")
        solo.set_fold(False)
        solo.set_split(False)
        solo.set_rho(rho0)
        solo.step(25)
        assert np.array_equal(s.get_rho()[0], solo.get_rho()[0]), lib["name"]
        solo.close()
    b.close()
    for s in sols:
        s.close()


# ------------------------------------------------ gradients of general models

from oracle import gradients as GR  # noqa: E402
from workloads import hydrogen_bond as hb  # noqa: E402

GRAD_TOL = {"fp64": 1e-9, "fp32": 1e-4}


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _small_collective():
    structured, channels = CO.tch_collective(atoms=(1, 2), cap=1, g=0.2, mu=0.1,
                                             gamma_collective=0.1, gamma_leak=0.05, dt=0.05)
    return collective_pair(structured, channels)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_general_adjoint_collective_decay(precision):
    """qme_adjoint on a general-form context with collective decay (N = 32,
    sparse channels): every gradient entry (H's symmetric entries, then the
    rates) against the oracle's tangent-linear gradient."""
    lib, orc, rho0 = _small_collective()
    obs = np.random.default_rng(20240311 + 45).uniform(0.0, 1.0, 32)
    print("oracle: tangent gradient of the N = 32 collective model", flush=True)
    f_ref, g_ref = GR.gradient(ev.GeneralSystem(orc), rho0, 30, obs)
    sol = P.Solver(lib, precision)
    sol.set_rho(rho0)
    f, g = sol.adjoint(30, obs, checkpoint_every=7)
    sol.close()
    assert g.shape == g_ref.shape
    assert abs(f - f_ref) < (1e-12 if precision == "fp64" else 1e-6)
    assert _rel(g, g_ref) < GRAD_TOL[precision]
    n_h = len(GR.general_pattern(orc))
    assert _rel(g[n_h:], g_ref[n_h:]) < GRAD_TOL[precision]       # the rates alone


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_general_adjoint_hydrogen_bond(precision):
    """The hydrogen-bond model (N = 64, monomial operators in gather form):
    gradients with respect to H's entries and the leak rates against the
    oracle's tangent-linear gradient; the autograd binding gives the same."""
    wl = hb.hb_model(1, steps=60)
    rho0 = hb.initial_rho(wl)
    obs = np.zeros(64)
    obs[np.arange(0, 64, 3)] = 1.0
    print("oracle: tangent gradient of the hydrogen-bond model", flush=True)
    f_ref, g_ref = GR.gradient(ev.GeneralSystem(wl), rho0, 60, obs)
    sol = P.Solver(wl, precision)
    sol.set_rho(rho0)
    f, g = sol.adjoint(60, obs, checkpoint_every=16)
    sol.close()
    assert abs(f - f_ref) < (1e-12 if precision == "fp64" else 1e-6)
    assert _rel(g, g_ref) < GRAD_TOL[precision]


def test_general_adjoint_restricted_basis():
    """Gradients on a qme_subspace context of a collective-decay model (the
    adjoint takes K formed before the projection); parameters whose entries
    touch removed states have zero gradient."""
    lib, orc, rho0 = _small_collective()
    occ = ev.System(CO.tch_collective(atoms=(1, 2), cap=1)[0]).occ
    removed = (occ[:, 0] == 0) & (occ[:, 1] == 0)
    keep = np.nonzero(~removed)[0].astype(np.int32)
    rk = rho0[np.ix_(keep, keep)]
    rk = rk / np.trace(rk).real
    obs = np.linspace(0.0, 1.0, keep.size)
    f_ref, g_ref = GR.gradient(ev.GeneralSystem(orc, keep=keep), rk, 25, obs)
    sol = P.Solver(lib, "fp64")
    sub = sol.subspace(keep)
    sub.set_rho(rk)
    f, g = sub.adjoint(25, obs, checkpoint_every=5)
    sub.close()
    sol.close()
    assert abs(f - f_ref) < 1e-12
    assert _rel(g, g_ref) < 1e-9
    zero = [i for i, (r, c) in enumerate(GR.general_pattern(orc)) if removed[r] or removed[c]]
    assert zero and np.all(g[zero] == 0.0)
