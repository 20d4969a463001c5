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
    lib = CO.general_workload(structured, s.n, P.hamiltonian_coo(structured), jumps)
    h = s.h
    r, c = np.nonzero(h)
    orc = CO.general_workload(structured, s.n, (r, c, h[r, c]), jumps)
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
