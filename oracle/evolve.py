"""Propagator, one time step and observables (oracle; test infrastructure).

Paper passages followed:

* Sec. II, Eq. 2: i hbar d(rho)/dt = [H, rho] + i L(rho), read with hbar = 1
  as d(rho)/dt = -i [H, rho] + L(rho).
* Sec. II, Eq. 3: L(rho) = sum_j gamma_j (A_j rho A_j^dag
  - 1/2 {A_j^dag A_j, rho}); the printed anticommutator lacks its rho and is
  read as {A_j^dag A_j, rho}.
* Sec. IV.B and Table III: the solve has a "Taylor approximation" stage that
  builds the propagator U = exp(-i H dt) once, and a "unitary evolution"
  stage that applies U rho U^dag repeatedly.  The paper gives no time
  discretisation for the dissipator; the reading used is one Lie-Trotter
  step per iteration -- rotate with U, then an explicit-Euler dissipator step
  on the rotated matrix:

      rho_u      = U rho_k U^dag
      rho_d      = rho_u + dt * sum_j gamma_j (A_j rho_u A_j^dag
                                       - 1/2 (A_j^dag A_j rho_u + rho_u A_j^dag A_j))
      sink      += dt * sum_j gamma_j [tr(A_j^dag A_j rho_u) - tr(A_j rho_u A_j^dag)]
      rho_{k+1}  = Herm(rho_d) * (1 - sink) / tr Herm(rho_d),
                   Herm(X) = (X + X^dag) / 2

  The last two lines are identities in exact arithmetic: they book the
  probability that a decoherence operator moves out of a truncated basis
  (the "sink") and remove rounding drift of the trace and of Hermiticity.

* Sec. IV.B: the photon plane without leakage is closed, so its state stays
  pure; ``evolve_pure`` takes the same step on psi (rho = psi psi^dag), the
  O(N^2)-per-step form of the unitary evolution stage for closed models.

The oracle's propagator comes from an eigendecomposition of H, deliberately
not the Taylor series the library uses.
"""
from __future__ import annotations

import numpy as np

from . import model


class System:
    """Everything the oracle needs about one workload, built from its dict.
    occ: an explicit occupation table (a subset of the window basis, as the
    state-space selection produces); default: the whole window basis."""

    def __init__(self, wl, occ=None):
        self.wl = wl
        if occ is None:
            occ = model.basis(wl["atoms"], wl["photon_cap"],
                              wl.get("exc_min", 0), wl.get("exc_max", -1))
        self.occ = np.asarray(occ)
        self.n = self.occ.shape[0]
        self.terms = model.hamiltonian_terms(wl, self.occ)
        h = None
        for coef, _, w in self.terms:
            h = coef * w if h is None else h + coef * w
        self.h = h.toarray()
        self.jumps = model.jump_operators(wl, self.occ)
        self.dt = float(wl["dt"])
        self.u = propagator(self.h, self.dt)


class GeneralSystem:
    """A model given directly as matrices (a general-form workload: real
    symmetric H as COO triplets, each decoherence operator A_j as moves
    A|source> = sum of coef |target> over its moves, target -1 for a
    component outside the basis), optionally restricted to the states
    `keep` (indices into its basis).

    Sec. II, Eq. 3 puts no restriction on the operators A_j: a state may
    have several images and several preimages (for example collective
    decay, A = sum of the lowering operators of several atoms).  Readings:
    moves with the same (source, target) add up (they are the matrix entries
    of A); every move with target -1 leads to its own state outside the
    basis, orthogonal to every other state, so it adds coef^2 to the
    diagonal of A^dag A and nothing else.  Restriction follows the window
    basis reading: P A P on the kept states and A^dag A formed from the
    whole operator before the projection, so probability that an operator
    moves onto removed states -- including the cross terms of two kept
    states moving onto the same removed state -- leaves through the sink."""

    def __init__(self, wl, keep=None):
        import scipy.sparse as sp
        self.wl = wl
        n = int(wl["n"])
        rows, cols, vals = wl["h"]
        h = sp.coo_matrix((np.asarray(vals, float), (np.asarray(rows), np.asarray(cols))),
                          shape=(n, n)).toarray()
        keep = np.arange(n) if keep is None else np.asarray(keep)
        self.keep = keep
        self.n = keep.size
        self.h = h[np.ix_(keep, keep)]
        self.jumps = []
        for gamma, src, dst, coef in wl["jumps"]:
            src = np.asarray(src, dtype=np.int64)
            dst = np.asarray(dst, dtype=np.int64)
            coef = np.asarray(coef, float)
            # image rows: the n basis states, then one private row per move
            # whose image leaves the basis
            image = np.where(dst >= 0, dst, n + np.arange(dst.size))
            a_full = sp.csr_matrix((coef, (image, src)), shape=(n + dst.size, n))
            k_full = (a_full.T @ a_full).tocsr()
            a_p = a_full[keep][:, keep].tocsr()
            k_p = k_full[keep][:, keep].tocsr()
            a_p.eliminate_zeros()
            k_p.eliminate_zeros()
            self.jumps.append((float(gamma), a_p, k_p))
        self.dt = float(wl["dt"])
        self.u = propagator(self.h, self.dt)


def propagator(h, dt):
    """U = exp(-i H dt) for real symmetric H, via H = V diag(lam) V^T."""
    lam, v = np.linalg.eigh(h)
    return (v * np.exp(-1j * lam * dt)) @ v.T


def _sandwich(a, x):
    """A x A^dag for a real sparse A (so A^dag = A^T): (A (A x)^T)^T."""
    y = a @ x
    return (a @ np.ascontiguousarray(y.T)).T


def _right(m, x):
    """x M for a real symmetric sparse M: (M x^T)^T."""
    return (m @ np.ascontiguousarray(x.T)).T


def _anticommutator_operator(jumps):
    """K = sum_j gamma_j A_j^dag A_j (a sparse sum)."""
    k = None
    for gamma, _, ada in jumps:
        k = gamma * ada if k is None else k + gamma * ada
    return k


def dissipator(rho, jumps):
    """D(rho) = sum_j gamma_j A_j rho A_j^dag - 1/2 (K rho + rho K),
    K = sum_j gamma_j A_j^dag A_j.

    Every decoherence operator here has real matrix elements, so A^dag is A^T
    and K is real symmetric.  A channel whose projected A_j has no non-zero
    element (every arrival outside the basis) contributes no jump term."""
    out = np.zeros_like(rho)
    if not jumps:
        return out
    k = _anticommutator_operator(jumps)
    out -= 0.5 * (k @ rho + _right(k, rho))
    for gamma, a, _ in jumps:
        if a.nnz:
            out += gamma * _sandwich(a, rho)
    return out


def lost_rate(rho, jumps):
    """sum_j gamma_j [tr(A^dag A rho) - tr(A rho A^dag)]: probability per unit
    time that the decoherence operators move out of the basis.  Uses
    tr(M X) = sum_ij M_ij X_ji and tr(A X A^T) = sum_ij A_ij (A X)_ij."""
    if not jumps:
        return 0.0
    total = _anticommutator_operator(jumps).multiply(rho.T).sum().real
    for gamma, a, _ in jumps:
        if a.nnz:
            total -= gamma * a.multiply(a @ rho).sum().real
    return float(total)


def step(rho, sink, u, jumps, dt):
    """One time step (rotate, dissipate, book sink, symmetrise, renormalise).
    Returns (rho_{k+1}, sink_{k+1})."""
    rho_u = u @ rho @ u.conj().T
    rho_d = rho_u + dt * dissipator(rho_u, jumps)
    sink = sink + dt * lost_rate(rho_u, jumps)
    herm = 0.5 * (rho_d + rho_d.conj().T)
    rho_next = herm * ((1.0 - sink) / herm.trace().real)
    return rho_next, sink


def evolve(sysm: System, rho0, n_steps, sink0=0.0, record_every=0):
    """n_steps time steps from rho0.  Returns (rho, sink[, records]) where
    records holds (k, rho_k, sink_k) every record_every steps."""
    rho, sink = rho0.astype(np.complex128), float(sink0)
    rec = []
    for k in range(1, n_steps + 1):
        rho, sink = step(rho, sink, sysm.u, sysm.jumps, sysm.dt)
        if record_every and k % record_every == 0:
            rec.append((k, rho.copy(), sink))
    return (rho, sink, rec) if record_every else (rho, sink)


def is_closed(jumps):
    """True when no decoherence operator acts on the basis: every channel has
    rate 0 or a projected A_j and A_j^dag A_j with no non-zero element."""
    return all(gamma == 0.0 or (a.nnz == 0 and ada.nnz == 0) for gamma, a, ada in jumps)


def step_pure(psi, u):
    """One time step of a closed model in pure-state form.

    Sec. IV.B: the photon on the plane of cavities with no leakage is a
    closed system, so a pure start stays pure.  With rho_k = psi_k psi_k^dag
    the step above becomes: rotation U psi psi^dag U^dag; the dissipator and
    the sink are zero; Herm leaves psi psi^dag unchanged; the trace
    renormalisation divides by tr = |U psi|^2.  Hence rho_{k+1} =
    psi_{k+1} psi_{k+1}^dag with psi_{k+1} = U psi_k / |U psi_k| (up to a
    global phase, which rho does not see)."""
    y = u @ psi
    return y / np.linalg.norm(y)


def evolve_pure(sysm: System, psi0, n_steps):
    """n_steps pure-state steps from psi0 ([n]); raises ValueError for a model
    with decoherence (its state does not stay pure)."""
    if not is_closed(sysm.jumps):
        raise ValueError("pure-state steps need a closed model")
    psi = np.asarray(psi0, dtype=np.complex128).copy()
    for _ in range(n_steps):
        psi = step_pure(psi, sysm.u)
    return psi


def observe(rho, sink):
    """Populations Re rho_ss, trace and sink."""
    pops = np.real(np.diag(rho)).copy()
    return pops, float(pops.sum()), float(sink)


def superoperator(sysm: System):
    """Matrix M of the step map on row-major vec(rho), for tiny N:
    M = (I + dt L_D) (U kron conj(U)), with L_D the dissipator's
    superoperator.  Uses vec(A X B) = (A kron B^T) vec(X) (row-major)."""
    n = sysm.n
    eye = np.eye(n)
    ld = np.zeros((n * n, n * n), dtype=np.complex128)
    for gamma, a, ada in sysm.jumps:
        ad = a.toarray().astype(np.complex128)
        add = ada.toarray().astype(np.complex128)
        ld += gamma * (np.kron(ad, ad.conj())
                       - 0.5 * (np.kron(add, eye) + np.kron(eye, add.T)))
    rot = np.kron(sysm.u, sysm.u.conj())
    return (np.eye(n * n) + sysm.dt * ld) @ rot
