"""Analytic solutions that pin the oracle (test infrastructure).

Each function is the textbook solution of a special case of the master
equation of Sec. II (Eqs. 2-3) with the Jaynes-Cummings / hopping Hamiltonians
of Sec. IV (Eq. 8b, Eq. 12), hbar = 1, omega_a = omega_c.

* ``rabi``: resonant JC, start |n photons, atom ground>, no decoherence:
  P(t) = cos^2(g sqrt(n) t).  U^k = exp(-i H k dt) makes the discrete map
  exact, so this pins U and the rotation to rounding level.
* ``damped_jc``: one photon + ground atom with photon leak gamma; the
  single-excitation amplitudes obey i c1' = -i gamma/2 c1 + g c2,
  i c2' = g c1 (rotating frame), solved with Omega = sqrt(g^2 - gamma^2/16).
  The time-discrete scheme differs from it at O(dt gamma), i.e. ~1e-7 for
  the first workload.
* ``bare_leak_mean``: a cavity with no coupling keeps a diagonal rho; the
  discrete dissipator maps <n> to (1 - gamma dt) <n> exactly per step.
* ``dephasing_factor``: sigma^dag sigma dephasing multiplies the atomic
  coherence by (1 - gamma dt / 2) exactly per step.
* ``lattice``: the open-boundary L x W lattice (Sec. IV.B) with nearest-
  neighbour hopping mu has sine eigenmodes with energies
  2 mu (cos(pi p/(L+1)) + cos(pi q/(W+1))); with one atom per site, uniform g
  and omega, the single-excitation Hamiltonian splits into one 2 x 2 block
  per mode, solved in closed form.  Also the derivatives of a photon
  population with respect to mu and g.
"""
from __future__ import annotations

import numpy as np


def rabi(g, n, t):
    return np.cos(g * np.sqrt(n) * t) ** 2


def damped_jc(g, gamma, t):
    """(P_{1,g}, P_{0,e}, P_{0,g}) at time t, for g > gamma / 4."""
    om = np.sqrt(g * g - gamma * gamma / 16.0)
    env = np.exp(-gamma * t / 4.0)
    c1 = env * (np.cos(om * t) - gamma / (4.0 * om) * np.sin(om * t))
    c2 = env * (g / om) * np.sin(om * t)
    p1, p2 = c1 * c1, c2 * c2
    return p1, p2, 1.0 - p1 - p2


def bare_leak_mean(n0, gamma, dt, k):
    return n0 * (1.0 - gamma * dt) ** k


def dephasing_factor(gamma, dt, k):
    return (1.0 - gamma * dt / 2.0) ** k


def _sine_modes(length, height):
    """Orthonormal eigenvectors phi[q, s] of the open-grid adjacency (site
    s = i * height + j) and their eigenvalues lam_q / 2 of (adjacency / 2)."""
    p = np.arange(1, length + 1)
    q = np.arange(1, height + 1)
    i = np.arange(length)
    j = np.arange(height)
    a = np.sqrt(2.0 / (length + 1)) * np.sin(np.pi * np.outer(p, i + 1) / (length + 1))
    b = np.sqrt(2.0 / (height + 1)) * np.sin(np.pi * np.outer(q, j + 1) / (height + 1))
    phi = np.einsum("pi,qj->pqij", a, b).reshape(length * height, length * height)
    lam = (np.cos(np.pi * p / (length + 1))[:, None]
           + np.cos(np.pi * q / (height + 1))[None, :]).reshape(-1)
    return phi, lam


def lattice_amplitudes(length, height, mu, g, omega, t, start, with_atoms=True):
    """Single-excitation amplitudes at time t for a photon started at site
    ``start``: returns (photon[s], atom[s]) (atom is zeros without atoms).

    Photon mode q has energy omega + eps_q, eps_q = 2 mu lam_q; it couples only
    to the atomic mode with the same sine profile (energy omega), strength g.
    With theta = eps/2 and Omega = sqrt(theta^2 + g^2), the 2 x 2 block
    started in the photon gives
        h_P = e^{-i(omega+theta)t} (cos Omega t - i theta/Omega sin Omega t)
        h_A = e^{-i(omega+theta)t} (-i g/Omega sin Omega t)."""
    phi, lam = _sine_modes(length, height)
    w = phi[:, start]
    if with_atoms:
        theta = mu * lam
        om = np.sqrt(theta ** 2 + g ** 2)
        ph = np.exp(-1j * (omega + theta) * t)
        hp = ph * (np.cos(om * t) - 1j * theta / om * np.sin(om * t))
        ha = ph * (-1j * g / om * np.sin(om * t))
    else:
        hp = np.exp(-1j * (omega + 2.0 * mu * lam) * t)
        ha = np.zeros_like(hp)
    photon = phi.T @ (w * hp)
    atom = phi.T @ (w * ha)
    return photon, atom


def lattice_population_grad(length, height, mu, g, omega, t, start, site):
    """Photon population at ``site`` and its derivatives d/dmu, d/dg (with all
    hops tied to mu and all couplings tied to g)."""
    phi, lam = _sine_modes(length, height)
    w = phi[:, start] * phi[:, site]
    theta = mu * lam
    om = np.sqrt(theta ** 2 + g ** 2)
    e = np.exp(-1j * (omega + theta) * t)
    c, s = np.cos(om * t), np.sin(om * t)
    r = theta / om
    h = e * (c - 1j * r * s)
    # derivatives of h with respect to theta and g
    dr_dth = g ** 2 / om ** 3
    dr_dg = -theta * g / om ** 3
    dh_dth = -1j * t * h + e * (-t * s * r - 1j * dr_dth * s - 1j * r * t * c * r)
    dh_dg = e * (-t * s * (g / om) - 1j * dr_dg * s - 1j * r * t * c * (g / om))
    amp = np.sum(w * h)
    damp_mu = np.sum(w * dh_dth * lam)
    damp_g = np.sum(w * dh_dg)
    pop = abs(amp) ** 2
    return (pop, 2.0 * np.real(np.conj(amp) * damp_mu),
            2.0 * np.real(np.conj(amp) * damp_g))


def lattice_rho(occ, atoms_per_site, length, height, mu, g, omega, t, start):
    """Density matrix psi psi^dag of the closed lattice at time t in the basis
    ``occ`` (single-excitation window, one photon mode then the atoms per
    site, as the basis enumerator orders modes)."""
    photon, atom = lattice_amplitudes(length, height, mu, g, omega, t, start,
                                      with_atoms=atoms_per_site > 0)
    stride = 1 + atoms_per_site
    n = occ.shape[0]
    psi = np.zeros(n, dtype=np.complex128)
    for idx in range(n):
        m = int(np.nonzero(occ[idx])[0][0])
        site, off = divmod(m, stride)
        psi[idx] = photon[site] if off == 0 else atom[site]
    return np.outer(psi, psi.conj())
