"""The approximate hydrogen-bond model of Sec. IV.A (Eqs. 4-9) as a
general-form workload: basis, Hamiltonian and decoherence operators written
out as matrices for qme_hamiltonian_general and the oracle.

This is input construction (like the other workloads), not the method: both
the library and the oracle take the matrices as given.

Reading of the model (the paper names the parts but not every condition or
value; each choice is listed in the design notes):

* Six two-level modes per hydrogen bond, in this order: the tunnelling
  phonon m (omega_tun), the proton l (0: |Phi_0>, bond formed; 1: |Phi_1>,
  no bond), the bond phonon n (omega_hyd), the photon p (omega_e), the
  electron e and the distance d (0: close, 1: far).  One bond: 2^6 = 64
  states; two bonds (three molecules): 2^12 = 4096, the paper's sizes.
  Basis order: Kronecker, mode 0 of bond 0 most significant.
* H = sum over bonds of H_dist + H_elec + H_tun + H_hyd (Eq. 8):
    H_dist = omega_d [d=1] + g_d (sigma_d + sigma_d^dag)   only when e = 1 and l = 1
    H_elec = omega_e (p + e) + g_e (a sigma_e^dag + a^dag sigma_e)   only when l = 0
    H_tun  = omega_tun (m + [l=1]) + g_tun (b sigma^dag + b^dag sigma)   only when d = 1, e = 0
    H_hyd  = omega_hyd (n + [l=1]) + g_hyd (b sigma^dag + b^dag sigma)   only when d = 0, e = 0
  (molecules move when the electron is excited and there is no bond; the
  electron changes state when the bond exists; the proton tunnels with the
  phonon of its distance only when the electron is in its ground state).
  sigma acts on l (1 -> 0).  The distance term is not rotating-wave: it
  changes the excitation number.  Bonds do not interact, so under the
  master equation a product initial state stays a product of one-bond
  states, which matches the paper's three-molecule limits 1/2, 1/4, 1/4
  when one bond tends to 1/2.  (The time-stepping scheme keeps this exactly
  for the unitary part; its explicit dissipator step adds a cross term of
  order dt^2 gamma^2 per step.)
* Decoherence per bond: leaks of the photon and of both phonons (monomial
  lowering operators), rates gamma_photon and gamma_phonon.
"""
from __future__ import annotations

import numpy as np

MODES = ("m", "l", "n", "p", "e", "d")
M, L, NPH, P, E, D = range(6)


def _bits(index, n_bonds):
    """Mode levels of basis state `index`: array [bond][mode]."""
    nb = 6 * n_bonds
    return np.array([(index >> (nb - 1 - k)) & 1 for k in range(nb)]).reshape(n_bonds, 6)


def _index(levels):
    flat = np.asarray(levels).reshape(-1)
    out = 0
    for b in flat:
        out = (out << 1) | int(b)
    return out


def hb_model(n_bonds=1, omega=1.0, g=0.1, gamma_photon=0.01, gamma_phonon=0.01, dt=0.05,
             steps=2000, init=None):
    """General-form workload dict of the hydrogen-bond model with n_bonds
    bonds (1: two molecules, N = 64; 2: three molecules, N = 4096).  init:
    per-bond levels of the initial basis state (default: far apart, no bond,
    electron ground, one photon, no phonons)."""
    n = 2 ** (6 * n_bonds)
    rows, cols, vals = [], [], []

    def add(i, j, v):
        rows.append(i); cols.append(j); vals.append(v)

    for s in range(n):
        lv = _bits(s, n_bonds)
        diag = 0.0
        for b in range(n_bonds):
            x = lv[b]
            diag += omega * x[D]                          # H_dist
            diag += omega * (x[P] + x[E])                 # H_elec
            diag += omega * (x[M] + x[L])                 # H_tun
            diag += omega * (x[NPH] + x[L])               # H_hyd
            # off-diagonal terms, added from the state with the smaller index
            # for each pair and mirrored below
            if x[E] == 1 and x[L] == 1:                   # g_d (sigma_d + sigma_d^dag)
                y = x.copy(); y[D] ^= 1
                t = lv.copy(); t[b] = y
                add(s, _index(t), g)
            if x[L] == 0 and x[P] == 1 and x[E] == 0:     # a sigma_e^dag: photon -> electron
                y = x.copy(); y[P] = 0; y[E] = 1
                t = lv.copy(); t[b] = y
                j = _index(t); add(s, j, g); add(j, s, g)
            for phonon, dist in ((M, 1), (NPH, 0)):       # b sigma^dag: phonon -> proton 0 -> 1
                if x[D] == dist and x[E] == 0 and x[phonon] == 1 and x[L] == 0:
                    y = x.copy(); y[phonon] = 0; y[L] = 1
                    t = lv.copy(); t[b] = y
                    j = _index(t); add(s, j, g); add(j, s, g)
        add(s, s, diag)
    jumps = []
    for b in range(n_bonds):
        for mode, gam in ((P, gamma_photon), (M, gamma_phonon), (NPH, gamma_phonon)):
            src, dst, coef = [], [], []
            for s in range(n):
                lv = _bits(s, n_bonds)
                if lv[b, mode] == 1:
                    t = lv.copy(); t[b, mode] = 0
                    src.append(s); dst.append(_index(t)); coef.append(1.0)
            jumps.append((gam, src, dst, coef))
    if init is None:
        init = [0, 1, 0, 1, 0, 1]                          # m, l, n, p, e, d
    start = _index(np.array([init] * n_bonds))
    return {
        "general": True, "name": f"hydrogen_bond_{n_bonds}", "n": n, "n_bonds": n_bonds,
        "h": (np.array(rows, np.int32), np.array(cols, np.int32), np.array(vals)),
        "jumps": jumps, "dt": dt, "steps": steps, "start": start,
    }


def initial_rho(wl):
    rho = np.zeros((wl["n"], wl["n"]), dtype=np.complex128)
    rho[wl["start"], wl["start"]] = 1.0
    return rho


def bond_probabilities(wl, pops):
    """Probabilities of 0, 1, ... bonds formed (proton in |Phi_0>, l = 0),
    the grouping {0>, {1>, {2> of Figs. 4-5."""
    nb = wl["n_bonds"]
    out = np.zeros(nb + 1)
    for s, ps in enumerate(pops):
        lv = _bits(s, nb)
        out[int(np.sum(lv[:, L] == 0))] += ps
    return out
