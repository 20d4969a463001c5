"""Decoherence operators that are not monomial, as general-form inputs.

Sec. II, Eq. 3 allows any operators A_j; the structured channels (photon
leak, atom decay, dephasing) each map a basis state onto at most one other.
Collective atomic decay, A_c = sum_k sigma_ck over the atoms of cavity c, is
the standard channel of Tavis-Cummings models that does not: a state with two
excited atoms has two images, and two states share an image.  This module
writes such operators out as moves (A|source> = sum of coef |target>) over a
basis given by its occupation table, and assembles general-form workload
dicts; both the library and the oracle take the matrices as given.  It holds
input construction only.

Occupation tables follow the structured workloads' mode order: for cavity c,
its photon mode, then its atoms.
"""
from __future__ import annotations

import numpy as np

from . import mode_list


def _index_of(occ: np.ndarray) -> dict:
    return {tuple(int(x) for x in row): i for i, row in enumerate(occ)}


def collective_decay_moves(wl: dict, occ: np.ndarray, cavity: int):
    """Moves of A = sum_k sigma_ck (every atom of `cavity` lowered, coefficient
    1 each); an image outside the basis gets target -1."""
    modes = mode_list(wl["atoms"])
    cols = [i for i, m in enumerate(modes) if m[0] == "atom" and m[1] == cavity]
    where = _index_of(occ)
    src, dst, coef = [], [], []
    for s, row in enumerate(occ):
        for col in cols:
            if row[col] == 1:
                t = list(int(x) for x in row)
                t[col] = 0
                src.append(s)
                dst.append(where.get(tuple(t), -1))
                coef.append(1.0)
    return src, dst, coef


def photon_leak_moves(wl: dict, occ: np.ndarray, cavity: int):
    """Moves of A = a_c (coefficient sqrt(n)); an image outside the basis gets
    target -1."""
    modes = mode_list(wl["atoms"])
    col = modes.index(("photon", cavity))
    where = _index_of(occ)
    src, dst, coef = [], [], []
    for s, row in enumerate(occ):
        n = int(row[col])
        if n > 0:
            t = list(int(x) for x in row)
            t[col] = n - 1
            src.append(s)
            dst.append(where.get(tuple(t), -1))
            coef.append(float(np.sqrt(n)))
    return src, dst, coef


def general_workload(wl: dict, n: int, h_coo, jumps, name: str | None = None) -> dict:
    """General-form dict of n states with Hamiltonian h_coo = (rows, cols,
    vals) and jumps [(gamma, src, dst, coef)], the time step, step count and
    initial state of the structured workload wl."""
    rows, cols, vals = h_coo
    return {"general": True, "name": name or (wl["name"] + "_collective"), "n": int(n),
            "h": (np.asarray(rows, np.int32), np.asarray(cols, np.int32), np.asarray(vals, float)),
            "jumps": [(float(g), list(s), list(d), list(c)) for g, s, d, c in jumps],
            "dt": wl["dt"], "steps": wl.get("steps", 100), "init": wl.get("init")}


def tch_collective(atoms=(2, 2), cap=2, g=0.01, mu=0.005, gamma_collective=0.002,
                   gamma_leak=0.001, dt=0.01, steps=500, seed=20240311 + 6):
    """A Tavis-Cummings-Hubbard chain (structured description) whose atoms
    decay collectively per cavity (rate gamma_collective) and whose photons
    leak (gamma_leak), with a seeded Haar-random pure start.  Returns the
    structured dict (without the collective channels, which the structured
    jump kinds cannot express) and the list of decoherence channels as
    callables of the occupation table: [(gamma, moves(occ))]."""
    atoms = list(atoms)
    n_cav = len(atoms)
    n_atoms = int(sum(atoms))
    wl = {
        "name": f"tch_collective_{'x'.join(map(str, atoms))}_cap{cap}",
        "atoms": atoms, "photon_cap": [cap] * n_cav, "exc_min": 0, "exc_max": -1,
        "omega_c": [1.0] * n_cav, "omega_a": [1.0] * n_atoms, "g": [g] * n_atoms,
        "hops": [(c, c + 1, mu) for c in range(n_cav - 1)], "jumps": [],
        "dt": dt, "steps": steps, "init": {"kind": "haar", "seed": seed},
    }
    channels = []
    for c in range(n_cav):
        channels.append((gamma_leak, lambda occ, c=c: photon_leak_moves(wl, occ, c)))
        if atoms[c] > 0:
            channels.append((gamma_collective, lambda occ, c=c: collective_decay_moves(wl, occ, c)))
    return wl, channels


def dicke_pair(gamma=0.05, omega=1.0, dt=0.01, steps=200, start="symmetric"):
    """Two bare two-level atoms (no cavity; basis |gg>, |ge>, |eg>, |ee> in
    Kronecker order, atom 0 most significant) with H = omega (n_0 + n_1) and
    collective decay A = sigma_0 + sigma_1 at rate gamma.  start: 'symmetric'
    ((|eg> + |ge>)/sqrt 2), 'antisymmetric' ((|eg> - |ge>)/sqrt 2) or
    'excited' (|ee>).  Returns (general-form dict, rho0)."""
    h = ([1, 2, 3], [1, 2, 3], [omega, omega, 2.0 * omega])
    # sigma_0 lowers atom 0 (index bit 1), sigma_1 lowers atom 1 (bit 0)
    src = [2, 3, 1, 3]
    dst = [0, 1, 0, 2]
    coef = [1.0, 1.0, 1.0, 1.0]
    psi = np.zeros(4, dtype=np.complex128)
    if start == "symmetric":
        psi[2] = psi[1] = 1.0 / np.sqrt(2.0)
    elif start == "antisymmetric":
        psi[2], psi[1] = 1.0 / np.sqrt(2.0), -1.0 / np.sqrt(2.0)
    elif start == "excited":
        psi[3] = 1.0
    else:
        raise ValueError(start)
    wl = {"general": True, "name": f"dicke_pair_{start}", "n": 4,
          "h": (np.array(h[0], np.int32), np.array(h[1], np.int32), np.array(h[2], float)),
          "jumps": [(gamma, src, dst, coef)], "dt": dt, "steps": steps}
    return wl, np.outer(psi, psi.conj())
