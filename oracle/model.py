"""Basis, Hamiltonian and decoherence operators (oracle; test infrastructure).

Paper passages followed:

* Sec. II, first point: a basis of joint atom and photon states and the matrix of
  the Hamiltonian H.
* Sec. IV.A, Eq. 8b: the resonant Jaynes-Cummings form
  omega (a^dag a + sigma^dag sigma) + g (a sigma^dag + a^dag sigma).
* Sec. IV.B, Eqs. 10-12: occupation basis of a cavity lattice, its
  single-photon (window) subspace, and nearest-neighbour photon hopping
  zeta (a_1^dag a_2 + a_1 a_2^dag) (called mu here).
* Sec. II, Eq. 3: decoherence operators A_j with rates gamma_j.

A state is a tuple of occupation levels, one per mode.  Modes are ordered
cavity by cavity: the photon mode of cavity c, then the atoms of cavity c.
The basis is every tuple whose total excitation lies in the window
[exc_min, exc_max], in ascending lexicographic order (mode 0 most
significant); for a full tensor product this is the Kronecker order.

Operators are built the textbook way: apply ladder operators to an
occupation tuple on the untruncated space and keep the matrix element only if
the final tuple lies in the basis (P A P).  Nothing here is blocked or fused.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

PHOTON_LEAK = 0
ATOM_DECAY = 1
ATOM_DEPHASE = 2


@dataclass
class Modes:
    kind: list      # "photon" or "atom" per mode
    cavity: list    # owning cavity per mode
    cap: list       # largest level per mode
    photon_mode: list   # mode index of each cavity's photon
    atom_mode: list     # mode index of each atom (cavity-major)


def make_modes(atoms, photon_cap) -> Modes:
    kind, cavity, cap, pm, am = [], [], [], [], []
    for c, m in enumerate(atoms):
        pm.append(len(kind))
        kind.append("photon"); cavity.append(c); cap.append(int(photon_cap[c]))
        for _ in range(m):
            am.append(len(kind))
            kind.append("atom"); cavity.append(c); cap.append(1)
    return Modes(kind, cavity, cap, pm, am)


def basis(atoms, photon_cap, exc_min=0, exc_max=-1) -> np.ndarray:
    """Occupation table (N x n_modes, int64) of the basis, lexicographic.

    Every state with exc_min <= total excitation <= exc_max (no upper bound
    when exc_max < 0) and 0 <= level <= cap per mode.  States are generated
    as sparse assignments of excitations to modes, then sorted.
    """
    md = make_modes(atoms, photon_cap)
    n_modes = len(md.cap)
    total_cap = sum(md.cap)
    hi = total_cap if exc_max < 0 else min(exc_max, total_cap)
    lo = max(exc_min, 0)
    rows = []

    # depth-first over (mode, level) choices; a stack avoids deep recursion
    stack = [(0, hi, ())]
    while stack:
        start, budget, assign = stack.pop()
        used = hi - budget
        if used >= lo:
            rows.append(assign)
        if budget == 0:
            continue
        for m in range(start, n_modes):
            for level in range(1, min(md.cap[m], budget) + 1):
                stack.append((m + 1, budget - level, assign + ((m, level),)))

    occ = np.zeros((len(rows), n_modes), dtype=np.int64)
    for r, assign in enumerate(rows):
        for m, level in assign:
            occ[r, m] = level
    if len(rows) == 0:
        return occ
    # lexsort: the last key is primary, so mode 0 must come last
    order = np.lexsort(occ.T[::-1])
    return occ[order]


# --- ladder operators on occupation states --------------------------------
# A state is held sparsely as {mode: level} for its non-zero levels, so that a
# lattice of thousands of modes costs no more than a few-mode system.  Each
# operator returns the amplitude and the new state, or None for zero.


def _lower(state, m):
    n = state.get(m, 0)
    if n == 0:
        return None
    s = dict(state)
    if n == 1:
        del s[m]
    else:
        s[m] = n - 1
    return math.sqrt(n), s


def _raise(state, m):
    n = state.get(m, 0)
    s = dict(state); s[m] = n + 1
    return math.sqrt(n + 1), s


def _sigma_minus(state, m):      # |g><e|
    if state.get(m, 0) != 1:
        return None
    s = dict(state); del s[m]
    return 1.0, s


def _sigma_plus(state, m):       # |e><g|
    if state.get(m, 0) != 0:
        return None
    s = dict(state); s[m] = 1
    return 1.0, s


_OPS = {"a": _lower, "adag": _raise, "sm": _sigma_minus, "sp": _sigma_plus}
_LOWERING = ("a", "sm")


def apply_word(state, word):
    """Apply a product of ladder operators, rightmost first.  ``word`` is a
    list of (op, mode).  Returns (amplitude, state) or None."""
    amp = 1.0
    for op, m in reversed(word):
        r = _OPS[op](state, m)
        if r is None:
            return None
        a, state = r
        amp *= a
    return amp, state


def _key(state):
    return tuple(sorted(state.items()))


class _Basis:
    """Sparse view of an occupation table with a state -> index map."""

    def __init__(self, occ):
        self.n = occ.shape[0]
        self.states = []
        self.index = {}
        self.with_mode = {}
        for i, row in enumerate(occ):
            nz = np.nonzero(row)[0]
            st = {int(m): int(row[m]) for m in nz}
            self.states.append(st)
            self.index[_key(st)] = i
            for m in st:
                self.with_mode.setdefault(m, []).append(i)


def word_matrix(occ, word, bs=None):
    """P W P as a sparse N x N matrix (real), with W a ladder-operator word.

    Only states on which the rightmost operator can act are visited when that
    operator lowers a level (a state with level 0 there gives zero)."""
    if bs is None:
        bs = _Basis(occ)
    op, m = word[-1]
    cand = bs.with_mode.get(m, []) if op in _LOWERING else range(bs.n)
    rows, cols, vals = [], [], []
    for j in cand:
        r = apply_word(bs.states[j], word)
        if r is None:
            continue
        amp, tgt = r
        i = bs.index.get(_key(tgt))
        if i is None:
            continue
        rows.append(i); cols.append(j); vals.append(amp)
    return sp.csr_matrix((vals, (rows, cols)), shape=(bs.n, bs.n), dtype=np.float64)


def hamiltonian_terms(wl, occ):
    """The Hamiltonian as a list of (coefficient, label, sparse P W P) terms.

    H = sum_c omega_c a_c^dag a_c + sum_atoms omega_a sigma^dag sigma
      + sum_atoms g (a_c^dag sigma + a_c sigma^dag)
      + sum_hops mu (a_c^dag a_d + a_d^dag a_c)          (hbar = 1)

    Labels: ("omega_c", c), ("omega_a", k), ("g", k), ("mu", h).
    """
    md = make_modes(wl["atoms"], wl["photon_cap"])
    bs = _Basis(occ)
    terms = []
    for c, m in enumerate(md.photon_mode):
        terms.append((wl["omega_c"][c], ("omega_c", c),
                      word_matrix(occ, [("adag", m), ("a", m)], bs)))
    for k, m in enumerate(md.atom_mode):
        terms.append((wl["omega_a"][k], ("omega_a", k),
                      word_matrix(occ, [("sp", m), ("sm", m)], bs)))
    for k, m in enumerate(md.atom_mode):
        pm = md.photon_mode[md.cavity[m]]
        # a sigma^dag is written sigma^dag a (the two act on different modes)
        w = (word_matrix(occ, [("adag", pm), ("sm", m)], bs)
             + word_matrix(occ, [("sp", m), ("a", pm)], bs))
        terms.append((wl["g"][k], ("g", k), w))
    for h, (c, d, mu) in enumerate(wl["hops"]):
        pc, pd = md.photon_mode[c], md.photon_mode[d]
        w = (word_matrix(occ, [("adag", pc), ("a", pd)], bs)
             + word_matrix(occ, [("adag", pd), ("a", pc)], bs))
        terms.append((mu, ("mu", h), w))
    return terms


def hamiltonian(wl, occ) -> np.ndarray:
    """Dense real symmetric H (float64)."""
    h = None
    for coef, _, w in hamiltonian_terms(wl, occ):
        h = coef * w if h is None else h + coef * w
    return h.toarray()


def jump_word(md: Modes, kind, cavity, atom_in_cavity):
    """Ladder-operator word of a decoherence operator A_j."""
    if kind == PHOTON_LEAK:
        return [("a", md.photon_mode[cavity])]
    m = [a for a in md.atom_mode if md.cavity[a] == cavity][atom_in_cavity]
    if kind == ATOM_DECAY:
        return [("sm", m)]
    if kind == ATOM_DEPHASE:
        return [("sp", m), ("sm", m)]
    raise ValueError(kind)


def jump_operators(wl, occ):
    """For each decoherence channel j: (gamma_j, P A_j P, P A_j^dag A_j P),
    both sparse.  The anticommutator uses A^dag A on the untruncated space
    projected afterwards, so population that A moves out of the basis still
    leaves through it (and is booked as sink)."""
    md = make_modes(wl["atoms"], wl["photon_cap"])
    bs = _Basis(occ)
    out = []
    for kind, cavity, atom, gamma in wl["jumps"]:
        w = jump_word(md, kind, cavity, atom)
        dag = [({"a": "adag", "adag": "a", "sm": "sp", "sp": "sm"}[op], m)
               for op, m in reversed(w)]
        a = word_matrix(occ, w, bs)
        ada = word_matrix(occ, dag + w, bs)
        out.append((gamma, a, ada))
    return out


def excitation_number(occ) -> np.ndarray:
    return occ.sum(axis=1)


def photon_number(wl, occ) -> np.ndarray:
    """Total photon number of each basis state."""
    md = make_modes(wl["atoms"], wl["photon_cap"])
    return occ[:, md.photon_mode].sum(axis=1)
