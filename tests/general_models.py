"""Helpers for the general-form tests: export a structured workload (cavities,
atoms, hops) to the matrix form of qme_hamiltonian_general, using the
oracle's operators.  Test infrastructure only."""
import numpy as np
import scipy.sparse as sp

from oracle import evolve as ev


def export_general(wl, h_coo=None):
    """General-form dict with the same H and decoherence operators as the
    structured workload wl: H from h_coo = (rows, cols, vals) when given
    (e.g. the library's own qme_hamiltonian_coo), else from the oracle's
    dense matrix; moves from the oracle's P A P and the pre-projection
    A^dag A diagonal."""
    s = ev.System(wl)
    h = sp.coo_matrix(s.h) if h_coo is None else sp.coo_matrix(
        (np.asarray(h_coo[2], float), (np.asarray(h_coo[0]), np.asarray(h_coo[1]))), shape=(s.n, s.n))
    jumps = []
    for gamma, a, ada in s.jumps:
        a = a.tocsc()
        src, dst, coef = [], [], []
        ada_d = ada.diagonal()
        for w in range(s.n):
            col = a.getcol(w)
            inside = 0.0
            for t, c in zip(col.indices, col.data):
                src.append(w); dst.append(int(t)); coef.append(float(c))
                inside += c * c
            rest = ada_d[w] - inside
            if rest > 1e-12:                     # image outside the basis
                src.append(w); dst.append(-1); coef.append(float(np.sqrt(rest)))
        jumps.append((gamma, src, dst, coef))
    return {"general": True, "name": wl["name"] + "_general", "n": s.n,
            "h": (h.row.astype(np.int32), h.col.astype(np.int32), h.data.astype(float)),
            "jumps": jumps, "dt": wl["dt"], "steps": wl.get("steps", 100)}
