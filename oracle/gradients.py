"""Derivatives of a final observable with respect to g, mu and gamma
(oracle; test infrastructure).

The paper's fourth modelling point (Sec. II) is fitting Hamiltonian parameters
to experiment; it does not do it.  Gradients of a final observable with
respect to the couplings make that fit possible.  The oracle computes them two
independent ways:

* tangent-linear (forward mode): differentiate each operation of the time
  step of ``evolve.step`` exactly, carrying d(rho) and d(sink) alongside rho;
  the derivative of U = exp(-i H dt) along dH is the Frechet derivative of the
  matrix exponential, evaluated with the Daleckii-Krein formula in the
  eigenbasis of H;
* central finite differences of the whole evolution.

Observable: f = sum_s o_s Re rho_K[s, s] for a diagonal weight vector o.

Parameter order (per term): g per atom (cavity-major), mu per hop (in the
given order), gamma per jump (in the given order).  For a model given as
matrices (evolve.GeneralSystem) the Hamiltonian parameters are its symmetric
entries instead: one per pair (r, c), r <= c, of the pattern of the given H
triplets, in (r, c) order, moving H[r][c] and H[c][r] together; then gamma
per jump.
"""
from __future__ import annotations

import copy

import numpy as np

from . import evolve, model


def _phi1(z):
    """(e^z - 1) / z, continuous at z = 0."""
    out = np.ones_like(z)
    nz = np.abs(z) > 1e-8
    out[nz] = np.expm1(z[nz]) / z[nz]
    small = ~nz
    out[small] = 1.0 + z[small] / 2.0 + z[small] ** 2 / 6.0
    return out


def frechet_exp_minus_i_h_dt(h, dt, dh):
    """Derivative of U(H) = exp(-i H dt) along the real symmetric direction dH.

    With H = V diag(lam) V^T and a_i = -i lam_i dt, the Daleckii-Krein formula
    gives dU = V (F o (V^T E V)) V^T with E = -i dt dH and the divided
    differences F_ij = (e^{a_i} - e^{a_j}) / (a_i - a_j) (F_ii = e^{a_i}),
    evaluated as e^{a_j} phi1(a_i - a_j)."""
    lam, v = np.linalg.eigh(h)
    a = -1j * lam * dt
    diff = a[:, None] - a[None, :]
    f = np.exp(a)[None, :] * _phi1(diff)
    e = -1j * dt * (v.T @ dh @ v)
    return v @ (f * e) @ v.T


def general_pattern(wl):
    """The symmetric entries (r, c), r <= c, of a general-form workload's H
    pattern, in (r, c) order: its Hamiltonian parameters."""
    rows, cols, _ = wl["h"]
    return sorted({(int(r), int(c)) for r, c in zip(rows, cols) if r <= c})


def parameter_directions(sysm):
    """Per-term derivative data: a list of ("h", dH) for g and mu terms (or
    a general model's symmetric H entries) and ("gamma", j) for jump rates,
    in the documented parameter order."""
    dirs = []
    if isinstance(sysm, evolve.GeneralSystem):
        pos = -np.ones(int(sysm.wl["n"]), dtype=np.int64)
        pos[sysm.keep] = np.arange(sysm.n)
        for r, c in general_pattern(sysm.wl):
            dh = np.zeros((sysm.n, sysm.n))
            a, b = pos[r], pos[c]
            if a >= 0 and b >= 0:
                dh[a, b] = 1.0
                dh[b, a] = 1.0
            dirs.append(("h", dh))
        for j in range(len(sysm.jumps)):
            dirs.append(("gamma", j))
        return dirs
    for coef, label, w in sysm.terms:
        if label[0] == "g":
            dirs.append(("h", w.toarray()))
    for coef, label, w in sysm.terms:
        if label[0] == "mu":
            dirs.append(("h", w.toarray()))
    for j in range(len(sysm.jumps)):
        dirs.append(("gamma", j))
    return dirs


def n_params(wl):
    if wl.get("general"):
        return len(general_pattern(wl)) + len(wl["jumps"])
    return int(sum(wl["atoms"])) + len(wl["hops"]) + len(wl["jumps"])


def tangent(sysm: evolve.System, rho0, n_steps, obs, dtheta):
    """Directional derivative df[dtheta] of f = sum_s obs_s Re rho_K[s,s].

    ``dtheta`` is a vector over all per-term parameters (documented order).
    Returns (f, df)."""
    n = sysm.n
    dirs = parameter_directions(sysm)
    dh = np.zeros((n, n))
    dgam = np.zeros(len(sysm.jumps))
    for w, (kind, item) in zip(dtheta, dirs):
        if w == 0.0:
            continue
        if kind == "h":
            dh += w * item
        else:
            dgam[item] += w
    u = sysm.u
    du = frechet_exp_minus_i_h_dt(sysm.h, sysm.dt, dh)
    dt = sysm.dt
    unit = [(1.0, a, ada) for _, a, ada in sysm.jumps]
    rho = rho0.astype(np.complex128)
    drho = np.zeros_like(rho)
    sink, dsink = 0.0, 0.0
    for _ in range(n_steps):
        rho_u = u @ rho @ u.conj().T
        drho_u = (du @ rho @ u.conj().T + u @ drho @ u.conj().T
                  + u @ rho @ du.conj().T)
        rho_d = rho_u + dt * evolve.dissipator(rho_u, sysm.jumps)
        drho_d = drho_u + dt * evolve.dissipator(drho_u, sysm.jumps)
        new_sink = sink + dt * evolve.lost_rate(rho_u, sysm.jumps)
        new_dsink = dsink + dt * evolve.lost_rate(drho_u, sysm.jumps)
        for j, dg in enumerate(dgam):
            if dg != 0.0:
                drho_d = drho_d + dt * dg * evolve.dissipator(rho_u, [unit[j]])
                new_dsink += dt * dg * evolve.lost_rate(rho_u, [unit[j]])
        x = 0.5 * (rho_d + rho_d.conj().T)
        dx = 0.5 * (drho_d + drho_d.conj().T)
        tau = x.trace().real
        dtau = dx.trace().real
        scale = (1.0 - new_sink) / tau
        dscale = -new_dsink / tau - (1.0 - new_sink) * dtau / tau ** 2
        rho = x * scale
        drho = dx * scale + x * dscale
        sink, dsink = new_sink, new_dsink
    f = float(np.dot(obs, np.real(np.diag(rho))))
    df = float(np.dot(obs, np.real(np.diag(drho))))
    return f, df


def gradient(sysm: evolve.System, rho0, n_steps, obs):
    """Full per-term gradient by one tangent pass per parameter (small N)."""
    p = n_params(sysm.wl)
    grad = np.zeros(p)
    f = None
    for i in range(p):
        e = np.zeros(p); e[i] = 1.0
        f, grad[i] = tangent(sysm, rho0, n_steps, obs, e)
    return f, grad


def perturbed(wl, dtheta, h):
    """Copy of a workload with per-term parameters moved by h * dtheta."""
    if wl.get("general"):
        return _perturbed_general(wl, dtheta, h)
    w = copy.deepcopy(wl)
    n_atoms = int(sum(wl["atoms"]))
    n_hops = len(wl["hops"])
    g = list(w["g"])
    hops = [list(x) for x in w["hops"]]
    jumps = [list(x) for x in w["jumps"]]
    for i, d in enumerate(dtheta):
        if d == 0.0:
            continue
        if i < n_atoms:
            g[i] += h * d
        elif i < n_atoms + n_hops:
            hops[i - n_atoms][2] += h * d
        else:
            jumps[i - n_atoms - n_hops][3] += h * d
    w["g"] = g
    w["hops"] = [tuple(x) for x in hops]
    w["jumps"] = [tuple(x) for x in jumps]
    return w


def _perturbed_general(wl, dtheta, h):
    """A general-form workload with its symmetric H entries and rates moved
    by h * dtheta (entries appended as extra triplets, which add up)."""
    w = copy.deepcopy(wl)
    pattern = general_pattern(wl)
    rows, cols, vals = (list(x) for x in wl["h"])
    for i, (r, c) in enumerate(pattern):
        d = dtheta[i]
        if d == 0.0:
            continue
        rows.append(r); cols.append(c); vals.append(h * d)
        if r != c:
            rows.append(c); cols.append(r); vals.append(h * d)
    w["h"] = (np.asarray(rows), np.asarray(cols), np.asarray(vals, float))
    jumps = [list(x) for x in wl["jumps"]]
    for j in range(len(jumps)):
        jumps[j][0] += h * dtheta[len(pattern) + j]
    w["jumps"] = [tuple(x) for x in jumps]
    return w


def finite_difference(wl, rho0, n_steps, obs, dtheta, h):
    """Central difference (f(theta + h d) - f(theta - h d)) / 2h."""
    vals = []
    make = evolve.GeneralSystem if wl.get("general") else evolve.System
    for s in (+1.0, -1.0):
        sysm = make(perturbed(wl, dtheta, s * h))
        rho, _ = evolve.evolve(sysm, rho0, n_steps)
        vals.append(float(np.dot(obs, np.real(np.diag(rho)))))
    return (vals[0] - vals[1]) / (2.0 * h)


def tied_direction(wl, name):
    """dtheta that moves every per-term parameter tied to a scalar knob
    ("g", "mu" or "gamma") by one unit."""
    n_atoms = int(sum(wl["atoms"]))
    n_hops = len(wl["hops"])
    d = np.zeros(n_params(wl))
    if name == "g":
        d[:n_atoms] = 1.0
    elif name == "mu":
        d[n_atoms:n_atoms + n_hops] = 1.0
    elif name == "gamma":
        d[n_atoms + n_hops:] = 1.0
    else:
        raise ValueError(name)
    return d
