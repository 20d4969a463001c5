"""Seeded synthetic workloads for the cavity-QED master-equation solver.

This module only *describes* inputs: system structure (cavities, atoms,
photon caps, excitation window), Hamiltonian parameters (omega, g, hopping mu),
decoherence channels (kind, site, rate gamma), time step, step count and the
initial state.  It holds none of the method's arithmetic; both the CPU oracle
and the GPU library consume these descriptions and build their own basis,
Hamiltonian and propagator from them.

All random draws use ``numpy.random.default_rng(20240311 + k)`` for workload k.

A workload is a plain dict::

    {
      "name": str,
      "atoms": [m_c per cavity], "photon_cap": [cap_c per cavity],
      "exc_min": int, "exc_max": int (-1: no excitation window),
      "omega_c": [per cavity], "omega_a": [per atom], "g": [per atom],
      "hops": [(c, d, mu)], "jumps": [(kind, cavity, atom, gamma)],
      "dt": float, "steps": int, "init": {...}
    }

Atoms are numbered cavity-major (all atoms of cavity 0, then cavity 1, ...).
Jump kinds: 0 photon leak a_c, 1 atom decay sigma_ck, 2 atom dephasing
sigma_ck^dag sigma_ck (the decoherence operators A_j of the Lindblad term,
Sec. II, Eq. 3).  The Hamiltonian form these parameters feed is the
Jaynes-/Tavis-Cummings-Hubbard form of Sec. IV (Eq. 8b on-site coupling,
Eq. 12 hopping).
"""
from __future__ import annotations

import numpy as np

PHOTON_LEAK = 0
ATOM_DECAY = 1
ATOM_DEPHASE = 2

SEED_BASE = 20240311


def rng_for(k: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + k)


def _uniform_params(atoms, omega=1.0, g=0.01):
    n_atoms = int(sum(atoms))
    return ([omega] * len(atoms), [omega] * n_atoms, [g] * n_atoms)


def _chain_hops(n_cav, mu):
    return [(c, c + 1, mu) for c in range(n_cav - 1)]


def jc_single(g=0.01, gamma=0.001, cap=3, dt=0.01, steps=10000, omega=1.0):
    """Workload 1: one cavity, one two-level atom, photon cap 3 (N = 8),
    start |1 photon, atom ground>, photon leak a with rate gamma."""
    oc, oa, gg = _uniform_params([1], omega, g)
    return {
        "name": "jc_n8",
        "atoms": [1], "photon_cap": [cap], "exc_min": 0, "exc_max": -1,
        "omega_c": oc, "omega_a": oa, "g": gg,
        "hops": [], "jumps": [(PHOTON_LEAK, 0, -1, gamma)] if gamma > 0 else [],
        "dt": dt, "steps": steps,
        "init": {"kind": "basis", "occ": {("photon", 0): 1}},
    }


def tch_2x2(dt=0.01, steps=5000):
    """Workload 2: Tavis-Cummings-Hubbard, 2 cavities x 2 atoms, cap 2
    (N = 144), g = 0.01, hopping mu = 0.005, leak 0.001 per cavity, seeded
    Haar-random pure initial state."""
    atoms = [2, 2]
    oc, oa, gg = _uniform_params(atoms)
    return {
        "name": "tch_2x2_n144",
        "atoms": atoms, "photon_cap": [2, 2], "exc_min": 0, "exc_max": -1,
        "omega_c": oc, "omega_a": oa, "g": gg,
        "hops": _chain_hops(2, 0.005),
        "jumps": [(PHOTON_LEAK, c, -1, 0.001) for c in range(2)],
        "dt": dt, "steps": steps,
        "init": {"kind": "haar", "seed": SEED_BASE + 2},
    }


def tch_chain3(dt=0.005, steps=2000):
    """Workload 3: TCH chain of 3 cavities x 1 atom, cap 5 (N = 1728);
    g_k ~ U(0.005, 0.02) seeded, mu = 0.005, leak 0.001 per cavity and atom
    dephasing 0.0005 per atom; seeded Haar-random pure initial state."""
    rng = rng_for(3)
    atoms = [1, 1, 1]
    g = [float(x) for x in rng.uniform(0.005, 0.02, size=3)]
    return {
        "name": "tch_chain3_n1728",
        "atoms": atoms, "photon_cap": [5, 5, 5], "exc_min": 0, "exc_max": -1,
        "omega_c": [1.0] * 3, "omega_a": [1.0] * 3, "g": g,
        "hops": _chain_hops(3, 0.005),
        "jumps": [(PHOTON_LEAK, c, -1, 0.001) for c in range(3)]
        + [(ATOM_DEPHASE, c, 0, 0.0005) for c in range(3)],
        "dt": dt, "steps": steps,
        "init": {"kind": "haar", "seed": SEED_BASE + 3},
    }


def lattice_sites(length, height):
    """Row-major site numbering: site (i, j) -> i * height + j."""
    return [(i, j) for i in range(length) for j in range(height)]


def lattice_hops(length, height, mu):
    """Unordered nearest-neighbour pairs (|di| + |dj| = 1), open boundary."""
    hops = []
    for i in range(length):
        for j in range(height):
            s = i * height + j
            if i + 1 < length:
                hops.append((s, (i + 1) * height + j, mu))
            if j + 1 < height:
                hops.append((s, i * height + j + 1, mu))
    return hops


def lattice_boundary(length, height):
    return [i * height + j for i in range(length) for j in range(height)
            if i in (0, length - 1) or j in (0, height - 1)]


def photon_lattice(length=32, height=32, mu=0.01, g=0.01, gamma=0.001,
                   dt=0.01, steps=1000, atoms_per_site=1, start=None):
    """Workload 4: 2D photon motion on a length x height lattice of cavities
    with one two-level atom each, single-excitation window (N = 2048 for
    32 x 32), hopping mu, coupling g, photon leak on boundary sites, photon
    initially at site (16, 16).  With atoms_per_site = 0 this is the
    photon-only lattice of Sec. IV.B."""
    n_cav = length * height
    atoms = [atoms_per_site] * n_cav
    oc, oa, gg = _uniform_params(atoms, 1.0, g)
    if start is None:
        start = (length // 2, height // 2)
    site = start[0] * height + start[1]
    return {
        "name": f"lattice_{length}x{height}",
        "atoms": atoms, "photon_cap": [1] * n_cav, "exc_min": 1, "exc_max": 1,
        "omega_c": oc, "omega_a": oa, "g": gg,
        "hops": lattice_hops(length, height, mu),
        "jumps": [(PHOTON_LEAK, c, -1, gamma) for c in lattice_boundary(length, height)]
        if gamma > 0 else [],
        "dt": dt, "steps": steps,
        "init": {"kind": "basis", "occ": {("photon", site): 1}},
        "lattice": (length, height), "centre_site": site,
    }


def photon_plane(start=(40, 0), zeta=0.2, omega=1.0, dt=0.25, steps=1000):
    """The paper's 2D photon motion (Sec. IV.B): an 81 x 51 plane of cavities
    without atoms, one photon (N = 4131), hopping zeta, closed (no leak),
    start (40, 0) (symmetric) or (20, 0) (asymmetric).  The paper does not
    give omega, zeta, dt or the step count; with these, 1000 steps carry the
    wavefront about 2 zeta t = 100 sites, past the boundaries and back."""
    wl = photon_lattice(81, 51, mu=zeta, g=0.0, gamma=0.0, dt=dt, steps=steps,
                        atoms_per_site=0, start=start)
    wl["omega_c"] = [omega] * (81 * 51)
    wl["name"] = f"photon_plane_81x51_{start[0]}_{start[1]}"
    return wl


# structures of the batched sweep, keyed by N (all photon caps 3, chain hops)
BATCH_STRUCTURES = {64: [1, 1], 128: [1, 2], 256: [2, 2], 512: [1, 1, 1]}


def batch_sweep(per_size=64, steps=500, dt=0.01, sizes=(64, 128, 256, 512)):
    """Workload 5: uneven-size TCH instances (per_size of each N), shuffled
    by seed; per instance one scalar g ~ U(0.005, 0.02), mu ~ U(0.001, 0.01),
    gamma ~ U(0.0005, 0.002) shared by all atoms / hops / cavity leaks;
    start: one photon in cavity 0, atoms in the ground state."""
    rng = rng_for(5)
    order = np.repeat(np.array(sizes), per_size)
    rng.shuffle(order)
    out = []
    for idx, n in enumerate(order):
        atoms = BATCH_STRUCTURES[int(n)]
        g = float(rng.uniform(0.005, 0.02))
        mu = float(rng.uniform(0.001, 0.01))
        gamma = float(rng.uniform(0.0005, 0.002))
        n_cav = len(atoms)
        out.append({
            "name": f"batch_{idx}_n{int(n)}",
            "atoms": list(atoms), "photon_cap": [3] * n_cav,
            "exc_min": 0, "exc_max": -1,
            "omega_c": [1.0] * n_cav, "omega_a": [1.0] * int(sum(atoms)),
            "g": [g] * int(sum(atoms)),
            "hops": _chain_hops(n_cav, mu),
            "jumps": [(PHOTON_LEAK, c, -1, gamma) for c in range(n_cav)],
            "dt": dt, "steps": steps,
            "init": {"kind": "basis", "occ": {("photon", 0): 1}},
            "expected_n": int(n),
            "tied": {"g": g, "mu": mu, "gamma": gamma},
        })
    return out


def workload(k: int, **kw):
    return {1: jc_single, 2: tch_2x2, 3: tch_chain3, 4: photon_lattice}[k](**kw)


# ----------------------------------------------------------------------------
# initial states


def mode_list(atoms):
    """Mode order: for cavity c, its photon mode, then its atoms."""
    modes = []
    for c, m in enumerate(atoms):
        modes.append(("photon", c))
        for k in range(m):
            modes.append(("atom", c, k))
    return modes


def haar_psi(n: int, seed: int) -> np.ndarray:
    """Normalised complex Gaussian vector (Haar-random pure state)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return v / np.linalg.norm(v)


def initial_psi(wl: dict, occ: np.ndarray) -> np.ndarray:
    """State vector of the workload's initial pure state in the basis whose
    occupation table (N x n_modes, one row per basis state) is ``occ``."""
    n = occ.shape[0]
    init = wl["init"]
    if init["kind"] == "haar":
        return haar_psi(n, init["seed"])
    if init["kind"] == "basis":
        modes = mode_list(wl["atoms"])
        want = np.zeros(len(modes), dtype=np.int64)
        for key, level in init["occ"].items():
            want[modes.index(key)] = level
        hit = np.nonzero((occ == want[None, :]).all(axis=1))[0]
        if len(hit) != 1:
            raise ValueError("initial basis state not in the basis")
        psi = np.zeros(n, dtype=np.complex128)
        psi[hit[0]] = 1.0
        return psi
    raise ValueError(init["kind"])


def initial_rho(wl: dict, occ: np.ndarray) -> np.ndarray:
    psi = initial_psi(wl, occ)
    return np.outer(psi, psi.conj())


def tied_parameter_maps(wl: dict):
    """Index lists that tie per-term gradients (g per atom, mu per hop,
    gamma per jump, in that order) into the workload's scalar knobs."""
    n_atoms = int(sum(wl["atoms"]))
    n_hops = len(wl["hops"])
    n_jumps = len(wl["jumps"])
    return {
        "g": list(range(0, n_atoms)),
        "mu": list(range(n_atoms, n_atoms + n_hops)),
        "gamma": list(range(n_atoms + n_hops, n_atoms + n_hops + n_jumps)),
    }
