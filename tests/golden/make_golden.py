"""Writes the stored expected values of the long oracle runs.

Only the CPU oracle is called.  Usage (from the repository root):

    python tests/golden/make_golden.py tch_chain3     # ~1 h on 8 cores

Output: tests/golden/<name>.json with, at the recorded steps, the diagonal
of rho, a seeded sample of off-diagonal entries, the trace and the sink.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import evolve as ev  # noqa: E402

SAMPLE_SEED = 99
N_SAMPLE = 512


def sample_pairs(n, count, seed=SAMPLE_SEED):
    rng = np.random.default_rng(seed)
    return rng.integers(0, n, size=(count, 2))


def record(rho, sink, pairs):
    vals = rho[pairs[:, 0], pairs[:, 1]]
    return {
        "diag": np.real(np.diag(rho)).tolist(),
        "sample_re": np.real(vals).tolist(),
        "sample_im": np.imag(vals).tolist(),
        "trace": float(np.trace(rho).real),
        "sink": float(sink),
    }


def run(name, wl, record_at):
    t0 = time.time()
    s = ev.System(wl)
    rho = W.initial_rho(wl, s.occ)
    pairs = sample_pairs(s.n, N_SAMPLE)
    out = {"workload": name, "n": s.n, "steps": wl["steps"], "dt": wl["dt"],
           "pairs": pairs.tolist(), "records": {}}
    sink = 0.0
    for k in range(1, wl["steps"] + 1):
        rho, sink = ev.step(rho, sink, s.u, s.jumps, s.dt)
        if k in record_at:
            out["records"][str(k)] = record(rho, sink, pairs)
            print(f"{name}: step {k} recorded ({time.time() - t0:.0f} s)", flush=True)
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, flush=True)


def main():
    which = sys.argv[1:] or ["tch_chain3"]
    if "tch_chain3" in which:
        wl = W.tch_chain3()
        run("tch_chain3", wl, {1, 10, 1000, wl["steps"]})


if __name__ == "__main__":
    main()
