"""Writes the stored expected values of the long oracle runs.

Only the CPU oracle is called.  Usage (from the repository root):

    python tests/golden/make_golden.py tch_chain3          # ~1 h on 8 cores
    python tests/golden/make_golden.py tch_chain3_blocks   # ~40 min on 8 cores

Outputs:

* tests/golden/tch_chain3.json: at the recorded steps, the diagonal of rho, a
  seeded sample of off-diagonal entries, the trace and the sink;
* tests/golden/tch_chain3_blocks.npz: whole 64 x 64 blocks of rho at steps
  1000 and 2000 (arrays ``blocks`` [block, 2 steps, 64, 64] complex128,
  ``block_rc`` the (row, column) of each block in units of 64, ``steps``,
  ``sink``, ``trace``), for blocks of every class a product tiling of the
  N = 1728 state has: diagonal blocks, interior blocks of the lower triangle,
  lower-triangle blocks past the first 256 tiles of 64 in row-major order (the
  k-split tail of a 64-tile lower-triangle product on 256 compute units),
  the corner block (26, 0) and upper-triangle blocks (mirror writes).
  Read with numpy.load(allow_pickle=False).
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

# (row, column) of the stored 64 x 64 blocks of the N = 1728 state (27 x 27
# blocks): diagonal; interior lower; lower-triangle tiles from row-major tile
# index 256 on ((22, 3) is index 256); upper triangle
CHAIN3_BLOCKS = [(0, 0), (13, 13), (21, 21), (22, 22), (26, 26),
                 (13, 5), (21, 0),
                 (22, 3), (24, 10), (26, 25), (26, 0),
                 (5, 13), (10, 24), (0, 26)]
CHAIN3_BLOCK_STEPS = (1000, 2000)


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


def run_blocks(wl, blocks, at_steps, path, bs=64):
    t0 = time.time()
    s = ev.System(wl)
    rho = W.initial_rho(wl, s.occ)
    sink = 0.0
    got = np.zeros((len(blocks), len(at_steps), bs, bs), dtype=np.complex128)
    sinks, traces = [], []
    for k in range(1, max(at_steps) + 1):
        rho, sink = ev.step(rho, sink, s.u, s.jumps, s.dt)
        if k in at_steps:
            i = list(at_steps).index(k)
            for b, (r, c) in enumerate(blocks):
                got[b, i] = rho[r * bs:(r + 1) * bs, c * bs:(c + 1) * bs]
            sinks.append(sink)
            traces.append(float(np.trace(rho).real))
            print(f"blocks: step {k} recorded ({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(path, blocks=got, block_rc=np.array(blocks, dtype=np.int64),
                        steps=np.array(at_steps, dtype=np.int64), sink=np.array(sinks),
                        trace=np.array(traces), n=np.int64(s.n), block=np.int64(bs))
    print("wrote", path, flush=True)


def main():
    which = sys.argv[1:] or ["tch_chain3"]
    if "tch_chain3" in which:
        wl = W.tch_chain3()
        run("tch_chain3", wl, {1, 10, 1000, wl["steps"]})
    if "tch_chain3_blocks" in which:
        run_blocks(W.tch_chain3(), CHAIN3_BLOCKS, CHAIN3_BLOCK_STEPS,
                   os.path.join(HERE, "tch_chain3_blocks.npz"))


if __name__ == "__main__":
    main()
