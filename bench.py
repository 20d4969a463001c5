#!/usr/bin/env python3
"""Throughput of the quantum-master-equation time step on one MI355X.

Workload: 2D photon motion (Sec. IV.B) on a 32 x 32 lattice of cavities with
one two-level atom each, single-excitation subspace (N = 2048), hopping
mu = 0.01, coupling g = 0.01, photon leak 0.001 on the 124 boundary sites,
dt = 0.01, photon started at site (16, 16).  One "step" is one full time step
of the method: rho_u = U rho U^dag as two planar complex MFMA products (the
first T = rho + dU rho, the second on the lower-triangle tiles only), the
decoherence step, the FP64 symmetrisation, trace and sink, and the
renormalisation.  Every boundary leak maps the single-excitation basis out of
itself, so the decoherence step is one factor per element: it runs in the
lower-triangle product's epilogue ("folded" steps), the one-workgroup FP64
trace pass computes the renormalisation factor from the stored diagonal, and
the next step's first product applies it.  Inputs are resident in HBM before
the timed region starts.

Prints one JSON line (rank 0, N = 1): value = FP32 time steps per second from
a run with no profiling, plus the FP64 and split-BF16x3 rates, per-kernel
durations from a second, profiled run of the same steps (every 8th step's
kernels launched with start / stop events stamped by their own dispatch),
the roofline entry of the dominant kernel (the first product) and the CPU
oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QME steps/sec at N=2048 (FP32 MFMA vs FP64) + adjoint grad time/step"
PEAK_FP32_MFMA = 157.3      # TFLOP/s, MI355X dense FP32 matrix
PEAK_FP64_MFMA = 78.6       # TFLOP/s, MI355X dense FP64 matrix
PEAK_BF16_MFMA = 2500.0     # TFLOP/s, MI355X dense bf16 matrix
PEAK_HBM = 8000.0           # GB/s

# HBM bytes per launch of the first FP32 product, from the FETCH_SIZE /
# WRITE_SIZE counters (scaled by a plain-copy calibration) recorded in
# profiles/cgemm_f32_lattice_n2048_hbm_counters.md for this source hash of
# the kernel's sources; reported as null once they differ.
TRAFFIC_FP32_PRODUCT = {"bytes": 275295.0 * 1024,
                        "sha256": "40983a9412742329d3f48aa538ab647a095912872d7d900097592fb380a469f8",
                        "source": "profiles/cgemm_f32_lattice_n2048_hbm_counters.md"}
KERNEL_SOURCES = ("cgemm.hip", "cgemm_tile.hpp", "dissipate_tile.hpp")


def measured_traffic():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2403_07042_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return TRAFFIC_FP32_PRODUCT["bytes"] if h.hexdigest() == TRAFFIC_FP32_PRODUCT["sha256"] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--fp64-steps", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=15,
                    help="oracle steps timed for the CPU baseline (0: skip)")
    ap.add_argument("--legs", default="fp32,fp64,bf16x3", help="comma list of fp32, fp64, bf16x3")
    ap.add_argument("--bf16x3-steps", type=int, default=1000)
    ap.add_argument("--adjoint-steps", type=int, default=200,
                    help="steps of the timed FP32 adjoint (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=500,
                    help="steps of the batched sweep of 256 uneven instances (0: skip)")
    ap.add_argument("--latency", type=int, default=1,
                    help="time the latency-bound N = 8 and N = 144 workloads (0: skip)")
    ap.add_argument("--configs", type=int, default=1,
                    help="time FP32 / BF16x3 / FP64 on the N = 144 and N = 1728 configurations (0: skip)")
    ap.add_argument("--config-steps", type=int, default=0,
                    help="steps per precision there (0: 2000 at N = 144, 200 at N = 1728)")
    ap.add_argument("--selection", type=int, default=1,
                    help="time the state-space selection loop on the N = 2048 lattice (0: skip)")
    ap.add_argument("--plane-steps", type=int, default=100,
                    help="steps timed on the N = 4131 photon plane (0: skip)")
    ap.add_argument("--pure-steps", type=int, default=2000,
                    help="steps timed on the N = 4131 plane in pure-state form (0: skip)")
    ap.add_argument("--hb-steps", type=int, default=100,
                    help="steps timed on the N = 4096 hydrogen-bond model (0: skip)")
    ap.add_argument("--checkpoint-every", type=int, default=32)
    ap.add_argument("--adjoint-all-resident", type=int, default=1,
                    help="also time the adjoint with every state kept in HBM (no recompute)")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="MiB moved by one plain device copy after the legs (counter calibration)")
    ap.add_argument("--tiles32", default="", help="tile1,tile2 override for the FP32 leg")
    ap.add_argument("--tiles64", default="", help="tile1,tile2 override for the FP64 leg")
    return ap.parse_args()


PROFILE_EVERY = 8


def timed_leg(P, W, torch, wl, precision, steps, warmup, tiles="", tune=False):
    """steps/s of `steps` time steps with no profiling (the throughput), then
    the same steps again from the same state with per-kernel events on every
    PROFILE_EVERY-th step (the kernel durations).  tune: tile pair and split
    picked first by the autotuner (timed on a scratch state, no cache)."""
    occ = P.basis(wl)
    rho0 = W.initial_rho(wl, occ)
    sol = P.Solver(wl, precision)
    if tiles:
        sol.set_tiles(*[int(x) for x in tiles.split(",")])
    sol.set_rho(rho0)
    tuned = None
    if tune:
        from paper_2403_07042_amd import autotune as A
        tuned = A.tune_solver(sol, steps=8, trials=3, use_cache=False)
    sol.step(warmup)
    torch.cuda.synchronize()
    sol.set_rho(rho0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pops, trace, sink = sol.observe()
    # profiled pass: each sampled step's kernels carry start / stop events
    # stamped by their own dispatch, so a duration is the kernel alone
    sol.set_rho(rho0)
    sol.profile(PROFILE_EVERY)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    sol.step(steps)
    torch.cuda.synchronize()
    p1 = time.perf_counter()
    prof = sol.profile_read()
    sol.profile(False)
    # per sampled step (one first product each): a kind launched on fewer
    # steps (the folded steps' trace, once per call) counts at its share
    sampled = max(prof["product_full"][1], 1)
    kern = {k: (1e3 * ms / sampled) for k, (ms, cnt) in prof.items()}
    out = {
        "seconds": t1 - t0,
        "steps_per_s": steps / (t1 - t0),
        "ms_per_step": 1e3 * (t1 - t0) / steps,
        "kernels_us": kern,
        "kernels_us_sum": sum(kern.values()),
        "profiled_ms_per_step": 1e3 * (p1 - p0) / steps,
        "tiles": tiles or ("autotuned" if tune else "default"),
        "tile1": sol.tile1,
        "tile2": sol.tile2,
        "tuned_split": None if tuned is None else bool(tuned[2]),
        "pops": pops, "trace": trace, "sink": sink, "n": sol.n, "ld": sol.ld,
    }
    sol.close()
    return out


# Real flops the matrix cores execute per complex multiply-add: the FP32 and
# FP64 products use three real products (Gauss's 3M form), 2 flop each.
MFMA_FLOP_PER_CMAC = 6.0


def lower_flops(leg):
    """MFMA flops the lower-triangle product executes: every tile on or below
    the diagonal (tile edge t2, padding included)."""
    ld, t2 = leg["ld"], leg["tile2"]
    t = ld // t2
    return MFMA_FLOP_PER_CMAC * ld * t2 * t2 * t * (t + 1) / 2


def executed_flops(leg):
    """Flops one step executes on the matrix cores: the full product plus the
    lower-triangle tiles."""
    return MFMA_FLOP_PER_CMAC * leg["ld"] ** 3 + lower_flops(leg)


def adjoint_leg(P, W, torch, wl, steps, every):
    """Wall time of one qme_adjoint call (forward with checkpoints, segment
    recompute, three adjoint products per step, FP64 finalisation) for the
    centre photon population, per step; and the tied gradients it returns."""
    import numpy as np
    occ = P.basis(wl)
    site = wl["centre_site"]
    obs = np.zeros(occ.shape[0])
    obs[int(np.nonzero(occ[:, 2 * site] == 1)[0][0])] = 1.0
    sol = P.Solver(wl, "fp32")
    sol.set_rho(W.initial_rho(wl, occ))
    sol.adjoint(min(steps, 8), obs, every)      # warm-up (allocations, kernels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f, g = sol.adjoint(steps, obs, every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sol.close()
    maps = W.tied_parameter_maps(wl)
    return {"ms_per_step": 1e3 * (t1 - t0) / steps, "steps": steps, "checkpoint_every": every,
            "value": f, "dvalue_dmu": float(g[maps["mu"]].sum()),
            "dvalue_dg": float(g[maps["g"]].sum())}


def batch_leg(P, W, torch, steps):
    """256 TCH instances (64 each of N = 64, 128, 256, 512), FP32, one graph
    replay of `steps` batched steps (one launch per phase over all
    instances), with the tile edges per size, graph replay and instance
    order picked by the autotuner first."""
    from paper_2403_07042_amd import autotune as A
    wls = W.batch_sweep(steps=steps)
    sols = []
    for wl in wls:
        s = P.Solver(wl, "fp32")
        s.set_rho(W.initial_rho(wl, P.basis(wl)))
        sols.append(s)
    b = P.Batch(sols)
    (use_graph, largest, per_n), tune = A.tune_batch(b, steps=4, trials=3)
    for wl, s in zip(wls, sols):
        s.set_rho(W.initial_rho(wl, P.basis(wl)))
    b.step(steps)                    # capture + warm-up run
    torch.cuda.synchronize()
    for wl, s in zip(wls, sols):
        s.set_rho(W.initial_rho(wl, P.basis(wl)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    flops = sum(16.0 * s.n ** 3 for s in sols)
    # what the matrix cores execute per batched step: both products of every
    # instance in the 3M form (6 flop per complex multiply-add) over its padded
    # ld, the lower product over its lower-triangle tiles
    executed = 0.0
    for s in sols:
        t1_, t2_ = s.tiles
        k = s.ld // t2_
        executed += MFMA_FLOP_PER_CMAC * (s.ld ** 3 + s.ld * t2_ * t2_ * k * (k + 1) / 2)
    b.close()
    for s in sols:
        s.close()
    rate = steps / (t1 - t0)
    return {"instances": len(wls), "steps": steps, "batched_steps_per_s": rate,
            "tuned": {"use_graph": use_graph, "largest_first": largest,
                      "tiles_per_n": {str(n): list(t) for n, t in sorted(per_n.items())}},
            "executed_tflops": executed * rate / 1e12,
            "executed_frac_of_fp32_peak": executed * rate / 1e12 / PEAK_FP32_MFMA,
            "instance_steps_per_s": rate * len(wls), "ms_per_batched_step": 1e3 / rate,
            "dense_equivalent_tflops": flops * rate / 1e12,
            "dense_equivalent_frac_of_fp32_peak": flops * rate / 1e12 / PEAK_FP32_MFMA}


def _timed(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def latency_leg(P, W, torch, warmup=20):
    """The launch-latency-bound workloads: the Jaynes-Cummings model (N = 8,
    FP64, 10000 steps) on the single-workgroup path and on the four-launch
    step; the 2 x 2 Tavis-Cummings-Hubbard model (N = 144, FP32, 5000 steps)
    stepped eagerly, replayed from a captured hipGraph of the whole run
    (qme_set_graph), and as a one-instance batch replayed from a hipGraph."""
    out = {}
    wl = W.jc_single()
    rho0 = W.initial_rho(wl, P.basis(wl))
    for fused in (True, False):
        sol = P.Solver(wl, "fp64")
        sol.set_fused(fused)
        sol.set_rho(rho0)
        sol.step(warmup)
        sol.set_rho(rho0)
        dt = _timed(torch, lambda: sol.step(wl["steps"]))
        sol.close()
        out["jc_n8_fp64_" + ("single_launch" if fused else "four_launch")] = {
            "steps": wl["steps"], "steps_per_s": wl["steps"] / dt}
    wl = W.tch_2x2()
    rho0 = W.initial_rho(wl, P.basis(wl))
    sol = P.Solver(wl, "fp32")
    sol.set_rho(rho0)
    sol.step(warmup)
    sol.set_rho(rho0)
    dt = _timed(torch, lambda: sol.step(wl["steps"]))
    out["tch_n144_fp32_eager"] = {"steps": wl["steps"], "steps_per_s": wl["steps"] / dt}
    sol.set_graph(True)
    sol.set_rho(rho0)
    sol.step(wl["steps"])                    # capture + warm-up run
    sol.set_rho(rho0)
    dt = _timed(torch, lambda: sol.step(wl["steps"]))
    out["tch_n144_fp32_graph"] = {"steps": wl["steps"], "steps_per_s": wl["steps"] / dt}
    sol.set_graph(False)
    b = P.Batch([sol])
    b.config(use_graph=True, largest_first=True)
    b.step(wl["steps"])                      # capture + warm-up run
    sol.set_rho(rho0)
    dt = _timed(torch, lambda: b.step(wl["steps"]))
    out["tch_n144_fp32_batch_graph"] = {"steps": wl["steps"], "steps_per_s": wl["steps"] / dt}
    b.close()
    sol.close()
    return out


def selection_leg(P, W, torch, steps=1000, eps=1e-20):
    """State-space selection (Sec. III.B) on the N = 2048 lattice, FP32,
    compared after every step: the first solve (step, populations, selection,
    subset context with its propagator, compaction), then the remaining steps
    on the selected basis with a comparison after each, decided on the host
    and, again, on the device with the next solve queued ahead; plus the
    compaction kernel alone on a half-size gather of the full state (HIP
    events)."""
    wl = W.photon_lattice(steps=steps)
    occ = P.basis(wl)
    rho0 = W.initial_rho(wl, occ)
    sol = P.Solver(wl, "fp32")
    sol.set_rho(rho0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out, kept, sizes = P.evolve_with_selection(sol, 1, eps, 1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out2, kept2, sizes2 = P.evolve_with_selection(out, steps - 1, eps, 1)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    final_n = sizes2[-1] if sizes2 else sizes[-1]
    if out2 is not out:
        out2.close()
    if out is not sol:
        out.close()
    # the same loop with the decisions on the device, one solve queued ahead
    sol.set_rho(rho0)
    out, _, _ = P.evolve_with_selection(sol, 1, eps, 1, device=True)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    out2, _, sizes3 = P.evolve_with_selection(out, steps - 1, eps, 1, device=True)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    same = sizes3 == sizes2
    if out2 is not out:
        out2.close()
    if out is not sol:
        out.close()
    # compaction kernel: keep every other state of the full 2048 basis
    sol.set_rho(rho0)
    sub = sol.subspace(np.arange(0, sol.n, 2))
    sol.compact_into(sub)                       # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        sol.compact_into(sub)
    e1.record()
    torch.cuda.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / reps
    moved = 2 * 4 * sub.n * sub.n * 2           # FP32 re+im gathered and written
    sub.close()
    sol.close()
    return {"workload": "jch_lattice_32x32_n2048", "precision": "fp32", "eps": eps,
            "steps": steps, "compare_every": 1, "basis_after_first_solve": sizes[0],
            "final_basis": int(final_n),
            "first_solve_s": t1 - t0, "remaining_steps_per_s": (steps - 1) / (t2 - t1),
            "remaining_steps_per_s_device_decision": (steps - 1) / (t4 - t3),
            "device_decision_same_sizes": same,
            "compact_2048_to_1024_us": us, "compact_gbs": moved / (us * 1e-6) / 1e9}


def configs_leg(P, W, torch, warmup=10, steps_override=0):
    """FP32, split-BF16x3 and plain FP64 steps/s, with the speedups over FP64,
    on the other parity configurations: the 2 x 2 Tavis-Cummings-Hubbard
    model (N = 144, 2000 steps) and the three-cavity chain (N = 1728, 200
    steps), each context's tile pair and split picked by the autotuner;
    steps_override > 0 runs that many steps on both."""
    out = {}
    for name, wl, steps in (("tch_2x2_n144", W.tch_2x2(), steps_override or 2000),
                            ("tch_chain3_n1728", W.tch_chain3(), steps_override or 200)):
        rates, picked = {}, {}
        for prec in ("fp32", "bf16x3", "fp64"):
            leg = timed_leg(P, W, torch, wl, prec, steps, warmup, tune=True)
            rates[prec] = leg["steps_per_s"]
            picked[prec] = {"tiles": [leg["tile1"], leg["tile2"]], "split": leg["tuned_split"]}
        out[name] = {"steps": steps, "steps_per_s": rates, "autotuned": picked,
                     "fp32_speedup_over_fp64": rates["fp32"] / rates["fp64"],
                     "bf16x3_speedup_over_fp64": rates["bf16x3"] / rates["fp64"]}
    return out


def plane_leg(P, W, torch, steps=100, warmup=5):
    """The paper's own 2D photon-motion plane (81 x 51 cavities, one photon,
    N = 4131, ld = 4160), FP32, symmetric start: steps/s and per-kernel
    durations (HIP events on the launch stream)."""
    wl = W.photon_plane(steps=steps)
    out = timed_leg(P, W, torch, wl, "fp32", steps, warmup)
    flops = executed_flops(out)
    return {"workload": "photon_plane_81x51_n4131", "precision": "fp32", "N": out["n"],
            "ld": out["ld"], "steps": steps, "steps_per_s": out["steps_per_s"],
            "ms_per_step": out["ms_per_step"], "kernels_us": out["kernels_us"],
            "executed_tflops": flops * out["steps_per_s"] / 1e12,
            "executed_frac_of_fp32_peak": flops * out["steps_per_s"] / 1e12 / PEAK_FP32_MFMA}


def pure_leg(P, W, torch, steps=2000, warmup=20):
    """The same plane as a pure state (qme_pure_step: psi <- U psi / |psi|,
    one launch per step), FP32 and FP64: steps/s from HIP events on the
    launch stream, and the dU bytes each step streams (algorithmic: 2 planes
    of N x N, the padding columns of each row excluded) against the HBM
    peak.  The final states are kept (key "_psi") for the parity check of the
    CPU-baseline leg."""
    wl = W.photon_plane()
    occ = P.basis(wl)
    site = np.argmax(occ, axis=1)
    psi0 = W.initial_psi(wl, occ)
    out = {"workload": "photon_plane_81x51_n4131_pure_state", "steps": steps}
    for prec in ("fp32", "fp64"):
        sol = P.Solver(wl, prec)
        sol.set_psi(psi0)
        sol.step_pure(warmup)
        sol.set_psi(psi0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        sol.step_pure(steps)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        us = 1e3 * e0.elapsed_time(e1) / steps
        per_step = 2.0 * sol.elem * sol.n * sol.n
        out[prec] = {"steps_per_s": steps / wall, "us_per_step": us,
                     "du_bytes_per_step": per_step,
                     "achieved_tb_s": per_step / (us * 1e-6) / 1e12,
                     "frac_of_hbm_peak": per_step / (us * 1e-6) / 1e9 / PEAK_HBM,
                     "_psi": (sol.get_psi(), site, wl)}
        sol.close()
    return out


def hydrogen_bond_leg(P, torch, steps=100, warmup=5):
    """The hydrogen-bond model of Sec. IV.A with two bonds (three molecules,
    N = 4096), built as a general-form model: FP32 steps/s, and the basis
    left by the state-space selection loop (compared every 10 steps over
    200 steps) at the two epsilons of Table I."""
    from workloads import hydrogen_bond as hb
    wl = hb.hb_model(2, steps=steps)
    rho0 = hb.initial_rho(wl)
    sol = P.Solver(wl, "fp32")
    sol.set_rho(rho0)
    sol.step(warmup)
    sol.set_rho(rho0)
    dt = _timed(torch, lambda: sol.step(steps))
    sol.set_rho(rho0)                     # profiled pass of the same steps
    sol.profile(PROFILE_EVERY)
    _timed(torch, lambda: sol.step(steps))
    prof = sol.profile_read()
    sol.profile(False)
    sizes = {}
    for eps in (1e-35, 1e-20):
        sol.set_rho(rho0)
        out, kept, hist = P.evolve_with_selection(sol, 200, eps, 10)
        sizes[str(eps)] = int(hist[-1])
        if out is not sol:
            out.close()
    sol.close()
    return {"workload": "hydrogen_bond_3_molecules_n4096", "precision": "fp32", "N": wl["n"],
            "steps": steps, "steps_per_s": steps / dt, "ms_per_step": 1e3 * dt / steps,
            "kernels_us": {k: (1e3 * ms / max(cnt, 1)) for k, (ms, cnt) in prof.items()},
            "selected_basis_after_200_steps": sizes}


def cpu_baseline(W, wl, gpu_leg, steps, pure=None):
    """The CPU oracle (NumPy complex128) timed on the host cores on a bounded
    sample of the same workload, plus the parity of the GPU run's final
    populations with the lattice's closed form (and of the pure-state plane
    runs, when given, with the plane's closed form)."""
    from oracle import closed_forms as cf
    from oracle import evolve as ev
    blas = "unknown"
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        info = [p for p in threadpool_info() if p.get("user_api") == "blas"] or threadpool_info()
        threads = max([p.get("num_threads", 1) for p in info] or [1])
        if info:
            blas = f"{info[0].get('internal_api', '?')} {info[0].get('version', '')}".strip()
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count() or 1
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next(ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name"))
    except Exception:
        pass
    s = ev.System(wl)
    rho0 = W.initial_rho(wl, s.occ)

    def run(k):
        rho, sink = rho0, 0.0
        t0 = time.perf_counter()
        for _ in range(k):
            rho, sink = ev.step(rho, sink, s.u, s.jumps, s.dt)
        return k / (time.perf_counter() - t0)

    rate = run(steps)
    base = {"value": rate, "unit": "steps/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{steps} time steps of the N=2048 lattice workload (NumPy complex128, "
                      f"BLAS threads={threads}); propagator build excluded",
            "host": {"cpu_model": cpu_model, "nproc": os.cpu_count(), "blas": blas}}
    if threadpool_limits is not None and steps > 0:
        with threadpool_limits(limits=1, user_api="blas"):
            base["single_thread"] = {"value": run(1), "unit": "steps/s", "steps": 1}
    parity = None
    if gpu_leg is not None:
        k = gpu_leg["k"]
        ref = cf.lattice_rho(s.occ, 1, 32, 32, 0.01, 0.01, 1.0, k * wl["dt"], wl["centre_site"])
        import numpy as np
        dpop = float(np.abs(gpu_leg["pops"] - np.real(np.diag(ref))).max())
        parity = {"after_steps": k, "max_abs_dpop_vs_closed_form": dpop,
                  "trace_error": abs(gpu_leg["trace"] - (1.0 - gpu_leg["sink"]))}
    if pure is not None:
        import numpy as np
        for prec in ("fp32", "fp64"):
            psi, site, pwl = pure[prec].pop("_psi")
            photon, _ = cf.lattice_amplitudes(81, 51, pwl["hops"][0][2], 0.0, pwl["omega_c"][0],
                                              pure["steps"] * pwl["dt"], pwl["centre_site"],
                                              with_atoms=False)
            pure[prec]["max_abs_dpsi_vs_closed_form"] = float(np.abs(psi - photon[site]).max())
    return base, parity


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the solver is single-GPU); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2403_07042_amd as P
    import workloads as W

    legs = [x.strip() for x in args.legs.split(",") if x.strip()]
    wl = W.photon_lattice(steps=args.steps)
    n = 2048
    flops_product = 8.0 * n ** 3          # one complex N^3 product
    flops_step = 2 * flops_product        # 16 N^3: both products counted dense
    res = {}
    if "fp32" in legs:
        res["fp32"] = timed_leg(P, W, torch, wl, "fp32", args.steps, args.warmup, args.tiles32)
    if "bf16x3" in legs and args.bf16x3_steps > 0:
        res["bf16x3"] = timed_leg(P, W, torch, wl, "bf16x3", args.bf16x3_steps, args.warmup)
    if "fp64" in legs and args.fp64_steps > 0:
        res["fp64"] = timed_leg(P, W, torch, wl, "fp64", args.fp64_steps, min(args.warmup, 5),
                                args.tiles64)

    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    batch = batch_leg(P, W, torch, args.batch_steps) if args.batch_steps > 0 else None
    latency = latency_leg(P, W, torch) if args.latency else None
    configs = configs_leg(P, W, torch, steps_override=args.config_steps) if args.configs else None
    selection = selection_leg(P, W, torch) if args.selection else None
    plane = plane_leg(P, W, torch, args.plane_steps) if args.plane_steps > 0 else None
    pure = pure_leg(P, W, torch, args.pure_steps) if args.pure_steps > 0 else None
    hbond = hydrogen_bond_leg(P, torch, args.hb_steps) if args.hb_steps > 0 else None

    adj = None
    if args.adjoint_steps > 0:
        adj = adjoint_leg(P, W, torch, wl, args.adjoint_steps, args.checkpoint_every)
        if args.adjoint_all_resident:
            full = adjoint_leg(P, W, torch, wl, args.adjoint_steps, args.adjoint_steps)
            adj["all_resident_ms_per_step"] = full["ms_per_step"]
            adj["all_resident_matches"] = (full["dvalue_dmu"] == adj["dvalue_dmu"]
                                           and full["dvalue_dg"] == adj["dvalue_dg"])

    if "fp32" not in res and "fp64" not in res:
        print(json.dumps({"metric": METRIC, "value": None,
                          "note": "the fp32 or fp64 leg is needed for the headline value",
                          "bf16x3": {k: v for k, v in res.get("bf16x3", {}).items() if k != "pops"}}))
        return
    main_leg = res.get("fp32") or res.get("fp64")
    prec = "fp32" if "fp32" in res else "fp64"
    peak = PEAK_FP32_MFMA if prec == "fp32" else PEAK_FP64_MFMA
    avg_us = main_leg["kernels_us"]["product_full"]
    ld = main_leg["ld"]
    # the first product executes 3 real ld^3 products (Gauss's 3M form), 6 ld^3 flop
    executed_per_launch = MFMA_FLOP_PER_CMAC * ld ** 3
    achieved = executed_per_launch / (avg_us * 1e-6) / 1e12
    roofline = {"bound": "mfma",
                "kernel": f"cgemm_{prec}_kernel<{main_leg['tile1']}, conj_b> "
                          "(first product T = rho + dU rho, full tiles)",
                "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak,
                "traffic": measured_traffic() if prec == "fp32" else None,
                "per_launch_flop": executed_per_launch,
                "per_launch_basis": "three real ld x ld x ld products (3M form of the complex "
                                    f"product), 6*ld^3 flop, ld = {ld}; equal to the MFMA "
                                    "operations the counters read per launch",
                "avg_launch_us": avg_us,
                "duration_source": "HIP start / stop events stamped by the kernel's own "
                                   "dispatch, every 8th step of a profiled pass of the same "
                                   "steps (the throughput pass runs without events)",
                "zgemm_equivalent_tflops": 8.0 * n ** 3 / (avg_us * 1e-6) / 1e12,
                "zgemm_equivalent_note": "8*N^3 (four-real-product convention) over the same "
                                         "duration; not a roofline fraction",
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                "copy-calibrated; " + TRAFFIC_FP32_PRODUCT["source"] + ")",
                "operand_bytes_per_launch": 24.0 * n * n}

    cpu, parity = None, None
    if args.cpu_steps > 0:
        gl = {"k": args.steps, **main_leg} if prec == "fp32" else {"k": args.fp64_steps, **main_leg}
        cpu, parity = cpu_baseline(W, wl, gl, args.cpu_steps, pure)
    if pure is not None:
        for key in ("fp32", "fp64"):
            pure[key].pop("_psi", None)
        pure["speedup_over_density_path_fp32"] = (
            pure["fp32"]["steps_per_s"] / plane["steps_per_s"] if plane else None)

    line = {
        "metric": METRIC,
        "value": main_leg["steps_per_s"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "jch_lattice_32x32_single_excitation_n2048", "N": n,
                   "ld": main_leg["ld"], "dt": 0.01, "mu": 0.01, "g": 0.01,
                   "boundary_leak": 0.001, "precision": prec},
        "dense_equivalent_tflops": flops_step * main_leg["steps_per_s"] / 1e12,
        "executed_tflops": executed_flops(main_leg) * main_leg["steps_per_s"] / 1e12,
        "executed_frac_of_peak": executed_flops(main_leg) * main_leg["steps_per_s"] / 1e12 / peak,
        "lower_product_frac_of_peak": lower_flops(main_leg) / (main_leg["kernels_us"]["product_lower"]
                                                               * 1e-6) / 1e12 / peak,
        "kernels_us": main_leg["kernels_us"],
        "kernels_us_sum": main_leg["kernels_us_sum"],
        "profiled_ms_per_step": main_leg["profiled_ms_per_step"],
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "adjoint_ms_per_step": adj["ms_per_step"] if adj else None,
        "adjoint": adj,
        "batch_sweep": batch,
        "latency_bound": latency,
        "other_configs": configs,
        "state_selection": selection,
        "photon_plane": plane,
        "photon_plane_pure_state": pure,
        "hydrogen_bond": hbond,
    }
    if "bf16x3" in res:
        b = res["bf16x3"]
        line["bf16x3"] = {"steps_per_s": b["steps_per_s"], "ms_per_step": b["ms_per_step"],
                          "steps": args.bf16x3_steps, "kernels_us": b["kernels_us"],
                          "dense_equivalent_frac_of_fp32_peak":
                              flops_step * b["steps_per_s"] / 1e12 / PEAK_FP32_MFMA,
                          "tiles": [b["tile1"], b["tile2"]],
                          "bf16_mfma_tflops_first_product":
                              6 * flops_product / (b["kernels_us"]["product_full"] * 1e-6) / 1e12,
                          "first_product_frac_of_bf16_peak":
                              6 * flops_product / (b["kernels_us"]["product_full"] * 1e-6) / 1e12
                              / PEAK_BF16_MFMA}
    if "fp64" in res:
        f = res["fp64"]
        line["fp64"] = {"steps_per_s": f["steps_per_s"], "ms_per_step": f["ms_per_step"],
                        "steps": args.fp64_steps, "kernels_us": f["kernels_us"],
                        "executed_frac_of_fp64_peak":
                            executed_flops(f) * f["steps_per_s"] / 1e12 / PEAK_FP64_MFMA,
                        "lower_product_frac_of_fp64_peak":
                            lower_flops(f) / (f["kernels_us"]["product_lower"] * 1e-6) / 1e12
                            / PEAK_FP64_MFMA}
        if "fp32" in res:
            line["fp32_speedup_over_fp64"] = res["fp32"]["steps_per_s"] / f["steps_per_s"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
