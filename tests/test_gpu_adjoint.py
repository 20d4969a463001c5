"""Adjoint gradients (qme_adjoint) against the oracle's tangent-linear FP64
gradients, the lattice's analytic gradient at full size, and the GPU
forward's own finite differences; plus checkpoint invariance and the
torch.autograd wiring.  Gradient error is the vector-norm relative error."""
import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as cf
from oracle import evolve as ev
from oracle import gradients as gr
from oracle import model as md

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2403_07042_amd")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def small_open():
    return {
        "name": "adj_small", "atoms": [1, 1], "photon_cap": [2, 2], "exc_min": 0, "exc_max": -1,
        "omega_c": [1.0, 1.0], "omega_a": [1.0, 1.0], "g": [0.09, 0.06],
        "hops": [(0, 1, 0.04)],
        "jumps": [(W.PHOTON_LEAK, 0, -1, 0.03), (W.PHOTON_LEAK, 1, -1, 0.01),
                  (W.ATOM_DEPHASE, 1, 0, 0.02), (W.ATOM_DECAY, 0, 0, 0.015)],
        "dt": 0.1, "steps": 40, "init": {"kind": "haar", "seed": 5},
    }


def windowed():
    wl = small_open()
    return dict(wl, name="adj_window", exc_min=1, exc_max=2)


@pytest.mark.parametrize("make", [small_open, windowed])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-4), ("bf16x3", 1e-4)])
def test_adjoint_matches_tangent_linear(make, precision, tol):
    wl = make()
    s = ev.System(wl)
    rho0 = W.initial_rho(wl, s.occ)
    obs = md.photon_number(wl, s.occ).astype(float)
    f_ref, g_ref = gr.gradient(s, rho0, wl["steps"], obs)
    sol = P.Solver(wl, precision)
    sol.set_rho(rho0)
    print(f"adjoint {wl['name']} {precision}", flush=True)
    f, g = sol.adjoint(wl["steps"], obs, checkpoint_every=7)
    sol.close()
    assert abs(f - f_ref) < {"fp64": 1e-12, "fp32": 1e-6, "bf16x3": 1e-5}[precision]
    assert rel(g, g_ref) < tol, (g, g_ref)


def test_checkpoint_interval_does_not_change_the_gradient():
    wl = small_open()
    occ = P.basis(wl)
    rho0 = W.initial_rho(wl, occ)
    obs = np.arange(occ.shape[0], dtype=float) / occ.shape[0]
    sol = P.Solver(wl, "fp32")
    sol.set_rho(rho0)
    outs = [sol.adjoint(40, obs, checkpoint_every=k) for k in (1, 6, 40, 1000)]
    sol.close()
    for f, g in outs[1:]:
        assert f == outs[0][0]
        assert np.array_equal(g, outs[0][1])


def test_adjoint_matches_gpu_finite_differences_fp64():
    wl = small_open()
    occ = P.basis(wl)
    rho0 = W.initial_rho(wl, occ)
    obs = md.photon_number(wl, occ).astype(float)
    sol = P.Solver(wl, "fp64")
    sol.set_rho(rho0)
    _, g = sol.adjoint(40, obs, checkpoint_every=8)
    sol.close()
    from paper_2403_07042_amd.autograd import parameters_of, with_parameters
    theta = parameters_of(wl).numpy()
    h = 1e-5
    fd = []
    for i in range(len(theta)):
        vals = []
        for sgn in (1, -1):
            t = theta.copy()
            t[i] += sgn * h
            s2 = P.Solver(with_parameters(wl, t), "fp64")
            s2.set_rho(rho0)
            s2.step(40)
            pops, _, _ = s2.observe()
            s2.close()
            vals.append(float(obs @ pops))
        fd.append((vals[0] - vals[1]) / (2 * h))
    assert rel(g, fd) < 1e-6


def test_lattice_2048_adjoint_against_closed_form_gradient():
    """Full-size 32 x 32 lattice, 1000 FP32 steps, checkpoint every 32: the
    derivative of the centre photon population with respect to the tied
    hopping mu and coupling g, against the analytic sine-mode gradient."""
    wl = W.photon_lattice()
    occ = P.basis(wl)
    site = wl["centre_site"]
    centre = int(np.nonzero(occ[:, 2 * site] == 1)[0][0])
    obs = np.zeros(occ.shape[0])
    obs[centre] = 1.0
    sol = P.Solver(wl, "fp32")
    sol.set_rho(W.initial_rho(wl, occ))
    print("adjoint lattice 2048 fp32 1000 steps", flush=True)
    f, g = sol.adjoint(1000, obs, checkpoint_every=32)
    sol.close()
    pop, dmu, dg = cf.lattice_population_grad(32, 32, 0.01, 0.01, 1.0, 10.0, site, site)
    maps = W.tied_parameter_maps(wl)
    gmu = g[maps["mu"]].sum()
    gg = g[maps["g"]].sum()
    assert abs(f - pop) < 1e-5
    assert rel([gmu, gg], [dmu, dg]) < 1e-4, (gmu, dmu, gg, dg)


def test_autograd_function():
    from paper_2403_07042_amd.autograd import evolve, parameters_of
    wl = small_open()
    occ = P.basis(wl)
    rho0 = W.initial_rho(wl, occ)
    obs = md.photon_number(wl, occ).astype(float)
    theta = parameters_of(wl).requires_grad_(True)
    f = evolve(theta, wl, rho0, 40, obs, precision="fp64", checkpoint_every=10)
    f.backward()
    s = ev.System(wl)
    f_ref, g_ref = gr.gradient(s, rho0, 40, obs)
    assert abs(f.item() - f_ref) < 1e-12
    assert rel(theta.grad.numpy(), g_ref) < 1e-9


def test_adjoint_with_scaling_and_squaring_fp64():
    """|H dt| > 1/2: the propagator needs squarings and the Frechet
    finalisation undoes them (host FP64 path)."""
    wl = dict(small_open(), dt=1.3, steps=12)
    s = ev.System(wl)
    rho0 = W.initial_rho(wl, s.occ)
    obs = md.photon_number(wl, s.occ).astype(float)
    f_ref, g_ref = gr.gradient(s, rho0, 12, obs)
    sol = P.Solver(wl, "fp64")
    sol.set_rho(rho0)
    f, g = sol.adjoint(12, obs, checkpoint_every=5)
    sol.close()
    assert abs(f - f_ref) < 1e-11
    assert rel(g, g_ref) < 1e-9


@pytest.mark.parametrize("size", [64, 128, 256, 512])
def test_batched_sweep_instance_gradients_against_finite_differences(size):
    """Instances of the batched sweep (one per N): FP32 adjoint of the final
    total photon number after 500 steps (checkpoint every 32) with respect to
    every g, mu and gamma term, against central finite differences of FP64
    forward runs on the device (step 1e-6)."""
    wl = next(w for w in W.batch_sweep(per_size=1) if w["expected_n"] == size)
    occ = P.basis(wl)
    assert occ.shape[0] == size
    rho0 = W.initial_rho(wl, occ)
    obs = md.photon_number(wl, occ).astype(float)
    steps = wl["steps"]
    sol = P.Solver(wl, "fp32")
    sol.set_rho(rho0)
    print(f"sweep instance N={size}: fp32 adjoint {steps} steps", flush=True)
    f, g = sol.adjoint(steps, obs, checkpoint_every=32)
    sol.close()
    from paper_2403_07042_amd.autograd import parameters_of, with_parameters
    theta = parameters_of(wl).numpy()

    def forward(t):
        s2 = P.Solver(with_parameters(wl, t), "fp64")
        s2.set_rho(rho0)
        s2.step(steps)
        pops, _, _ = s2.observe()
        s2.close()
        return float(obs @ pops)

    h = 1e-6
    fd = []
    for i in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd.append((forward(tp) - forward(tm)) / (2 * h))
    assert abs(f - forward(theta)) < 1e-5
    assert rel(g, fd) < 1e-4, (g, fd)
