"""torch.autograd binding of the time-stepping solver and its adjoint.

``evolve(theta, wl, rho0, n_steps, obs)`` returns f = sum_s obs[s] Re rho_K[s,s]
as a differentiable scalar of the parameter vector theta = [g per atom,
mu per hop, gamma per jump].  The forward pass runs qme_step on the GPU; the
backward pass runs qme_adjoint (checkpointed recomputation + adjoint
products + FP64 Frechet finalisation).  theta is a float64 CPU tensor: the
propagator is rebuilt on the host in FP64 for every new parameter set.
"""
from __future__ import annotations

import copy

import torch

from .api import Solver


def with_parameters(wl: dict, theta) -> dict:
    """Copy of a workload with g, mu and gamma taken from theta."""
    theta = [float(x) for x in theta]
    n_atoms = int(sum(wl["atoms"]))
    n_hops = len(wl.get("hops", []))
    n_jumps = len(wl.get("jumps", []))
    if len(theta) != n_atoms + n_hops + n_jumps:
        raise ValueError("theta must hold g per atom, mu per hop and gamma per jump")
    out = copy.deepcopy(wl)
    out["g"] = theta[:n_atoms]
    out["hops"] = [(a, b, theta[n_atoms + h]) for h, (a, b, _) in enumerate(wl.get("hops", []))]
    out["jumps"] = [(k, c, at, theta[n_atoms + n_hops + j])
                    for j, (k, c, at, _) in enumerate(wl.get("jumps", []))]
    return out


def parameters_of(wl: dict) -> torch.Tensor:
    theta = list(wl["g"]) + [m for _, _, m in wl.get("hops", [])] + \
        [gm for _, _, _, gm in wl.get("jumps", [])]
    return torch.tensor(theta, dtype=torch.float64)


class QMEEvolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, wl, rho0, n_steps, obs, precision, checkpoint_every):
        sol = Solver(with_parameters(wl, theta.detach().cpu().numpy()), precision)
        sol.set_rho(rho0)
        state0 = sol.state.clone()
        sol.step(n_steps)
        f = sol.observe_weighted(obs)
        ctx.sol = sol
        ctx.state0 = state0
        ctx.n_steps = n_steps
        ctx.obs = obs
        ctx.every = checkpoint_every
        return torch.tensor(f, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        _, grad = ctx.sol.adjoint(ctx.n_steps, ctx.obs, ctx.every, state=ctx.state0)
        ctx.sol.close()
        g = torch.from_numpy(grad).to(torch.float64) * grad_out.detach().cpu()
        return g, None, None, None, None, None, None


def evolve(theta: torch.Tensor, wl: dict, rho0, n_steps: int, obs, precision: str = "fp32",
           checkpoint_every: int = 32) -> torch.Tensor:
    return QMEEvolve.apply(theta, wl, rho0, n_steps, obs, precision, checkpoint_every)
