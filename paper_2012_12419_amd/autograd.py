"""torch.autograd.Function over the GPU solver: the optimal expected discounted
reward from the empty system and its gradient with respect to the arrival
rates, the unit-release rate, the host-leave rate and the placement rewards.

Forward (all on the GPU through the C ABI): value iteration (FP32 values,
FP64 sums) -> greedy policy -> FP64 evaluation of that policy -> FP64
improvement steps until the policy is stable -> J = sum_e c_e V_pi(0, e).
Backward: vi_adjoint solves (I - gamma P_pi)^T w = c with transposed sweeps
and forms dJ/dtheta in one FP64 pass; the result is scaled by the incoming
gradient.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import MDP


class MdpValue(torch.autograd.Function):
    @staticmethod
    def forward(ctx, lam, mu, nu, reward, spec):
        K, C, size, gamma = spec["K"], spec["C"], spec["size"], spec["gamma"]
        mdp = MDP(K, C, size, lam.detach().double().cpu().tolist(), float(mu), float(nu),
                  reward.detach().double().cpu().tolist(), gamma, spec.get("reject_cost"),
                  spec.get("idle_unit_cost", 0.0))
        dev = spec.get("device", "cuda")
        V = torch.zeros(mdp.num_states, dtype=torch.float32, device=dev)
        if spec.get("V0") is not None:
            V.copy_(spec["V0"])
        mdp.vi_solve(V, tol=spec.get("tol", 1e-6))
        pi, _ = mdp.policy_extract(V, want_gap=False)
        Vp = V.double()
        for _ in range(spec.get("improve_steps", 8)):
            mdp.policy_eval(pi, Vp, tol=spec.get("eval_tol", 1e-11))
            pi2, _ = mdp.policy_extract(Vp, want_gap=False)
            if torch.equal(pi2, pi):
                break
            pi = pi2
        Jv = mdp.objective(Vp)
        ctx.mdp = mdp
        ctx.spec = spec
        ctx.save_for_backward(pi, Vp)
        ctx.shapes = (lam, mu, nu, reward)
        return torch.tensor(Jv, dtype=torch.float64, device=lam.device)

    @staticmethod
    def backward(ctx, gJ):
        pi, Vp = ctx.saved_tensors
        grad, _, _, _ = ctx.mdp.vi_adjoint(pi, Vp, tol=ctx.spec.get("adjoint_tol", 1e-10))
        lam, mu, nu, reward = ctx.shapes
        J = len(ctx.spec["size"])
        g = torch.tensor(grad, dtype=torch.float64, device=lam.device) * gJ.to(torch.float64)
        return (g[:J].to(lam.dtype), g[J].to(mu.dtype).reshape(mu.shape),
                g[J + 1].to(nu.dtype).reshape(nu.shape), g[J + 2:].to(reward.dtype), None)


def expected_reward(lam: torch.Tensor, mu: torch.Tensor, nu: torch.Tensor, reward: torch.Tensor,
                    K: int, C: int, size: Sequence[int], gamma: float,
                    reject_cost: Optional[Sequence[float]] = None, idle_unit_cost: float = 0.0,
                    **opts) -> torch.Tensor:
    """Optimal J(lambda, mu, nu, r) as a differentiable scalar tensor.  The
    paid-cloud costs and the under-utilisation penalty per free unit are held
    fixed (not differentiated)."""
    known = {"tol", "eval_tol", "adjoint_tol", "improve_steps", "device", "V0"}
    unknown = set(opts) - known
    if unknown:
        raise TypeError(f"unknown options {sorted(unknown)}")
    spec = dict(K=K, C=C, size=list(size), gamma=gamma, reject_cost=reject_cost,
                idle_unit_cost=float(idle_unit_cost), **opts)
    return MdpValue.apply(lam, mu, nu, reward, spec)
