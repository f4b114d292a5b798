"""Gradient of the expected discounted reward from the empty system (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Objective: J(theta) = sum_e c_e V_pi*(0, e), c_e = lambda_e / sum_j lambda_j,
with theta = (lambda_1..lambda_J, mu, nu, r_1..r_J) and pi* the optimal
policy of Eq. (18) held fixed (the envelope argument: where the optimal
action is unique up to exact ties between equivalent actions, the derivative
of the maximum equals the derivative at the maximising policy).

Three independent routes:

* ``gradient_dense``: the uniformised chain of ``oracle.model`` built as a
  dense float64 torch matrix P_pi(theta), V = (I - gamma P)^{-1} r and J
  differentiated by torch autograd (tiny instances).
* ``gradient_adjoint``: w solves (I - gamma P_pi)^T w = c; then
  dJ/dtheta = d/dtheta [ w^T (r_pi(theta) + gamma P_pi(theta) V) + c(theta)^T V ]
  with w and V held constant, the inner derivative taken by torch autograd
  over the edge probabilities (any size that fits in memory).
* ``finite_difference``: central differences of J with the policy
  re-optimised at every perturbed theta (value iteration + evaluation).
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import scipy.sparse as sp
import torch

from . import model, vi


def theta_of(p) -> np.ndarray:
    return np.array(list(p.lam) + [p.mu, p.nu] + list(p.reward), dtype=np.float64)


def with_theta(p, theta: np.ndarray):
    J = p.J
    return p.replace(lam=tuple(float(x) for x in theta[:J]), mu=float(theta[J]),
                     nu=float(theta[J + 1]),
                     reward=tuple(float(x) for x in theta[J + 2:]))


def _edges(p, pi: np.ndarray, theta: torch.Tensor, g: vi.Grid):
    """Edges (row, col, probability(theta)) of P_pi and r_pi(theta), in torch
    float64, branch by branch as in ``oracle.model.transitions``."""
    J, K = p.J, p.K
    lam = theta[:J]
    mu = theta[J]
    nu = theta[J + 1]
    rew = theta[J + 2:]
    cost = torch.tensor(p.reject_cost, dtype=torch.float64)
    Lam = lam.sum() + K * p.C * mu + K * nu
    P_arr = lam.sum() / Lam
    pi = np.asarray(pi, dtype=np.int64).reshape(J, g.n_occ)
    occ = np.arange(g.n_occ, dtype=np.int64)
    rows, cols, vals = [], [], []
    r_parts = []
    load = torch.from_numpy(g.load.astype(np.float64))
    for e in range(J):
        se = p.size[e]
        src = occ + e * g.n_occ
        a = pi[e]
        place = a < K
        m = occ.copy()
        m[place] += se * g.stride[a[place]]
        place_t = torch.from_numpy(place)
        r_parts.append(torch.where(place_t, P_arr * rew[e], -P_arr * cost[e])
                       - p.idle_unit_cost * (p.K * p.C - load))
        for j in range(J):
            rows.append(src); cols.append(m + j * g.n_occ)
            vals.append((lam[j] / Lam).expand(g.n_occ))
        for k in range(K):
            nk = g.digits[:, k]
            has = nk >= 1
            rows.append(src[has]); cols.append(src[has] - g.stride[k])
            vals.append(mu * torch.from_numpy(nk[has].astype(np.float64)) / Lam)
            rows.append(src); cols.append(src - nk * g.stride[k])
            vals.append((nu / Lam).expand(g.n_occ))
        rows.append(src); cols.append(src)
        vals.append(1.0 - P_arr - (mu * load + K * nu) / Lam)
    c = lam / lam.sum()
    return (np.concatenate(rows), np.concatenate(cols), torch.cat(vals),
            torch.cat(r_parts), c)


def objective_dense(p, pi: np.ndarray, theta: torch.Tensor) -> torch.Tensor:
    """J(theta) at fixed pi with a dense solve (tiny instances only)."""
    g = vi.grid(p)
    N = p.J * g.n_occ
    rows, cols, vals, r, c = _edges(p, pi, theta, g)
    P = torch.zeros((N, N), dtype=torch.float64)
    P = P.index_put((torch.from_numpy(rows), torch.from_numpy(cols)), vals, accumulate=True)
    V = torch.linalg.solve(torch.eye(N, dtype=torch.float64) - p.gamma * P, r)
    return c @ V[torch.arange(p.J) * g.n_occ]


def gradient_dense(p, pi: np.ndarray) -> np.ndarray:
    theta = torch.tensor(theta_of(p), dtype=torch.float64, requires_grad=True)
    Jv = objective_dense(p, pi, theta)
    Jv.backward()
    return theta.grad.numpy().copy()


def adjoint_weights(p, pi: np.ndarray, tol: float = 1e-13, g: Optional[vi.Grid] = None,
                    max_iter: int = 10_000_000) -> np.ndarray:
    """w = (I - gamma P_pi)^{-T} c by transposed sweeps w <- c + gamma P_pi^T w
    (a contraction in the 1-norm since every row of P_pi sums to 1)."""
    g = g or vi.grid(p)
    P, _ = vi.policy_system(p, pi, g)
    N = P.shape[0]
    c = np.zeros(N)
    lam = np.asarray(p.lam)
    c[np.arange(p.J) * g.n_occ] = lam / lam.sum()
    if N <= 4096:
        return np.linalg.solve((np.eye(N) - p.gamma * P.toarray()).T, c)
    PT = P.T.tocsr()
    w = c.copy()
    for _ in range(max_iter):
        wn = c + p.gamma * (PT @ w)
        if np.abs(wn - w).sum() < tol:
            return wn
        w = wn
    raise RuntimeError("adjoint did not converge")


def gradient_adjoint(p, pi: np.ndarray, V: Optional[np.ndarray] = None,
                     w: Optional[np.ndarray] = None, tol: float = 1e-12) -> np.ndarray:
    g = vi.grid(p)
    if V is None:
        V = vi.policy_eval(p, pi, tol=tol, g=g)
    if w is None:
        w = adjoint_weights(p, pi, g=g)
    theta = torch.tensor(theta_of(p), dtype=torch.float64, requires_grad=True)
    rows, cols, vals, r, c = _edges(p, pi, theta, g)
    Vt = torch.from_numpy(np.asarray(V, dtype=np.float64))
    wt = torch.from_numpy(np.asarray(w, dtype=np.float64))
    f = (wt * r).sum() + p.gamma * (wt[torch.from_numpy(rows)] * vals * Vt[torch.from_numpy(cols)]).sum()
    f = f + c @ Vt[torch.arange(p.J) * g.n_occ]
    f.backward()
    return theta.grad.numpy().copy()


def solve_objective(p, tol: float = 1e-12) -> float:
    """J with the policy re-optimised: VI to tol, extract, exact evaluation."""
    g = vi.grid(p)
    res = vi.value_iteration(p, tol, g=g)
    pi, _ = vi.extract(p, res.V, g)
    V = vi.policy_eval(p, pi, tol=tol * 1e-2, V0=res.V, g=g)
    return vi.objective(p, V)


def finite_difference(p, h: float = 1e-6, tol: float = 1e-13) -> np.ndarray:
    th = theta_of(p)
    out = np.empty_like(th)
    for i in range(th.size):
        tp = th.copy(); tp[i] += h
        tm = th.copy(); tm[i] -= h
        out[i] = (solve_objective(with_theta(p, tp), tol) -
                  solve_objective(with_theta(p, tm), tol)) / (2 * h)
    return out
