"""Whole-state-space FP64 value iteration, extraction and evaluation (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

The same model as ``oracle.model`` (read its header for the readings of
Sec. V-B..V-E), computed for all states at once with NumPy index arithmetic.
Nothing here is blocked, fused or reordered beyond grouping the successor
terms of Eq. (18) by branch:

  sum_s' P(s'|s,a) V(s') = A(m) + D(n, e),
    A(m)   = sum_j lambda_j/Lam V(m, j)                      (arrival branch)
    D(n,e) = sum_k mu n_k/Lam V(n - 1_k, e)                  (unit release)
           + sum_k nu/Lam V(n with n_k = 0, e)               (host leaves)
           + (1 - P_arr - (mu |n| + K nu)/Lam) V(n, e)       (idle)

Value iteration follows Alg. 3: V^0 = 0 (or a given V^0), V^{k+1} = T V^k for
every state from the old iterate (synchronous), stop at the first k with
||V^{k+1} - V^k||_inf < tol and return V^{k+1}; the policy is the argmax of
Q computed from that returned iterate (Alg. 3, step 4).  Ties go to the
lowest action index (hosts in order, paid cloud last).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Tuple

import numpy as np
import scipy.sparse as sp

NEG_INF = -np.inf


@dataclass
class Grid:
    """Digit table and strides of the mixed-radix occupancy layout."""

    K: int
    C: int
    J: int
    n_occ: int
    digits: np.ndarray   # [n_occ, K] int64
    stride: np.ndarray   # [K] int64
    load: np.ndarray     # [n_occ] sum_k n_k


def grid(p) -> Grid:
    R = p.C + 1
    n_occ = R ** p.K
    stride = R ** np.arange(p.K, dtype=np.int64)
    occ = np.arange(n_occ, dtype=np.int64)
    digits = (occ[:, None] // stride[None, :]) % R
    return Grid(p.K, p.C, p.J, n_occ, digits, stride, digits.sum(axis=1))


def rates(p):
    lam = np.asarray(p.lam, dtype=np.float64)
    Lam = lam.sum() + p.K * p.C * p.mu + p.K * p.nu
    return lam, Lam, lam.sum() / Lam


def _branch_terms(p, g: Grid, V: np.ndarray):
    """A[occ] and D[e, occ] of the grouped Bellman sum (header)."""
    lam, Lam, P_arr = rates(p)
    Vc = V.reshape(p.J, g.n_occ)
    A = (lam / Lam) @ Vc
    idle = 1.0 - P_arr - (p.mu * g.load + p.K * p.nu) / Lam
    D = idle[None, :] * Vc
    occ = np.arange(g.n_occ, dtype=np.int64)
    for k in range(p.K):
        nk = g.digits[:, k]
        has = nk >= 1
        D[:, has] += (p.mu * nk[has] / Lam)[None, :] * Vc[:, occ[has] - g.stride[k]]
        D += (p.nu / Lam) * Vc[:, occ - nk * g.stride[k]]
    return A, D


def q_table(p, V: np.ndarray, g: Optional[Grid] = None) -> np.ndarray:
    """Q[s, a] of Eq. (18) for every state and action; -inf where infeasible."""
    g = g or grid(p)
    lam, Lam, P_arr = rates(p)
    A, D = _branch_terms(p, g, np.asarray(V, dtype=np.float64))
    occ = np.arange(g.n_occ, dtype=np.int64)
    hold = p.idle_unit_cost * (p.K * p.C - g.load)   # under-utilisation penalty, Eq. (16)
    Q = np.full((p.J, g.n_occ, p.K + 1), NEG_INF)
    for e in range(p.J):
        se = p.size[e]
        for a in range(p.K):
            feas = g.digits[:, a] + se <= p.C
            m = occ[feas] + se * g.stride[a]
            Q[e, feas, a] = P_arr * p.reward[e] - hold[feas] + p.gamma * (A[m] + D[e, feas])
        Q[e, :, p.K] = -P_arr * p.reject_cost[e] - hold + p.gamma * (A + D[e])
    return Q.reshape(p.J * g.n_occ, p.K + 1)


def bellman(p, V: np.ndarray, g: Optional[Grid] = None) -> np.ndarray:
    """(T V)(s) = max over feasible a of Q(s, a)."""
    return q_table(p, V, g).max(axis=1)


@dataclass
class VIResult:
    V: np.ndarray
    iterations: int
    residual: float
    converged: bool


def value_iteration(p, tol: float, max_iter: int = 1_000_000,
                    V0: Optional[np.ndarray] = None,
                    g: Optional[Grid] = None) -> VIResult:
    """Synchronous value iteration, Alg. 3 steps 1-3 (infinity norm, strict <)."""
    g = g or grid(p)
    N = p.J * g.n_occ
    V = np.zeros(N) if V0 is None else np.array(V0, dtype=np.float64)
    res = np.inf
    for k in range(1, max_iter + 1):
        Vn = bellman(p, V, g)
        res = float(np.max(np.abs(Vn - V)))
        V = Vn
        if res < tol:
            return VIResult(V, k, res, True)
    return VIResult(V, max_iter, res, False)


def extract(p, V: np.ndarray, g: Optional[Grid] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Alg. 3 step 4: pi(s) = lowest-index argmax of Q(s, .) computed from V;
    gap(s) = best Q minus second-best Q over feasible actions (+inf when only
    the paid cloud is feasible)."""
    Q = q_table(p, V, g)
    pi = np.argmax(Q, axis=1).astype(np.uint8)
    best = Q.max(axis=1)
    Qs = np.sort(Q, axis=1)
    second = Qs[:, -2]
    gap = np.where(np.isfinite(second), best - second, np.inf)
    return pi, gap


def greedy_policy(p, kind: str = "least_loaded", g: Optional[Grid] = None) -> np.ndarray:
    """Fixed policies from the fast greedy heuristic (Alg. 2).

    least_loaded: place the pending task on the feasible host with the fewest
        occupied units (lowest index on ties), paid cloud iff no host fits.
    first_fit:    place it on the lowest-index host that fits (Alg. 2 scans
        the VCs in order and takes the first with an available VM), paid
        cloud iff none fits.
    """
    g = g or grid(p)
    pi = np.full((p.J, g.n_occ), p.K, dtype=np.int64)
    for e in range(p.J):
        feas = g.digits + p.size[e] <= p.C          # [n_occ, K]
        any_f = feas.any(axis=1)
        if kind == "least_loaded":
            key = np.where(feas, g.digits, p.C + 1)
            choice = np.argmin(key, axis=1)
        elif kind == "first_fit":
            choice = np.argmax(feas, axis=1)
        else:
            raise ValueError(kind)
        pi[e] = np.where(any_f, choice, p.K)
    return pi.reshape(-1).astype(np.uint8)


def policy_system(p, pi: np.ndarray, g: Optional[Grid] = None):
    """Sparse P_pi (CSR, N x N) and r_pi of a deterministic policy, built
    branch by branch from the same definitions as ``q_table``."""
    g = g or grid(p)
    lam, Lam, P_arr = rates(p)
    N = p.J * g.n_occ
    pi = np.asarray(pi, dtype=np.int64).reshape(p.J, g.n_occ)
    occ = np.arange(g.n_occ, dtype=np.int64)
    rows, cols, vals = [], [], []
    r = np.empty((p.J, g.n_occ))
    for e in range(p.J):
        se = p.size[e]
        src = occ + e * g.n_occ
        a = pi[e]
        place = a < p.K
        if np.any(place):
            ak = a[place]
            if np.any(g.digits[place, ak] + se > p.C):
                raise ValueError("policy chooses an infeasible placement")
        m = occ.copy()
        m[place] += se * g.stride[a[place]]
        r[e] = (np.where(place, P_arr * p.reward[e], -P_arr * p.reject_cost[e])
                - p.idle_unit_cost * (p.K * p.C - g.load))
        for j in range(p.J):
            rows.append(src); cols.append(m + j * g.n_occ)
            vals.append(np.full(g.n_occ, lam[j] / Lam))
        for k in range(p.K):
            nk = g.digits[:, k]
            has = nk >= 1
            rows.append(src[has]); cols.append(src[has] - g.stride[k])
            vals.append(p.mu * nk[has] / Lam)
            rows.append(src); cols.append(src - nk * g.stride[k])
            vals.append(np.full(g.n_occ, p.nu / Lam))
        rows.append(src); cols.append(src)
        vals.append(1.0 - P_arr - (p.mu * g.load + p.K * p.nu) / Lam)
    P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    P.sum_duplicates()
    return P, r.reshape(-1)


def policy_eval(p, pi: np.ndarray, tol: float = 1e-12, max_iter: int = 10_000_000,
                V0: Optional[np.ndarray] = None, g: Optional[Grid] = None,
                dense_limit: int = 4096) -> np.ndarray:
    """V_pi = (I - gamma P_pi)^{-1} r_pi: a dense LU solve when N <= dense_limit,
    else fixed-policy Jacobi sweeps V <- r_pi + gamma P_pi V until
    ||dV||_inf < tol."""
    P, r = policy_system(p, pi, g)
    N = r.size
    if N <= dense_limit:
        Mx = np.eye(N) - p.gamma * P.toarray()
        return np.linalg.solve(Mx, r)
    V = np.zeros(N) if V0 is None else np.array(V0, dtype=np.float64)
    for _ in range(max_iter):
        Vn = r + p.gamma * (P @ V)
        if np.max(np.abs(Vn - V)) < tol:
            return Vn
        V = Vn
    raise RuntimeError("policy evaluation did not converge")


def objective(p, V: np.ndarray) -> float:
    """J = sum_e lambda_e / sum_j lambda_j * V(0, e): expected discounted reward
    of a system that starts with every host empty."""
    lam = np.asarray(p.lam, dtype=np.float64)
    n_occ = (p.C + 1) ** p.K
    V = np.asarray(V, dtype=np.float64)
    return float((lam / lam.sum()) @ V[np.arange(p.J) * n_occ])


def feasible_pairs(p) -> int:
    """Feasible (state, action) pairs per sweep: every state has the paid
    cloud plus one placement per host with room for its pending class."""
    g = grid(p)
    total = 0
    for e in range(p.J):
        total += g.n_occ + int((g.digits + p.size[e] <= p.C).sum())
    return total
