"""Exact and exhaustive solves for tiny instances (oracle; test only).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Built from the per-state definitions in ``oracle.model``:

* ``policy_value_exact``: V_pi solving (I - gamma P_pi) V = r_pi in rational
  arithmetic (``fractions.Fraction``) by Gaussian elimination.
* ``brute_force``: V_pi for every deterministic stationary policy (the product
  of the feasible-action sets), each by an FP64 dense solve.  The optimal
  value of Eq. (18) is the elementwise maximum over them.
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from typing import List, Sequence, Tuple

import numpy as np

from . import model


def solve_fraction(M: List[List[Fraction]], b: List[Fraction]) -> List[Fraction]:
    """Gaussian elimination with exact rationals (row pivoting on nonzero)."""
    n = len(b)
    A = [row[:] + [b[i]] for i, row in enumerate(M)]
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        inv = 1 / A[col][col]
        A[col] = [x * inv for x in A[col]]
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [x - f * y for x, y in zip(A[r], A[col])]
    return [A[i][n] for i in range(n)]


def policy_value_exact(p, pi: Sequence[int]) -> List[Fraction]:
    """Exact V_pi for a deterministic policy (one action per state)."""
    N = model.num_states(p)
    g = Fraction(p.gamma)
    M = [[Fraction(0)] * N for _ in range(N)]
    b = [Fraction(0)] * N
    for s in range(N):
        M[s][s] += 1
        for t, q in model.transitions(p, s, int(pi[s]), exact=True).items():
            M[s][t] -= g * q
        b[s] = model.reward(p, s, int(pi[s]), exact=True)
    return solve_fraction(M, b)


def dense_system(p, pi: Sequence[int]) -> Tuple[np.ndarray, np.ndarray]:
    """Dense FP64 P_pi and r_pi from the per-state transition lists."""
    N = model.num_states(p)
    P = np.zeros((N, N))
    r = np.zeros(N)
    for s in range(N):
        for t, q in model.transitions(p, s, int(pi[s])).items():
            P[s, t] += q
        r[s] = model.reward(p, s, int(pi[s]))
    return P, r


def action_sets(p) -> List[List[int]]:
    return [model.feasible_actions(p, s) for s in range(model.num_states(p))]


def count_policies(p) -> int:
    out = 1
    for acts in action_sets(p):
        out *= len(acts)
    return out


def brute_force(p, limit: int = 200_000):
    """Every deterministic policy's value by a dense solve.

    Returns (Vmax, values, policies): Vmax is the elementwise maximum of V_pi
    over all policies, values[i] = V_{policies[i]}.
    """
    sets = action_sets(p)
    total = count_policies(p)
    if total > limit:
        raise ValueError(f"{total} policies exceed limit {limit}")
    N = len(sets)
    # per-state, per-action rows so that each policy is a row selection
    rows = {}
    for s, acts in enumerate(sets):
        for a in acts:
            row = np.zeros(N)
            for t, q in model.transitions(p, s, a).items():
                row[t] += q
            rows[(s, a)] = (row, model.reward(p, s, a))
    policies = np.array(list(itertools.product(*sets)), dtype=np.int64)
    P = np.empty((total, N, N))
    r = np.empty((total, N))
    for s in range(N):
        for a in sets[s]:
            sel = policies[:, s] == a
            P[sel, s, :] = rows[(s, a)][0]
            r[sel, s] = rows[(s, a)][1]
    M = np.eye(N)[None, :, :] - p.gamma * P
    values = np.linalg.solve(M, r[:, :, None])[:, :, 0]
    return values.max(axis=0), values, policies
