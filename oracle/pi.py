"""Policy iteration (Howard), FP64: the improvement loop around the fixed-
policy evaluation and the greedy extraction of Alg. 3 step 4.

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

pi_0 given; round k: V_k = V_{pi_k} (vi.policy_eval: a dense solve for small
instances, else Jacobi to the given tolerance); pi_{k+1}(s) = pi_k(s) unless
some action's Q(s, .) computed from V_k (vi.q_table) beats Q(s, pi_k(s)) by
more than improve_tol, else the lowest-index argmax; stop when
pi_{k+1} = pi_k.  Keeping the current action on near-ties is the standard
guard against cycling between tied actions (rounding makes equivalent hosts
alternate otherwise).  Returns the final policy, its value and the number of
evaluations.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from .vi import Grid, grid, policy_eval, q_table


def improve(p, pi: np.ndarray, V: np.ndarray, improve_tol: float, g: Grid) -> np.ndarray:
    Q = q_table(p, V, g)
    arg = np.argmax(Q, axis=1)
    q_cur = Q[np.arange(Q.shape[0]), pi.astype(np.int64)]
    keep = q_cur >= Q.max(axis=1) - improve_tol
    return np.where(keep, pi, arg).astype(np.uint8)


def policy_iteration(p, pi0: np.ndarray, tol: float = 1e-13, improve_tol: float = 1e-9,
                     max_rounds: int = 1000, g: Optional[Grid] = None):
    g = g or grid(p)
    pi = np.array(pi0, dtype=np.uint8)
    V = None
    for k in range(1, max_rounds + 1):
        V = policy_eval(p, pi, tol=tol, V0=V, g=g)
        pi_next = improve(p, pi, V, improve_tol, g)
        if np.array_equal(pi_next, pi):
            return pi, V, k
        pi = pi_next
    raise RuntimeError("policy iteration did not stabilise")
