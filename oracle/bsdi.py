"""Block-asynchronous value iteration: the paper's BSDI scheme (Alg. 4), FP64.

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Reading of Alg. 4 (its listing is garbled: the max sits inside the action
loop, "V_s <- v" restores the old value, "pi <- max Delta_s"): the state
space is divided into blocks of states with no dependence between blocks
inside one pass; a pass copies each block's values, runs ``inner`` episodes
of the Bellman backup of Eq. (18) on the block's states, in which a
successor inside the block contributes the block's latest value and a
successor outside the block the value of the previous pass, and writes the
block back.  Passes repeat until the largest change of a pass is below tol
(infinity norm, strict <, as Alg. 3 step 3).

Blocks here are the (C+1)^T occupancies that share the high digits
n_T..n_{K-1}, with all J classes.  A successor along a low digit (k < T:
release, host reset, placement) stays in the block; a successor along a high
digit (k >= T) leaves it, except the reset of a host that is already empty,
which is the state itself; the paid cloud and the idle branch stay at n.
Within an episode the block's states are updated synchronously (each reads
the previous episode's block values), so the scheme is deterministic.  With
inner = 1 a pass is one synchronous Jacobi sweep (``vi.value_iteration``).
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from .vi import NEG_INF, Grid, VIResult, grid, rates


def backup_mixed(p, g: Grid, Vcur: np.ndarray, Vold: np.ndarray, T: int) -> np.ndarray:
    """One episode: (T V)(s) with in-block successors from Vcur and the
    others from Vold.  Same grouping and order of terms as vi._branch_terms
    and vi.q_table, so that Vcur == Vold gives vi.bellman bit for bit."""
    lam, Lam, P_arr = rates(p)
    Vc = Vcur.reshape(p.J, g.n_occ)
    Vo = Vold.reshape(p.J, g.n_occ)
    A_cur = (lam / Lam) @ Vc
    A_old = (lam / Lam) @ Vo
    idle = 1.0 - P_arr - (p.mu * g.load + p.K * p.nu) / Lam
    D = idle[None, :] * Vc
    occ = np.arange(g.n_occ, dtype=np.int64)
    for k in range(p.K):
        nk = g.digits[:, k]
        has = nk >= 1
        src = Vc if k < T else Vo
        D[:, has] += (p.mu * nk[has] / Lam)[None, :] * src[:, occ[has] - g.stride[k]]
        reset = occ - nk * g.stride[k]
        if k < T:
            D += (p.nu / Lam) * Vc[:, reset]
        else:
            D += (p.nu / Lam) * np.where((nk == 0)[None, :], Vc[:, reset], Vo[:, reset])
    # Q of every action, then the max (vi.q_table's layout and order)
    hold = p.idle_unit_cost * (p.K * p.C - g.load)
    N = p.J * g.n_occ
    Q = np.full((N, p.K + 1), NEG_INF)
    for e in range(p.J):
        rows = slice(e * g.n_occ, (e + 1) * g.n_occ)
        s = p.size[e]
        Q[rows, p.K] = -P_arr * p.reject_cost[e] - hold + p.gamma * (A_cur + D[e])
        for a in range(p.K):
            room = g.digits[:, a] + s <= p.C
            m = occ[room] + s * g.stride[a]
            A = A_cur if a < T else A_old
            q = np.full(g.n_occ, NEG_INF)
            q[room] = P_arr * p.reward[e] - hold[room] + p.gamma * (A[m] + D[e][room])
            Q[rows, a] = q
    return Q.max(axis=1)


def bsdi(p, T: int, inner: int, tol: float, max_iter: int = 1_000_000,
         V0: Optional[np.ndarray] = None, g: Optional[Grid] = None) -> VIResult:
    """Passes of `inner` block episodes until the change of a pass is < tol."""
    if not (1 <= T <= p.K) or inner < 1:
        raise ValueError("need 1 <= T <= K and inner >= 1")
    g = g or grid(p)
    V = np.zeros(p.J * g.n_occ) if V0 is None else np.array(V0, dtype=np.float64)
    res = np.inf
    for k in range(1, max_iter + 1):
        Vold = V
        Vcur = V
        for _ in range(inner):
            Vcur = backup_mixed(p, g, Vcur, Vold, T)
        res = float(np.max(np.abs(Vcur - Vold)))
        V = Vcur
        if res < tol:
            return VIResult(V, k, res, True)
    return VIResult(V, max_iter, res, False)
