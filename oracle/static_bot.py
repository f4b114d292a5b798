"""Static bag-of-task placement: the fast greedy heuristic (Alg. 2), the
reward of a placement (Eqs. (14)-(16) summed over the cloud) and the best
placement by exhaustive search.

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Alg. 2 as read here: bags in order, tasks of a bag in order; a task of n VMs
goes to the first VC (in the cloud's order) that still has n free VMs, and
takes n of them; if none has, it goes to the paid cloud.  A placement is
scored with the three constants of Eqs. (15)-(16) applied to the whole
cloud: beta_vc per VM used in a VC, minus beta_tc per VM bought in the paid
cloud, minus gamma_vc per VM left idle in a VC.  With the example's
constants (1, 1.2, 1) the published totals are 116 (greedy) and 202.4 (MDP).

The per-VC reward dots of the example's figure do not add up to those
totals; they equal beta_vc c_i - beta_tc u_i (c_i the VC's capacity, u_i its
idle VMs), which ``per_vc_reward`` computes as a reading of that figure.

Place codes: VC index >= 0, PAID = -1, EMPTY = -2 (need 0: no task).
"""
from __future__ import annotations

import itertools
from typing import Optional, Sequence

import numpy as np

PAID = -1
EMPTY = -2


def first_fit(caps: Sequence[int], need: Sequence[int]):
    """Alg. 2 on one scenario.  Returns (place int32[T], used int64[K])."""
    free = [int(c) for c in caps]
    place = []
    for n in need:
        n = int(n)
        if n <= 0:
            place.append(EMPTY)
            continue
        where = PAID
        for k in range(len(free)):
            if free[k] >= n:
                free[k] -= n
                where = k
                break
        place.append(where)
    used = np.array([int(c) - f for c, f in zip(caps, free)], dtype=np.int64)
    return np.array(place, dtype=np.int32), used


def score(caps, need, place, beta_vc: float, beta_tc: float, gamma_vc: float):
    """Totals of one placement: dict with used int64[K], vc (VMs in VCs),
    paid (VMs in the paid cloud), idle (free VMs left in VCs) and reward =
    beta_vc vc - beta_tc paid - gamma_vc idle.  Raises ValueError if a VC is
    over its capacity or a place code is out of range."""
    K = len(caps)
    used = np.zeros(K, dtype=np.int64)
    paid = 0
    for n, p in zip(need, place):
        n, p = int(n), int(p)
        if n <= 0:
            continue
        if p == PAID:
            paid += n
        elif 0 <= p < K:
            used[p] += n
        else:
            raise ValueError(f"place code {p} out of range")
    if np.any(used > np.asarray(caps, dtype=np.int64)):
        raise ValueError("a VC is over its capacity")
    vc = int(used.sum())
    idle = int(np.sum(np.asarray(caps, dtype=np.int64)) - vc)
    reward = beta_vc * vc - beta_tc * paid - gamma_vc * idle
    return {"used": used, "vc": vc, "paid": paid, "idle": idle, "reward": reward}


def per_vc_reward(caps, used, beta_vc: float, beta_tc: float) -> np.ndarray:
    """Reading of the per-VC reward dots: beta_vc c_i - beta_tc (c_i - used_i)."""
    caps = np.asarray(caps, dtype=np.float64)
    return beta_vc * caps - beta_tc * (caps - np.asarray(used, dtype=np.float64))


def best_by_enumeration(caps, need, beta_vc: float, beta_tc: float, gamma_vc: float):
    """Highest reward over every assignment of each task to a VC or the paid
    cloud (K+1)^T assignments; tiny scenarios only.  Returns (reward, place)."""
    tasks = [t for t, n in enumerate(need) if int(n) > 0]
    K = len(caps)
    best, arg = None, None
    for choice in itertools.product(range(-1, K), repeat=len(tasks)):
        place = np.full(len(need), EMPTY, dtype=np.int32)
        place[tasks] = choice
        try:
            s = score(caps, need, place, beta_vc, beta_tc, gamma_vc)
        except ValueError:
            continue
        if best is None or s["reward"] > best:
            best, arg = s["reward"], place
    return best, arg


def full_packing(caps, need) -> Optional[np.ndarray]:
    """A placement that fills every VC exactly (so no placement uses more VC
    VMs), found by depth-first search over VCs, largest first, each filled
    with a multiset of the remaining tasks; None if there is none."""
    caps = [int(c) for c in caps]
    tasks = sorted(((int(n), t) for t, n in enumerate(need) if int(n) > 0), reverse=True)
    place = np.full(len(need), EMPTY, dtype=np.int32)
    order = sorted(range(len(caps)), key=lambda k: -caps[k])
    taken = [False] * len(tasks)

    def fill(i: int, k_pos: int, room: int) -> bool:
        if k_pos == len(order):
            return True
        if room == 0:
            nxt = k_pos + 1
            return fill(0, nxt, caps[order[nxt]]) if nxt < len(order) else True
        last = None
        for j in range(i, len(tasks)):
            n, t = tasks[j]
            if taken[j] or n > room or n == last:
                continue
            last = n
            taken[j] = True
            place[t] = order[k_pos]
            if fill(j + 1, k_pos, room - n):
                return True
            taken[j] = False
            place[t] = EMPTY
        return False

    if not order or not fill(0, 0, caps[order[0]]):
        return None
    for j, (n, t) in enumerate(tasks):
        if not taken[j]:
            place[t] = PAID
    return place
