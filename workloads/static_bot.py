"""Inputs of the static bag-of-task placement example (Sec. VII) and seeded
random static scenarios.  Data only: no placement or reward arithmetic.

The example's eleven vehicular clouds have the VM capacities that label the
per-VC reward figure (5 ... 45 VMs, 272 in all).  Its eleven bags of tasks
need 5, 10, ..., 55 VMs (330 in all).  The task granularity inside a bag is
not stated.  Bag i (1-based) is read here as five tasks of i VMs each,
the only one of the readings tried that reproduces the published greedy
figure exactly: per-bag VC VMs, the 85 paid VMs (30 of bag 10, all 55 of bag
11), the 27 idle VMs and each per-VC reward.

Scenario layout shared by both sides: caps[b, k] = free VMs of VC k in
scenario b; need[b, t] = VMs of task t in arrival order (bag by bag), 0 =
empty slot (ragged scenarios are padded with zeros).
"""
from __future__ import annotations

from typing import Tuple

import numpy as np

EXAMPLE_CAPS = (5, 7, 10, 15, 20, 25, 28, 35, 40, 42, 45)
EXAMPLE_BOTS = 11
EXAMPLE_TASKS_PER_BOT = 5
# reward constants of the example: VM reward per VC, paid VM cost, idle VM penalty
EXAMPLE_BETA_VC = 1.0
EXAMPLE_BETA_TC = 1.2
EXAMPLE_GAMMA_VC = 1.0


def example() -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """caps int32[11], need int32[55] (bag i = 5 tasks of i VMs, bags in
    order), bag int32[55] (the 1-based bag of each task)."""
    caps = np.array(EXAMPLE_CAPS, dtype=np.int32)
    bag = np.repeat(np.arange(1, EXAMPLE_BOTS + 1), EXAMPLE_TASKS_PER_BOT).astype(np.int32)
    need = bag.copy()
    return caps, need, bag


def random_scenarios(B: int, K: int, T: int, seed: int, cap_max: int = 48,
                     need_max: int = 12, empty_frac: float = 0.1) -> Tuple[np.ndarray, np.ndarray]:
    """B scenarios of K VCs and up to T tasks: caps ~ U{0..cap_max}, need ~
    U{1..need_max}, then each task slot emptied (need 0) with probability
    empty_frac and every scenario's tail cut at a random length (ragged)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    caps = rng.integers(0, cap_max + 1, size=(B, K)).astype(np.int32)
    need = rng.integers(1, need_max + 1, size=(B, T)).astype(np.int32)
    need[rng.random(size=(B, T)) < empty_frac] = 0
    if T:
        length = rng.integers(0, T + 1, size=B)
        need[np.arange(T)[None, :] >= length[:, None]] = 0
    return caps, need
