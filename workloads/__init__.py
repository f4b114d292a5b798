"""Seeded synthetic instances of the occupancy MDP.

This module only draws model parameters (host count K, per-host capacity C,
task classes with their sizes, rates and rewards, discount).  It contains none
of the method's arithmetic: it is the one place that both the GPU library's
tests and the CPU oracle take their inputs from, so that both sides see the
same instance for the same seed.

The paper (Sec. V-B..V-E) leaves the workload unspecified beyond "tasks of
bag-of-tasks need VMs in vehicular clouds".  The instances below stand in for
it: hosts are vehicular clouds of C VM units each, task class j needs size_j
units, arrives as a Poisson stream of rate lambda_j, every occupied unit is
released at rate mu, and every host leaves (its VMs are dropped and it is
replaced empty) at rate nu.

Draw order (every draw from ``numpy.random.Generator(PCG64(seed))``):
per instance, optionally (K, C, J) as integers, then lambda_1..lambda_J,
mu, nu, u_1..u_J (reward r_j = size_j * u_j), then optionally gamma.
"""
from __future__ import annotations

from dataclasses import dataclass, field, asdict
from typing import List, Optional, Sequence

import numpy as np


@dataclass(frozen=True)
class Instance:
    """One MDP instance: K hosts of capacity C, J task classes."""

    K: int
    C: int
    J: int
    size: tuple
    lam: tuple
    mu: float
    nu: float
    reward: tuple
    reject_cost: tuple
    gamma: float
    idle_unit_cost: float = 0.0

    def as_dict(self) -> dict:
        return asdict(self)

    @property
    def num_states(self) -> int:
        return self.J * (self.C + 1) ** self.K

    def replace(self, **kw) -> "Instance":
        d = self.as_dict()
        d.update(kw)
        for key in ("size", "lam", "reward", "reject_cost"):
            d[key] = tuple(d[key])
        return Instance(**d)


def make(K: int, C: int, size: Sequence[int], lam: Sequence[float], mu: float,
         nu: float, reward: Sequence[float], gamma: float,
         reject_cost: Optional[Sequence[float]] = None, idle_unit_cost: float = 0.0) -> Instance:
    J = len(size)
    if reject_cost is None:
        reject_cost = [0.0] * J
    return Instance(K=int(K), C=int(C), J=J, size=tuple(int(s) for s in size),
                    lam=tuple(float(x) for x in lam), mu=float(mu), nu=float(nu),
                    reward=tuple(float(x) for x in reward),
                    reject_cost=tuple(float(x) for x in reject_cost),
                    gamma=float(gamma), idle_unit_cost=float(idle_unit_cost))


def _draw_rates(rng: np.random.Generator, K: int, C: int, J: int, gamma: Optional[float]):
    size = list(range(1, J + 1))
    lam = rng.uniform(0.2, 1.0, size=J)
    mu = rng.uniform(0.05, 0.2)
    nu = rng.uniform(0.005, 0.05)
    u = rng.uniform(0.8, 1.2, size=J)
    reward = [s * x for s, x in zip(size, u)]
    if gamma is None:
        gamma = rng.uniform(0.9, 0.99)
    return make(K, C, size, lam, mu, nu, reward, gamma)


def small_parity() -> Instance:
    """K=3, C=8, J=2 (sizes 1,2): 729 x 2 = 1458 states, gamma 0.95."""
    return make(3, 8, (1, 2), (0.6, 0.3), 0.1, 0.02, (1.0, 2.5), 0.95)


def large_single(seed: int = 2, K: int = 6, C: int = 10, J: int = 3) -> Instance:
    """K=6, C=10, J=3 (sizes 1,2,3): 11^6 x 3 = 5,314,683 states, gamma 0.99.

    With K=7 the same draws give the 58,461,513-state instance whose two
    FP32 value buffers (468 MB) exceed the 256 MB last-level cache.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    return _draw_rates(rng, K, C, J, 0.99)


def batch(n: int = 512, seed: int = 3) -> List[Instance]:
    """Parameter sweep: K ~ U{2..5}, C ~ U{4..12}, J ~ U{1..3}, gamma ~ U(.9,.99)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        K = int(rng.integers(2, 6))
        C = int(rng.integers(4, 13))
        J = int(rng.integers(1, 4))
        out.append(_draw_rates(rng, K, C, J, None))
    return out


def gradient_instance(K: int = 5, C: int = 10) -> Instance:
    """K=5, C=10, J=2 (sizes 1, 2), gamma 0.98: 161,051 x 2 states.

    The small-parity release, leave and reward rates with the arrival rates
    scaled by 5, lambda = (3.0, 1.5): the offered load (60 units) exceeds the
    50 units of capacity, so the optimal policy reserves room for the larger
    class and sends some small tasks to the paid cloud.  (At lambda =
    (0.6, 0.3) the system almost never fills and J reduces to
    P_arr E[r] / (1 - gamma) = 11.25, which would not exercise the policy.)
    ``gradient_instance(2, 6)`` is the 98-state copy used for dense checks.
    """
    return make(K, C, (1, 2), (3.0, 1.5), 0.1, 0.02, (1.0, 2.5), 0.98)


def random_small(seed: int, K_max: int = 3, C_max: int = 5, J_max: int = 3) -> Instance:
    """Tiny random instance for brute-force style checks (sizes 1..J, C >= J)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    K = int(rng.integers(1, K_max + 1))
    J = int(rng.integers(1, J_max + 1))
    C = int(rng.integers(max(J, 1), C_max + 1))
    inst = _draw_rates(rng, K, C, J, None)
    return inst


def random_rewards_with_reject(seed: int, inst: Instance) -> Instance:
    """Same structure, rewards drawn so that rejection is sometimes optimal
    (a high-reward large class competes with a low-reward small class), and a
    positive reject cost on some classes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    reward = tuple(float(x) for x in rng.uniform(0.1, 6.0, size=inst.J))
    cost = tuple(float(x) for x in rng.uniform(0.0, 0.5, size=inst.J))
    return inst.replace(reward=reward, reject_cost=cost)
