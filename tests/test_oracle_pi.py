"""Pins of the policy-iteration oracle (oracle/pi.py).

- on tiny instances the final value is the elementwise maximum over every
  deterministic policy (brute force, oracle/exact.py) and the final policy
  attains it;
- on larger ones the final value is the value-iteration fixed point, and the
  final policy is greedy with respect to its own value (no improving action);
- each round improves the value elementwise (policy improvement theorem);
- without the near-tie guard the plain argmax alternates between
  equivalent hosts on the small parity instance (why the guard exists).
"""
import numpy as np
import pytest

import workloads as W
from oracle import exact, pi as pio, vi


@pytest.mark.parametrize("seed", [1, 4, 9])
def test_brute_force_optimum(seed):
    p = W.random_small(seed, K_max=2, C_max=3, J_max=2)
    p = W.random_rewards_with_reject(seed, p)
    if exact.count_policies(p) > 100_000:
        pytest.skip("too many policies")
    vmax, _, _ = exact.brute_force(p)
    g = vi.grid(p)
    pol, V, rounds = pio.policy_iteration(p, vi.greedy_policy(p, "least_loaded", g), g=g)
    assert np.max(np.abs(V - vmax)) <= 1e-10 * max(1.0, np.max(np.abs(vmax)))
    assert rounds >= 1


CASES = [("small_parity", W.small_parity()),
         ("K3C5J3", W.make(3, 5, (1, 2, 3), (0.5, 0.4, 0.3), 0.12, 0.03, (1.0, 2.2, 3.1), 0.96)),
         ("reject", W.make(2, 6, (1, 2), (0.7, 0.5), 0.1, 0.02, (0.3, 4.0), 0.95, reject_cost=(0.2, 0.6)))]


@pytest.mark.parametrize("name,p", CASES, ids=[c[0] for c in CASES])
def test_fixed_point_and_improvement(name, p):
    g = vi.grid(p)
    star = vi.value_iteration(p, 1e-13, g=g).V
    pi0 = vi.greedy_policy(p, "first_fit", g)
    pol, V, rounds = pio.policy_iteration(p, pi0, g=g)
    assert np.max(np.abs(V - star)) <= 1e-9 * np.max(np.abs(star))
    # greedy with respect to its own value: no action improves on it
    Q = vi.q_table(p, V, g)
    assert np.all(Q.max(axis=1) <= V + 1e-10 * np.max(np.abs(V)))
    # the value improves round by round
    pol_k = pi0.copy()
    V_prev = vi.policy_eval(p, pol_k, tol=1e-13, g=g)
    for _ in range(rounds - 1):
        pol_k = pio.improve(p, pol_k, V_prev, 1e-9, g)
        V_k = vi.policy_eval(p, pol_k, tol=1e-13, g=g)
        assert np.all(V_k >= V_prev - 1e-10 * np.max(np.abs(V_prev)))
        V_prev = V_k
    assert np.array_equal(pol_k, pol)


def test_plain_argmax_cycles_on_ties():
    # exact ties between equivalent hosts: the plain lowest-index argmax of a
    # rounded Q flips between them from round to round; the guard stops it
    p = W.small_parity()
    g = vi.grid(p)
    pi = vi.greedy_policy(p, "first_fit", g)
    stable = False
    for _ in range(40):
        V = vi.policy_eval(p, pi, tol=1e-13, g=g)
        pi_next, _ = vi.extract(p, V, g)
        if np.array_equal(pi_next, pi):
            stable = True
            break
        pi = pi_next
    assert not stable
    pol, V, rounds = pio.policy_iteration(p, vi.greedy_policy(p, "first_fit", g), g=g)
    assert rounds < 40
