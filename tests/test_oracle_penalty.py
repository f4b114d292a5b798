"""Pins of the under-utilisation penalty (Eq. (16): a cost on every free VM
unit of every host, per uniformised step) in the oracle.

- closed form: one host with arrivals only (mu = nu = 0, Lam = lambda, every
  step is an arrival) and no rewards fills one unit per step, so
  V(n) = -u sum_{t < C-n} gamma^t (C - n - t);
- brute force over every policy (per-state model.reward and transitions)
  equals vectorised value iteration (vi.q_table);
- per-state and vectorised backups agree at random values;
- with no rewards and no paid-cloud cost the optimum never uses the paid
  cloud while a host has room (placing removes free units), and V <= 0;
- evaluation is linear in the penalty: V_pi(u) - V_pi(0) = -u (I - gamma
  P_pi)^-1 (K C - |n|), with the right-hand side solved densely;
- the gradient routes (dense autograd, adjoint, central differences) agree.
"""
import numpy as np
import pytest

import workloads as W
from oracle import exact, grad, model, vi


@pytest.mark.parametrize("C,g,u", [(1, 0.9, 0.5), (4, 0.95, 0.2), (7, 0.8, 1.3)])
def test_single_host_fill_closed_form(C, g, u):
    p = W.make(1, C, (1,), (0.7,), 0.0, 0.0, (0.0,), g, idle_unit_cost=u)
    res = vi.value_iteration(p, 1e-14)
    for n in range(C + 1):
        ref = -u * sum(g ** t * (C - n - t) for t in range(C - n))
        assert abs(res.V[n] - ref) <= 1e-12 * max(1.0, abs(ref))


@pytest.mark.parametrize("seed", [0, 1])
def test_brute_force_with_penalty(seed):
    rng = np.random.default_rng(seed)
    p = W.make(2, 2, (1,), (rng.uniform(0.3, 1.0),), rng.uniform(0.05, 0.3), rng.uniform(0.01, 0.1),
               (rng.uniform(0.2, 2.0),), 0.9, reject_cost=(rng.uniform(0.0, 0.5),),
               idle_unit_cost=rng.uniform(0.05, 0.5))
    vmax, values, policies = exact.brute_force(p)
    assert len(policies) == 1_296
    res = vi.value_iteration(p, 1e-13)
    assert np.max(np.abs(res.V - vmax)) < 1e-9


def test_per_state_backup_with_penalty():
    p = W.random_rewards_with_reject(5, W.random_small(4, K_max=3, C_max=4)).replace(idle_unit_cost=0.37)
    rng = np.random.default_rng(0)
    V = rng.normal(size=model.num_states(p))
    Q = vi.q_table(p, V)
    for s in range(model.num_states(p)):
        best, arg, qs = model.bellman_backup(p, V, s)
        acts = model.feasible_actions(p, s)
        assert np.allclose(Q[s, acts], qs, atol=1e-13)


def test_penalty_alone_favours_placement():
    p = W.make(3, 4, (1, 2), (0.6, 0.4), 0.1, 0.02, (0.0, 0.0), 0.95, idle_unit_cost=0.3)
    g = vi.grid(p)
    res = vi.value_iteration(p, 1e-12, g=g)
    assert np.all(res.V <= 0)
    pi, _ = vi.extract(p, res.V, g)
    Q = vi.q_table(p, res.V, g)
    for e in range(p.J):
        room = np.any(g.digits + p.size[e] <= p.C, axis=1)
        rows = np.arange(g.n_occ)[room] + e * g.n_occ
        assert np.all(pi[rows] < p.K)
        # strictly: the best placement beats the paid cloud (ties only between hosts)
        assert np.all(Q[rows, :p.K].max(axis=1) > Q[rows, p.K])


def test_evaluation_is_linear_in_the_penalty():
    base = W.make(2, 4, (1, 2), (0.8, 0.3), 0.12, 0.04, (1.0, 2.5), 0.93, reject_cost=(0.1, 0.2))
    g = vi.grid(base)
    pi = vi.greedy_policy(base, "first_fit", g)
    u = 0.41
    V0 = vi.policy_eval(base, pi, g=g)
    Vu = vi.policy_eval(base.replace(idle_unit_cost=u), pi, g=g)
    P, _ = vi.policy_system(base, pi, g)
    free = np.tile(base.K * base.C - g.load, base.J).astype(np.float64)
    H = np.linalg.solve(np.eye(P.shape[0]) - base.gamma * P.toarray(), free)
    assert np.max(np.abs((Vu - V0) + u * H)) <= 1e-10 * np.max(np.abs(Vu))


def test_gradient_routes_with_penalty():
    p = W.gradient_instance(2, 6).replace(idle_unit_cost=0.15)
    res = vi.value_iteration(p, 1e-13)
    pi, _ = vi.extract(p, res.V)
    gd = grad.gradient_dense(p, pi)
    ga = grad.gradient_adjoint(p, pi)
    fd = grad.finite_difference(p, h=1e-6)
    assert np.allclose(gd, ga, rtol=1e-10, atol=1e-10)
    assert np.allclose(gd, fd, rtol=1e-6, atol=1e-6)
    # scaling every rate leaves the chain and the per-step penalty unchanged
    th = grad.theta_of(p)
    assert abs(th[:p.J + 2] @ gd[:p.J + 2]) < 1e-9
