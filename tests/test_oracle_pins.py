"""Pins of the FP64 oracle to mathematics (no GPU).

Each test checks the oracle against something other than itself: a closed
form, a textbook queueing identity, brute force over every policy, an exact
rational solve, or an invariant of the model.  They are chosen so that a
dropped branch, a wrong rate, a wrong index or a transposed operand in the
oracle fails at least one of them.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import exact, grad, model, vi


# ---------------------------------------------------------------- layout

def test_encode_decode_roundtrip_and_layout():
    p = W.small_parity()
    N = model.num_states(p)
    assert N == 729 * 2
    for s in [0, 1, 8, 9, 80, 728, 729, 1457, 555]:
        n, e = model.decode(p, s)
        assert model.encode(p, n, e) == s
    # host 0 is the fastest digit, the class the slowest
    assert model.decode(p, 1) == ((1, 0, 0), 0)
    assert model.decode(p, 9) == ((0, 1, 0), 0)
    assert model.decode(p, 729) == ((0, 0, 0), 1)
    g = vi.grid(p)
    for occ in [0, 5, 100, 728]:
        n, _ = model.decode(p, occ)
        assert tuple(g.digits[occ]) == n


@pytest.mark.parametrize("K,C,sizes", [(3, 8, (1, 2)), (6, 10, (1, 2, 3)), (5, 10, (1, 2)), (2, 4, (1,))])
def test_feasible_pair_count_closed_form(K, C, sizes):
    # every state has the paid cloud; host a is feasible for class e on the
    # (C+1-s_e) of its C+1 occupancy values that leave room
    p = W.make(K, C, sizes, [0.5] * len(sizes), 0.1, 0.01, [1.0] * len(sizes), 0.9)
    n_occ = (C + 1) ** K
    closed = sum(n_occ + K * n_occ * (C + 1 - s) // (C + 1) for s in sizes)
    if K <= 5:
        assert vi.feasible_pairs(p) == closed
    if (K, C, sizes) == (3, 8, (1, 2)):
        assert closed == 5103
    if (K, C, sizes) == (6, 10, (1, 2, 3)):
        assert closed == 31_404_945


# ---------------------------------------------------------------- model rows

@pytest.mark.parametrize("seed", range(4))
def test_transition_rows_are_exact_distributions(seed):
    p = W.random_small(seed, K_max=3, C_max=4)
    for s in range(model.num_states(p)):
        for a in model.feasible_actions(p, s):
            row = model.transitions(p, s, a, exact=True)
            assert all(q >= 0 for q in row.values())
            assert sum(row.values()) == 1


def test_infeasible_action_is_refused():
    p = W.small_parity()
    s = model.encode(p, (8, 0, 0), 0)       # host 0 full
    assert 0 not in model.feasible_actions(p, s)
    with pytest.raises(ValueError):
        model.transitions(p, s, 0)
    s2 = model.encode(p, (7, 8, 8), 1)      # size-2 task fits nowhere
    assert model.feasible_actions(p, s2) == [p.K]


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("K,C,s,c", [(1, 6, 1, 0.0), (2, 5, 2, 0.0), (3, 4, 1, 0.7), (2, 7, 3, 0.25)])
def test_pure_arrival_closed_form(K, C, s, c):
    # mu = nu = 0, one class: every step is an arrival, the system fills
    # up after m = sum_k floor((C - n_k)/s) placements and rejects forever:
    # V*(n) = r (1 - g^m)/(1 - g) - c g^m/(1 - g)
    r, g = 1.3, 0.9
    p = W.make(K, C, (s,), (0.8,), 0.0, 0.0, (r,), g, reject_cost=(c,))
    res = vi.value_iteration(p, 1e-13)
    gr = vi.grid(p)
    m = ((C - gr.digits) // s).sum(axis=1)
    closed = r * (1 - g ** m) / (1 - g) - c * g ** m / (1 - g)
    assert np.max(np.abs(res.V - closed)) < 1e-11


def _erlang_b(C, a):
    terms = [a ** n / math.factorial(n) for n in range(C + 1)]
    return terms[-1] / sum(terms)


@pytest.mark.parametrize("C,lam,mu,g", [(4, 0.7, 0.2, 0.9), (8, 2.0, 0.3, 0.97), (10, 0.5, 0.5, 0.5)])
def test_single_host_erlang_identity(C, lam, mu, g):
    # K=1, one class of size 1, nu=0: accepting when there is room is
    # optimal and the occupancy is the M/M/C/C queue, whose stationary law is
    # the truncated Poisson pi_B (uniformisation keeps it stationary).  The
    # stationary identity then gives
    #   sum_n pi_B(n) V*(n) = P_arr r (1 - ErlangB(C, lam/mu)) / (1 - g).
    r = 1.7
    p = W.make(1, C, (1,), (lam,), mu, 0.0, (r,), g)
    res = vi.value_iteration(p, 1e-13)
    a = lam / mu
    piB = np.array([a ** n / math.factorial(n) for n in range(C + 1)])
    piB /= piB.sum()
    P_arr = lam / (lam + C * mu)
    lhs = piB @ res.V
    rhs = P_arr * r * (1 - _erlang_b(C, a)) / (1 - g)
    assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(rhs))
    pi, _ = vi.extract(p, res.V)
    assert np.all(pi[:C] == 0) and pi[C] == 1


@pytest.mark.parametrize("C,lam,nu,g", [(3, 0.6, 0.1, 0.9), (6, 1.0, 0.05, 0.95)])
def test_single_host_reset_identity(C, lam, nu, g):
    # K=1, one class of size 1, mu=0: the occupancy climbs by one per
    # accepted arrival and drops to 0 when the host leaves (rate nu).
    # Balance of the continuous-time chain: pi(n) = pi(0) rho^n (n < C),
    # rho = lam/(lam+nu), pi(C) = pi(0) rho^(C-1) lam/nu.  Stationary identity:
    #   sum_n pi(n) V*(n) = P_arr r (1 - pi(C)) / (1 - g).
    r = 0.9
    p = W.make(1, C, (1,), (lam,), 0.0, nu, (r,), g)
    res = vi.value_iteration(p, 1e-13)
    rho = lam / (lam + nu)
    w = np.array([rho ** n for n in range(C)] + [rho ** (C - 1) * lam / nu])
    w /= w.sum()
    P_arr = lam / (lam + nu)
    assert abs(w @ res.V - P_arr * r * (1 - w[-1]) / (1 - g)) < 1e-10


def test_single_host_exact_rational():
    # K=1: the value of accept-when-possible in exact rationals agrees with
    # FP64 value iteration to its tolerance.
    p = W.make(1, 5, (1,), (Fraction(3, 5),), Fraction(1, 10), Fraction(1, 50), (1.0,), 0.95)
    p = p.replace(lam=(0.6,), mu=0.1, nu=0.02)
    pi = [0] * 5 + [1]
    Vx = exact.policy_value_exact(p, pi)
    res = vi.value_iteration(p, 1e-14)
    assert max(abs(float(x) - y) for x, y in zip(Vx, res.V)) < 1e-12


# ---------------------------------------------------------------- brute force

BRUTE = [
    (1, 3, (1, 2)),
    (2, 2, (1,)),
    (2, 2, (1, 2)),
]


@pytest.mark.parametrize("K,C,sizes", BRUTE)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_over_all_policies(K, C, sizes, seed):
    J = len(sizes)
    rng = np.random.default_rng(seed)
    lam = rng.uniform(0.2, 1.0, J)
    reward = [1.0, 5.0][:J] if seed == 2 else list(rng.uniform(0.5, 3.0, J))
    cost = [0.0] * J if seed == 0 else list(rng.uniform(0.0, 0.5, J))
    p = W.make(K, C, sizes, lam, rng.uniform(0.05, 0.3), rng.uniform(0.01, 0.1), reward,
               0.9, reject_cost=cost)
    Vmax, values, policies = exact.brute_force(p)
    if (K, C, sizes) == (2, 2, (1, 2)):
        assert len(policies) == 62_208
    if (K, C, sizes) == (2, 2, (1,)):
        assert len(policies) == 1_296
    if (K, C, sizes) == (1, 3, (1, 2)):
        assert len(policies) == 32
    res = vi.value_iteration(p, 1e-13)
    assert np.max(np.abs(res.V - Vmax)) < 1e-9
    # a single policy attains the maximum everywhere
    best = np.all(values >= Vmax[None, :] - 1e-9, axis=1)
    assert best.any()
    # the extracted policy is one of them
    pi, _ = vi.extract(p, res.V)
    idx = np.where(np.all(policies == pi[None, :].astype(np.int64), axis=1))[0]
    assert idx.size == 1 and best[idx[0]]


def test_rejection_can_be_optimal():
    # a large, valuable class competes with a cheap small one: the optimal
    # policy sends some small tasks to the paid cloud while hosts have room
    p = W.make(2, 2, (1, 2), (0.9, 0.5), 0.1, 0.02, (0.1, 5.0), 0.95)
    res = vi.value_iteration(p, 1e-13)
    pi, _ = vi.extract(p, res.V)
    Vmax, _, _ = exact.brute_force(p)
    assert np.max(np.abs(res.V - Vmax)) < 1e-9
    n_occ = 9
    small = pi[:n_occ]
    feasible_place = [any(d + 1 <= 2 for d in model.decode(p, s)[0]) for s in range(n_occ)]
    assert any(f and a == p.K for f, a in zip(feasible_place, small))


# ---------------------------------------------------------------- invariants

def test_contraction_certificate():
    p = W.small_parity()
    star = vi.value_iteration(p, 1e-13).V
    for tol in [1e-1, 1e-3, 1e-6]:
        V = np.zeros(model.num_states(p))
        while True:
            Vn = vi.bellman(p, V)
            d = np.max(np.abs(Vn - V))
            V = Vn
            if d < tol:
                break
        assert np.max(np.abs(V - star)) <= p.gamma / (1 - p.gamma) * d + 1e-12


def test_host_permutation_symmetry():
    p = W.make(3, 4, (1, 2), (0.6, 0.3), 0.1, 0.02, (1.0, 2.5), 0.95)
    V = vi.value_iteration(p, 1e-12).V
    g = vi.grid(p)
    rng = np.random.default_rng(0)
    for perm in [(1, 0, 2), (2, 1, 0), (1, 2, 0)]:
        for occ in rng.integers(0, g.n_occ, 40):
            n = g.digits[occ]
            for e in range(p.J):
                a = model.encode(p, tuple(n), e)
                b = model.encode(p, tuple(n[list(perm)]), e)
                assert abs(V[a] - V[b]) < 1e-12


@pytest.mark.parametrize("inst", ["small", "seeded"])
def test_optimality_order_and_bounds(inst):
    p = W.small_parity() if inst == "small" else W.random_small(7, K_max=3, C_max=5)
    star = vi.value_iteration(p, 1e-12).V
    _, Lam, P_arr = vi.rates(p)
    for kind in ["least_loaded", "first_fit"]:
        Vg = vi.policy_eval(p, vi.greedy_policy(p, kind))
        assert np.all(Vg <= star + 1e-9)
    rng = np.random.default_rng(1)
    for _ in range(3):
        pi = np.array([rng.choice(model.feasible_actions(p, s)) for s in range(model.num_states(p))])
        assert np.all(vi.policy_eval(p, pi) <= star + 1e-9)
    hi = P_arr * max(p.reward) / (1 - p.gamma)
    lo = -P_arr * max(p.reject_cost) / (1 - p.gamma)
    assert star.max() <= hi + 1e-12 and star.min() >= lo - 1e-12
    if inst == "small":
        assert hi == pytest.approx(13.392857142857, rel=1e-12)


@pytest.mark.parametrize("seed", [0, 3])
def test_stationary_identity_any_policy(seed):
    # d^T V_pi = d^T r_pi / (1 - gamma) for the stationary law d of P_pi:
    # fails if any row of P_pi (arrival, release, reset or idle) is wrong
    p = W.random_small(seed + 11, K_max=3, C_max=4)
    rng = np.random.default_rng(seed)
    pi = np.array([rng.choice(model.feasible_actions(p, s)) for s in range(model.num_states(p))])
    P, r = vi.policy_system(p, pi)
    d = np.full(P.shape[0], 1.0 / P.shape[0])
    PT = P.T.tocsr()
    for _ in range(20000):
        dn = PT @ d
        if np.abs(dn - d).sum() < 1e-15:
            break
        d = dn
    V = vi.policy_eval(p, pi)
    assert abs(d @ V - d @ r / (1 - p.gamma)) < 1e-9


def test_vectorised_backup_matches_per_state_definition():
    p = W.random_rewards_with_reject(5, W.random_small(4, K_max=3, C_max=4))
    rng = np.random.default_rng(0)
    V = rng.normal(size=model.num_states(p))
    Q = vi.q_table(p, V)
    for s in range(model.num_states(p)):
        best, arg, qs = model.bellman_backup(p, V, s)
        acts = model.feasible_actions(p, s)
        assert np.allclose(Q[s, acts], qs, atol=1e-13)
        assert np.all(np.isneginf(np.delete(Q[s], acts)))


def test_extract_ties_and_gap():
    p = W.small_parity()
    V = vi.value_iteration(p, 1e-12).V
    pi, gap = vi.extract(p, V)
    # empty system: all hosts are equivalent, so the tie goes to host 0
    assert pi[0] == 0 and gap[0] == 0.0
    # only the paid cloud is feasible
    s = model.encode(p, (7, 8, 8), 1)
    assert pi[s] == p.K and np.isinf(gap[s])


def test_greedy_policy_definitions():
    p = W.small_parity()
    ll = vi.greedy_policy(p, "least_loaded")
    ff = vi.greedy_policy(p, "first_fit")
    s = model.encode(p, (5, 2, 2), 0)
    assert ll[s] == 1 and ff[s] == 0
    s = model.encode(p, (7, 8, 3), 1)
    assert ll[s] == 2 and ff[s] == 2
    s = model.encode(p, (8, 8, 8), 0)
    assert ll[s] == p.K and ff[s] == p.K
    # K=1: both are "accept when there is room", optimal by the Erlang pin
    q = W.make(1, 6, (1,), (0.7,), 0.2, 0.0, (1.0,), 0.9)
    star = vi.value_iteration(q, 1e-13).V
    for kind in ["least_loaded", "first_fit"]:
        assert np.max(np.abs(vi.policy_eval(q, vi.greedy_policy(q, kind)) - star)) < 1e-10


# ---------------------------------------------------------------- gradient

@pytest.fixture(scope="module")
def dense_copy():
    p = W.gradient_instance(2, 6)
    res = vi.value_iteration(p, 1e-13)
    pi, gap = vi.extract(p, res.V)
    return p, pi, gap


def test_gradient_routes_agree(dense_copy):
    p, pi, _ = dense_copy
    gd = grad.gradient_dense(p, pi)
    ga = grad.gradient_adjoint(p, pi)
    fd = grad.finite_difference(p, h=1e-6)
    assert np.allclose(gd, ga, rtol=1e-10, atol=1e-10)
    assert np.allclose(gd, fd, rtol=1e-6, atol=1e-6)


def test_gradient_identities(dense_copy):
    p, pi, _ = dense_copy
    gd = grad.gradient_dense(p, pi)
    th = grad.theta_of(p)
    J = p.J
    # every probability is a ratio of rates to Lam: scaling all rates leaves
    # the chain, and hence J, unchanged
    assert abs(th[:J + 2] @ gd[:J + 2]) < 1e-9
    # with zero reject cost the reward is linear in r
    V = vi.policy_eval(p, pi)
    assert abs(th[J + 2:] @ gd[J + 2:] - vi.objective(p, V)) < 1e-9
