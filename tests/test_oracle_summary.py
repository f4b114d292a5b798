"""Pins of the tie-invariant summaries (oracle/summary.py; no GPU).

The summaries are what the full-size parity tests compare when the two sides
may route exact ties between equivalent hosts differently.  They are pinned
here on instances small enough for exact solves: re-routing every tie to the
highest-index equivalent host (a different, equally optimal policy) leaves
the target loads, the values and the orbit sums of the adjoint weights
unchanged, while the raw adjoint weights do change; routing one placement to
a host of another load changes the target loads.
"""
import numpy as np
import pytest

import workloads as W
from oracle import grad, summary, vi


def _reroute_highest(p, pi, g):
    """The same target loads, each placement moved to the highest-index host
    with the chosen host's occupancy (an equivalent host)."""
    pi = np.asarray(pi, dtype=np.int64).reshape(p.J, g.n_occ).copy()
    for e in range(p.J):
        for o in range(g.n_occ):
            a = pi[e, o]
            if a < p.K:
                same = np.flatnonzero(g.digits[o] == g.digits[o, a])
                pi[e, o] = same[-1]
    return pi.reshape(-1).astype(np.uint8)


INSTS = [W.make(3, 5, (1, 2), (0.9, 0.5), 0.1, 0.02, (1.0, 2.5), 0.95),
         W.make(4, 3, (1,), (0.8,), 0.12, 0.03, (1.0,), 0.96),
         W.make(3, 4, (1, 2, 3), (0.6, 0.4, 0.3), 0.1, 0.02, (1.0, 2.2, 3.1), 0.94,
                reject_cost=(0.1, 0.2, 0.3))]


@pytest.mark.parametrize("p", INSTS)
def test_summaries_invariant_under_equivalent_tie_routing(p):
    g = vi.grid(p)
    star = vi.value_iteration(p, 1e-13, g=g).V
    pi, _ = vi.extract(p, star, g)
    pi2 = _reroute_highest(p, pi, g)
    assert not np.array_equal(pi, pi2)           # the routing really differs
    tl, tl2 = summary.target_load(p, pi, g), summary.target_load(p, pi2, g)
    assert np.array_equal(tl, tl2)
    V1 = vi.policy_eval(p, pi, tol=1e-14, g=g)
    V2 = vi.policy_eval(p, pi2, tol=1e-14, g=g)
    assert np.max(np.abs(V1 - V2)) <= 1e-11 * np.max(np.abs(V1))
    assert np.max(np.abs(V1 - star)) <= 1e-10 * np.max(np.abs(star))
    w1 = grad.adjoint_weights(p, pi, g=g)
    w2 = grad.adjoint_weights(p, pi2, g=g)
    assert np.max(np.abs(w1 - w2)) > 1e-3 * np.max(np.abs(w1))   # raw weights move
    o1, o2 = summary.orbit_sum(p, w1, g), summary.orbit_sum(p, w2, g)
    assert np.max(np.abs(o1 - o2)) <= 1e-11 * np.max(np.abs(o1))
    assert abs(o1.sum() - w1.sum()) <= 1e-11 * abs(w1.sum())
    # total discounted mass of the adjoint weights: sum_s w(s) = 1 / (1 - gamma)
    assert abs(w1.sum() - 1.0 / (1.0 - p.gamma)) <= 1e-9 / (1.0 - p.gamma)
    # exact ties between equivalent hosts are not near ties of target loads
    amb = summary.ambiguous(p, star, g=g)
    assert amb.size < 0.01 * p.num_states
    assert summary.masked_digest(tl, amb) == summary.masked_digest(tl2, amb)


def test_target_load_detects_a_non_equivalent_move():
    p = INSTS[0]
    g = vi.grid(p)
    star = vi.value_iteration(p, 1e-13, g=g).V
    pi, _ = vi.extract(p, star, g)
    tl = summary.target_load(p, pi, g)
    # a state whose chosen host has a lower-loaded feasible alternative
    occ = np.arange(g.n_occ)
    for s in range(p.num_states):
        e, o = divmod(s, g.n_occ)
        a = int(pi[s])
        if a < p.K:
            alt = [b for b in range(p.K)
                   if g.digits[o, b] != g.digits[o, a] and g.digits[o, b] + p.size[e] <= p.C]
            if alt:
                pi_bad = pi.copy()
                pi_bad[s] = alt[0]
                tl_bad = summary.target_load(p, pi_bad, g)
                assert not np.array_equal(tl, tl_bad)
                assert summary.masked_digest(tl, []) != summary.masked_digest(tl_bad, [])
                break
    else:
        pytest.fail("no state with a non-equivalent alternative")
    assert occ.size == g.n_occ


def test_orbit_ids_are_permutation_classes():
    p = W.make(3, 2, (1,), (0.5,), 0.1, 0.01, (1.0,), 0.9)
    g = vi.grid(p)
    ids = summary.orbit_ids(p, g)
    # orbits of 3 digits in 0..2: multisets of size 3 from 3 values = 10
    assert np.unique(ids).size == 10
    for o in range(g.n_occ):
        key = np.sort(g.digits[o]) @ g.stride
        assert ids[o] == key
    # an orbit id is itself the sorted state, so orbit sums of an indicator
    # count the orbit's size (3!/multiplicities)
    sizes = summary.orbit_sum(p, np.ones(p.num_states), g)
    assert sizes[0] == 1
    assert sizes[np.array([0, 0, 1]) @ g.stride] == 3   # digits sorted ascending
    assert sizes[np.array([1, 0, 0]) @ g.stride] == 0   # not a representative
    assert sizes[np.array([0, 1, 2]) @ g.stride] == 6


def test_orbit_table_roundtrip_and_policy_reconstruction():
    p = INSTS[2]
    g = vi.grid(p)
    star = vi.value_iteration(p, 1e-13, g=g).V
    pi, _ = vi.extract(p, star, g)
    tl = summary.target_load(p, pi, g)
    amb = summary.ambiguous(p, star, g=g)
    table = summary.orbit_table(p, tl, amb, g)
    back = summary.expand_orbit_table(p, table, g)
    known = back != -2
    assert known.sum() >= p.num_states - 6 * amb.size
    assert np.array_equal(back[known], tl[known])
    # a policy rebuilt from the target loads is optimal (same values as pi*)
    pi_r = summary.policy_from_target_load(p, np.where(known, back, tl), g)
    assert np.array_equal(summary.target_load(p, pi_r, g), np.where(known, back, tl))
    V_r = vi.policy_eval(p, pi_r, tol=1e-14, g=g)
    assert np.max(np.abs(V_r - star)) <= 1e-10 * np.max(np.abs(star))
    # a corrupted table character changes the expansion
    bad = ("b" if table[5] != "b" else "c") + table[1:]
    assert not np.array_equal(summary.expand_orbit_table(p, bad, g), back)
