"""Pins of the BSDI oracle (oracle/bsdi.py), the block-asynchronous scheme of
Alg. 4 as read in the module header.

- one episode per pass is synchronous Jacobi (the pinned vi.value_iteration),
  bit for bit;
- one block holding every state (T = K) turns a pass of m episodes into m
  Jacobi sweeps, bit for bit;
- a pass computed state by state from the per-state transition lists of
  oracle.model, with each successor's value taken from the block's latest
  values or the previous pass by the block rule, matches backup_mixed;
- from V = 0 with no reject cost the passes dominate Jacobi's iterates and
  stay below V* (monotonicity of the Bellman operator), and they reach the
  same fixed point in fewer passes.
"""
import numpy as np
import pytest

import workloads as W
from oracle import bsdi, model, vi


def _per_state_pass(p, Vold, T, inner):
    """Episodes of the block scheme written one state at a time."""
    R = p.C + 1
    n_occ = R ** p.K
    low = R ** T
    N = p.J * n_occ

    def block(s):
        return (s % n_occ) // low

    Vcur = np.array(Vold, dtype=np.float64)
    for _ in range(inner):
        Vn = np.empty(N)
        for s in range(N):
            best = -np.inf
            for a in model.feasible_actions(p, s):
                q = model.reward(p, s, a)
                for s2, pr in model.transitions(p, s, a).items():
                    q += p.gamma * pr * (Vcur[s2] if block(s2) == block(s) else Vold[s2])
                best = max(best, q)
            Vn[s] = best
        Vcur = Vn
    return Vcur


CASES = [("small_parity", W.small_parity()),
         ("K3C4J3", W.make(3, 4, (1, 2, 3), (0.5, 0.4, 0.3), 0.12, 0.03, (1.0, 2.2, 3.1), 0.93,
                           reject_cost=(0.1, 0.0, 0.3))),
         ("random", W.random_small(11, K_max=3, C_max=4))]


@pytest.mark.parametrize("name,p", CASES, ids=[c[0] for c in CASES])
def test_one_episode_is_jacobi(name, p):
    for T in range(1, p.K + 1):
        a = bsdi.bsdi(p, T, 1, 1e-9)
        b = vi.value_iteration(p, 1e-9)
        assert a.iterations == b.iterations
        assert np.array_equal(a.V, b.V)


@pytest.mark.parametrize("name,p", CASES, ids=[c[0] for c in CASES])
def test_single_block_pass_is_m_sweeps(name, p):
    for m in (1, 3, 7):
        a = bsdi.bsdi(p, p.K, m, 0.0, max_iter=1)
        b = vi.value_iteration(p, 0.0, max_iter=m)
        assert np.array_equal(a.V, b.V)


@pytest.mark.parametrize("T,inner", [(1, 2), (1, 3), (2, 2)])
def test_block_rule_per_state(T, inner):
    p = W.make(3, 3, (1, 2), (0.7, 0.4), 0.15, 0.05, (1.0, 2.3), 0.9, reject_cost=(0.05, 0.2))
    g = vi.grid(p)
    rng = np.random.default_rng(5)
    Vold = rng.uniform(0.0, 3.0, size=p.J * g.n_occ)
    Vcur = Vold
    for _ in range(inner):
        Vcur = bsdi.backup_mixed(p, g, Vcur, Vold, T)
    ref = _per_state_pass(p, Vold, T, inner)
    assert np.max(np.abs(Vcur - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("T,inner", [(1, 4), (2, 3), (2, 8)])
def test_dominates_jacobi_and_same_fixed_point(T, inner):
    p = W.make(4, 5, (1, 2, 3), (0.6, 0.5, 0.3), 0.1, 0.02, (1.0, 2.1, 3.3), 0.96)
    g = vi.grid(p)
    star = vi.value_iteration(p, 1e-12, g=g)
    Vb = np.zeros(p.J * g.n_occ)
    Vj = np.zeros_like(Vb)
    for _ in range(15):
        Vb_next = bsdi.bsdi(p, T, inner, 0.0, max_iter=1, V0=Vb, g=g).V
        Vj = vi.bellman(p, Vj, g)
        assert np.all(Vb_next >= Vb)          # monotone increasing from a sub-solution
        assert np.all(Vb_next >= Vj)          # at least one Jacobi sweep per pass
        assert np.all(Vb_next <= star.V + 1e-9)
        Vb = Vb_next
    res = bsdi.bsdi(p, T, inner, 1e-12, g=g)
    assert res.converged
    assert res.iterations < star.iterations
    assert np.max(np.abs(res.V - star.V)) <= 1e-9 * np.max(np.abs(star.V))
