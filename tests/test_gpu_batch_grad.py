"""GPU parity of the batched gradient and greedy-scoring pipeline.

For every instance of a mixed batch: value iteration -> extraction -> FP64
policy iteration (per instance) -> adjoint gradient, and the
least-loaded greedy policy with its FP64 value.  Checked against the FP64
oracle instance by instance, and against the single-instance entry points
bit for bit (same per-state arithmetic, same tile order in the reductions).
"""
import numpy as np
import pytest

import workloads as W
from oracle import grad, vi
from tests.gpu_util import sub_solution, EVAL_REL, gap_mask, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdpvi():
    torch_cuda()
    import paper_2012_12419_amd as m
    m.load()
    return m


def _instances():
    out = list(W.batch(10, seed=5))
    out.append(W.gradient_instance(3, 6))
    out.append(W.make(4, 8, (1, 2), (1.2, 0.6), 0.1, 0.02, (1.0, 2.5), 0.97))        # 13,122 states
    out.append(W.make(2, 5, (1, 2), (0.9, 0.5), 0.1, 0.02, (0.3, 4.0), 0.95, reject_cost=(0.2, 0.5)))
    out.append(W.make(3, 4, (1, 2), (0.8, 0.4), 0.1, 0.02, (1.0, 2.5), 0.95, idle_unit_cost=0.1))
    return out


def _batch_pipeline(mdpvi, insts):
    import torch
    b = mdpvi.Batch(insts)
    N = b.num_states
    V = torch.zeros(N, device="cuda")
    lb = torch.zeros(N, device="cuda")
    for i, p in enumerate(insts):   # constant sub-solution start (reject costs, penalties)
        lb[b.offsets[i]:b.offsets[i + 1]] = sub_solution(p)
    V.copy_(lb)
    b.vi_solve(V, tol=1e-7)
    _batch_pipeline.last_V = V
    pi, _ = b.policy_extract(V, want_gap=False)
    Vp = V.double()
    # per-instance FP64 policy iteration from the FP32 greedy policy (an
    # action changes only when another beats it by more than 1e-9)
    _, rounds = b.policy_iteration(pi, Vp, eval_tol=1e-12, improve_tol=IMPROVE_TOL)
    _batch_pipeline.rounds = rounds
    grads, objs, w, st, its = b.vi_adjoint(pi, Vp, [p.J for p in insts], tol=1e-11)
    pig = b.policy_greedy("least_loaded")
    # the heuristic's evaluation starts from V_pi* (V_greedy <= V*, close to it)
    Vg, _, _, _ = b.policy_eval(pig, Vp.clone(), tol=1e-12)
    return b, pi, Vp, grads, objs, w, pig, Vg


def test_batch_gradient_and_greedy_vs_oracle(mdpvi):
    insts = _instances()
    b, pi, Vp, grads, objs, w, pig, Vg = _batch_pipeline(mdpvi, insts)
    pi_h, Vp_h, pig_h, Vg_h = (t.cpu().numpy() for t in (pi, Vp, pig, Vg))
    for i, p in enumerate(insts):
        sl = slice(b.offsets[i], b.offsets[i + 1])
        print(f"instance {i}: K={p.K} C={p.C} J={p.J} N={p.num_states}", flush=True)
        if p.num_states > 30_000:
            # the oracle needs minutes here; these instances are compared bit
            # for bit with the single-instance path in the next test
            continue
        g = vi.grid(p)
        star = vi.value_iteration(p, 1e-13, g=g).V
        pi_o, gap_o = vi.extract(p, star, g)
        V_o = vi.policy_eval(p, pi_o, tol=1e-13, g=g)
        mask = gap_mask(vi.q_table(p, star, g).max(axis=1), gap_o, star)
        assert np.array_equal(pi_h[sl][mask], pi_o[mask])
        # the GPU policy's value and gradient against the oracle's for that policy
        V_pi = vi.policy_eval(p, pi_h[sl], tol=1e-13, g=g)
        assert np.max(np.abs(Vp_h[sl] - V_pi)) <= EVAL_REL * np.max(np.abs(V_pi))
        assert abs(objs[i] - vi.objective(p, V_pi)) <= 1e-10 * max(1.0, abs(objs[i]))
        g_o = grad.gradient_adjoint(p, pi_h[sl], V=V_pi)
        assert np.max(np.abs(np.array(grads[i]) - g_o)) <= 1e-5 * np.max(np.abs(g_o))
        _near_optimal(p, Vp_h[sl], V_o)
        pg_o = vi.greedy_policy(p, "least_loaded", g)
        assert np.array_equal(pig_h[sl], pg_o)
        Vg_o = vi.policy_eval(p, pg_o, tol=1e-13, g=g)
        assert np.max(np.abs(Vg_h[sl] - Vg_o)) <= EVAL_REL * np.max(np.abs(Vg_o))
        assert np.all(Vg_h[sl] <= Vp_h[sl] + 1e-9 * np.max(np.abs(V_o)))


IMPROVE_TOL = 1e-9


def _near_optimal(p, V, V_star, eval_tol=1e-12):
    """A policy that no improvement by more than IMPROVE_TOL changes, with
    values from an evaluation stopped at eval_tol (error bound b =
    gamma/(1-gamma) eval_tol), is within (IMPROVE_TOL + 2 gamma b)/(1 - gamma)
    of optimal."""
    scale = np.max(np.abs(V_star))
    b = p.gamma / (1 - p.gamma) * eval_tol
    assert np.all(V <= V_star + EVAL_REL * scale)
    assert np.all(V >= V_star - (IMPROVE_TOL + 2 * p.gamma * b) / (1 - p.gamma) - EVAL_REL * scale)


def test_batch_gradient_equals_single_instance(mdpvi):
    import torch
    insts = _instances()
    b, pi, Vp, grads, objs, w, pig, Vg = _batch_pipeline(mdpvi, insts)
    for i, p in enumerate(insts):
        sl = slice(b.offsets[i], b.offsets[i + 1])
        mdp = mdpvi.MDP.from_instance(p)
        g1, J1, w1, _ = mdp.vi_adjoint(pi[sl].contiguous(), Vp[sl].contiguous(), tol=1e-11)
        assert np.array_equal(np.array(g1), np.array(grads[i])), i
        assert np.array_equal(w1.cpu().numpy().view(np.uint32), w[sl].cpu().numpy().view(np.uint32)), i
        V1, _ = mdp.policy_eval(pig[sl].contiguous(), Vp[sl].clone(), tol=1e-12)
        assert np.array_equal(V1.cpu().numpy().view(np.uint64), Vg[sl].cpu().numpy().view(np.uint64)), i


def test_batch_policy_iteration_equals_single_instance(mdpvi):
    """Batched policy iteration stops each instance at its own first stable
    improvement: per instance the same evaluations, final policy and value
    bits as policy_iteration on that instance alone."""
    import torch
    insts = _instances()
    b = mdpvi.Batch(insts)
    V = torch.zeros(b.num_states, device="cuda")
    for i, p in enumerate(insts):
        V[b.offsets[i]:b.offsets[i + 1]] = sub_solution(p)
    b.vi_solve(V, tol=1e-6)
    pi0, _ = b.policy_extract(V, want_gap=False)
    pi, Vp = pi0.clone(), V.double()
    _, rounds = b.policy_iteration(pi, Vp, eval_tol=1e-12, improve_tol=IMPROVE_TOL)
    print("rounds per instance", rounds, flush=True)
    assert max(rounds) > 1
    for i, p in enumerate(insts):
        sl = slice(b.offsets[i], b.offsets[i + 1])
        mdp = mdpvi.MDP.from_instance(p)
        pi1 = pi0[sl].clone()
        V1 = V[sl].double()
        _, _, _, r1 = mdp.policy_iteration(pi1, V1, eval_tol=1e-12, improve_tol=IMPROVE_TOL)
        assert r1 == rounds[i], (i, r1, rounds[i])
        assert torch.equal(pi1, pi[sl]), i
        assert np.array_equal(V1.cpu().numpy().view(np.uint64), Vp[sl].cpu().numpy().view(np.uint64)), i


def _eval_residual(p, pi, V):
    """||r_pi + gamma P_pi V - V||_inf with the oracle's P_pi and r_pi."""
    P, r = vi.policy_system(p, pi)
    V = np.asarray(V, dtype=np.float64)
    return np.max(np.abs(r + p.gamma * (P @ V) - V))


def _adjoint_residual(p, pi, w):
    P, _ = vi.policy_system(p, pi)
    n_occ = (p.C + 1) ** p.K
    c = np.zeros(P.shape[0])
    lam = np.asarray(p.lam)
    c[np.arange(p.J) * n_occ] = lam / lam.sum()
    w = np.asarray(w, dtype=np.float64)
    return np.abs(c + p.gamma * (P.T @ w) - w).sum()


@pytest.mark.timeout(900)
def test_batch_pipeline_first_256_of_sweep(mdpvi):
    """The batched gradient and greedy-scoring pipeline on the first 256
    instances of the 512-instance parameter sweep (the bench workload):

    * every instance's gradient, adjoint weights, greedy policy and greedy
      FP64 value equal the single-instance entry points' bit for bit;
    * every instance's values are a fixed point of the oracle's Bellman
      operator (half an FP32 ulp plus the stopping residual); its FP64 policy
      value satisfies the oracle's fixed-policy equation to 1e-10 relative;
      its policy is greedy with respect to that value under the oracle's Q
      (so it is optimal); its adjoint weights satisfy the adjoint equation;
    * the instances of at most 30,000 states (190 of them) against the
      oracle's full pipeline: policy on the parity gap mask of the oracle's
      optimal policy; FP64 value, objective and gradient against the oracle's
      for the GPU's policy, and the value within IMPROVE_TOL / (1 - gamma) of
      the optimal one; greedy policy and its value."""
    import torch

    from tests.oracle_pool import batch_oracle
    insts = W.batch(512, seed=3)[:256]
    small = [i for i, p in enumerate(insts) if p.num_states <= 30_000]
    b, pi, Vp, grads, objs, w, pig, Vg = _batch_pipeline(mdpvi, insts)
    V32 = _batch_pipeline.last_V.cpu().numpy()
    pi_h, Vp_h, pig_h, Vg_h, w_h = (t.cpu().numpy() for t in (pi, Vp, pig, Vg, w))
    for i, p in enumerate(insts):
        sl = slice(b.offsets[i], b.offsets[i + 1])
        mdp = mdpvi.MDP.from_instance(p)
        g1, J1, w1, _ = mdp.vi_adjoint(pi[sl].contiguous(), Vp[sl].contiguous(), tol=1e-11)
        assert np.array_equal(np.array(g1), np.array(grads[i])), i
        assert np.array_equal(w1.cpu().numpy().view(np.uint32), w_h[sl].view(np.uint32)), i
        pg1 = mdp.policy_greedy("least_loaded")
        assert np.array_equal(pg1.cpu().numpy(), pig_h[sl]), i
        V1, _ = mdp.policy_eval(pig[sl].contiguous(), Vp[sl].clone(), tol=1e-12)
        assert np.array_equal(V1.cpu().numpy().view(np.uint64), Vg_h[sl].view(np.uint64)), i
        # properties at any size, with the oracle's operators
        v = V32[sl].astype(np.float64)
        half_ulp = np.spacing(np.abs(V32[sl])).astype(np.float64) / 2
        assert np.max(np.abs(vi.bellman(p, v) - v) - 1.0001 * half_ulp) <= 1e-7, i
        scale = np.max(np.abs(Vp_h[sl]))
        assert _eval_residual(p, pi_h[sl], Vp_h[sl]) <= 1e-10 * scale, i
        Q = vi.q_table(p, Vp_h[sl])
        chosen = Q[np.arange(p.num_states), pi_h[sl].astype(np.int64)]
        assert np.all(chosen >= Q.max(axis=1) - 1e-9 * scale), i
        assert _adjoint_residual(p, pi_h[sl], w_h[sl]) <= 1e-6 * np.abs(w_h[sl]).sum(), i
        assert _eval_residual(p, pig_h[sl], Vg_h[sl]) <= 1e-10 * np.max(np.abs(Vg_h[sl])), i
        if i % 32 == 31:
            print(f"instances 0..{i}: checks hold", flush=True)
    print(f"256 instances: single-instance bit identity and oracle properties hold; "
          f"oracle pipeline on {len(small)} instances", flush=True)
    ref = batch_oracle(small, 512, 3, policies={i: pi_h[b.offsets[i]:b.offsets[i + 1]] for i in small})
    for i in small:
        p, o = insts[i], ref[i]
        sl = slice(b.offsets[i], b.offsets[i + 1])
        assert np.array_equal(pi_h[sl][o["mask"]], o["pi"][o["mask"]]), i
        assert np.max(np.abs(Vp_h[sl] - o["V_pi"])) <= EVAL_REL * np.max(np.abs(o["V_pi"])), i
        assert abs(objs[i] - o["J_pi"]) <= 1e-10 * max(1.0, abs(o["J_pi"])), i
        assert np.max(np.abs(np.array(grads[i]) - o["grad_pi"])) <= 1e-5 * np.max(np.abs(o["grad_pi"])), i
        _near_optimal(p, Vp_h[sl], o["V"])
        assert np.array_equal(pig_h[sl], o["greedy"]), i
        assert np.max(np.abs(Vg_h[sl] - o["V_greedy"])) <= EVAL_REL * np.max(np.abs(o["V_greedy"])), i


def _line_table_batch(with_k6):
    out = [
        W.make(1, 6, (1, 2), (0.8, 0.4), 0.1, 0.02, (1.0, 2.5), 0.95),                   # K = 1
        W.make(2, 16, (1, 2, 3), (0.5, 0.4, 0.3), 0.1, 0.02, (1.0, 2.0, 3.0), 0.96),     # C + 1 > 16
        W.make(5, 2, (1, 2), (0.6, 0.3), 0.1, 0.02, (1.0, 2.0), 0.95),                   # C + 1 = 3
        W.make(5, 3, (1, 2, 3), (0.6, 0.3, 0.2), 0.1, 0.02, (1.0, 2.0, 3.5), 0.95),
        W.make(4, 5, (2,), (1.0,), 0.1, 0.02, (2.0,), 0.95),                             # J = 1
        W.make(3, 9, (1, 1), (0.7, 0.5), 0.1, 0.02, (1.0, 1.5), 0.97, idle_unit_cost=0.05),
        W.gradient_instance(3, 6),
    ]
    if with_k6:   # a host count past the exact round backups: every instance generic
        out.append(W.make(6, 2, (1, 2), (0.8, 0.4), 0.1, 0.02, (1.0, 2.5), 0.95))
    return out


@pytest.mark.parametrize("with_k6", [False, True])
def test_batch_adjoint_line_table_equals_single_instance(mdpvi, with_k6):
    """The batched adjoint with its precomputed reset-line sums (exact round
    backups) and without them (a batch with K = 6 takes the generic backup)
    gives the single-instance adjoint's bits: K = 1, lines longer than 16,
    lines of 3, J = 1, equal task sizes."""
    insts = _line_table_batch(with_k6)
    b = mdpvi.Batch(insts)
    pig = b.policy_greedy("least_loaded")
    import torch
    V0 = torch.zeros(b.num_states, dtype=torch.float64, device="cuda")
    Vg, _, _, _ = b.policy_eval(pig, V0, tol=1e-12)
    grads, objs, w, st, its = b.vi_adjoint(pig, Vg, [p.J for p in insts], tol=1e-11)
    for i, p in enumerate(insts):
        sl = slice(b.offsets[i], b.offsets[i + 1])
        mdp = mdpvi.MDP.from_instance(p)
        g1, J1, w1, _ = mdp.vi_adjoint(pig[sl].contiguous(), Vg[sl].contiguous(), tol=1e-11)
        assert np.array_equal(w1.cpu().numpy().view(np.uint32), w[sl].cpu().numpy().view(np.uint32)), i
        assert np.allclose(np.array(g1), np.array(grads[i]), rtol=1e-12, atol=0.0), i
