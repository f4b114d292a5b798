"""GPU parity of the batched solver.

* A mixed batch (LDS-resident and round-form instances, ragged sizes) against
  the FP64 oracle instance by instance.
* The 512-instance parameter sweep: every instance's batched result equals
  the single-instance vi_solve result bit for bit (same backup arithmetic, same
  stopping test), and every instance is a fixed point of the oracle's
  Bellman operator up to one FP32 rounding.
"""
import numpy as np
import pytest

import workloads as W
from oracle import vi
from tests.gpu_util import sub_solution, torch_cuda, vi_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdpvi():
    torch_cuda()
    import paper_2012_12419_amd as m
    m.load()
    return m


def _mixed():
    out = list(W.batch(20, seed=7))
    out.append(W.make(4, 12, (1, 2, 3), (0.6, 0.5, 0.3), 0.08, 0.02, (1.0, 2.1, 3.3), 0.97))  # 85,683
    out.append(W.make(5, 6, (1, 2), (0.9, 0.4), 0.1, 0.02, (1.0, 2.4), 0.95))                 # 33,614
    out.append(W.make(1, 1, (1,), (0.5,), 0.3, 0.1, (1.0,), 0.9))                             # 2
    out.append(W.make(2, 4, (1,), (0.7,), 0.1, 0.02, (1.2,), 0.93))                           # 25
    out.append(W.make(3, 6, (1, 2), (0.8, 0.3), 0.1, 0.02, (1.0, 2.4), 0.94, idle_unit_cost=0.15))  # 686
    return out


def test_batch_mixed_vs_oracle(mdpvi):
    import torch
    insts = _mixed()
    b = mdpvi.Batch(insts)
    V = torch.zeros(b.num_states, device="cuda")
    for i, p in enumerate(insts):
        V[b.offsets[i]:b.offsets[i + 1]] = sub_solution(p)
    st, its, res = b.vi_solve(V, tol=1e-7)
    Vh = V.cpu().numpy()
    assert b.feasible_pairs == sum(vi.feasible_pairs(p) for p in insts)
    for i, p in enumerate(insts):
        print(f"instance {i}: K={p.K} C={p.C} J={p.J} N={p.num_states} sweeps={its[i]}", flush=True)
        assert res[i] < 1e-7
        Vi = Vh[b.offsets[i]:b.offsets[i + 1]]
        if p.num_states <= 20_000:
            star = vi.value_iteration(p, 1e-12).V
            vi_close(Vi, star)
        else:
            # one oracle sweep from the GPU's values: a fixed point up to one
            # FP32 rounding plus gamma times the stopping residual
            Vg = Vi.astype(np.float64)
            TV = vi.bellman(p, Vg)
            half_ulp = np.spacing(np.abs(Vi)).astype(np.float64) / 2
            assert np.all(np.abs(TV - Vg) <= 1.0001 * half_ulp + 1e-7)


def test_batch_equals_per_instance(mdpvi):
    """All 512 instances of the parameter sweep: the batched iterate equals the
    single-instance vi_solve iterate bit for bit, with the same sweep count,
    and every instance is a fixed point of the oracle's Bellman operator up
    to half an FP32 ulp plus the stopping residual (one vectorised oracle
    sweep per instance), which bounds ||V - V*|| by that over (1 - gamma)."""
    import torch
    insts = W.batch(512, seed=3)
    b = mdpvi.Batch(insts)
    V = torch.zeros(b.num_states, device="cuda")
    st, its, res = b.vi_solve(V, tol=1e-6)
    print(f"batch: {b.n} instances, {b.num_states} states, {st['seconds']:.3f} s", flush=True)
    Vh = V.cpu().numpy()
    worst = 0.0
    for i, p in enumerate(insts):
        mdp = mdpvi.MDP.from_instance(p)
        Vi = torch.zeros(mdp.num_states, device="cuda")
        sti = mdp.vi_solve(Vi, tol=1e-6)
        assert sti["iterations"] == its[i], (i, sti["iterations"], its[i])
        got = Vh[b.offsets[i]:b.offsets[i + 1]]
        assert np.array_equal(got.view(np.uint32), Vi.cpu().numpy().view(np.uint32)), i
        Vg = got.astype(np.float64)
        TV = vi.bellman(p, Vg)
        half_ulp = np.spacing(np.abs(got)).astype(np.float64) / 2
        excess = np.max(np.abs(TV - Vg) - 1.0001 * half_ulp)
        assert excess <= 1e-6, (i, p.K, p.C, p.J, excess)
        worst = max(worst, excess)
    print(f"all 512 bit-identical; largest fixed-point excess over half an ulp {worst:.2e}", flush=True)


def _round_forms_cases():
    base = [W.make(4, 12, (1, 1), (0.6, 0.4), 0.1, 0.02, (1.0, 1.3), 0.95),     # repeated sizes, 57,122 states
            W.make(5, 6, (1, 2, 3), (0.9, 0.4, 0.3), 0.1, 0.02, (1.0, 2.4, 3.1), 0.96),  # 50,421
            W.make(3, 4, (1, 2), (0.8, 0.3), 0.1, 0.02, (1.0, 2.4), 0.94)]     # 250: LDS-resident
    return {"exact_kernel": base + list(W.batch(6, seed=11)),
            "generic_kernel": base + [W.make(6, 5, (1,), (1.1,), 0.1, 0.02, (1.0,), 0.95)]}  # K=6: 46,656


@pytest.mark.parametrize("case", ["exact_kernel", "generic_kernel"])
def test_batch_round_forms_bit_identical_and_tuned(mdpvi, case):
    """Round kernels with 1, 2 and 4 occupancies per thread give the same bits
    for value iteration, FP64 evaluation and the adjoint (instances of up to
    5 hosts through the exact-shape backups, with a repeated task size taking
    the generic one inside them; a 6-host instance sends the batch to the
    generic kernels); batch_autotune records a choice per operation that a
    second batch of the same instance shapes then uses."""
    import torch
    insts = _round_forms_cases()[case]
    b = mdpvi.Batch(insts)
    lb = torch.zeros(b.num_states, device="cuda")
    for i, p in enumerate(insts):
        lb[b.offsets[i]:b.offsets[i + 1]] = sub_solution(p)
    outs = {}
    for opt in (1, 2, 4):
        for op in ("vi", "eval", "adjoint"):
            b.set_round_form(op, opt)
        assert b.round_forms() == {"vi": opt, "eval": opt, "adjoint": opt}
        V = lb.clone()
        b.vi_solve(V, tol=1e-6)
        pi, _ = b.policy_extract(V, want_gap=False)
        Vp, _, _, _ = b.policy_eval(pi, V.double(), tol=1e-11)
        grads, objs, w, _, _ = b.vi_adjoint(pi, Vp, [p.J for p in insts], tol=1e-10)
        outs[opt] = (V.cpu().numpy().view(np.uint32), Vp.cpu().numpy().view(np.uint64),
                     w.cpu().numpy().view(np.uint32), np.concatenate([np.array(g) for g in grads]))
    for opt in (2, 4):
        for x, y in zip(outs[1], outs[opt]):
            assert np.array_equal(x, y), opt
    for op in ("vi", "eval", "adjoint"):
        b.set_round_form(op, 0)
    rec = b.autotune(trials=3)
    print(f"{case}: tuned {rec}", flush=True)
    for op, (opt, us) in rec.items():
        assert opt in (1, 2, 4) and us > 0, (op, opt, us)
    other = mdpvi.Batch(insts)
    assert other.round_forms() == {op: rec[op][0] for op in rec}
    # the tile forms' choices recorded for these shapes reach a new batch too
    for op in ("vi", "eval"):
        b.set_tile_form(op, -1)
        assert other.tile_form_instances(op) == b.tile_form_instances(op), op
    with pytest.raises(mdpvi.MdpviError):
        other.set_round_form("vi", 3)
    with pytest.raises(mdpvi.MdpviError):
        other.set_tile_form("adjoint", 1)


def test_batch_tile_forms_bit_identical(mdpvi):
    """The tile forms of the round kernels (instances of 4 or 5 hosts and up
    to 3 distinct sizes, one (C+1)^3 tile per workgroup) give the direct round
    forms' results bit for bit, with the same sweep counts: value iteration to
    convergence from a sub-solution and stopped after an odd number of sweeps
    (the iterate then comes back from the second buffer), FP64 evaluation of
    the extracted policy and of the least-loaded one, and policy iteration.
    The batch mixes covered instances with ones the direct forms keep (a
    repeated task size, small tiles) and LDS-resident ones."""
    import torch
    insts = list(W.batch(64, seed=3)) + [
        W.make(4, 12, (1, 1), (0.6, 0.4), 0.1, 0.02, (1.0, 1.3), 0.95),      # repeated sizes: direct
        W.make(5, 6, (1, 2, 3), (0.9, 0.4, 0.3), 0.1, 0.02, (1.0, 2.4, 3.1), 0.96),
        W.make(4, 12, (2,), (0.9,), 0.1, 0.02, (2.0,), 0.95, idle_unit_cost=0.05)]   # J = 1, penalty
    b = mdpvi.Batch(insts)
    lb = torch.zeros(b.num_states, device="cuda")
    for i, p in enumerate(insts):
        lb[b.offsets[i]:b.offsets[i + 1]] = sub_solution(p)
    outs = {}
    for mode in (0, 1):
        b.set_tile_form("vi", mode)
        b.set_tile_form("eval", mode)
        n_vi, n_ev = b.tile_form_instances("vi"), b.tile_form_instances("eval")
        assert (n_vi > 0) == (mode == 1) and (n_ev > 0) == (mode == 1), (mode, n_vi, n_ev)
        V = lb.clone()
        st, its, res = b.vi_solve(V, tol=1e-6)
        V7 = lb.clone()
        with pytest.raises(mdpvi.MdpviError) as e:
            b.vi_solve(V7, tol=1e-30, max_iter=7)
        assert e.value.code == mdpvi.ENOCONV
        pi, _ = b.policy_extract(V, want_gap=False)
        Vp, _, eits, _ = b.policy_eval(pi, V.double(), tol=1e-11)
        pig = b.policy_greedy("least_loaded")
        Vg, _, gits, _ = b.policy_eval(pig, torch.zeros_like(Vp), tol=1e-11)
        Vpi = V.double()
        _, rounds = b.policy_iteration(pi, Vpi, eval_tol=1e-11, improve_tol=1e-9)
        outs[mode] = [V.cpu().numpy().view(np.uint32), list(its), V7.cpu().numpy().view(np.uint32),
                      Vp.cpu().numpy().view(np.uint64), list(eits), Vg.cpu().numpy().view(np.uint64), list(gits),
                      Vpi.cpu().numpy().view(np.uint64), pi.cpu().numpy(), list(rounds)]
        print(f"tile mode {mode}: {n_vi} value-iteration and {n_ev} evaluation instances in the tile form, "
              f"VI {st['seconds'] * 1e3:.1f} ms", flush=True)
    for k, (x, y) in enumerate(zip(outs[0], outs[1])):
        if isinstance(x, list):
            assert x == y, k
        else:
            assert np.array_equal(x, y), k
