"""GPU parity of the adjoint gradient (vi_adjoint) and the autograd Function.

Small instances: the adjoint weights w and dJ/dtheta against the oracle's
sparse adjoint route and its dense autograd route; the gradient instance at
full size (322,102 states) against the oracle's stored adjoint gradient and
central finite differences (tests/golden/gradient_K5C10.json, written by the
oracle-only script beside it); two exact identities on the GPU result.

Tolerance: w is FP32 with FP64 sums (one rounding per state and sweep), so
its error is bounded by 2^-24 ||w|| / (1 - gamma) plus the stopping error;
the gradient then carries a relative error of the same order (<= 1e-5 for
gamma <= 0.98), while the FD reference itself is good to about 1e-7.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import grad, vi
from tests.gpu_util import gap_mask, torch_cuda

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def mdpvi():
    torch_cuda()
    import paper_2012_12419_amd as m
    m.load()
    return m


def _gpu_pipeline(mdpvi, inst, tol=1e-7, adjoint_tol=1e-11):
    import torch
    mdp = mdpvi.MDP.from_instance(inst)
    V = torch.zeros(mdp.num_states, device="cuda")
    mdp.vi_solve(V, tol=tol)
    pi, _ = mdp.policy_extract(V, want_gap=False)
    Vp = V.double()
    for _ in range(8):
        mdp.policy_eval(pi, Vp, tol=1e-12)
        pi2, _ = mdp.policy_extract(Vp, want_gap=False)
        if torch.equal(pi2, pi):
            break
        pi = pi2
    g, Jv, w, st = mdp.vi_adjoint(pi, Vp, tol=adjoint_tol)
    return mdp, pi, Vp, np.array(g), Jv, w, st


SMALL = [("dense_copy_K2C6", W.gradient_instance(2, 6)),
         ("small_parity", W.small_parity()),
         ("K3C5J3", W.make(3, 5, (1, 2, 3), (0.5, 0.4, 0.3), 0.12, 0.03, (1.0, 2.2, 3.1), 0.96)),
         ("reject_cost", W.make(2, 6, (1, 2), (0.7, 0.5), 0.1, 0.02, (0.3, 4.0), 0.95,
                                reject_cost=(0.2, 0.6))),
         ("penalty", W.make(3, 5, (1, 2), (0.9, 0.5), 0.1, 0.02, (1.0, 2.5), 0.95, idle_unit_cost=0.1))]


@pytest.mark.parametrize("name,inst", SMALL, ids=[s[0] for s in SMALL])
def test_adjoint_small(mdpvi, name, inst):
    gd = vi.grid(inst)
    star = vi.value_iteration(inst, 1e-13, g=gd).V
    pi_o, _ = vi.extract(inst, star, gd)
    V_o = vi.policy_eval(inst, pi_o, tol=1e-13, g=gd)
    w_o = grad.adjoint_weights(inst, pi_o, g=gd)
    g_o = grad.gradient_adjoint(inst, pi_o, V=V_o, w=w_o)

    mdp, pi, Vp, g, Jv, w, st = _gpu_pipeline(mdpvi, inst)
    # policies agree wherever the oracle's best-vs-second gap is clear (exact
    # ties between equivalent hosts may resolve either way in FP64)
    gap_o = vi.extract(inst, star, gd)[1]
    Q1 = vi.q_table(inst, star, gd).max(axis=1)
    mask = gap_mask(Q1, gap_o, star)
    assert np.array_equal(pi.cpu().numpy()[mask], pi_o[mask])
    assert abs(Jv - vi.objective(inst, V_o)) <= 1e-10 * abs(Jv)
    if np.array_equal(pi.cpu().numpy(), pi_o):
        # the adjoint weights depend on how ties are routed; compare them
        # element by element when both sides resolved every tie alike
        w_g = w.cpu().numpy().astype(np.float64)
        assert np.max(np.abs(w_g - w_o)) <= 1e-5 * np.max(np.abs(w_o))
        assert np.abs(w_g - w_o).sum() <= 1e-5 * np.abs(w_o).sum()
    scale = np.max(np.abs(g_o))
    assert np.max(np.abs(g - g_o)) <= 1e-5 * scale, (g, g_o)
    if inst.num_states <= 200:
        assert np.allclose(g, grad.gradient_dense(inst, pi_o), rtol=1e-5, atol=1e-5 * scale)
    # identities: rate scale invariance; reward homogeneity when c = 0
    th = grad.theta_of(inst)
    J = inst.J
    assert abs(th[:J + 2] @ g[:J + 2]) <= 1e-5 * scale * np.abs(th[:J + 2]).sum()
    if max(inst.reject_cost) == 0 and inst.idle_unit_cost == 0:
        assert abs(th[J + 2:] @ g[J + 2:] - Jv) <= 1e-5 * abs(Jv)


def test_adjoint_gradient_instance_vs_golden(mdpvi):
    with open(os.path.join(HERE, "golden", "gradient_K5C10.json")) as f:
        gold = json.load(f)
    inst = W.gradient_instance()
    mdp, pi, Vp, g, Jv, w, st = _gpu_pipeline(mdpvi, inst)
    print(f"adjoint sweeps {st['iterations']}, {st['seconds']:.4f} s", flush=True)
    assert abs(Jv - gold["J"]) <= 1e-9 * abs(gold["J"])
    ga = np.array(gold["grad_adjoint"])
    fd = np.array(gold["grad_fd"])
    scale = np.max(np.abs(ga))
    assert np.max(np.abs(g - ga)) <= 1e-5 * scale, (g, ga)
    assert np.max(np.abs(g - fd)) <= 1e-4 * scale, (g, fd)
    assert sum(np.bincount(pi.cpu().numpy(), minlength=inst.K + 1)) == inst.num_states


def test_adjoint_deterministic(mdpvi):
    inst = W.make(4, 7, (1, 2), (0.6, 0.3), 0.1, 0.02, (1.0, 2.5), 0.97)
    a = _gpu_pipeline(mdpvi, inst)
    b = _gpu_pipeline(mdpvi, inst)
    assert np.array_equal(a[3], b[3])
    assert np.array_equal(a[5].cpu().numpy().view(np.uint32), b[5].cpu().numpy().view(np.uint32))


def test_autograd_function(mdpvi):
    import torch
    from paper_2012_12419_amd.autograd import expected_reward
    inst = W.gradient_instance(3, 6)
    lam = torch.tensor(inst.lam, dtype=torch.float64, requires_grad=True)
    mu = torch.tensor(inst.mu, dtype=torch.float64, requires_grad=True)
    nu = torch.tensor(inst.nu, dtype=torch.float64, requires_grad=True)
    r = torch.tensor(inst.reward, dtype=torch.float64, requires_grad=True)
    Jt = expected_reward(lam, mu, nu, r, inst.K, inst.C, inst.size, inst.gamma, tol=1e-7)
    (2.0 * Jt).backward()
    gd = vi.grid(inst)
    star = vi.value_iteration(inst, 1e-13, g=gd).V
    pi_o, _ = vi.extract(inst, star, gd)
    g_o = grad.gradient_adjoint(inst, pi_o)
    got = np.concatenate([lam.grad.numpy(), [mu.grad.item(), nu.grad.item()], r.grad.numpy()])
    assert np.max(np.abs(got - 2.0 * g_o)) <= 1e-5 * np.max(np.abs(2.0 * g_o))
    assert abs(Jt.item() - vi.objective(inst, vi.policy_eval(inst, pi_o))) <= 1e-9 * abs(Jt.item())
