"""GPU parity of the adjoint gradient (vi_adjoint) and the autograd Function.

Small instances: the adjoint weights w and dJ/dtheta against the oracle's
sparse adjoint route and its dense autograd route; the gradient instance at
full size (322,102 states) against the oracle's stored adjoint gradient and
central finite differences (tests/golden/gradient_K5C10.json) and its
optimal policy (tests/golden/policy_gradient.json), both written by the
oracle-only scripts beside them; two exact identities on the GPU result.
Adjoint weights are compared summed over host-permutation orbits, which does
not depend on how either side routed exact ties between equivalent hosts,
and through the residual of the adjoint equation.

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
from oracle import grad, summary, vi
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


def _adjoint_residual(inst, pi, w):
    """1-norm of c + gamma P_pi^T w - w with the oracle's P_pi for the policy
    the GPU used (a property of the GPU's w at any size)."""
    P, _ = vi.policy_system(inst, pi)
    n_occ = (inst.C + 1) ** inst.K
    c = np.zeros(P.shape[0])
    lam = np.asarray(inst.lam)
    c[np.arange(inst.J) * n_occ] = lam / lam.sum()
    w = np.asarray(w, dtype=np.float64)
    return np.abs(c + inst.gamma * (P.T @ w) - w).sum()


@pytest.mark.parametrize("name,inst", SMALL, ids=[s[0] for s in SMALL])
def test_adjoint_small(mdpvi, name, inst):
    gd = vi.grid(inst)
    star = vi.value_iteration(inst, 1e-13, g=gd).V
    pi_o, gap_o = vi.extract(inst, star, gd)
    V_o = vi.policy_eval(inst, pi_o, tol=1e-13, g=gd)
    w_o = grad.adjoint_weights(inst, pi_o, g=gd)
    g_o = grad.gradient_adjoint(inst, pi_o, V=V_o, w=w_o)
    # these instances have no near tie between actions of different target
    # loads down to 1e-10 relative, so the FP64-polished GPU policy must
    # choose the oracle's target load at every state
    assert summary.ambiguous(inst, star, 1e-10, gd).size == 0

    mdp, pi, Vp, g, Jv, w, st = _gpu_pipeline(mdpvi, inst)
    pi_h = pi.cpu().numpy()
    # policies agree wherever the oracle's best-vs-second gap is clear (exact
    # ties between equivalent hosts may resolve either way in FP64)
    Q1 = vi.q_table(inst, star, gd).max(axis=1)
    mask = gap_mask(Q1, gap_o, star)
    assert np.array_equal(pi_h[mask], pi_o[mask])
    assert np.array_equal(summary.target_load(inst, pi_h, gd), summary.target_load(inst, pi_o, gd))
    assert abs(Jv - vi.objective(inst, V_o)) <= 1e-10 * abs(Jv)
    # adjoint weights: summed over host-permutation orbits they do not depend
    # on how ties between equivalent hosts were routed
    w_g = w.cpu().numpy().astype(np.float64)
    og, oo = summary.orbit_sum(inst, w_g, gd), summary.orbit_sum(inst, w_o, gd)
    assert np.max(np.abs(og - oo)) <= 1e-5 * np.max(np.abs(oo))
    assert np.abs(og - oo).sum() <= 1e-5 * np.abs(oo).sum()
    if np.array_equal(pi_h, pi_o):
        assert np.max(np.abs(w_g - w_o)) <= 1e-5 * np.max(np.abs(w_o))
    assert _adjoint_residual(inst, pi_h, w_g) <= 1e-6 * np.abs(w_g).sum()
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
    """The gradient instance at full size (322,102 states) against oracle-only
    stored values: J and dJ/dtheta (adjoint and central differences); the
    policy through its target loads per host-permutation orbit
    (policy_gradient.json), on every state outside the oracle's near ties at
    1e-6 relative (the policy parity bar) and at 1e-10; the adjoint weights
    through their orbit sums against the oracle's weights of the stored
    optimal policy, and through the residual of the adjoint equation."""
    with open(os.path.join(HERE, "golden", "gradient_K5C10.json")) as f:
        gold = json.load(f)
    with open(os.path.join(HERE, "golden", "policy_gradient.json")) as f:
        pol = json.load(f)
    inst = W.gradient_instance()
    gd = vi.grid(inst)
    mdp, pi, Vp, g, Jv, w, st = _gpu_pipeline(mdpvi, inst)
    print(f"adjoint sweeps {st['iterations']}, {st['seconds']:.4f} s", flush=True)
    assert abs(Jv - gold["J"]) <= 1e-9 * abs(gold["J"])
    assert abs(Jv - pol["J"]) <= 1e-9 * abs(pol["J"])
    ga = np.array(gold["grad_adjoint"])
    fd = np.array(gold["grad_fd"])
    scale = np.max(np.abs(ga))
    assert np.max(np.abs(g - ga)) <= 1e-5 * scale, (g, ga)
    assert np.max(np.abs(g - fd)) <= 1e-4 * scale, (g, fd)

    pi_h = pi.cpu().numpy()
    tl = summary.target_load(inst, pi_h, gd)
    for key in ("orbit_target_load", "orbit_target_load_strict"):
        want = summary.expand_orbit_table(inst, pol[key], gd)
        known = want != -2
        bad = np.flatnonzero(known & (tl != want))
        print(f"{key}: {known.sum()} states compared, {bad.size} differ", flush=True)
        assert bad.size == 0, bad[:10]
    all_tl = summary.expand_orbit_table(inst, pol["orbit_target_load_all"], gd)
    assert summary.histogram(inst, all_tl) == pol["target_load_histogram"]
    pi_o = summary.policy_from_target_load(inst, all_tl, gd)
    w_o = grad.adjoint_weights(inst, pi_o, tol=1e-12, g=gd)
    w_g = w.cpu().numpy().astype(np.float64)
    og, oo = summary.orbit_sum(inst, w_g, gd), summary.orbit_sum(inst, w_o, gd)
    print(f"orbit-summed w: max rel diff {np.max(np.abs(og - oo)) / np.max(np.abs(oo)):.2e}", flush=True)
    assert np.max(np.abs(og - oo)) <= 1e-5 * np.max(np.abs(oo))
    assert np.abs(og - oo).sum() <= 1e-5 * np.abs(oo).sum()
    assert _adjoint_residual(inst, pi_h, w_g) <= 1e-6 * np.abs(w_g).sum()


def test_adjoint_deterministic(mdpvi):
    inst = W.make(4, 7, (1, 2), (0.6, 0.3), 0.1, 0.02, (1.0, 2.5), 0.97)
    a = _gpu_pipeline(mdpvi, inst)
    b = _gpu_pipeline(mdpvi, inst)
    assert np.array_equal(a[3], b[3])
    assert np.array_equal(a[5].cpu().numpy().view(np.uint32), b[5].cpu().numpy().view(np.uint32))


AUTOGRAD = [("K3C6", W.gradient_instance(3, 6)),
            ("penalty", W.make(3, 5, (1, 2), (0.9, 0.5), 0.1, 0.02, (1.0, 2.5), 0.95,
                               idle_unit_cost=0.1))]


@pytest.mark.parametrize("name,inst", AUTOGRAD, ids=[a[0] for a in AUTOGRAD])
def test_autograd_function(mdpvi, name, inst):
    import torch
    from paper_2012_12419_amd.autograd import expected_reward
    lam = torch.tensor(inst.lam, dtype=torch.float64, requires_grad=True)
    mu = torch.tensor(inst.mu, dtype=torch.float64, requires_grad=True)
    nu = torch.tensor(inst.nu, dtype=torch.float64, requires_grad=True)
    r = torch.tensor(inst.reward, dtype=torch.float64, requires_grad=True)
    Jt = expected_reward(lam, mu, nu, r, inst.K, inst.C, inst.size, inst.gamma,
                         reject_cost=inst.reject_cost, idle_unit_cost=inst.idle_unit_cost, tol=1e-7)
    (2.0 * Jt).backward()
    gd = vi.grid(inst)
    star = vi.value_iteration(inst, 1e-13, g=gd).V
    pi_o, _ = vi.extract(inst, star, gd)
    g_o = grad.gradient_adjoint(inst, pi_o)
    got = np.concatenate([lam.grad.numpy(), [mu.grad.item(), nu.grad.item()], r.grad.numpy()])
    assert np.max(np.abs(got - 2.0 * g_o)) <= 1e-5 * np.max(np.abs(2.0 * g_o))
    assert abs(Jt.item() - vi.objective(inst, vi.policy_eval(inst, pi_o))) <= 1e-9 * abs(Jt.item())


FORM_SHAPES = [("gradient_K5C10J2", W.gradient_instance()),
               ("K3C5J3", W.make(3, 5, (1, 2, 3), (0.5, 0.4, 0.3), 0.12, 0.03, (1.0, 2.2, 3.1), 0.96)),
               ("K4C15J1", W.make(4, 15, (2,), (2.0,), 0.1, 0.02, (1.0,), 0.97)),
               ("K6C4J3", W.make(6, 4, (1, 2, 3), (0.9, 0.6, 0.3), 0.1, 0.02, (1.0, 2.0, 3.5), 0.97)),
               ("K8C3J2", W.make(8, 3, (1, 2), (1.5, 0.8), 0.1, 0.03, (1.0, 2.5), 0.95,
                                 idle_unit_cost=0.05)),
               ("K7C2J1", W.make(7, 2, (1,), (1.2,), 0.1, 0.02, (1.0,), 0.96))]


@pytest.mark.parametrize("name,inst", FORM_SHAPES, ids=[f[0] for f in FORM_SHAPES])
def test_adjoint_forms_bit_identical(mdpvi, name, inst):
    """Every adjoint sweep form (group, exact-shape with 1/2/4 occupancies
    per thread, generic with 1/4) gives the same w bit for bit and the same
    gradient, for the least-loaded policy: groups per workgroup from 1
    (C = 15) to 28 (C = 2), a last workgroup with groups past the end, and
    lanes past the last whole group."""
    import torch
    mdp = mdpvi.MDP.from_instance(inst)
    pi = mdp.policy_greedy("least_loaded")
    Vp = torch.zeros(mdp.num_states, dtype=torch.float64, device="cuda")
    mdp.policy_eval(pi, Vp, tol=1e-11)
    ref = None
    for form in (mdpvi.ADJOINT_GROUP, mdpvi.ADJOINT_EXACT + 1, mdpvi.ADJOINT_EXACT + 2,
                 mdpvi.ADJOINT_EXACT + 4, 1, 4):
        mdp.set_adjoint_form(form)
        assert mdp.adjoint_form() == form
        g, Jv, w, st = mdp.vi_adjoint(pi, Vp, tol=1e-9)
        got = (np.array(g), Jv, w.cpu().numpy().view(np.uint32).copy(), st["iterations"])
        if ref is None:
            ref = got
            continue
        assert got[3] == ref[3], (form, got[3], ref[3])
        assert np.array_equal(got[2], ref[2]), form
        assert np.array_equal(got[0], ref[0]) and got[1] == ref[1], form
    mdp.set_adjoint_form(0)


def test_adjoint_form_rejected_where_it_does_not_apply(mdpvi):
    big_c = mdpvi.MDP.from_instance(W.make(3, 16, (1,), (1.0,), 0.1, 0.02, (1.0,), 0.95))
    with pytest.raises(mdpvi.MdpviError) as e:
        big_c.set_adjoint_form(mdpvi.ADJOINT_GROUP)
    assert e.value.code == mdpvi.EINVAL
    big_c.set_adjoint_form(mdpvi.ADJOINT_EXACT + 1)
    assert big_c.adjoint_form() == mdpvi.ADJOINT_EXACT + 1
    with pytest.raises(mdpvi.MdpviError):
        big_c.set_adjoint_form(3)
