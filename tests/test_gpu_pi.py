"""GPU parity of policy iteration (policy_iteration: FP64 evaluation sweeps
plus the tie-guarded improvement kernel) against the oracle's policy
iteration (oracle/pi.py) and value iteration."""
import numpy as np
import pytest

import workloads as W
from oracle import pi as pio, vi
from tests.gpu_util import EVAL_REL, VI_REL, gap_mask, torch_cuda, vi_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdpvi():
    torch_cuda()
    import paper_2012_12419_amd as m
    m.load()
    return m


CASES = [("small_parity", W.small_parity()),
         ("K3C5J3", W.make(3, 5, (1, 2, 3), (0.5, 0.4, 0.3), 0.12, 0.03, (1.0, 2.2, 3.1), 0.96)),
         ("reject", W.make(2, 6, (1, 2), (0.7, 0.5), 0.1, 0.02, (0.3, 4.0), 0.95, reject_cost=(0.2, 0.6))),
         ("tile_K4C9J3", W.make(4, 9, (1, 2, 3), (0.5, 0.4, 0.3), 0.1, 0.02, (1.0, 2.2, 3.1), 0.95)),
         ("penalty", W.make(3, 5, (1, 2), (0.6, 0.4), 0.1, 0.02, (1.0, 2.5), 0.95, idle_unit_cost=0.2))]


@pytest.mark.parametrize("name,p", CASES, ids=[c[0] for c in CASES])
def test_vs_oracle(mdpvi, name, p):
    import torch
    g = vi.grid(p)
    pi0 = vi.greedy_policy(p, "first_fit", g)
    pol_o, V_o, rounds_o = pio.policy_iteration(p, pi0, tol=1e-13, improve_tol=1e-8, g=g)
    star = vi.value_iteration(p, 1e-13, g=g).V
    mdp = mdpvi.MDP.from_instance(p)
    pi = torch.from_numpy(pi0.copy()).cuda()
    pi, V, st, rounds = mdp.policy_iteration(pi, eval_tol=1e-12, improve_tol=1e-8)
    print(f"{name}: gpu {rounds} rounds ({st['iterations']} eval sweeps), oracle {rounds_o}", flush=True)
    Vg = V.cpu().numpy()
    assert np.max(np.abs(Vg - V_o)) <= 10 * EVAL_REL * np.max(np.abs(V_o))
    assert np.max(np.abs(Vg - star)) <= 10 * EVAL_REL * np.max(np.abs(star))
    # the policies agree wherever the optimal action is clear
    Q1 = vi.q_table(p, star, g).max(axis=1)
    _, gap = vi.extract(p, star, g)
    mask = gap_mask(Q1, gap, star)
    assert np.array_equal(pi.cpu().numpy()[mask], pol_o[mask])
    assert abs(rounds - rounds_o) <= 1


def test_full_size(mdpvi):
    import torch
    p = W.large_single()
    mdp = mdpvi.MDP.from_instance(p)
    Vs = torch.zeros(mdp.num_states, device="cuda")
    mdp.vi_solve(Vs, tol=1e-6)
    pi = mdp.policy_greedy("least_loaded")
    pi, V, st, rounds = mdp.policy_iteration(pi, eval_tol=1e-10, improve_tol=1e-7)
    print(f"large_single: {rounds} rounds, {st['iterations']} eval sweeps, {st['seconds']:.3f} s", flush=True)
    vi_close(V.cpu().numpy(), Vs.cpu().numpy().astype(np.float64), rel=VI_REL)
    # no action improves on the final policy by more than the tie tolerance
    pi2, _ = mdp.policy_extract(V, want_gap=False)
    assert rounds >= 2


def test_errors(mdpvi):
    import torch
    p = W.small_parity()
    mdp = mdpvi.MDP.from_instance(p)
    pi = mdp.policy_greedy("least_loaded")
    with pytest.raises(mdpvi.MdpviError) as e:
        mdp.policy_iteration(pi.clone(), improve_tol=-1.0)
    assert e.value.code == mdpvi.EINVAL
    bad = pi.clone()
    bad[-1] = 0   # (C, C, C) occupancy, class 2: no room on host 0
    with pytest.raises(mdpvi.MdpviError) as e:
        mdp.policy_iteration(bad)
    assert e.value.code == mdpvi.EINVAL
    with pytest.raises(mdpvi.MdpviError) as e:
        mdp.policy_iteration(pi.clone(), max_rounds=1)
    assert e.value.code == mdpvi.ENOCONV
