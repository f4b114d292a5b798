"""GPU parity of the static bag-of-task kernels (static_first_fit: Alg. 2;
static_score: the cloud-wide reward of Eqs. (14)-(16)) against the oracle
(oracle/static_bot.py), which is pinned to the paper's worked example.

Integer outputs (placements, VMs per VC, totals, status) are compared bit
for bit; the reward is the same three rounded products subtracted left to
right on both sides, so it is compared bit for bit too.
"""
import json
import os

import numpy as np
import pytest

from oracle import static_bot as sb
from tests.gpu_util import torch_cuda
from workloads import static_bot as ws

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "static_bot_example.json")))
CONST = (GOLD["constants"]["beta_vc"], GOLD["constants"]["beta_tc"], GOLD["constants"]["gamma_vc"])


@pytest.fixture(scope="module")
def mdpvi():
    torch_cuda()
    import paper_2012_12419_amd as m
    m.load()
    return m


def _gpu(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.int32)).cuda()


def _host(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def _check_first_fit(caps, need, got, rows=None):
    for b in (range(caps.shape[0]) if rows is None else rows):
        place, used = sb.first_fit(caps[b], need[b])
        s = sb.score(caps[b], need[b], place, *CONST)
        assert got["status"][b] == 0
        assert np.array_equal(got["place"][b], place), f"scenario {b}"
        assert np.array_equal(got["used"][b], used), f"scenario {b}"
        assert got["totals"][b].tolist() == [s["vc"], s["paid"], s["idle"]]
        assert got["reward"][b] == s["reward"]


def test_example(mdpvi):
    caps, need, _ = ws.example()
    got = _host(mdpvi.static_first_fit(_gpu(caps[None]), _gpu(need[None]), *CONST))
    _check_first_fit(caps[None], need[None], got)
    g = GOLD["greedy"]
    assert got["totals"][0].tolist() == [int(caps.sum()) - g["idle_vms"], g["paid_vms"], g["idle_vms"]]
    assert abs(got["reward"][0] - g["total_reward"]) < 1e-12
    # the best placement (every VC full) scored on the GPU: the MDP total
    best = sb.full_packing(caps, need)
    sc = _host(mdpvi.static_score(_gpu(caps[None]), _gpu(need[None]), _gpu(best[None]), *CONST))
    assert sc["status"][0] == 0
    assert np.array_equal(sc["used"][0], caps)
    assert sc["totals"][0].tolist() == [int(caps.sum()), GOLD["mdp"]["paid_vms"], 0]
    assert abs(sc["reward"][0] - GOLD["mdp"]["total_reward"]) < 1e-12


@pytest.mark.parametrize("K,T", [(1, 0), (1, 5), (7, 63), (11, 64), (11, 65), (33, 130), (64, 200)])
def test_random_vs_oracle(mdpvi, K, T):
    caps, need = ws.random_scenarios(300, K, T, seed=K * 1000 + T)
    got = _host(mdpvi.static_first_fit(_gpu(caps), _gpu(need), *CONST))
    _check_first_fit(caps, need, got)


def test_score_vs_oracle(mdpvi):
    rng = np.random.default_rng(5)
    B, K, T = 400, 9, 70
    caps, need = ws.random_scenarios(B, K, T, seed=17, cap_max=120, need_max=6)
    place = rng.integers(-1, K, size=(B, T)).astype(np.int32)
    place[rng.random(size=(B, T)) < 0.005] = K + 3      # out-of-range codes in some scenarios
    got = _host(mdpvi.static_score(_gpu(caps), _gpu(need), _gpu(place), *CONST))
    seen = set()
    for b in range(B):
        try:
            s = sb.score(caps[b], need[b], place[b], *CONST)
        except ValueError as e:
            code = 4 if "range" in str(e) else 3
            assert got["status"][b] == code, f"scenario {b}"
            seen.add(code)
            continue
        seen.add(0)
        assert got["status"][b] == 0
        assert np.array_equal(got["used"][b], s["used"])
        assert got["totals"][b].tolist() == [s["vc"], s["paid"], s["idle"]]
        assert got["reward"][b] == s["reward"]
    assert seen == {0, 3, 4}
    # the first-fit placement scores what first fit reports
    ff = mdpvi.static_first_fit(_gpu(caps), _gpu(need), *CONST)
    sc = _host(mdpvi.static_score(_gpu(caps), _gpu(need), ff["place"], *CONST))
    ffh = _host(ff)
    assert np.array_equal(sc["status"], np.zeros(B, dtype=np.int32))
    for k in ("used", "totals", "reward"):
        assert np.array_equal(sc[k], ffh[k])


def test_invalid_inputs_set_status(mdpvi):
    caps = np.array([[3, 4], [3, -1], [3, 4], [1 << 30, 0], [(1 << 30) + 1, 0]], dtype=np.int32)
    need = np.array([[1, 2, 3], [1, 1, 1], [1, -2, 1], [5, 0, 0], [1, 1, 1]], dtype=np.int32)
    got = _host(mdpvi.static_first_fit(_gpu(caps), _gpu(need), *CONST))
    assert got["status"].tolist() == [0, 1, 2, 0, 1]
    _check_first_fit(caps, need, got, rows=[0, 3])


def test_full_size(mdpvi):
    import torch
    # one million scenarios of the example's shape (11 VCs, 55 task slots)
    B, K, T = 1_000_000, 11, 55
    caps, need = ws.random_scenarios(B, K, T, seed=99, cap_max=45, need_max=11)
    got = mdpvi.static_first_fit(_gpu(caps), _gpu(need), *CONST)
    torch.cuda.synchronize()
    h = _host(got)
    assert np.all(h["status"] == 0)
    # properties at every scenario
    vc, paid, idle = h["totals"].T
    assert np.array_equal(vc + paid, need.sum(axis=1, dtype=np.int64))
    assert np.array_equal(vc + idle, caps.sum(axis=1, dtype=np.int64))
    assert np.array_equal(h["used"].sum(axis=1, dtype=np.int64), vc)
    assert np.all(h["used"] <= caps)
    assert np.array_equal(h["place"] == sb.EMPTY, need == 0)
    # a sample against the oracle, one scenario at a time
    rows = np.random.default_rng(0).choice(B, size=400, replace=False)
    _check_first_fit(caps, need, h, rows=rows)


def test_errors(mdpvi):
    import torch
    caps = torch.zeros((2, 65), dtype=torch.int32, device="cuda")
    need = torch.zeros((2, 4), dtype=torch.int32, device="cuda")
    with pytest.raises(mdpvi.MdpviError) as e:
        mdpvi.static_first_fit(caps, need)
    assert e.value.code == mdpvi.EINVAL
    with pytest.raises(ValueError):
        mdpvi.static_first_fit(caps[:, :3], need[:1])
    with pytest.raises(ValueError):
        mdpvi.static_first_fit(caps[:, :3].cpu(), need.cpu())
    # B = 0 and T = 0 are valid
    out = mdpvi.static_first_fit(caps[:0, :3], need[:0])
    assert out["reward"].numel() == 0
