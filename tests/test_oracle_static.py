"""Pins of the static bag-of-task oracle (oracle/static_bot.py).

- the published example (tests/golden/static_bot_example.json): Alg. 2
  with bag i read as five tasks of i VMs gives the greedy figure's per-bag VC
  and paid VMs, its 27 idle VMs, its per-VC reward dots and the total 116;
  a placement that fills every VC exists, pays for 58 VMs and scores the
  MDP total 202.4 (no placement scores more: every VC is full and the
  reward grows with the VMs placed in VCs);
- on tiny scenarios the exhaustive optimum is never below the greedy
  score, and equals it when every task fits;
- conservation: vc + paid = VMs asked for, vc + idle = capacity;
- one VC: first fit takes each task while it fits (closed form of a scan);
- score rejects an over-full VC and an out-of-range place code.
"""
import json
import os

import numpy as np
import pytest

from oracle import static_bot as sb
from workloads import static_bot as ws

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "static_bot_example.json")))
C = GOLD["constants"]
B = (C["beta_vc"], C["beta_tc"], C["gamma_vc"])


def test_example_inputs_match_the_figures():
    caps, need, bag = ws.example()
    assert caps.tolist() == GOLD["vc_capacities"]
    per_bag = [int(need[bag == i].sum()) for i in range(1, 12)]
    assert per_bag == GOLD["bag_vms"]


def test_greedy_reproduces_the_published_figure():
    caps, need, bag = ws.example()
    place, used = sb.first_fit(caps, need)
    g = GOLD["greedy"]
    vc_per_bag = [int(need[(bag == i) & (place >= 0)].sum()) for i in range(1, 12)]
    paid_per_bag = [int(need[(bag == i) & (place == sb.PAID)].sum()) for i in range(1, 12)]
    assert vc_per_bag == g["vc_vms_per_bag"]
    assert paid_per_bag == g["paid_vms_per_bag"]
    s = sb.score(caps, need, place, *B)
    assert s["paid"] == g["paid_vms"] and s["idle"] == g["idle_vms"]
    assert abs(s["reward"] - g["total_reward"]) < 1e-9
    dots = sb.per_vc_reward(caps, used, B[0], B[1])
    assert np.allclose(dots, g["per_vc_reward"], atol=1e-9)


def test_full_packing_reproduces_the_mdp_total():
    caps, need, _ = ws.example()
    place = sb.full_packing(caps, need)
    assert place is not None
    s = sb.score(caps, need, place, *B)
    m = GOLD["mdp"]
    assert s["idle"] == m["idle_vms"] and s["paid"] == m["paid_vms"]
    assert abs(s["reward"] - m["total_reward"]) < 1e-9
    assert np.array_equal(s["used"], caps)
    assert np.allclose(sb.per_vc_reward(caps, s["used"], B[0], B[1]), m["per_vc_reward"])
    # the greedy leaves reward on the table
    g = sb.score(caps, need, sb.first_fit(caps, need)[0], *B)
    assert s["reward"] > g["reward"]


@pytest.mark.parametrize("seed", range(12))
def test_exhaustive_optimum_dominates_greedy(seed):
    rng = np.random.default_rng(seed)
    K = int(rng.integers(1, 4))
    T = int(rng.integers(1, 6))
    caps = rng.integers(0, 7, size=K)
    need = rng.integers(0, 5, size=T)
    place, used = sb.first_fit(caps, need)
    g = sb.score(caps, need, place, *B)
    best, arg = sb.best_by_enumeration(caps, need, *B)
    assert best >= g["reward"] - 1e-12
    if np.all((place >= 0) | (place == sb.EMPTY)):
        # every task fit: nothing is paid, so no placement scores more
        assert abs(best - g["reward"]) < 1e-12
    fp = sb.full_packing(caps, need)
    if fp is not None:
        assert abs(sb.score(caps, need, fp, *B)["reward"] - best) < 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_conservation(seed):
    caps, need = ws.random_scenarios(8, 5, 30, seed)
    for b in range(8):
        place, used = sb.first_fit(caps[b], need[b])
        s = sb.score(caps[b], need[b], place, *B)
        assert np.array_equal(s["used"], used)
        assert s["vc"] + s["paid"] == int(need[b].sum())
        assert s["vc"] + s["idle"] == int(caps[b].sum())
        assert np.all(used <= caps[b]) and np.all(used >= 0)
        assert np.array_equal(place == sb.EMPTY, need[b] == 0)


def test_single_vc_scan():
    cap, need = 10, [3, 4, 5, 2, 1, 6]
    place, used = sb.first_fit([cap], need)
    room, expect = cap, []
    for n in need:
        expect.append(0 if n <= room else sb.PAID)
        room -= n if n <= room else 0
    assert place.tolist() == expect and int(used[0]) == cap - room


def test_score_rejects_invalid():
    with pytest.raises(ValueError):
        sb.score([3], [2, 2], [0, 0], *B)
    with pytest.raises(ValueError):
        sb.score([3], [2], [1], *B)
