"""GPU parity of the block-asynchronous value iteration (vi_solve_bsdi, the
paper's BSDI scheme of Alg. 4 on the tiles of the tile form).

- inner = 1 is vi_solve's Jacobi iteration: same bits, same sweep count;
- run to a zero residual, BSDI and Jacobi reach the same FP32 fixed point
  bit for bit (both increase monotonically from a sub-solution to the least
  fixed point of the same rounded, monotone operator);
- pass counts and values against the FP64 BSDI oracle on the same blocks;
- the 5.3M-state instance: fewer passes than Jacobi sweeps and the same
  values within the FP32 bound.
"""
import numpy as np
import pytest

import workloads as W
from oracle import bsdi, vi
from tests.gpu_util import VI_REL, sub_solution, torch_cuda, vi_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdpvi():
    torch_cuda()
    import paper_2012_12419_amd as m
    m.load()
    return m


def bsdi_digits(p):
    """Tile depth the library picks for the block-asynchronous form: the
    deepest T in 2..min(4, K-1) whose two LDS images fit 64 KB."""
    R = p.C + 1
    for T in range(min(4, p.K - 1), 1, -1):
        occ = R ** T
        if occ * 2 * (4 * p.J + 8) + 16 <= 64 * 1024 and occ <= 4096:
            return T
    return None




CASES = [("K4C12J3", W.make(4, 12, (3, 1, 2), (0.4, 0.7, 0.2), 0.09, 0.03, (2.0, 0.7, 1.6), 0.96)),
         ("K4C9J3", W.make(4, 9, (1, 2, 3), (0.5, 0.4, 0.3), 0.1, 0.02, (1.0, 2.2, 3.1), 0.95)),
         ("K6C4J2_reject", W.make(6, 4, (1, 3), (0.5, 0.3), 0.12, 0.03, (1.0, 2.9), 0.94,
                                  reject_cost=(0.1, 0.4))),
         ("K3C7J1", W.make(3, 7, (2,), (0.9,), 0.1, 0.05, (1.5,), 0.93)),
         ("K5C6J2", W.make(5, 6, (1, 2), (0.8, 0.5), 0.1, 0.02, (1.0, 2.4), 0.95)),
         ("K4C9J2_penalty", W.make(4, 9, (1, 2), (0.6, 0.5), 0.1, 0.02, (1.0, 2.4), 0.95, idle_unit_cost=0.1))]


@pytest.mark.parametrize("name,p", CASES, ids=[c[0] for c in CASES])
def test_inner1_is_jacobi(mdpvi, name, p):
    import torch
    mdp = mdpvi.MDP.from_instance(p)
    lb = sub_solution(p)
    V1 = torch.full((mdp.num_states,), lb, device="cuda")
    V2 = V1.clone()
    a = mdp.vi_solve(V1, tol=1e-7)
    b = mdp.vi_solve_bsdi(V2, tol=1e-7, inner=1)
    print(f"{name}: jacobi {a['iterations']} sweeps, bsdi(1) {b['iterations']} passes", flush=True)
    assert a["iterations"] == b["iterations"]
    assert torch.equal(V1.view(torch.int32), V2.view(torch.int32))


@pytest.mark.parametrize("name,p", CASES, ids=[c[0] for c in CASES])
def test_same_fixed_point_at_zero_residual(mdpvi, name, p):
    import torch
    mdp = mdpvi.MDP.from_instance(p)
    lb = sub_solution(p)
    Vj = torch.full((mdp.num_states,), lb, device="cuda")
    Vb = Vj.clone()
    sj = mdp.vi_solve(Vj, tol=1e-300, max_iter=200_000)
    sb = mdp.vi_solve_bsdi(Vb, tol=1e-300, inner=4, max_iter=200_000)
    print(f"{name}: zero residual after {sj['iterations']} sweeps / {sb['iterations']} passes", flush=True)
    assert sj["residual_inf"] == 0.0 and sb["residual_inf"] == 0.0
    assert torch.equal(Vj.view(torch.int32), Vb.view(torch.int32))
    assert sb["iterations"] < sj["iterations"]


@pytest.mark.parametrize("name,p", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("inner", [2, 5])
def test_vs_oracle(mdpvi, name, p, inner):
    import torch
    T = bsdi_digits(p)
    assert T is not None
    # tol far above the FP32 spacing of the values (a few 1e-6 here), so that
    # both sides stop by the same test rather than at FP32's exact fixed point
    tol = 1e-3
    ref = bsdi.bsdi(p, T, inner, tol, V0=np.full(p.num_states, sub_solution(p)))
    mdp = mdpvi.MDP.from_instance(p)
    V = torch.full((mdp.num_states,), sub_solution(p), device="cuda")
    st = mdp.vi_solve_bsdi(V, tol=tol, inner=inner)
    print(f"{name} T={T} inner={inner}: gpu {st['iterations']} passes, oracle {ref.iterations}", flush=True)
    # FP32 storage against FP64: a change within rounding of tol may stop one
    # side a pass earlier
    assert abs(st["iterations"] - ref.iterations) <= 1
    vi_close(V.cpu().numpy(), ref.V, rel=VI_REL)


def test_full_size(mdpvi):
    import torch
    p = W.large_single()
    mdp = mdpvi.MDP.from_instance(p)
    Vj = torch.zeros(mdp.num_states, device="cuda")
    sj = mdp.vi_solve(Vj, tol=1e-6)
    for inner in (2, 4):
        Vb = torch.zeros(mdp.num_states, device="cuda")
        sb = mdp.vi_solve_bsdi(Vb, tol=1e-6, inner=inner)
        print(f"large_single: jacobi {sj['iterations']} sweeps {sj['seconds']:.4f} s; "
              f"bsdi({inner}) {sb['iterations']} passes {sb['seconds']:.4f} s", flush=True)
        assert sb["iterations"] < sj["iterations"]
        # both are within gamma/(1-gamma) tol plus the FP32 bound of V*
        vi_close(Vb.cpu().numpy(), Vj.cpu().numpy().astype(np.float64), rel=VI_REL)


def test_errors(mdpvi):
    import torch
    p = W.small_parity()   # K = 3, C = 8: (C+1)^2 = 81 fits, so the form applies
    mdp = mdpvi.MDP.from_instance(p)
    V = torch.zeros(mdp.num_states, device="cuda")
    with pytest.raises(mdpvi.MdpviError) as e:
        mdp.vi_solve_bsdi(V, inner=0)
    assert e.value.code == mdpvi.EINVAL
    q = W.make(2, 5, (1,), (0.5,), 0.1, 0.02, (1.0,), 0.9)   # K = 2: no tile with T >= 2 below K
    mdq = mdpvi.MDP.from_instance(q)
    Vq = torch.zeros(mdq.num_states, device="cuda")
    with pytest.raises(mdpvi.MdpviError) as e:
        mdq.vi_solve_bsdi(Vq, inner=2)
    assert e.value.code == mdpvi.EINVAL
