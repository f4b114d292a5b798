"""The allocation-free value iteration (vi_solve_noalloc) against vi_solve.

Called through the C ABI with ctypes: two calls in a row on one device,
the second on a smaller instance (the static scratch array keeps the first
call's contents, so the second call shows that everything that must start
cleared is cleared), each compared bit for bit with vi_solve on the same
input (same kernels and stopping test: identical iterates and sweep counts).
Also: an instance beyond the array's size is refused with MDPVI_ERANGE, and
the refused call leaves the next call unaffected."""
import ctypes

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdpvi():
    torch_cuda()
    import paper_2012_12419_amd as m
    m.load()
    return m


def _noalloc(mdpvi, mdp, V, tol):
    st = mdpvi.Stats()
    rc = mdpvi.load().vi_solve_noalloc(mdp._h, ctypes.c_void_p(V.data_ptr()), ctypes.c_double(tol),
                                       ctypes.c_int64(1_000_000), None, ctypes.byref(st))
    return rc, st


CASES = [  # (instance, tol), largest first: the tile form (5,314,683 states, about 51 MB
           # of the 64 MiB), the exact-shape direct form, the small instances
    (W.large_single(), 1e-6),
    (W.make(5, 10, (1, 2, 3), (0.7, 0.5, 0.3), 0.1, 0.02, (1.0, 2.2, 3.1), 0.97), 1e-6),   # 483,153
    (W.small_parity(), 1e-9),                                                              # 1,458
    (W.make(2, 5, (1, 2), (0.7, 0.5), 0.1, 0.02, (0.3, 4.0), 0.95, reject_cost=(0.2, 0.6)), 1e-8),
]


def test_noalloc_matches_vi_solve_two_calls_shrinking(mdpvi):
    import torch
    for inst, tol in CASES:
        print(f"noalloc K={inst.K} C={inst.C} J={inst.J} N={inst.num_states}", flush=True)
        mdp = mdpvi.MDP.from_instance(inst)
        V0 = torch.zeros(mdp.num_states, device="cuda")
        if max(inst.reject_cost) > 0:
            V0.fill_(-10.0)
        Va = V0.clone()
        Vb = V0.clone()
        sa = mdp.vi_solve(Va, tol=tol)
        rc, sb = _noalloc(mdpvi, mdp, Vb, tol)
        torch.cuda.synchronize()
        assert rc == mdpvi.OK, mdpvi.load().mdpvi_last_error()
        assert sb.iterations == sa["iterations"]
        assert sb.residual_inf == sa["residual_inf"]
        assert np.array_equal(Va.cpu().numpy().view(np.uint32), Vb.cpu().numpy().view(np.uint32))


def test_noalloc_refuses_beyond_its_array(mdpvi):
    import torch
    big = W.large_single(K=7)   # 58 million states: far beyond 64 MiB of scratch
    mdp = mdpvi.MDP.from_instance(big)
    V = torch.zeros(16, device="cuda")   # never touched: the size check comes first
    rc, _ = _noalloc(mdpvi, mdp, V, 1e-6)
    assert rc == mdpvi.ERANGE
    assert b"allocation-free" in mdpvi.load().mdpvi_last_error()
    small = W.small_parity()
    m2 = mdpvi.MDP.from_instance(small)
    Va = torch.zeros(m2.num_states, device="cuda")
    Vb = torch.zeros(m2.num_states, device="cuda")
    m2.vi_solve(Va, tol=1e-9)
    rc, _ = _noalloc(mdpvi, m2, Vb, 1e-9)
    assert rc == mdpvi.OK
    assert np.array_equal(Va.cpu().numpy().view(np.uint32), Vb.cpu().numpy().view(np.uint32))
