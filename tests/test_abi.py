"""The C-ABI library loads, exports every symbol the header declares, and
validates parameters on the host (no GPU needed for any of this)."""
import ctypes
import os
import re

import pytest

import paper_2012_12419_amd as mdpvi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[\w ]+?\**\s*\b(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    lib = mdpvi.load()
    declared = _declared()
    assert "vi_solve" in declared and "mdp_build" in declared
    for name in declared:
        assert hasattr(lib, name), f"{name} declared in include/ but not exported"
    assert set(declared) <= set(mdpvi.SIGNATURES), set(declared) - set(mdpvi.SIGNATURES)


def _build(**kw):
    base = dict(K=3, C=8, size=[1, 2], lam=[0.6, 0.3], mu=0.1, nu=0.02, reward=[1.0, 2.5],
                gamma=0.95, reject_cost=None)
    base.update(kw)
    p, keep = mdpvi.make_params(**base)
    h = ctypes.c_void_p()
    rc = mdpvi.load().mdp_build(ctypes.byref(p), ctypes.byref(h))
    return rc, h


def test_build_and_counts():
    rc, h = _build()
    lib = mdpvi.load()
    assert rc == mdpvi.OK
    assert lib.mdp_num_states(h) == 1458
    assert lib.mdp_num_actions(h) == 4
    assert lib.mdp_feasible_pairs(h) == 5103
    lib.mdp_free(h)
    lib.mdp_free(None)
    assert lib.mdp_num_states(None) == -1


@pytest.mark.parametrize("kw,code,text", [
    (dict(gamma=1.0), mdpvi.EINVAL, "gamma"),
    (dict(gamma=-0.1), mdpvi.EINVAL, "gamma"),
    (dict(gamma=float("nan")), mdpvi.EINVAL, "gamma"),
    (dict(size=[1, 9]), mdpvi.EINVAL, "size[1]"),
    (dict(size=[0, 2]), mdpvi.EINVAL, "size[0]"),
    (dict(lam=[-0.1, 0.3]), mdpvi.EINVAL, "lambda[0]"),
    (dict(lam=[0.0, 0.0]), mdpvi.EINVAL, "sum of lambda"),
    (dict(lam=[float("inf"), 0.3]), mdpvi.EINVAL, "lambda[0]"),
    (dict(mu=-1.0), mdpvi.EINVAL, "mu"),
    (dict(nu=float("nan")), mdpvi.EINVAL, "nu"),
    (dict(reward=[1.0, float("nan")]), mdpvi.EINVAL, "reward[1]"),
    (dict(reject_cost=[0.0, float("inf")]), mdpvi.EINVAL, "reject_cost[1]"),
    (dict(K=0), mdpvi.EINVAL, "K=0"),
    (dict(K=17), mdpvi.EINVAL, "K=17"),
    (dict(C=0, size=[1, 1]), mdpvi.EINVAL, "C=0"),
    (dict(size=[1] * 9, lam=[0.1] * 9, reward=[1.0] * 9), mdpvi.EINVAL, "J=9"),
    (dict(K=16, C=20, size=[1], lam=[1.0], reward=[1.0]), mdpvi.ERANGE, "2^"),
    (dict(K=11, C=8, size=[1], lam=[1.0], reward=[1.0]), mdpvi.ERANGE, "occupancies"),
])
def test_validation(kw, code, text):
    rc, h = _build(**kw)
    assert rc == code
    assert h.value is None
    assert text in mdpvi.load().mdpvi_last_error().decode()


def test_null_arguments():
    lib = mdpvi.load()
    h = ctypes.c_void_p()
    assert lib.mdp_build(None, ctypes.byref(h)) == mdpvi.EINVAL
    assert lib.vi_solve(None, None, 1e-6, 10, None, None) == mdpvi.EINVAL
    assert lib.policy_extract(None, None, None, None, None) == mdpvi.EINVAL
    assert lib.policy_eval(None, None, None, 1e-6, 10, None, None) == mdpvi.EINVAL
    assert lib.policy_greedy(None, 0, None, None) == mdpvi.EINVAL
    rc, h = _build()
    assert lib.vi_solve(h, None, 1e-6, 10, None, None) == mdpvi.EINVAL
    fake = ctypes.c_void_p(16)
    assert lib.vi_solve(h, fake, 0.0, 10, None, None) == mdpvi.EINVAL
    assert lib.vi_solve(h, fake, float("nan"), 10, None, None) == mdpvi.EINVAL
    assert lib.vi_solve(h, fake, 1e-6, 0, None, None) == mdpvi.EINVAL
    assert lib.policy_greedy(h, 2, fake, None) == mdpvi.EINVAL
    lib.mdp_free(h)


def test_python_binding_refuses_cpu_tensors():
    import torch
    m = mdpvi.MDP(3, 8, [1, 2], [0.6, 0.3], 0.1, 0.02, [1.0, 2.5], 0.95)
    with pytest.raises(ValueError, match="GPU tensor"):
        m.vi_solve(torch.zeros(m.num_states))


@pytest.mark.parametrize("K,C,J", [(8, 10, 3), (6, 24, 3), (7, 10, 3), (6, 10, 3)])
def test_tile_form_only_below_2gib_values(K, C, J):
    """The tile and row kernels address the FP32 values through 32-bit
    buffer offsets, so the automatic choice (and an explicit request) must
    not take them once J (C+1)^K reaches 2^29 states.  Host-only: mdp_build and the
    form query launch nothing."""
    rc, h = _build(K=K, C=C, size=list(range(1, J + 1)), lam=[0.5] * J, reward=[1.0] * J)
    assert rc == mdpvi.OK
    lib = mdpvi.load()
    try:
        n = lib.mdp_num_states(h)
        assert n == J * (C + 1) ** K
        vi_f, ev_f = ctypes.c_int32(), ctypes.c_int32()
        assert lib.mdp_sweep_forms(h, ctypes.byref(vi_f), ctypes.byref(ev_f)) == mdpvi.OK
        def is_tile(f):   # the tile, row and walk forms (32-bit buffer offsets)
            return any(b <= f <= b + 8 for b in (mdpvi.FORM_TILE, mdpvi.FORM_ROW))
        if n >= 2 ** 29:
            assert not is_tile(vi_f.value) and not is_tile(ev_f.value)
            for form in (mdpvi.FORM_TILE, mdpvi.FORM_ROW):
                assert lib.mdp_set_sweep_form(h, form) == mdpvi.EINVAL
        else:
            assert is_tile(vi_f.value)
    finally:
        lib.mdp_free(h)


def test_adjoint_form_choice_on_the_host():
    """mdp_set_adjoint_form validates forms against the shape; the automatic
    form is the group form where it applies (C <= 15, K 3..8, J <= 3)."""
    lib = mdpvi.load()
    rc, h = _build(K=5, C=10)
    assert rc == mdpvi.OK
    try:
        assert lib.mdp_adjoint_form(h) == mdpvi.ADJOINT_GROUP
        for bad in (3, 5, 16 + 3, 33, -1):
            assert lib.mdp_set_adjoint_form(h, bad) == mdpvi.EINVAL, bad
        for good in (mdpvi.ADJOINT_EXACT + 1, mdpvi.ADJOINT_EXACT + 4, 1, 2, 4, mdpvi.ADJOINT_GROUP):
            assert lib.mdp_set_adjoint_form(h, good) == mdpvi.OK, good
            assert lib.mdp_adjoint_form(h) == good
        assert lib.mdp_set_adjoint_form(h, 0) == mdpvi.OK
    finally:
        lib.mdp_free(h)
    rc, h = _build(K=3, C=16, size=[1], lam=[1.0], reward=[1.0])
    assert rc == mdpvi.OK
    try:
        assert lib.mdp_adjoint_form(h) == mdpvi.ADJOINT_EXACT + 1   # (C+1)^2 = 289 > 256
        assert lib.mdp_set_adjoint_form(h, mdpvi.ADJOINT_GROUP) == mdpvi.EINVAL
    finally:
        lib.mdp_free(h)


def test_batch_round_form_choice_on_the_host():
    """batch_set_round_form validates the operation and the occupancies per
    thread; with nothing recorded every operation uses 4."""
    import workloads as W
    lib = mdpvi.load()
    insts = W.batch(6, seed=11)
    arr = (mdpvi.Params * len(insts))()
    keep = []
    for i, p in enumerate(insts):
        arr[i], k = mdpvi.make_params(p.K, p.C, p.size, p.lam, p.mu, p.nu, p.reward, p.gamma,
                                      p.reject_cost, p.idle_unit_cost)
        keep.append(k)
    h = ctypes.c_void_p()
    assert lib.mdp_build_batch(arr, len(insts), ctypes.byref(h)) == mdpvi.OK
    try:
        out = (ctypes.c_int32 * 3)()
        assert lib.batch_round_forms(h, out) == mdpvi.OK
        assert list(out) == [4, 4, 4]
        for op, opt in ((-1, 1), (3, 1), (0, 3), (1, 8), (2, -1)):
            assert lib.batch_set_round_form(h, op, opt) == mdpvi.EINVAL, (op, opt)
        assert lib.batch_set_round_form(h, 0, 1) == mdpvi.OK
        assert lib.batch_set_round_form(h, 2, 2) == mdpvi.OK
        assert lib.batch_round_forms(h, out) == mdpvi.OK
        assert list(out) == [1, 4, 2]
    finally:
        lib.mdp_free_batch(h)


def test_batch_tile_form_choice_on_the_host():
    """batch_set_tile_form validates the operation and the mode.  Value
    iteration's tile form covers the round-form instances (more states than
    two FP32 copies in 159 KB of LDS hold) of 4 or 5 hosts and up to 3
    distinct sizes whose (C+1)^3 tile of values and arrival terms fits 60 KB;
    evaluation's covers the instances of 4 or 5 hosts and up to 3 distinct
    sizes whose tile has 1,000 or more occupancies and whose FP64 values fit
    32 KB.  Unless set, value iteration's is on and evaluation's off."""
    import workloads as W
    lib = mdpvi.load()
    insts = W.batch(40, seed=3)
    arr = (mdpvi.Params * len(insts))()
    keep = []
    for i, p in enumerate(insts):
        arr[i], k = mdpvi.make_params(p.K, p.C, p.size, p.lam, p.mu, p.nu, p.reward, p.gamma,
                                      p.reject_cost, p.idle_unit_cost)
        keep.append(k)
    lds_states = (160 * 1024 - 1024) // 8
    expect = [0, 0]
    for p in insts:
        R = p.C + 1
        shape = p.K in (4, 5) and p.J <= 3 and len(set(p.size)) == p.J
        if shape and p.num_states > lds_states and (R ** 3 + 1) * 8 + R ** 3 * 4 * p.J <= 60 * 1024:
            expect[0] += 1
        if shape and R ** 3 >= 1000 and R ** 3 * 8 * p.J <= 32 * 1024:
            expect[1] += 1
    assert expect[0] > 0 and expect[1] > 0
    h = ctypes.c_void_p()
    assert lib.mdp_build_batch(arr, len(insts), ctypes.byref(h)) == mdpvi.OK
    try:
        assert lib.batch_tile_form_instances(h, 0) == expect[0]
        assert lib.batch_tile_form_instances(h, 1) == 0
        assert lib.batch_set_tile_form(h, 1, 1) == mdpvi.OK
        assert lib.batch_tile_form_instances(h, 1) == expect[1]
        for op, mode in ((0, -2), (1, 2), (2, 1), (-1, 0)):
            assert lib.batch_set_tile_form(h, op, mode) == mdpvi.EINVAL, (op, mode)
        assert lib.batch_tile_form_instances(h, 2) == -1
        assert lib.batch_set_tile_form(h, 0, 0) == mdpvi.OK
        assert lib.batch_tile_form_instances(h, 0) == 0
        assert lib.batch_tile_form_instances(h, 1) == expect[1]
        assert lib.batch_set_tile_form(h, 1, 0) == mdpvi.OK
        assert lib.batch_tile_form_instances(h, 1) == 0
        assert lib.batch_set_tile_form(h, 0, 1) == mdpvi.OK
        assert lib.batch_tile_form_instances(h, 0) == expect[0]
    finally:
        lib.mdp_free_batch(h)
    assert lib.batch_tile_form_instances(None, 0) == -1
