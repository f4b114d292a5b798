"""The oracle's results for many batch instances, computed in worker
processes (spawned, so that no worker inherits the GPU context of the test
process).  Test infrastructure only."""
from __future__ import annotations

import multiprocessing as mp
from concurrent.futures import ProcessPoolExecutor

import numpy as np


def _pipeline(args):
    """VI to 1e-13, extraction with the parity gap mask, FP64 evaluation,
    adjoint gradient and the least-loaded heuristic's FP64 value of batch
    instance i of (n, seed); with a policy pi (uint8 array), also its FP64
    value, objective and adjoint gradient."""
    import workloads as W
    from oracle import grad, vi
    from tests.gpu_util import gap_mask
    i, n, seed, pi = args
    p = W.batch(n, seed=seed)[i]
    g = vi.grid(p)
    star = vi.value_iteration(p, 1e-13, g=g).V
    pi_o, gap_o = vi.extract(p, star, g)
    V_o = vi.policy_eval(p, pi_o, tol=1e-13, g=g)
    mask = gap_mask(vi.q_table(p, star, g).max(axis=1), gap_o, star)
    g_o = grad.gradient_adjoint(p, pi_o, V=V_o)
    pg_o = vi.greedy_policy(p, "least_loaded", g)
    Vg_o = vi.policy_eval(p, pg_o, tol=1e-13, g=g)
    out = dict(i=i, pi=pi_o, mask=mask, V=V_o, J=vi.objective(p, V_o), grad=g_o,
               greedy=pg_o, V_greedy=Vg_o)
    if pi is not None:
        V_pi = vi.policy_eval(p, pi, tol=1e-13, g=g)
        out.update(V_pi=V_pi, J_pi=vi.objective(p, V_pi), grad_pi=grad.gradient_adjoint(p, pi, V=V_pi))
    return out


def batch_oracle(indices, n: int, seed: int, policies=None, workers: int = 8):
    """policies: optional {i: uint8 policy of instance i} to evaluate too."""
    ctx = mp.get_context("spawn")
    pols = policies or {}
    with ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        out = list(ex.map(_pipeline, [(int(i), n, seed, pols.get(int(i))) for i in indices]))
    return {r["i"]: r for r in out}


def as_f64(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64)
