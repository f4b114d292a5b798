"""Helpers for the GPU parity tests: device availability and tolerances.

Tolerances (derived from the arithmetic of the kernels):

* Value iteration stores FP32 values and forms every backup in FP64, rounding
  once per state and sweep (relative error <= 2^-24).  The Bellman operator is
  a gamma-contraction, so the FP32 fixed point V_hat satisfies
  ||V_hat - V*||_inf <= 2^-24 ||V*||_inf / (1 - gamma) (+ the stopping error
  gamma/(1-gamma) tol), i.e. 6e-6 relative at gamma = 0.99: within the
  1e-5 relative bound used below.
* Fixed-policy evaluation is FP64 end to end: 1e-10 relative.
* Policies are compared bit-exactly on the states where the oracle's
  best-vs-second Q gap exceeds 1e-6 relative (max(|Q1|, 1e-3 ||V*||));
  elsewhere both sides must choose an action whose Q is within that gap.
"""
import numpy as np
import pytest

VI_REL = 1e-5
EVAL_REL = 1e-10
GAP_REL = 1e-6


def sub_solution(inst) -> float:
    """A constant sub-solution of the Bellman operator: the lowest one-step
    reward (paid-cloud cost on the arrival branch and the under-utilisation
    penalty of every unit) over the discount horizon.  Value iteration from
    it increases monotonically to an exact FP32 fixed point."""
    lam = np.asarray(inst.lam)
    Lam = lam.sum() + inst.K * inst.C * inst.mu + inst.K * inst.nu
    worst = lam.sum() / Lam * max(inst.reject_cost) + inst.idle_unit_cost * inst.K * inst.C
    return -worst / (1 - inst.gamma)


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def vi_close(V_gpu: np.ndarray, V_ref: np.ndarray, rel: float = VI_REL):
    scale = np.max(np.abs(V_ref))
    err = np.max(np.abs(V_gpu.astype(np.float64) - V_ref))
    assert err <= rel * scale, f"max |V_gpu - V_ref| = {err:.3e} > {rel:.1e} * {scale:.3e}"
    return err / scale


def gap_mask(Q1: np.ndarray, gap: np.ndarray, Vstar: np.ndarray) -> np.ndarray:
    denom = np.maximum(np.abs(Q1), 1e-3 * np.max(np.abs(Vstar)))
    return gap / denom > GAP_REL
