"""Write tests/golden/gradient_K5C10.json with the FP64 oracle only.

    python tests/golden/make_gradient_golden.py [--procs 8]

Instance (workloads.gradient_instance): K=5 hosts, C=10 units, J=2
classes of sizes 1, 2, lambda = (3.0, 1.5), mu = 0.1, nu = 0.02,
r = (1, 2.5), gamma = 0.98: 322,102 states.

Stored: J, the gradient dJ/d(lambda_1, lambda_2, mu, nu, r_1, r_2) from the
oracle's sparse adjoint route and from central finite differences (h = 1e-6)
with the policy re-optimised at every perturbed parameter vector (value
iteration warm-started from the unperturbed fixed point), and a summary of
the optimal policy.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import grad, vi  # noqa: E402

H = 1e-6
_BASE = None


def _solve_at(theta_and_v0):
    theta, V0 = theta_and_v0
    p = grad.with_theta(W.gradient_instance(), theta)
    g = vi.grid(p)
    res = vi.value_iteration(p, 1e-12, V0=V0, g=g)
    pi, _ = vi.extract(p, res.V, g)
    V = vi.policy_eval(p, pi, tol=1e-13, V0=res.V, g=g)
    return vi.objective(p, V)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    args = ap.parse_args()
    t0 = time.time()
    p = W.gradient_instance()
    g = vi.grid(p)
    res = vi.value_iteration(p, 1e-12, g=g)
    pi, gap = vi.extract(p, res.V, g)
    V = vi.policy_eval(p, pi, tol=1e-13, V0=res.V, g=g)
    Jv = vi.objective(p, V)
    print(f"VI {res.iterations} sweeps, J = {Jv:.12f} ({time.time() - t0:.0f} s)", flush=True)
    w = grad.adjoint_weights(p, pi, g=g)
    ga = grad.gradient_adjoint(p, pi, V=V, w=w)
    print("adjoint", ga, f"({time.time() - t0:.0f} s)", flush=True)
    th = grad.theta_of(p)
    jobs = []
    for i in range(th.size):
        for sgn in (+1, -1):
            t = th.copy()
            t[i] += sgn * H
            jobs.append((t, res.V))
    with Pool(args.procs) as pool:
        vals = pool.map(_solve_at, jobs)
    fd = np.array([(vals[2 * i] - vals[2 * i + 1]) / (2 * H) for i in range(th.size)])
    print("fd     ", fd, f"({time.time() - t0:.0f} s)", flush=True)
    out = {
        "instance": {"K": p.K, "C": p.C, "size": list(p.size), "lam": list(p.lam), "mu": p.mu,
                     "nu": p.nu, "reward": list(p.reward), "gamma": p.gamma},
        "theta_order": ["lambda_1", "lambda_2", "mu", "nu", "r_1", "r_2"],
        "J": Jv,
        "grad_adjoint": ga.tolist(),
        "grad_fd": fd.tolist(),
        "fd_h": H,
        "vi_sweeps_1e-12": res.iterations,
        "policy_counts": np.bincount(pi, minlength=p.K + 1).tolist(),
        "min_gap_nonzero": float(np.min(gap[(gap > 0) & np.isfinite(gap)])),
        "source": "oracle only (tests/golden/make_gradient_golden.py)",
    }
    with open(os.path.join(HERE, "gradient_K5C10.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote gradient_K5C10.json", flush=True)


if __name__ == "__main__":
    main()
