"""Write tests/golden/policy_<workload>.json with the FP64 oracle only.

    python tests/golden/make_policy_golden.py gradient|large_single [--tol T]

The optimal policy of a full-size instance, reduced to what does not depend
on how exact ties between equivalent hosts are broken (oracle/summary.py):
for every host-permutation orbit of states, the occupancy of the host the
policy places on ('?' where the orbit holds a state whose best and best
other-target-load Q are within 1e-6 relative, the parity threshold for
policies).  With --strict r, the same table at threshold r and the table
with no orbit masked are stored too.  Also stored: the sweep count, the objective J of the policy
(FP64 evaluation), and per-class target-load histograms.

Workloads (workloads/__init__.py):
  gradient      K=5, C=10, J=2, lambda=(3.0, 1.5), mu=0.1, nu=0.02,
                r=(1, 2.5), gamma=0.98: 322,102 states
                (stored with --tol 1e-12 --strict 1e-10)
  large_single  K=6, C=10, J=3, sizes (1,2,3), seeded draws (seed 2),
                gamma=0.99: 5,314,683 states (about 1.5 hours on one core)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import summary, vi  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["gradient", "large_single"])
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--strict", type=float, default=0.0,
                    help="also store the table at this smaller ambiguity threshold, and the "
                         "unmasked table (needs --tol well below it)")
    args = ap.parse_args()
    p = W.gradient_instance() if args.workload == "gradient" else W.large_single()
    t0 = time.time()
    g = vi.grid(p)
    res = vi.value_iteration(p, args.tol, g=g)
    print(f"VI {res.iterations} sweeps, residual {res.residual:.3e} ({time.time() - t0:.0f} s)", flush=True)
    V = res.V
    pi, _ = vi.extract(p, V, g)
    tl = summary.target_load(p, pi, g)
    amb = summary.ambiguous(p, V, 1e-6, g)
    table = summary.orbit_table(p, tl, amb, g)
    back = summary.expand_orbit_table(p, table, g)
    known = back != -2
    assert np.array_equal(back[known], tl[known])
    Vp = vi.policy_eval(p, pi, tol=1e-12, V0=V, g=g)
    out = {
        "instance": {"K": p.K, "C": p.C, "size": list(p.size), "lam": list(p.lam), "mu": p.mu,
                     "nu": p.nu, "reward": list(p.reward), "gamma": p.gamma},
        "vi_tol": args.tol,
        "vi_sweeps": res.iterations,
        "J": vi.objective(p, Vp),
        "V_inf": float(np.max(np.abs(V))),
        "ambiguous_states": int(amb.size),
        "unknown_states": int((~known).sum()),
        "target_load_histogram": summary.histogram(p, tl),
        "orbit_target_load": table,
        "source": "oracle only (tests/golden/make_policy_golden.py)",
    }
    if args.strict > 0:
        amb_s = summary.ambiguous(p, V, args.strict, g)
        full = summary.orbit_table(p, tl, [], g)
        assert "?" not in full, "the policy's target load is not constant on an orbit"
        out["strict_rel"] = args.strict
        out["ambiguous_states_strict"] = int(amb_s.size)
        out["orbit_target_load_strict"] = summary.orbit_table(p, tl, amb_s, g)
        out["orbit_target_load_all"] = full
    path = os.path.join(HERE, f"policy_{args.workload}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}: {amb.size} ambiguous, {(~known).sum()} unknown states "
          f"({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
