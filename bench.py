#!/usr/bin/env python
"""Throughput of the value-iteration hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step is one pass of the whole hot path over the large single instance
(K=6 hosts, C=10 units, J=3 classes of sizes 1,2,3: 5,314,683 states,
gamma 0.99, seeded rates), with every input already resident in HBM:

  1. V := 0; vi_solve to ||dV||_inf < 1e-6 (Jacobi sweeps, FP32 values,
     FP64 sums);
  2. policy_extract (greedy policy pi* and Q gap);
  3. policy_eval of pi* in FP64 (warm start from V) and one FP64
     improvement step (policy_extract_f64) that certifies pi*;
  4. policy_greedy (least-loaded heuristic) and its FP64 policy_eval.

value = state-action backups per second over the timed steps: feasible
(state, action) pairs per value-iteration sweep times its sweeps, plus one
backup per state per fixed-policy sweep, divided by the wall time of the
steps.  The JSON line also carries the time to ||dV||_inf < 1e-6, the
roofline of the dominant kernel (algorithmic bytes per launch over the
average launch duration: the timed solves' spans between the HIP events the
library records on the solver's stream, over their working sweeps; one
extra step with an event pair around every sweep is reported beside it) and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "state-action backups/s + time to ‖ΔV‖∞<1e-6; batched vs per-instance, 1 GPU"
HBM_PEAK_GBS = 8000.0
VI_BYTES_PER_STATE = 8.0      # FP32 value read once + written once per sweep
EVAL_BYTES_PER_STATE = 17.0   # FP64 value read + write, uint8 policy read


def workload(name: str):
    import workloads as W
    if name == "large_single":
        return W.large_single(), "K=6 C=10 J=3 sizes(1,2,3) seed 2, gamma 0.99: 5,314,683 states"
    if name == "large_single_k7":
        return (W.large_single(K=7),
                "K=7 C=10 J=3 sizes(1,2,3) seed 2, gamma 0.99: 58,461,513 states (exceeds the 256 MB last-level cache)")
    if name == "gradient":
        return W.gradient_instance(), "K=5 C=10 J=2 sizes(1,2), gamma 0.98: 322,102 states"
    raise SystemExit(f"unknown workload {name}")


def vi_kernel_name(form: int) -> str:
    """The value-iteration sweep kernel a form code runs."""
    if form >= 32:
        return "vi_row_kernel"
    if form >= 16:
        return "vi_tile_kernel"
    return "vi_slab_kernel" if form > 0 else "vi_exact_kernel"


def batched_vs_per_instance(mdpvi, n: int, tol: float) -> dict:
    """The 512-instance parameter sweep solved by one vi_solve_batch call and
    by one vi_solve call per instance on the same stream (handles built and
    value arrays allocated outside the timed regions)."""
    import torch

    import workloads as W
    insts = W.batch(n, seed=3)
    b = mdpvi.Batch(insts)
    tuned = b.autotune(trials=3)               # untimed: round-kernel tile sizes for these shapes
    V = torch.zeros(b.num_states, device="cuda")
    b.vi_solve(V, tol=tol)                     # warm-up (first-use allocations)
    V.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, its, _ = b.vi_solve(V, tol=tol)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    mdps = [mdpvi.MDP.from_instance(p) for p in insts]
    Vs = [torch.zeros(m.num_states, device="cuda") for m in mdps]
    for m, v in zip(mdps[:8], Vs[:8]):
        m.vi_solve(v, tol=tol)
        v.zero_()
    torch.cuda.synchronize()
    backups_single = 0.0
    t0 = time.perf_counter()
    for m, v in zip(mdps, Vs):
        backups_single += m.vi_solve(v, tol=tol)["backups"]
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    return {"instances": n, "states": b.num_states, "tol": tol,
            "batched_seconds": t_batch, "batched_backups_per_s": st["backups"] / t_batch,
            "per_instance_seconds": t_single, "per_instance_backups_per_s": backups_single / t_single,
            "speedup": t_single / t_batch, "max_sweeps": max(its),
            "round_kernel_occupancies_per_thread": b.round_forms(),
            "tile_form_instances": {op: b.tile_form_instances(op) for op in ("vi", "eval")},
            "autotuned_us_per_round": {k: v[1] for k, v in tuned.items()}}


def tolerance_runs(mdp, V, tol: float, t_abs: float, sweeps_abs) -> dict:
    """The stopping test ||dV||_inf < 1e-6 with FP32 values: at ||V||_inf
    above 16 the FP32 spacing exceeds 1e-6, so the absolute test passes only
    at an exact FP32 fixed point.  Reported side by side, each with its
    label: the timed absolute test; the relative test ||dV||_inf <= 1e-6
    ||V||_inf; and the exact FP32 fixed point (residual 0)."""
    import numpy as np
    import torch
    vmax = float(V.abs().max())
    spacing = float(np.spacing(np.float32(vmax)))
    out = {"V_inf": vmax, "fp32_spacing_at_V_inf": spacing,
           "abs": {"label": f"||dV||_inf < {tol:g} (FP32 spacing at ||V||_inf is {spacing:.2g}: "
                            + ("an exact FP32 fixed point" if spacing > tol else "a true tolerance") + ")",
                   "seconds": t_abs, "sweeps": sweeps_abs}}
    W = torch.zeros_like(V)
    st = mdp.vi_solve(W, tol=tol * vmax)
    out["rel"] = {"label": f"||dV||_inf < {tol:g} * ||V||_inf = {tol * vmax:.3g}",
                  "seconds": st["seconds"], "sweeps": st["iterations"]}
    W.zero_()
    st = mdp.vi_solve(W, tol=1e-300)
    out["fixed_point"] = {"label": "||dV||_inf = 0: the exact FP32 fixed point",
                          "seconds": st["seconds"], "sweeps": st["iterations"],
                          "equals_abs_result": bool(torch.equal(W, V))}
    return out


def supplementary_k7(mdpvi, tol: float) -> dict:
    """Value iteration on the instance beyond the last-level cache (K=7, C=10,
    J=3: 58,461,513 states, 468 MB of FP32 values read and written per sweep):
    its time to tolerance and the sweep kernel's achieved bandwidth."""
    import torch
    inst, desc = workload("large_single_k7")
    mdp = mdpvi.MDP.from_instance(inst)
    vi_form, _ = mdp.sweep_forms()
    V = torch.zeros(mdp.num_states, dtype=torch.float32, device="cuda")
    try:
        mdp.vi_solve(V, tol=tol, max_iter=8)   # first-use allocations, tile order
    except mdpvi.MdpviError:
        pass
    V.zero_()
    st = mdp.vi_solve(V, tol=tol)
    N = mdp.num_states
    avg = st["seconds"] / st["iterations"]
    ach = VI_BYTES_PER_STATE * N / avg / 1e9
    impl = vi_kernel_name(vi_form)
    srcs = {"vi_row_kernel": ["paper_2012_12419_amd/csrc/row_vi.hip", "paper_2012_12419_amd/csrc/row.hpp",
                              "paper_2012_12419_amd/csrc/tile.hpp"],
            "vi_tile_kernel": ["paper_2012_12419_amd/csrc/tile_vi.hip", "paper_2012_12419_amd/csrc/tile_vi.hpp",
                               "paper_2012_12419_amd/csrc/tile.hpp"]}
    return {"workload": f"large_single_k7: {desc}", "states": N, "form": vi_form, "kernel": impl,
            "sweeps": st["iterations"], "seconds": st["seconds"],
            "backups_per_s": st["backups"] / st["seconds"], "avg_us": avg * 1e6,
            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS,
                         "traffic": traffic_record(srcs[impl], f"{impl}_large_single_k7")
                         if impl in srcs else None}}


def bsdi_comparison(mdp, N: int, tol: float, inners=(1, 2, 4, 8)) -> dict:
    """Block-asynchronous value iteration (the paper's BSDI) against Jacobi
    on the same instance: passes and device seconds to the same tolerance
    from V = 0 (the Jacobi figure is the timed steps' time to tol)."""
    import torch
    out = {"inner": [], "passes": [], "seconds": [], "us_per_pass": []}
    V = torch.zeros(N, dtype=torch.float32, device="cuda")
    mdp.vi_solve_bsdi(V, tol=tol, inner=2)   # first-use allocations
    for inner in inners:
        V.zero_()
        st = mdp.vi_solve_bsdi(V, tol=tol, inner=inner)
        out["inner"].append(inner)
        out["passes"].append(st["iterations"])
        out["seconds"].append(st["seconds"])
        out["us_per_pass"].append(st["seconds"] / st["iterations"] * 1e6)
    return out


def policy_iteration_run(mdp, eval_tol: float) -> dict:
    """Howard's policy iteration from the least-loaded heuristic."""
    import torch
    pi = mdp.policy_greedy("least_loaded")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pi, V, st, rounds = mdp.policy_iteration(pi, eval_tol=eval_tol, improve_tol=1e-7)
    torch.cuda.synchronize()
    return {"start": "least-loaded heuristic", "rounds": rounds, "eval_sweeps": st["iterations"],
            "seconds": time.perf_counter() - t0, "eval_tol": eval_tol, "improve_tol": 1e-7}


def static_bot_run(mdpvi, n: int) -> dict:
    """Fast greedy placement (Alg. 2) of the static example (11 VCs, 11 bags,
    55 tasks) and of n random scenarios of the same shape, timed."""
    import numpy as np
    import torch
    from workloads import static_bot as ws
    caps, need, _ = ws.example()
    consts = (ws.EXAMPLE_BETA_VC, ws.EXAMPLE_BETA_TC, ws.EXAMPLE_GAMMA_VC)
    ex = mdpvi.static_first_fit(torch.from_numpy(caps[None]).cuda(), torch.from_numpy(need[None]).cuda(),
                                *consts)
    tot = ex["totals"][0].tolist()
    c, d = ws.random_scenarios(n, len(caps), need.size, seed=99, cap_max=45, need_max=11)
    c, d = torch.from_numpy(c).cuda(), torch.from_numpy(d).cuda()
    mdpvi.static_first_fit(c, d, *consts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        mdpvi.static_first_fit(c, d, *consts)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    return {"example": {"vc_vms": tot[0], "paid_vms": tot[1], "idle_vms": tot[2],
                        "greedy_reward": float(ex["reward"][0])},
            "scenarios": n, "tasks_per_scenario": int(need.size), "seconds": sec,
            "scenarios_per_s": n / sec}


def _sub_solution(p):
    """A constant sub-solution of the Bellman operator: the least one-step
    reward over the discount horizon (value iteration from it is monotone)."""
    import numpy as np
    lam = np.asarray(p.lam)
    Lam = lam.sum() + p.K * p.C * p.mu + p.K * p.nu
    worst = lam.sum() / Lam * max(p.reject_cost) + p.idle_unit_cost * p.K * p.C
    return -worst / (1 - p.gamma)


def gradient_workloads(mdpvi, n_batch: int, tol: float) -> dict:
    """The adjoint gradient (dJ/dtheta, theta = lambda, mu, nu, r) on the
    gradient instance (K=5 C=10 J=2, 322,102 states), and the batched
    pipeline on the first n_batch instances of the parameter sweep: value
    iteration, greedy policy, FP64 policy iteration (each instance until its
    improvement changes nothing, actions kept on near-ties within 1e-9),
    adjoint gradient, and the least-loaded heuristic's FP64 evaluation, all as
    batched calls.  Wall time on one stream."""
    import numpy as np
    import torch

    import workloads as W

    def single():
        inst = W.gradient_instance()
        mdp = mdpvi.MDP.from_instance(inst)
        V = torch.zeros(mdp.num_states, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mdp.vi_solve(V, tol=tol)
        pi, _ = mdp.policy_extract(V, want_gap=False)
        Vp = V.double()
        mdp.policy_iteration(pi, Vp, eval_tol=1e-12, improve_tol=1e-9)
        g, Jv, _, st = mdp.vi_adjoint(pi, Vp, tol=1e-10)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, g, Jv, st

    inst = W.gradient_instance()
    tuner = mdpvi.MDP.from_instance(inst)
    tuner.autotune(trials=5)          # untimed: records the forms for this shape
    adj_form = tuner.adjoint_form()
    single()   # first-use allocations
    t_single, g, Jv, st_adj = single()

    insts = W.batch(512, seed=3)[:n_batch]
    b = mdpvi.Batch(insts)
    b_tuned = b.autotune(trials=3)     # untimed: round-kernel tile sizes for these shapes
    N = b.num_states
    lb = torch.zeros(N, device="cuda")
    for i, p in enumerate(insts):
        lb[b.offsets[i]:b.offsets[i + 1]] = _sub_solution(p)

    def batched():
        stages = {}
        V = lb.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t = t0

        def mark(name):
            nonlocal t
            torch.cuda.synchronize()
            now = time.perf_counter()
            stages[name] = stages.get(name, 0.0) + now - t
            t = now

        b.vi_solve(V, tol=tol)
        mark("value_iteration")
        pi, _ = b.policy_extract(V, want_gap=False)
        Vp = V.double()
        _, per_inst = b.policy_iteration(pi, Vp, eval_tol=1e-12, improve_tol=1e-9)
        rounds = max(per_inst)
        mark("evaluation_and_improvement")
        grads, objs, _, _, _ = b.vi_adjoint(pi, Vp, [p.J for p in insts], tol=1e-10)
        mark("adjoint_gradient")
        pig = b.policy_greedy("least_loaded")
        Vg, _, _, _ = b.policy_eval(pig, Vp.clone(), tol=1e-12)   # from V_pi*: V_greedy <= V*
        mark("greedy_evaluation")
        return time.perf_counter() - t0, objs, Vg, stages, rounds

    batched()
    t_batch, objs, Vg, stages, pi_rounds = batched()
    Vg_h = Vg.cpu().numpy()
    gaps = []
    for i, p in enumerate(insts):
        c = np.asarray(p.lam) / sum(p.lam)
        n_occ = (p.C + 1) ** p.K
        J_g = float(sum(c[e] * Vg_h[b.offsets[i] + e * n_occ] for e in range(p.J)))
        gaps.append(objs[i] - J_g)
    return {"single": {"workload": "gradient: K=5 C=10 J=2 sizes(1,2), gamma 0.98: 322,102 states",
                       "seconds": t_single, "gradients_per_s": 1.0 / t_single, "J": Jv,
                       "adjoint_sweeps": st_adj["iterations"], "adjoint_seconds": st_adj["seconds"],
                       "adjoint_us_per_sweep": st_adj["seconds"] / st_adj["iterations"] * 1e6,
                       "adjoint_form": adj_form,
                       "dJ_dtheta": list(g)},
            "batched": {"instances": n_batch, "states": N, "seconds": t_batch,
                        "gradients_per_s": n_batch / t_batch,
                        "stage_seconds": stages, "evaluation_rounds": pi_rounds,
                        "round_kernel_occupancies_per_thread": b.round_forms(),
                        "tile_form_instances": {op: b.tile_form_instances(op) for op in ("vi", "eval")},
                        "autotuned_us_per_round": {k: v[1] for k, v in b_tuned.items()},
                        "mean_J_opt_minus_J_greedy": float(np.mean(gaps)),
                        "min_J_opt_minus_J_greedy": float(np.min(gaps))}}


def traffic_record(kernel_files, name: str):
    """HBM traffic of a kernel from the committed counter record, or None when
    the record is missing or its sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{name}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for fn in kernel_files:
        with open(os.path.join(ROOT, fn), "rb") as f:
            h.update(f.read())
    if rec.get("source_sha256") != h.hexdigest():
        return None
    return rec["bytes_per_launch"]


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(inst, sweeps: int, gpu_sweeps, gpu_seconds) -> dict:
    """The FP64 NumPy oracle's Jacobi sweep, single-threaded, on `sweeps`
    sweeps from V = 0 of the same instance; its time to the GPU's stopping
    sweep is extrapolated from the per-sweep time."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import vi
    with threadpool_limits(limits=1):
        g = vi.grid(inst)
        pairs = vi.feasible_pairs(inst)
        V = np.zeros(inst.num_states)
        t0 = time.perf_counter()
        for _ in range(sweeps):
            V = vi.bellman(inst, V, g)
        dt = time.perf_counter() - t0
    out = {"value": pairs * sweeps / dt, "unit": "backups/s", "cores": 1, "kind": "oracle",
           "sample": f"{sweeps} FP64 Jacobi sweeps from V=0 of the same instance "
                     f"({pairs} feasible pairs each, {dt:.1f} s), NumPy on one host thread",
           "cpu_model": _cpu_model(), "host_cores_available": len(os.sched_getaffinity(0)),
           "seconds_per_sweep": dt / sweeps}
    if gpu_sweeps:
        out["time_to_tol_extrapolated_s"] = dt / sweeps * gpu_sweeps
        out["time_to_tol_note"] = (f"per-sweep time x the {gpu_sweeps} sweeps the GPU ran to the same "
                                   f"stopping test (extrapolated; GPU: {gpu_seconds:.4f} s)")
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large_single")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--eval-tol", type=float, default=1e-10)
    ap.add_argument("--cpu-sweeps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true",
                    help="skip the extra event-bracketed step (roofline fields become null)")
    ap.add_argument("--sweep-form", type=int, default=-1,
                    help="sweep kernels: -1 automatic, 0 direct, t in 1..K-1 LDS slab of t digits, "
                         "16+w tile form (w workgroups per CU, 0: one per tile)")
    ap.add_argument("--batch", type=int, default=512,
                    help="instances of the batched-vs-per-instance comparison (0: skip)")
    ap.add_argument("--no-bsdi", dest="bsdi", action="store_false",
                    help="skip the block-asynchronous (BSDI) comparison")
    ap.add_argument("--grad-batch", type=int, default=256,
                    help="instances of the batched gradient pipeline (0: skip the gradient fields)")
    ap.add_argument("--static", type=int, default=1_000_000,
                    help="random static scenarios for the first-fit placement timing (0: skip)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="time the automatic forms without running the autotuner first")
    ap.add_argument("--no-k7", dest="k7", action="store_false",
                    help="skip the supplementary instance beyond the last-level cache (K=7)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(instances are independent; see the sharding design). Run with --gpus 1.",
              file=sys.stderr)
        return 2

    import torch

    import paper_2012_12419_amd as mdpvi

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    inst, desc = workload(args.workload)
    mdp = mdpvi.MDP.from_instance(inst)
    mdp.set_sweep_form(args.sweep_form)
    tuned = None
    if args.autotune and args.sweep_form == -1:
        # untimed: the autotuner records the fastest form of each sweep for
        # this shape, and the automatic choice of the timed steps takes it
        tf, tus = mdp.autotune(trials=5)
        tuned = {"vi_form": tf, "vi_us_per_sweep": tus}
    vi_form, ev_form = mdp.sweep_forms()
    if tuned is not None:
        tuned.update({"eval_form": ev_form, "adjoint_form": mdp.adjoint_form()})
    N = mdp.num_states
    dev = "cuda:0"
    V = torch.zeros(N, dtype=torch.float32, device=dev)
    Vp = torch.zeros(N, dtype=torch.float64, device=dev)
    Vg = torch.zeros(N, dtype=torch.float64, device=dev)
    pi = torch.empty(N, dtype=torch.uint8, device=dev)
    pi2 = torch.empty(N, dtype=torch.uint8, device=dev)
    pig = torch.empty(N, dtype=torch.uint8, device=dev)
    gap = torch.empty(N, dtype=torch.float32, device=dev)
    lam = torch.tensor(inst.lam, dtype=torch.float64)
    c = lam / lam.sum()
    empty = torch.arange(inst.J, device=dev) * mdp.n_occ

    def step():
        V.zero_()
        s_vi = mdp.vi_solve(V, tol=args.tol)
        mdp.policy_extract(V, pi=pi, gap=gap)
        Vp.copy_(V)
        _, s_ev = mdp.policy_eval(pi, Vp, tol=args.eval_tol)
        mdp.policy_extract(Vp, pi=pi2, gap=None, want_gap=False)
        mdp.policy_greedy("least_loaded", pi=pig)
        Vg.copy_(Vp)   # the heuristic's evaluation starts from V_pi* (V_greedy <= V*, close to it)
        _, s_g = mdp.policy_eval(pig, Vg, tol=args.eval_tol)
        return s_vi, s_ev, s_g

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        recs.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    t_tol = sum(r[0]["seconds"] for r in recs) / len(recs)
    tol_labels = tolerance_runs(mdp, V, args.tol, t_tol, recs[0][0]["iterations"] if recs else None)
    pi_run = policy_iteration_run(mdp, args.eval_tol)
    bsdi = None
    if args.bsdi:
        try:
            bsdi = bsdi_comparison(mdp, N, args.tol)
        except mdpvi.MdpviError as e:
            bsdi = {"skipped": str(e)}

    # one more step with every sweep bracketed by its own pair of HIP events
    # (outside the timed region): a cross-check of the per-launch durations,
    # which the event pairs inflate by their own cost
    meas = None
    if not args.no_timing:
        mdp.set_timing(True)
        meas = step()
        torch.cuda.synchronize()
        mdp.set_timing(False)

    if args.copy_calibration_mb:
        n = args.copy_calibration_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    backups = sum(r[0]["backups"] + N * (r[1]["iterations"] + r[2]["iterations"]) for r in recs)
    vi_sweeps = [r[0]["iterations"] for r in recs]
    ev_sweeps = [r[1]["iterations"] for r in recs]
    g_sweeps = [r[2]["iterations"] for r in recs]

    roof = None
    kernels = {}
    if recs:
        vi_impl = vi_kernel_name(vi_form)
        ev_impl = "eval_tile_kernel" if ev_form >= mdpvi.FORM_TILE else "eval_exact_kernel"
        srcs = {"vi_tile_kernel": ["paper_2012_12419_amd/csrc/tile_vi.hip", "paper_2012_12419_amd/csrc/tile_vi.hpp",
                                   "paper_2012_12419_amd/csrc/tile.hpp"],
                "vi_row_kernel": ["paper_2012_12419_amd/csrc/row_vi.hip", "paper_2012_12419_amd/csrc/row.hpp",
                                  "paper_2012_12419_amd/csrc/tile.hpp"],
                "vi_exact_kernel": ["paper_2012_12419_amd/csrc/sweep.hip",
                                    "paper_2012_12419_amd/csrc/sweep_impl.hpp"],
                "vi_slab_kernel": ["paper_2012_12419_amd/csrc/sweep.hip",
                                   "paper_2012_12419_amd/csrc/sweep_impl.hpp"],
                "eval_tile_kernel": ["paper_2012_12419_amd/csrc/tile_eval.hip",
                                     "paper_2012_12419_amd/csrc/tile_eval.hpp",
                                     "paper_2012_12419_amd/csrc/tile.hpp"],
                "eval_exact_kernel": ["paper_2012_12419_amd/csrc/policy.hip",
                                      "paper_2012_12419_amd/csrc/policy_impl.hpp"]}
        # per-launch duration over the timed steps: each solve's span between
        # the HIP events that the library records on the solver's stream
        # before its first and after its last sweep, divided by the sweeps
        # that did work (the span also holds the few launches issued after
        # the stopping test and the per-chunk control reads: an upper bound)
        n_vi = sum(r[0]["iterations"] for r in recs)
        n_ev = sum(r[1]["iterations"] + r[2]["iterations"] for r in recs)
        t_vi = sum(r[0]["seconds"] for r in recs)
        t_ev = sum(r[1]["seconds"] + r[2]["seconds"] for r in recs)
        for name, impl, tot, cnt, bps, bracketed in [
                ("vi_sweep_kernel", vi_impl, t_vi, n_vi, VI_BYTES_PER_STATE,
                 (meas[0]["sweep_seconds"], meas[0]["iterations"]) if meas else None),
                ("eval_sweep_kernel", ev_impl, t_ev, n_ev, EVAL_BYTES_PER_STATE,
                 (meas[1]["sweep_seconds"] + meas[2]["sweep_seconds"],
                  meas[1]["iterations"] + meas[2]["iterations"]) if meas else None)]:
            avg = tot / cnt
            ach = bps * N / avg / 1e9
            kernels[name] = {"kernel": impl, "launches": cnt, "avg_us": avg * 1e6, "bytes_per_launch": bps * N,
                             "achieved_GBs": ach, "frac": ach / HBM_PEAK_GBS,
                             "share_of_solve_time": tot / (t_vi + t_ev),
                             "avg_us_event_pair_per_sweep": bracketed[0] / bracketed[1] * 1e6 if bracketed else None,
                             "traffic": traffic_record(srcs[impl], f"{impl}_{args.workload}")}
        dom = max(kernels, key=lambda k: kernels[k]["share_of_solve_time"])
        kd = kernels[dom]
        roof = {"bound": "hbm", "achieved": kd["achieved_GBs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": kd["frac"], "traffic": kd["traffic"], "kernel": kd["kernel"]}

    Vh = V.double()
    J_opt = float((c.to(dev) * Vp[empty]).sum())
    J_greedy = float((c.to(dev) * Vg[empty]).sum())
    changed = int((pi2 != pi).sum())

    out = {
        "metric": METRIC,
        "value": backups / elapsed,
        "unit": "backups/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32-storage/fp64-sum",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "states": N,
                   "feasible_pairs_per_sweep": mdp.feasible_pairs, "tol": args.tol,
                   "eval_tol": args.eval_tol, "sweep_form": args.sweep_form,
                   "forms_in_use": {"vi": vi_form, "eval": ev_form},
                   "autotuned": tuned,
                   "values": "FP32 storage, FP64 sums (VI); FP64 (evaluation)",
                   "value_composition": "per step: value iteration's feasible (state, action) backups "
                                        "over its sweeps, plus one (state, policy action) backup per "
                                        "state per FP64 evaluation sweep of pi* and of the least-loaded "
                                        "heuristic; divided by the steps' wall time"},
        "time_to_tol_s": t_tol,
        "time_to_tol": tol_labels,
        "vi_sweeps": vi_sweeps,
        "eval_sweeps": ev_sweeps,
        "greedy_eval_sweeps": g_sweeps,
        "vi_backups_per_s": sum(r[0]["backups"] for r in recs) / sum(r[0]["seconds"] for r in recs),
        "J_optimal": J_opt,
        "J_greedy_least_loaded": J_greedy,
        "improvement_step_changed_states": changed,
        "roofline": roof,
        "kernels": kernels,
        "bsdi_vs_jacobi": bsdi,
        "policy_iteration": pi_run,
    }
    del Vh
    if args.batch:
        out["batched_vs_per_instance"] = batched_vs_per_instance(mdpvi, args.batch, args.tol)
    if args.grad_batch:
        out["gradient"] = gradient_workloads(mdpvi, args.grad_batch, args.tol)
    if args.static:
        out["static_bot"] = static_bot_run(mdpvi, args.static)
    if args.k7:
        out["supplementary_beyond_cache"] = supplementary_k7(mdpvi, args.tol)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_sweeps, vi_sweeps[0] if vi_sweeps else None,
                                           t_tol)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
