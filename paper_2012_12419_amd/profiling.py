"""Counter-collection driver and rocprofv3 post-processing for profiles/.

    # a fixed number of sweeps of one kernel, plus a plain device copy of
    # known size (the calibration of the byte counters), for --pmc runs
    python -m paper_2012_12419_amd.profiling run --kernel vi --sweeps 30 --copy-mb 1024

    # per-kernel duration summary of a --kernel-trace --stats run
    python -m paper_2012_12419_amd.profiling stats <kernel_stats.csv> --command "..." \
        [--trace <kernel_trace.csv> --kernels vi_exact_kernel ...] > profiles/X.md

    # HBM traffic per launch from two --pmc runs (FETCH_SIZE, WRITE_SIZE),
    # scaled by what the counters read for a plain device copy of known size
    python -m paper_2012_12419_amd.profiling traffic --fetch <dir> --write <dir> \
        --kernel vi_exact_kernel --name vi_sweep_kernel_large_single \
        --copy-bytes 1073741824 --sources <files...> --command "..."

    # per-dispatch medians of any counters, one or more --pmc runs per kernel
    python -m paper_2012_12419_amd.profiling counters --dirs <dir...> \
        --kernels vi_tile_kernel eval_tile_kernel --command "..." > profiles/X.md

The traffic record carries a SHA-256 of the kernel's source files; bench.py
reports the traffic only while the sources are unchanged.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _counter_rows(d: str):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    rows = []
    for fn in files:
        with open(fn) as f:
            rows += list(csv.DictReader(f))
    return rows


def _per_dispatch(rows, counter: str, match) -> list:
    vals = {}
    for r in rows:
        if r["Counter_Name"] == counter and match(r["Kernel_Name"]):
            key = r.get("Dispatch_Id") or r.get("Correlation_Id") or str(len(vals))
            vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    return list(vals.values())


def sources_sha256(files) -> str:
    h = hashlib.sha256()
    for fn in files:
        with open(os.path.join(ROOT, fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic(fetch_dir: str, write_dir: str, kernel: str, copy_bytes: int, sources, command: str) -> dict:
    """The copy of copy_bytes (torch's device-to-device copy: a runtime blit
    kernel or an elementwise copy kernel) is the largest copy dispatch in the
    files; its counter readings calibrate the kernel's."""
    fr = _counter_rows(fetch_dir)
    wr = _counter_rows(write_dir)
    is_k = lambda n: kernel in n                                    # noqa: E731
    is_copy = lambda n: "copyBuffer" in n or ("elementwise" in n and "copy" in n.lower())  # noqa: E731
    f_k = _per_dispatch(fr, "FETCH_SIZE", is_k)
    w_k = _per_dispatch(wr, "WRITE_SIZE", is_k)
    f_c = _per_dispatch(fr, "FETCH_SIZE", is_copy)
    w_c = _per_dispatch(wr, "WRITE_SIZE", is_copy)
    if not f_k or not w_k:
        raise ValueError(f"kernel {kernel} not found in the counter files")
    if not f_c or not w_c:
        raise ValueError("copy calibration kernel not found in the counter files")
    kib = copy_bytes / 1024.0
    ff = kib / max(f_c)     # the copy moves copy_bytes each way
    fw = kib / max(w_c)
    fetch = statistics.median(f_k) * ff * 1024.0
    write = statistics.median(w_k) * fw * 1024.0
    return {"kernel": kernel, "launches_measured": len(f_k),
            "fetch_kib_median": statistics.median(f_k), "write_kib_median": statistics.median(w_k),
            "copy_bytes": copy_bytes, "copy_fetch_kib": max(f_c), "copy_write_kib": max(w_c),
            "fetch_factor": ff, "write_factor": fw,
            "bytes_per_launch": fetch + write, "fetch_bytes_per_launch": fetch,
            "write_bytes_per_launch": write, "sources": list(sources),
            "source_sha256": sources_sha256(sources), "command": command}


def working_launches(trace_csv: str, kernels) -> list:
    """Per kernel: the launches that did a sweep's work.  A sweep launched
    after the stopping test has passed returns at once (a few microseconds);
    those launches are the ones shorter than half the kernel's median."""
    with open(trace_csv) as f:
        rows = list(csv.DictReader(f))
    out = []
    for k in kernels:
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
             for r in rows if k in r["Kernel_Name"]]
        if not d:
            continue
        cut = 0.5 * statistics.median(d)
        w = [x for x in d if x >= cut]
        out.append((k, len(d), len(w), statistics.mean(w), statistics.median(w)))
    return out


def stats_markdown(stats_csv: str, command: str, top: int = 12, trace_csv: str = None,
                   kernels=()) -> str:
    with open(stats_csv) as f:
        rows = list(csv.DictReader(f))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"Command: `{command}`", "",
           "| Kernel | Calls | Total ms | Average us | Min us | Max us | % |",
           "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        name = r["Name"].replace("|", "/")
        if len(name) > 90:
            name = name[:87] + "..."
        out.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    if trace_csv and kernels:
        out += ["", "Working launches (from the kernel trace; launches shorter than half the "
                "kernel's median are sweeps issued after the stopping test passed, which return at once):", "",
                "| Kernel | Launches | Working | Mean us | Median us |", "|---|---|---|---|---|"]
        for k, n, nw, mean, med in working_launches(trace_csv, kernels):
            out.append(f"| `{k}` | {n} | {nw} | {mean:.2f} | {med:.2f} |")
    return "\n".join(out) + "\n"


def run_sweeps(kernel: str, workload: str, sweeps: int, copy_mb: int, form: int,
               adjoint_form: int = 0) -> None:
    """`sweeps` sweeps of value iteration (kernel "vi"), of FP64 evaluation
    of the least-loaded policy (kernel "eval") or of the adjoint equation of
    that policy (kernel "adjoint") from zero, then a device copy of copy_mb
    MiB."""
    import torch

    import paper_2012_12419_amd as mdpvi
    sys.path.insert(0, ROOT)
    import workloads as W
    inst = {"large_single": W.large_single(), "large_single_k7": W.large_single(K=7),
            "gradient": W.gradient_instance()}[workload]
    mdp = mdpvi.MDP.from_instance(inst)
    mdp.set_sweep_form(form)
    mdp.set_adjoint_form(adjoint_form)
    try:
        if kernel == "vi":
            V = torch.zeros(mdp.num_states, device="cuda")
            mdp.vi_solve(V, tol=1e-300, max_iter=sweeps)
        elif kernel == "adjoint":
            pi = mdp.policy_greedy("least_loaded")
            Vp = torch.zeros(mdp.num_states, dtype=torch.float64, device="cuda")
            mdp.vi_adjoint(pi, Vp, tol=1e-300, max_iter=sweeps)
        else:
            pi = mdp.policy_greedy("least_loaded")
            V = torch.zeros(mdp.num_states, dtype=torch.float64, device="cuda")
            mdp.policy_eval(pi, V, tol=1e-300, max_iter=sweeps)
    except mdpvi.MdpviError as e:
        if e.code != mdpvi.ENOCONV:
            raise
    if copy_mb:
        a = torch.ones(copy_mb * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"ran {sweeps} {kernel} sweeps on {workload}, copy {copy_mb} MiB", flush=True)


def counters_markdown(dirs, kernels, command: str) -> str:
    """Median over dispatches of every counter found in the --pmc output
    directories, per kernel (a kernel name matches when it contains the given
    string), as a markdown table with one row per counter."""
    rows = []
    for d in dirs:
        rows += _counter_rows(d)
    names = sorted({r["Counter_Name"] for r in rows})
    table = {}
    for k in kernels:
        for c in names:
            v = _per_dispatch(rows, c, lambda n, k=k: k in n)
            if v:
                table[(c, k)] = (statistics.median(v), len(v))
    out = [f"Command: `{command}`", "", "Per-dispatch medians (dispatches in brackets).", "",
           "| Counter | " + " | ".join(f"`{k}`" for k in kernels) + " |",
           "|---|" + "---|" * len(kernels)]
    for c in names:
        cells = []
        for k in kernels:
            m = table.get((c, k))
            cells.append(f"{m[0]:.4g} ({m[1]})" if m else "")
        if any(cells):
            out.append(f"| {c} | " + " | ".join(cells) + " |")
    return "\n".join(out) + "\n"


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--kernel", choices=["vi", "eval", "adjoint"], default="vi")
    r.add_argument("--workload", default="large_single")
    r.add_argument("--sweeps", type=int, default=30)
    r.add_argument("--copy-mb", type=int, default=1024)
    r.add_argument("--form", type=int, default=-1)
    r.add_argument("--adjoint-form", type=int, default=0)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--command", required=True)
    s.add_argument("--trace", default=None, help="kernel_trace.csv of the same run")
    s.add_argument("--kernels", nargs="*", default=[], help="kernels to list working launches of")
    s.add_argument("--top", type=int, default=12, help="rows of the per-kernel table")
    c = sub.add_parser("counters")
    c.add_argument("--dirs", nargs="+", required=True)
    c.add_argument("--kernels", nargs="+", required=True)
    c.add_argument("--command", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--name", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--sources", nargs="+", required=True)
    t.add_argument("--command", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "run":
        run_sweeps(a.kernel, a.workload, a.sweeps, a.copy_mb, a.form, a.adjoint_form)
        return 0
    if a.cmd == "stats":
        sys.stdout.write(stats_markdown(a.csv, a.command, top=a.top, trace_csv=a.trace, kernels=a.kernels))
        return 0
    if a.cmd == "counters":
        sys.stdout.write(counters_markdown(a.dirs, a.kernels, a.command))
        return 0
    rec = traffic(a.fetch, a.write, a.kernel, a.copy_bytes, a.sources, a.command)
    path = os.path.join(ROOT, "profiles", f"{a.name}_traffic.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(path)
    return 0


if __name__ == "__main__":
    sys.exit(main())
