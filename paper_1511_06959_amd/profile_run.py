"""Fixed launch sequences for hardware-counter and kernel-trace profiles, and their summaries.

    python -m paper_1511_06959_amd.profile_run adjoint --n 64 --precision f32 --reps 5 [--stages]
        reverse steps (adjoint_step / adjoint_step_stages) on an n^3 Taylor-Green state, Mach 0.1,
        lambda 0: the reverse-stage kernel as the benchmark launches it
    python -m paper_1511_06959_amd.profile_run copy --mib 1024 --reps 5
        torch's device-to-device copy of a buffer of known size, the calibration of the byte
        counters (it reads and writes exactly mib MiB per launch)
    python -m paper_1511_06959_amd.profile_run summarize <rocprofv3 output dir> [--kernel SUBSTR]
        mean value per dispatch of every counter, per kernel, from the *_counter_collection.csv
        files under the directory

Run the first two under rocprofv3, e.g.
    rocprofv3 --pmc FETCH_SIZE -d gpurun_out/pmc_fetch -o run --output-format csv -- \
        python -m paper_1511_06959_amd.profile_run adjoint --n 64 --precision f32 --reps 5 --stages
"""
import argparse
import csv
import glob
import math
import os
import re
import sys
from collections import defaultdict


def run_adjoint(n, precision, reps, stages):
    import torch

    import paper_1511_06959_amd as adj
    import workloads as W

    prec = adj.F64 if precision == "f64" else adj.F32
    dt = torch.float64 if prec == adj.F64 else torch.float32
    L = (2 * math.pi,) * 3
    nn = (n, n, n)
    rho, u, v, w, p = W.tgv_fields(nn, L, 0.1)
    dx = [L[d] / n for d in range(3)]
    g = adj.Grid.make(nn, L, 1.0 / 1600.0, W.cfl_dt(rho, u, v, w, p, dx), precision=prec)
    w0 = torch.from_numpy(W.conservative(rho, u, v, w, p)).to("cuda", dt)
    ws = adj.workspace(g)
    obj = adj.Objective.make(adj.OBJ_KE_DISSIPATION)
    w1 = torch.empty_like(w0)
    st = torch.empty(3 * w0.numel(), dtype=dt, device="cuda") if stages else None
    if stages:
        adj.primal_step_stages(g, w0, None, w1, st, ws)
    else:
        adj.primal_step(g, w0, None, w1, ws)
    a = torch.randn(w0.numel(), dtype=dt, device="cuda") * 1e-3
    b = torch.empty_like(a)
    gs = torch.zeros_like(a)
    for _ in range(reps):
        if stages:
            adj.adjoint_step_stages(g, w0, st, None, a, b, ws, obj=obj, c_n=1e-3, grad_s=gs)
        else:
            adj.adjoint_step(g, w0, None, a, b, ws, obj=obj, c_n=1e-3, grad_s=gs)
        a, b = b, a
    torch.cuda.synchronize()
    print(f"adjoint: {reps} reverse steps on {n}^3 ({precision}, {'stored' if stages else 'recomputed'} stages)",
          flush=True)


def run_copy(mib, reps):
    import torch

    x = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copy: {reps} copies of {mib} MiB", flush=True)


def short_name(name):
    name = name.replace("(anonymous namespace)::", "").replace("adjns::", "")
    name = re.sub(r"^void ", "", name)
    m = re.match(r"([A-Za-z_0-9:]+)(<[^()]*>)?", name)
    return (m.group(1) + (m.group(2) or "")) if m else name


def summarize(outdir, kernel=None):
    files = glob.glob(os.path.join(outdir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        sys.exit(f"no counter_collection.csv under {outdir}")
    acc = defaultdict(lambda: defaultdict(float))
    disp = defaultdict(set)
    for f in files:
        with open(f) as fh:
            for row in csv.DictReader(fh):
                k = short_name(row.get("Kernel_Name", ""))
                if kernel and kernel not in k:
                    continue
                key = (k, row.get("Counter_Name"))
                acc[k][row.get("Counter_Name")] += float(row.get("Counter_Value", 0.0))
                disp[key].add(row.get("Dispatch_Id") or row.get("Correlation_Id"))
    counters = sorted({c for k in acc for c in acc[k]})
    print("| kernel | dispatches | " + " | ".join(f"{c} / dispatch" for c in counters) + " |")
    print("|---|---:|" + "---:|" * len(counters))
    for k in sorted(acc):
        nd = max(len(disp[(k, c)]) for c in counters if (k, c) in disp)
        vals = [acc[k][c] / max(1, len(disp[(k, c)])) if (k, c) in disp else float("nan") for c in counters]
        print(f"| `{k}` | {nd} | " + " | ".join(f"{v:.6g}" for v in vals) + " |")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("adjoint")
    a.add_argument("--n", type=int, default=64)
    a.add_argument("--precision", choices=("f32", "f64"), default="f32")
    a.add_argument("--reps", type=int, default=5)
    a.add_argument("--stages", action="store_true")
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    c.add_argument("--reps", type=int, default=5)
    s = sub.add_parser("summarize")
    s.add_argument("outdir")
    s.add_argument("--kernel", default=None)
    args = ap.parse_args()
    if args.cmd == "adjoint":
        run_adjoint(args.n, args.precision, args.reps, args.stages)
    elif args.cmd == "copy":
        run_copy(args.mib, args.reps)
    else:
        summarize(args.outdir, args.kernel)


if __name__ == "__main__":
    main()
