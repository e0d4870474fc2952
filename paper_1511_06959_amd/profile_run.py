"""Fixed launch sequences for hardware-counter and kernel-trace profiles, and their summaries.

    python -m paper_1511_06959_amd.profile_run adjoint --n 64 --precision f32 --reps 5 [--stages] [--tune]
        [--flux roe]
        reverse steps (adjoint_step / adjoint_step_stages) on an n^3 Taylor-Green state, Mach 0.1,
        lambda 0: the reverse-stage kernel as the benchmark launches it (with --tune, in the tile
        shapes of the tuning cache that a preceding bench.py run filled; with --flux roe, followed
        by the Roe flux kernels)
    python -m paper_1511_06959_amd.profile_run step384 --reps 3 [--cache FILE.npy]
        time steps of the 384^3 turbulence case as the benchmark runs them: primal step with BF16
        snapshot encoding, reverse step from the record (lambda 0.1 dx^2 sigma_1, mean pressure)
    python -m paper_1511_06959_amd.profile_run copy --mib 1024 --reps 5
        torch's device-to-device copy of a buffer of known size, the calibration of the byte
        counters (it reads and writes exactly mib MiB per launch)
    python -m paper_1511_06959_amd.profile_run summarize <rocprofv3 output dir> [--kernel SUBSTR]
        mean value per dispatch of every counter, per kernel, from the *_counter_collection.csv
        files under the directory
    python -m paper_1511_06959_amd.profile_run traffic --fetch D --write D --copy-fetch D --copy-write D
        --cells N [--kernel k_adjoint_stage]
        HBM bytes per launch of a kernel from FETCH_SIZE / WRITE_SIZE runs, calibrated on the copy runs
    python -m paper_1511_06959_amd.profile_run valu <dir> --cells N [--kernel k_adjoint_stage]
        vector-ALU instructions and FP32 operations per launch from one run with the SQ counters
        of VALU_COUNTERS
    python -m paper_1511_06959_amd.profile_run stall <dir> [<dir> ...] --cells N [--kernel _stage]
        issue, wait and LDS fractions per kernel from runs with SQ counters (STALL_COUNTERS and others)
    python -m paper_1511_06959_amd.profile_run trace <dir> --title T --command C [--note PARAGRAPH ...]
        markdown table of a --kernel-trace --stats run

Run the first two under rocprofv3, e.g.
    rocprofv3 --pmc FETCH_SIZE -d prof/pmc_fetch -o run --output-format csv -- \
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


def run_adjoint(n, precision, reps, stages, tune=False, flux="split"):
    import torch

    import paper_1511_06959_amd as adj
    import workloads as W

    prec = adj.F64 if precision == "f64" else adj.F32
    dt = torch.float64 if prec == adj.F64 else torch.float32
    L = (2 * math.pi,) * 3
    nn = (n, n, n)
    rho, u, v, w, p = W.tgv_fields(nn, L, 0.1)
    dx = [L[d] / n for d in range(3)]
    g = adj.Grid.make(nn, L, 1.0 / 1600.0, W.cfl_dt(rho, u, v, w, p, dx), precision=prec,
                      flux=adj.FLUX_ROE if flux == "roe" else adj.FLUX_SPLIT, roe_delta=0.1)
    w0 = torch.from_numpy(W.conservative(rho, u, v, w, p)).to("cuda", dt)
    ws = adj.workspace(g)
    if tune:
        # the tile shapes the benchmark runs (from the tuning cache when it holds this grid)
        from . import autotune
        autotune.tune(g)
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
    print(f"adjoint: {reps} reverse steps on {n}^3 ({precision}, {'stored' if stages else 'recomputed'} stages, "
          f"{flux} flux)", flush=True)


def run_step384(reps, cache=None, tune=True):
    """Time steps of the 384^3 decaying-turbulence case with the benchmark's kernels (FP32 states
    stored as deviations, BF16 snapshot records, lambda = 0.1 dx^2 sigma_1, mean pressure fused
    into the stages): each rep is a primal step that encodes its snapshot and accumulates J, and a
    reverse step from that record (which recomputes the stage states).  cache:
    an .npy file holding the initial field (written on the first run, read afterwards)."""
    import numpy as np
    import torch

    import paper_1511_06959_amd as adj
    import workloads as W

    wl = W.turb_384(nsteps=5000, lam_factor=0.1) if not (cache and os.path.exists(cache)) else None
    if wl is None:
        w0 = np.load(cache)
        wl = W.turbulence(8, mach_rms=0.4, nu=2.887e-3, seed=4, nsteps=5000, lam_factor=0.1)  # parameters only
        n, L = (384, 384, 384), (2 * math.pi,) * 3
        dx = L[0] / 384
        # the dt and lambda of the 384^3 field (dt from its realised velocities, as turb_384 sets it)
        u = w0.reshape(5, -1)[1:4] / w0.reshape(5, -1)[0]
        c0 = 1.0 / 0.4
        rate = float((np.abs(u).sum(axis=0) + 3 * c0).max()) / dx
        wl.n, wl.L, wl.w0, wl.dt, wl.lam = n, L, w0, 0.5 / rate, 0.1 * dx * dx
    elif cache:
        np.save(cache, wl.w0)
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, adj.F32, adj.CKPT_BF16,
                      adj.reference_state(wl.w0))
    if tune:
        from . import autotune
        autotune.tune(g)
    w = torch.from_numpy(g.to_stored(wl.w0)).to("cuda", torch.float32)
    nxt = torch.empty_like(w)
    ws = adj.workspace(g)
    rec = torch.empty(adj.ckpt_bytes(g), dtype=torch.uint8, device="cuda")
    obj = adj.Objective.make(adj.OBJ_MEAN_PRESSURE)
    a = torch.randn(w.numel(), dtype=torch.float32, device="cuda") * 1e-3
    b = torch.empty_like(a)
    gs = torch.zeros_like(a)
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(reps):
        adj.primal_step_obj(g, w, None, nxt, ws, obj, 1.0 / 5000, J, ckpt_out=rec)
        adj.adjoint_step(g, rec, None, a, b, ws, lam=wl.lam, obj=obj, c_n=1.0 / 5000, grad_s=gs)
        a, b = b, a
        w, nxt = nxt, w
    torch.cuda.synchronize()
    print(f"step384: {reps} primal + reverse steps on 384^3 (dt {wl.dt:.4e}, lambda {wl.lam:.3e})", flush=True)


def run_copy(mib, reps):
    """reps device copies of a buffer of mib MiB; prints the copy rate (bytes read + written per
    second, HIP events around the copies after one untimed copy)."""
    import torch

    x = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    print(f"copy: {reps} copies of {mib} MiB, {ms:.3f} ms each, {2 * (mib << 20) / ms / 1e6:.0f} GB/s read + write",
          flush=True)


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


def _counter_means(outdir, kernel):
    """{kernel name: (dispatches, mean value)} of the single counter in a rocprofv3 output dir."""
    acc, disp = defaultdict(float), defaultdict(set)
    for f in glob.glob(os.path.join(outdir, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                k = short_name(row.get("Kernel_Name", ""))
                if kernel in k:
                    acc[k] += float(row["Counter_Value"])
                    disp[k].add(row.get("Dispatch_Id"))
    return {k: (len(disp[k]), acc[k] / max(1, len(disp[k]))) for k in acc}


def traffic(fetch, write, copy_fetch, copy_write, mib, cells, kernel, commands):
    """key = value file of HBM bytes per cell and launch of `kernel` (all its instantiations,
    weighted by dispatch count), FETCH_SIZE / WRITE_SIZE scaled by what they read for a copy of
    mib MiB (which reads and writes exactly that much)."""
    cf = _counter_means(copy_fetch, "copyBuffer")
    cw = _counter_means(copy_write, "copyBuffer")
    (_, cfv), = cf.values()
    (_, cwv), = cw.values()
    sf, sw = mib * 1024.0 / cfv, mib * 1024.0 / cwv
    fm, wm = _counter_means(fetch, kernel), _counter_means(write, kernel)
    nd = sum(n for n, _ in fm.values())
    fkib = sum(n * v for n, v in fm.values()) / nd
    wkib = sum(n * v for n, v in wm.values()) / sum(n for n, _ in wm.values())
    byts = (fkib * sf + wkib * sw) * 1024.0
    print(f"# HBM traffic of {kernel} (rocprofv3 FETCH_SIZE and WRITE_SIZE, separate runs), {cells} cells")
    for c in commands:
        print(f"# command: {c}")
    print(f"# calibration: copy of {mib} MiB reads FETCH_SIZE {cfv:.0f} KiB, WRITE_SIZE {cwv:.0f} KiB per dispatch")
    print(f"# scale factors (true / counter): fetch {sf:.4f}, write {sw:.4f}")
    for k in sorted(fm):
        print(f"# {k}: {fm[k][0]} dispatches, FETCH_SIZE {fm[k][1]:.1f} KiB, WRITE_SIZE {wm.get(k, (0, 0))[1]:.1f} KiB")
    print(f"kernel_source_sha256 = {_src_hash(kernel)}")
    print(f"tile_f32 = {_tiles(fm)}")
    print(f"fetch_bytes_per_launch = {fkib * sf * 1024.0:.6g}")
    print(f"write_bytes_per_launch = {wkib * sw * 1024.0:.6g}")
    print(f"bytes_per_cell_launch_f32 = {byts / cells:.6g}")


def _tiles(names):
    """Tile shapes ("32x8x4") in the template arguments of k_*_stage kernel names."""
    out = set()
    for k in names:
        m = re.search(r"<[^<>]*?(\d+), (\d+), (\d+)>$", k)
        if m:
            out.add("x".join(m.groups()))
    return ",".join(sorted(out))


SOURCES = {"stage": ("stencil.hip", "common.hpp"), "roe": ("roe.hip", "roe_flux.hpp", "common.hpp")}


def _src_hash(kernel="k_adjoint_stage"):
    """sha256 of the sources of a kernel family: the Roe kernels (k_roe_*) are roe.hip with the
    flux core roe_flux.hpp, the stage kernels stencil.hip; all include common.hpp."""
    import hashlib
    h = hashlib.sha256()
    here = os.path.dirname(os.path.abspath(__file__))
    for name in SOURCES["roe" if kernel.startswith("k_roe") else "stage"]:
        h.update(open(os.path.join(here, "csrc", name), "rb").read())
    return h.hexdigest()


VALU_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32",
                 "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_TRANS_F32")


def valu(outdir, cells, kernel, commands):
    """key = value file of vector-ALU work per cell and launch of `kernel` (all its
    instantiations, weighted by dispatch count) from one run with VALU_COUNTERS: wave-level VALU
    instructions, and FP32 operations issued (64 lanes per wave instruction; an FMA counts 2)."""
    acc, disp = defaultdict(lambda: defaultdict(float)), defaultdict(set)
    for f in glob.glob(os.path.join(outdir, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                k = short_name(row.get("Kernel_Name", ""))
                if kernel in k:
                    acc[k][row["Counter_Name"]] += float(row["Counter_Value"])
                    disp[k].add(row.get("Dispatch_Id"))
    if not acc:
        sys.exit(f"no {kernel} dispatches under {outdir}")
    nd = sum(len(disp[k]) for k in acc)
    tot = defaultdict(float)
    for k in acc:
        for c, v in acc[k].items():
            tot[c] += v
    per = {c: tot[c] / nd for c in tot}  # per dispatch
    flops = 64.0 * (per.get("SQ_INSTS_VALU_ADD_F32", 0.0) + per.get("SQ_INSTS_VALU_MUL_F32", 0.0)
                    + 2.0 * per.get("SQ_INSTS_VALU_FMA_F32", 0.0) + per.get("SQ_INSTS_VALU_TRANS_F32", 0.0))
    print(f"# vector-ALU work of {kernel} (rocprofv3 SQ counters, one run), {cells} cells")
    for c in commands:
        print(f"# command: {c}")
    for k in sorted(acc):
        print(f"# {k}: {len(disp[k])} dispatches, " +
              ", ".join(f"{c} {acc[k][c] / len(disp[k]):.6g}" for c in VALU_COUNTERS if c in acc[k]))
    print("# FP32 operations = 64 x (ADD + MUL + TRANS + 2 FMA) wave instructions")
    print(f"kernel_source_sha256 = {_src_hash(kernel)}")
    print(f"tile_f32 = {_tiles(acc)}")
    print(f"waves_per_launch = {per.get('SQ_WAVES', 0.0):.6g}")
    print(f"valu_insts_per_launch = {per.get('SQ_INSTS_VALU', 0.0):.6g}")
    print(f"valu_insts_per_cell_launch_f32 = {per.get('SQ_INSTS_VALU', 0.0) / cells:.6g}")
    print(f"fp32_ops_per_cell_launch_f32 = {flops / cells:.6g}")


STALL_COUNTERS = ("SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU",
                  "SQ_INSTS_LDS", "SQ_WAIT_INST_LDS", "SQ_LDS_BANK_CONFLICT")


FRACTIONS = (("valu_active_frac", "SQ_ACTIVE_INST_VALU"), ("wait_issue_frac", "SQ_WAIT_INST_ANY"),
             ("wait_lds_frac", "SQ_WAIT_INST_LDS"), ("wait_any_frac", "SQ_WAIT_ANY"),
             ("lds_active_frac", "SQ_ACTIVE_INST_LDS"), ("active_any_frac", "SQ_ACTIVE_INST_ANY"))


def stall(outdirs, cells, kernel, commands):
    """Averages per dispatch of the SQ counters of one or more runs (each counter averaged over
    the dispatches of the run that took it) for every kernel whose name holds `kernel`, and their
    fractions of SQ_WAVE_CYCLES (the summed wave lifetimes, so the counters' common unit cancels):
    VALU issue, waiting to issue, waiting for LDS, waiting on any counter, LDS and any-unit
    activity, as far as the runs hold them; bank-conflict cycles per LDS instruction and per
    LDS-active cycle."""
    if isinstance(outdirs, str):
        outdirs = [outdirs]
    acc, disp = defaultdict(lambda: defaultdict(float)), defaultdict(lambda: defaultdict(set))
    for d in outdirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for row in csv.DictReader(fh):
                    k = short_name(row.get("Kernel_Name", ""))
                    if kernel in k:
                        c = row["Counter_Name"]
                        acc[k][c] += float(row["Counter_Value"])
                        disp[k][c].add((d, row.get("Dispatch_Id")))
    if not acc:
        sys.exit(f"no {kernel} dispatches under {', '.join(outdirs)}")
    print(f"# stall and issue counters of the *{kernel}* kernels (rocprofv3 SQ counters, "
          f"{len(outdirs)} run{'s' if len(outdirs) > 1 else ''}), {cells} cells")
    for c in commands:
        print(f"# command: {c}")
    print("# averages per dispatch; the fractions are of SQ_WAVE_CYCLES (summed wave lifetimes), so the counters' "
          "common unit")
    print("# cancels; lds_conflict_per_lds_inst = SQ_LDS_BANK_CONFLICT cycles per LDS instruction")
    print(f"# kernel_source_sha256 = {_src_hash(kernel)}")
    for k in sorted(acc):
        a = {c: v / len(disp[k][c]) for c, v in acc[k].items()}
        n = max(len(v) for v in disp[k].values())
        print(f"{k}: {n} dispatches, " + ", ".join(f"{c} {a[c]:.6g}" for c in sorted(a)))
        wc = a.get("SQ_WAVE_CYCLES", 0.0) or float("nan")
        parts = [f"{name} = {a[c] / wc:.3f}" for name, c in FRACTIONS if c in a]
        if "SQ_LDS_BANK_CONFLICT" in a and "SQ_INSTS_LDS" in a:
            parts.append(f"lds_conflict_per_lds_inst = {a['SQ_LDS_BANK_CONFLICT'] / max(a['SQ_INSTS_LDS'], 1.0):.3f}")
        if "SQ_LDS_BANK_CONFLICT" in a and "SQ_ACTIVE_INST_LDS" in a:
            parts.append("lds_conflict_per_lds_active_cycle = "
                         f"{a['SQ_LDS_BANK_CONFLICT'] / max(a['SQ_ACTIVE_INST_LDS'], 1.0):.3f}")
        print("  " + ", ".join(parts))


def trace_summary(outdir, title, command, notes=()):
    """Markdown table of a rocprofv3 --kernel-trace --stats run (*_kernel_stats.csv), after the
    paragraphs `notes`."""
    files = glob.glob(os.path.join(outdir, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        sys.exit(f"no kernel_stats.csv under {outdir}")
    rows = []
    for f in files:
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    print(f"# {title}\n")
    print("Command (from the repository root):\n")
    print("```\n" + command + "\n```\n")
    for n in notes:
        print(n + "\n")
    print("rocprofv3 kernel-trace statistics:\n")
    print("| kernel | calls | total (ms) | average (us) | % |")
    print("|---|---:|---:|---:|---:|")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        pct = float(r.get("Percentage", 0.0))
        if pct < 0.05:
            continue
        print(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
              f"{float(r['AverageNs']) / 1e3:.2f} | {pct:.1f} |")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("adjoint")
    a.add_argument("--n", type=int, default=64)
    a.add_argument("--precision", choices=("f32", "f64"), default="f32")
    a.add_argument("--reps", type=int, default=5)
    a.add_argument("--stages", action="store_true")
    a.add_argument("--tune", action="store_true", help="install the autotuned tiles (tuning cache) first")
    a.add_argument("--flux", choices=("split", "roe"), default="split",
                   help="roe: the Roe flux option (its kernels run after each stage kernel)")
    q = sub.add_parser("step384")
    q.add_argument("--reps", type=int, default=3)
    q.add_argument("--cache", default=None, help=".npy file of the initial field (written if missing)")
    q.add_argument("--no-tune", action="store_true")
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    c.add_argument("--reps", type=int, default=5)
    s = sub.add_parser("summarize")
    s.add_argument("outdir")
    s.add_argument("--kernel", default=None)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--mib", type=int, default=1024)
    t.add_argument("--cells", type=int, required=True)
    t.add_argument("--kernel", default="k_adjoint_stage")
    t.add_argument("--command", action="append", default=[])
    v = sub.add_parser("valu")
    v.add_argument("outdir")
    v.add_argument("--cells", type=int, required=True)
    v.add_argument("--kernel", default="k_adjoint_stage")
    v.add_argument("--command", action="append", default=[])
    st = sub.add_parser("stall")
    st.add_argument("outdir", nargs="+")
    st.add_argument("--cells", type=int, required=True)
    st.add_argument("--kernel", default="_stage")
    st.add_argument("--command", action="append", default=[])
    r = sub.add_parser("trace")
    r.add_argument("outdir")
    r.add_argument("--title", required=True)
    r.add_argument("--command", required=True)
    r.add_argument("--note", action="append", default=[], help="a paragraph printed before the table")
    args = ap.parse_args()
    if args.cmd == "traffic":
        traffic(args.fetch, args.write, args.copy_fetch, args.copy_write, args.mib, args.cells, args.kernel,
                args.command)
        return
    if args.cmd == "valu":
        valu(args.outdir, args.cells, args.kernel, args.command)
        return
    if args.cmd == "stall":
        stall(args.outdir, args.cells, args.kernel, args.command)
        return
    if args.cmd == "trace":
        trace_summary(args.outdir, args.title, args.command, args.note)
        return
    if args.cmd == "adjoint":
        run_adjoint(args.n, args.precision, args.reps, args.stages, args.tune, args.flux)
    elif args.cmd == "step384":
        run_step384(args.reps, args.cache, not args.no_tune)
    elif args.cmd == "copy":
        run_copy(args.mib, args.reps)
    else:
        summarize(args.outdir, args.kernel)


if __name__ == "__main__":
    main()
