#!/usr/bin/env python3
"""Throughput of the stabilised discrete unsteady adjoint on one MI355X.

Default workload (the large single case with autograd): 384^3 periodic decaying turbulence
(E(k) ~ k^4 exp(-2k^2/k0^2), k0 = 4, Mach_rms 0.4, nu = 2.887e-3), the window of 5000 RK4 steps
reversed with checkpointing sized to the free HBM, the snapshots BF16 records (block-scaled,
plane-predicted), lambda = 0.1 dx^2 sigma_1, objective the time-averaged volume-mean pressure,
gradient with respect to a 5 x 384^3 body force (base 0), FP32 stencils, FP64 reductions.
Synthetic data (seeded), inputs resident in HBM before the timed region.  The plan that fits is
two-level: a snapshot every ~28 steps, and in the reverse sweep one segment at a time re-advanced
from its snapshot with every state and stage state kept, then reversed without recomputation.

One benchmark step = one time step of that plan: its primal step, its re-advance (with the stage
states kept) and its reverse step (sigma_1, the four transposed stages, objective injection,
body-force gradient), with the snapshot encodings and decodings of the window.  `--steps K` times
one K-step window of the same schedule (one segment); `value` = cells x K / seconds of that
window (adjoint cell-steps/s).  The FP64 path (FP64 snapshots; the two-level plan does not fit,
so binomial checkpointing whose sample window recomputes no less per time step than the plan) is
timed the same way and reported beside it, with the FP32/BF16 error against it, and the 16^3
Taylor-Green window of every path is checked against the FP64 oracle.

Roofline: each kernel class's average launch duration is measured with the dispatch's own HIP
events (hipExtLaunchKernel) over a second, profiled run of the same window; `achieved` =
algorithmic bytes per launch (the hot-path byte counts per adjoint or primal cell-step, a
quarter of them per stage launch) / that duration, against 8 TB/s; `roofline_valu` sets the
same launches against the vector ALU.  Other workloads: --workload (see WORKLOADS).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ROE_DELTA = 0.1  # Roe flux option: |lam| smoothed within 0.1 c~ of zero
# FP32 vector peaks: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz = 78.6 TFLOP/s without packed
# FP32 instructions (this library is built without them), 157.3 TFLOP/s with them
VALU_PEAK_TFLOPS = 78.6
VALU_PEAK_PACKED_TFLOPS = 157.3
METRIC = "adjoint cell-steps/s + % HBM roofline, FP32/BF16-ckpt vs FP64 at stated rel err"
# Algorithmic bytes per cell-step (what the method must move): an adjoint step reads the stored
# snapshot, reads w^_{n+1}, writes w^_n and updates grad_s; a primal step reads w_n, writes w_{n+1}
# and writes the snapshot.  A stage launch does a quarter of a step.
ALG_BYTES = {"adjoint": {"f32": 90.0, "f64": 200.0}, "primal": {"f32": 50.0, "f64": 120.0}}
PLAN_STEPS = 5000  # the configured window of the 384^3 case

# Algorithmic values moved per cell by the four reverse-stage launches of one adjoint step
# (stage 4: W, a in, g4 out = 15; stages 3 and 2: W, a, g_next in, g out = 20 each;
# stage 1: W, a, g2, g3, g4 in, w^_n out, grad_s read+write = 40), i.e. 95 values per
# adjoint cell-step, 23.75 per launch and cell.
VALUES_PER_STAGE_LAUNCH = 95.0 / 4.0
# SSP-RK3: stage 3 (W, a in, g3 out) 15, stage 2 (W, a, g3 in, g2 out) 20, stage 1 (W, a, g2 + g3/4
# in, g1 out) 20 values per cell; the combination of the stages is a separate elementwise pass
VALUES_PER_STAGE_LAUNCH_RK3 = 55.0 / 3.0


def profile_values(name, kernel_src_hash, tile):
    """key = value pairs of a committed rocprofv3 summary of the reverse-stage kernel:
    profiles/<name>, or profiles/<stem>_<tile>.txt (summaries taken in another tile shape, for
    runs whose tuner keeps that shape), whichever was taken on this kernel source and tile;
    None if neither was."""
    stem, ext = os.path.splitext(name)
    for cand in (name, f"{stem}_{tile}{ext}"):
        path = os.path.join(ROOT, "profiles", cand)
        if not os.path.exists(path):
            continue
        vals = {}
        for line in open(path):
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
        if vals.get("kernel_source_sha256") == kernel_src_hash and vals.get("tile_f32") == tile:
            vals["profile"] = cand
            return vals
    return None


def valu_roofline(valu, cells, avg_us):
    """A kernel against the vector ALU: FP32 operations it issues per launch (committed SQ counter
    summary) / its live average launch duration, against 78.6 TFLOP/s (FP32 without packed
    instructions; 157.3 with them is stated beside it);
    issue_frac = wave-level VALU instructions x 4 cycles (a wave64 instruction on a 16-lane SIMD)
    / (1024 SIMDs x 2.4 GHz x duration), an upper bound of the issue share: some VALU instructions
    issue in fewer cycles on this part (a VALU-bound kernel can exceed 1 by this count)."""
    if valu is None:
        return None
    s = avg_us * 1e-6
    flops = float(valu["fp32_ops_per_cell_launch_f32"]) * cells
    insts = float(valu["valu_insts_per_cell_launch_f32"]) * cells
    return {"bound": "alu", "achieved": flops / s / 1e12, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": flops / s / 1e12 / VALU_PEAK_TFLOPS, "peak_packed_fp32": VALU_PEAK_PACKED_TFLOPS,
            "issue_frac": insts * 4.0 / (1024 * 2.4e9 * s),
            "fp32_ops_per_launch": flops, "valu_insts_per_launch": insts}


def record_format(args):
    """Checkpoint record format of the FP32 paths: BF16 codes (the configured form) unless
    --ckpt i16 asks for the 16-bit fixed-point codes of the same size."""
    import paper_1511_06959_amd as adj

    return adj.CKPT_I16 if getattr(args, "ckpt", "bf16") == "i16" else adj.CKPT_BF16


def device_copy_gbs(mib=4096, reps=10):
    """Bytes read + written per second by a device-to-device copy of mib MiB (HIP events around
    reps copies after an untimed one): the streaming rate a kernel can reach on this device."""
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
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * (mib << 20) / (ms * 1e-3) / 1e9


def kernel_hash(family="stage"):
    """sha256 of a kernel family's sources ("stage": the stage kernels, "roe": the Roe flux
    kernels), as the committed counter summaries record it."""
    from paper_1511_06959_amd.profile_run import SOURCES
    h = hashlib.sha256()
    for name in SOURCES[family]:
        h.update(open(os.path.join(ROOT, "paper_1511_06959_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def _tile_report(res, g, lnu):
    """Autotuner result as bench fields: the selected tile, the tile the launches of this
    workload really use (lnu: a lambda term is applied) and the timed candidates (us; for the
    primal stage, per stage of a whole RK step)."""
    import paper_1511_06959_amd as adj

    name = lambda t: "x".join(map(str, adj.TILES[t]))
    out = {}
    for kc, key in ((adj.PROF_ADJOINT_STAGE, "adjoint_stage"), (adj.PROF_PRIMAL_STAGE, "primal_stage")):
        best, times = res[kc]
        out[key] = {"tile": name(best), "launched": name(adj.tile_launched(kc, g.precision, g.bc_x, lnu, best)),
                    "us": {name(t): round(ms * 1e3, 2) for t, ms in times.items()}}
    return out


def run_gpu(wl, precision, steps, warmup, tune=True, stages=False, ckpt_bf16=False, time_scheme=0, flux=0,
            nu_weight=None, rec_fmt=None):
    import torch

    import paper_1511_06959_amd as adj
    from paper_1511_06959_amd import autotune, sweep

    dt = torch.float64 if precision == adj.F64 else torch.float32
    # FP32 states are stored as deviations from the mean initial state (see adj_grid.w_ref)
    w_ref = adj.reference_state(wl.w0) if precision == adj.F32 else None
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, precision,
                      (rec_fmt or adj.CKPT_BF16) if ckpt_bf16 else adj.CKPT_NATIVE, w_ref, time_scheme=time_scheme,
                      flux=flux,
                      roe_delta=ROE_DELTA, w_far=wl.extra.get("w_far"), nu_weight=nu_weight)
    tiles = {}
    if tune:
        tiles = _tile_report(autotune.tune(g), g, wl.lam > 0.0)
    obj = adj.Objective.make(wl.obj_kind, wl.plane_i, wl.pt_ref)
    w0 = torch.from_numpy(g.to_stored(wl.w0)).to("cuda", dt)
    s = torch.from_numpy(wl.s).to("cuda", dt)
    ws = adj.workspace(g)
    traj = sweep.Trajectory(g, wl.nsteps, stages=stages)  # the schedule the graphs replay
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    gs = torch.zeros(5 * g.ncells, dtype=dt, device="cuda")
    out = {}
    cells = g.ncells

    def window():
        J.zero_()
        gs.zero_()
        sweep.forward(g, w0, s, wl.nsteps, obj, wl.weights, ws, traj=traj, J=J)
        wh0, _, _ = sweep.backward(g, traj, s, obj, wl.weights, wl.lam, ws, grad_s=gs)
        return wh0

    # (1) eager windows with every kernel launch bracketed by HIP events on its stream: the
    #     per-kernel durations of the roofline entry come from these timed windows
    adj.profile_enable(True)  # one profiled window grows the event pool before timing
    window()
    torch.cuda.synchronize()
    adj.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        window()
    torch.cuda.synchronize()
    out["eager_ms_per_step"] = (time.perf_counter() - t0) * 1e3 / steps
    adj.profile_enable(False)
    prof = {}
    for name, cls in (("adjoint_stage", adj.PROF_ADJOINT_STAGE), ("primal_stage", adj.PROF_PRIMAL_STAGE),
                      ("objective", adj.PROF_OBJECTIVE), ("sigma1", adj.PROF_SIGMA1), ("codec", adj.PROF_CODEC),
                      ("reduce", adj.PROF_REDUCE), ("roe_primal", adj.PROF_ROE_PRIMAL),
                      ("roe_adjoint", adj.PROF_ROE_ADJOINT), ("boundary", adj.PROF_BOUNDARY)):
        prof[name] = adj.profile_read(cls)
    del traj, ws
    torch.cuda.empty_cache()

    # (2) the same window captured as two HIP graphs and replayed: the throughput (value)
    cw = sweep.CapturedWindow(g, w0, s, wl.nsteps, obj, wl.weights, lam=wl.lam, stages=stages)
    for _ in range(warmup):
        cw.run()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    mids = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record()
        cw.run_forward()
        mids[k].record()
        cw.run_backward()
        ends[k].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd = sum(starts[k].elapsed_time(mids[k]) for k in range(steps)) / steps
    bwd = sum(mids[k].elapsed_time(ends[k]) for k in range(steps)) / steps
    out["ms_per_step"] = wall * 1e3 / steps
    out["fwd_ms"] = fwd
    out["bwd_ms"] = bwd
    out["value"] = cells * wl.nsteps / (out["ms_per_step"] / 1e3)
    out["adjoint_sweep_cell_steps_per_s"] = cells * wl.nsteps / (bwd / 1e3)
    out["primal_cell_steps_per_s"] = cells * wl.nsteps / (fwd / 1e3)
    out["prof"] = prof
    esz = 8 if precision == adj.F64 else 4
    ms, n = prof["adjoint_stage"]
    avg_s = ms / n / 1e3
    nst = 3 if time_scheme == 1 else 4
    # the per-unit figure (90 B / 200 B per adjoint cell-step) spread over the step's stage launches,
    # and beside it the values this store-all schedule's stage launches read and write
    alg_bytes = ALG_BYTES["adjoint"]["f64" if precision == adj.F64 else "f32"] / nst * cells
    sched_bytes = (VALUES_PER_STAGE_LAUNCH_RK3 if time_scheme == 1 else VALUES_PER_STAGE_LAUNCH) * esz * cells
    out["stage_avg_us"] = avg_s * 1e6
    out["stage_alg_bytes"] = alg_bytes
    out["stage_achieved_gbs"] = alg_bytes / avg_s / 1e9
    out["stage_schedule_bytes"] = sched_bytes
    out["stage_schedule_gbs"] = sched_bytes / avg_s / 1e9
    if flux == 1:
        # Roe flux kernels: the primal kernel reads W and updates out (15 values per cell), the
        # reverse kernel reads W, a, gnext and updates out (25 values per cell)
        out["roe"] = {}
        for name, vals in (("roe_primal", 15), ("roe_adjoint", 25)):
            ms_k, n_k = prof[name]
            us = ms_k / n_k * 1e3
            byts = vals * esz * cells
            out["roe"][name] = {"avg_launch_us": us, "alg_bytes_per_launch": byts,
                                "achieved_gbs": byts / us / 1e3, "frac_hbm": byts / us / 1e3 / HBM_PEAK_GBS}
    Jt, wh0, gs = cw.J, cw.wh0, cw.grad_s
    out["tiles"] = tiles
    out["J"] = float(Jt.cpu()[0])
    out["wh0"] = wh0.double().cpu().numpy()
    out["grad_s"] = gs.double().cpu().numpy()
    del cw
    torch.cuda.empty_cache()
    return out


def make_ensemble():
    """The batched-ensemble configuration: 64 periodic decaying-turbulence boxes, sizes drawn from
    {32, 48, 64, 96}^3, windows of 50-400 steps and lambda factors from {0, 0.03, 0.1, 0.3, 1}
    (seeded draws), Mach_rms 0.3, nu 0.0175; ordered by decreasing window for the batched sweep."""
    import workloads as W
    sizes, windows, lams = W.ensemble_draws()
    order = sorted(range(len(sizes)), key=lambda i: -windows[i])
    return [W.turbulence(sizes[i], mach_rms=0.3, nu=0.0175, seed=4 + i, nsteps=windows[i], lam_factor=lams[i])
            for i in order]


def run_ensemble(boxes, precision, steps, warmup, tune=True):
    import torch

    import paper_1511_06959_amd as adj
    from paper_1511_06959_amd import autotune
    from paper_1511_06959_amd.ensemble import CapturedEnsemble, EnsembleWindow

    refs = [adj.reference_state(wl.w0) if precision == adj.F32 else None for wl in boxes]
    grids = [adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, precision, w_ref=r)
             for wl, r in zip(boxes, refs)]
    tiles = {}
    if tune:
        # tile shapes tuned on the largest box; the ensemble launches use the same kernel bodies
        big = max(grids, key=lambda g: g.ncells)
        tiles = _tile_report(autotune.tune(big), big, any(wl.lam > 0.0 for wl in boxes))
        for v in tiles.values():
            v["tuned_on"] = "x".join(map(str, big.n))
    win = EnsembleWindow(grids, [wl.nsteps for wl in boxes], [g.to_stored(wl.w0) for g, wl in zip(grids, boxes)], None,
                         list(range(len(boxes))), [wl.lam for wl in boxes])
    out = {"tiles": tiles}
    adj.profile_enable(True)
    win.forward()
    win.backward()
    torch.cuda.synchronize()
    adj.profile_enable(True)
    t0 = time.perf_counter()
    win.forward()
    win.backward()
    torch.cuda.synchronize()
    out["eager_ms_per_step"] = (time.perf_counter() - t0) * 1e3
    adj.profile_enable(False)
    prof = {}
    for name, cls in (("adjoint_stage", adj.PROF_ADJOINT_STAGE), ("primal_stage", adj.PROF_PRIMAL_STAGE),
                      ("objective", adj.PROF_OBJECTIVE), ("sigma1", adj.PROF_SIGMA1), ("reduce", adj.PROF_REDUCE)):
        prof[name] = adj.profile_read(cls)
    print("[bench] ensemble eager window done", file=sys.stderr, flush=True)
    cap = CapturedEnsemble(win)
    for _ in range(warmup):
        cap.run()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    mids = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record()
        cap.run_forward()
        mids[k].record()
        cap.run_backward()
        ends[k].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cs = win.cell_steps()
    acs = win.adjoint_cell_steps()
    fwd = sum(starts[k].elapsed_time(mids[k]) for k in range(steps)) / steps
    bwd = sum(mids[k].elapsed_time(ends[k]) for k in range(steps)) / steps
    out["ms_per_step"] = wall * 1e3 / steps
    out["value"] = cs / (out["ms_per_step"] / 1e3)
    out["adjoint_sweep_cell_steps_per_s"] = acs / (bwd / 1e3)
    out["primal_cell_steps_per_s"] = cs / (fwd / 1e3)
    out["prof"] = prof
    esz = 8 if precision == adj.F64 else 4
    ms, n = prof["adjoint_stage"]
    # every reverse step launches the four stages over the members still running: the per-unit
    # figure per member cell-step, and beside it the values the stage launches read and write
    alg = ALG_BYTES["adjoint"]["f64" if precision == adj.F64 else "f32"] * acs
    out["stage_achieved_gbs"] = alg / (ms / 1e3) / 1e9
    out["stage_schedule_gbs"] = VALUES_PER_STAGE_LAUNCH * esz * 4 * acs / (ms / 1e3) / 1e9
    out["stage_avg_us"] = ms / n * 1e3
    out["stage_launches"] = n
    out["cells"] = win.ens.offset(0, win.nbox)
    out["cell_steps"] = cs
    out["trajectory_gb"] = sum(t.numel() for t in win.slots) * esz / 1e9
    out["J_mean"] = float(win.J.mean().cpu())
    del cap, win
    torch.cuda.empty_cache()
    return out


def cpu_baseline(wl, budget_s, flux=0):
    """The FP64 oracle as it stands, on the host cores: whole primal + reverse steps of the
    same 64^3 field, repeated until about budget_s seconds have been spent."""
    import oracle

    p = wl.params()
    p["flux"], p["roe_delta"] = flux, ROE_DELTA
    og = oracle.grid_from(p)
    obj = oracle.make_obj(wl.obj_kind)
    w = wl.w0
    a = np.random.default_rng(0).standard_normal(w.size) * 1e-3
    gs = np.zeros_like(w)
    nsteps = 0
    t_pr = t_ad = 0.0
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        wn = oracle.primal_step(og, w, wl.s)
        t1 = time.perf_counter()
        a = oracle.adjoint_step(og, w, wl.s, a, 0.0, obj, 1.0 / wl.nsteps, gs)
        t2 = time.perf_counter()
        t_pr += t1 - t0
        t_ad += t2 - t1
        w = wn
        nsteps += 1
        if time.perf_counter() - t_start >= budget_s:
            break
    cells = wl.ncells
    return {
        "value": cells * nsteps / (t_pr + t_ad),
        "unit": "cell-steps/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"{nsteps} primal RK4 step(s) + {nsteps} reverse step(s) of the 64^3 Taylor-Green field "
                   f"(FP64, OpenMP), {t_pr + t_ad:.1f} s; rate = cells x steps / (primal + reverse time), "
                   f"the same per-step definition as value"),
        "primal_cell_steps_per_s": cells * nsteps / t_pr,
        "adjoint_cell_steps_per_s": cells * nsteps / t_ad,
    }


# ---------------------------------------------------------------------------------------------
# The 384^3 case: a window reversed with binomial checkpointing
# ---------------------------------------------------------------------------------------------
def window_slots(K, ratio):
    """Largest slot count whose K-step binomial schedule advances at least `ratio` primal steps per
    time step (first sweep included), so that the sample window recomputes no less than the plan."""
    from paper_1511_06959_amd import revolve
    best = 1
    for s_ in range(1, K + 2):
        if (revolve.min_advances(K, s_) + 1) / K >= ratio - 1e-12:
            best = s_
    return best


def plan_for(g, plan_steps, budget_bytes):
    """Checkpointing plan of the plan_steps window within budget_bytes of HBM (sweep.plan_window)
    and the primal steps it advances per time step."""
    from paper_1511_06959_amd import revolve, sweep
    kind, size = sweep.plan_window(g, plan_steps, budget_bytes)
    rec = sweep.snapshot_bytes(g)
    if kind == "segments":
        return {"schedule": "segments", "segment": size, "snapshots": -(-plan_steps // size), "record_bytes": rec,
                "hbm_gb": sweep.segment_bytes(g, plan_steps, size) / 1e9, "advances_per_step": 2.0,
                "stage_recomputes_per_step": 0}
    adv = revolve.min_advances(plan_steps, size) + 1
    return {"schedule": "binomial", "slots": size, "record_bytes": rec, "hbm_gb": size * rec / 1e9,
            "advances": adv, "advances_per_step": adv / plan_steps, "stage_recomputes_per_step": 3}


PROF_CLASSES = (("adjoint_stage", 0), ("primal_stage", 1), ("sigma1", 2), ("objective", 3), ("codec", 4),
                ("reduce", 5))


def run_plan(wl, precision, K, warmup, tune=True, bf16=True, rec_fmt=None):
    """K-step window of the 384^3 plan on the GPU, in the schedule the plan picks for the free HBM
    (segments of the plan's length, or binomial slots that recompute no less per time step than
    the plan does): timed once, then run again with per-kernel event timing.  Returns timings,
    the plan, per-kernel durations and the results."""
    import torch

    import paper_1511_06959_amd as adj
    from paper_1511_06959_amd import autotune
    from paper_1511_06959_amd.sweep import RevolveSweep, SegmentSweep
    import workloads as W

    f32 = precision == adj.F32
    ref = adj.reference_state(wl.w0) if f32 else None
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, precision,
                      (rec_fmt or adj.CKPT_BF16) if (f32 and bf16) else adj.CKPT_NATIVE, ref)
    tiles = _tile_report(autotune.tune(g), g, wl.lam > 0.0) if tune else {}
    obj = adj.Objective.make(wl.obj_kind)
    w0 = torch.from_numpy(g.to_stored(wl.w0)).to("cuda", g.dtype)
    ws = adj.workspace(g)
    torch.cuda.synchronize()
    import gc
    gc.collect()
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    held = torch.cuda.memory_allocated()
    print(f"[bench] {'f64' if precision == adj.F64 else 'f32'}: {free / 1e9:.1f} GB free of {total / 1e9:.1f}, torch "
          f"holds {held / 1e9:.1f} GB", file=sys.stderr, flush=True)
    # the plan of a process that runs this window alone: the device's memory less what this one
    # holds (grid, workspace), the window's working states and adjoints, and a margin for the
    # runtime (an earlier window of this process may leave memory that the runtime has not returned)
    plan = plan_for(g, PLAN_STEPS, max(0, total - held - 6 * 5 * g.ncells * g.dtype.itemsize - (6 << 30)))

    def sweep_of(steps, wts):
        if plan["schedule"] == "segments":
            return SegmentSweep(g, steps, min(steps, plan["segment"]), None, obj, wts, wl.lam, ws)
        return RevolveSweep(g, steps, window_slots(steps, plan["advances_per_step"]), None, obj, wts, wl.lam, ws)

    def window(steps):
        sw = sweep_of(steps, W.window_weights(steps, 1, steps))
        J = sw.forward(w0)
        wh0, gs = sw.backward()
        return sw, J, wh0, gs

    out = {"plan": plan, "tiles": tiles}
    if warmup > 0:
        window(warmup)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    sw, J, wh0, gs = window(K)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    out["window"] = ({"schedule": "segments", "segment": sw.seg, "snapshots": sw.nsnap} if plan["schedule"] == "segments"
                     else {"schedule": "binomial", "slots": sw.slots})
    out["ms_per_step"] = sec * 1e3 / K
    out["value"] = g.ncells * K / sec
    out["advances"] = sw.advanced
    out["J"] = float(J.cpu()[0])
    out["wh0"] = wh0.double().cpu().numpy()
    out["grad_s"] = gs.double().cpu().numpy()
    del sw, wh0, gs
    torch.cuda.empty_cache()
    # the same window with every launch timed by its own dispatch events
    adj.profile_enable(True)
    window(K)
    torch.cuda.synchronize()
    adj.profile_enable(False)
    out["prof"] = {name: adj.profile_read(cls) for name, cls in PROF_CLASSES}
    out["cells"] = g.ncells
    del ws
    torch.cuda.empty_cache()
    return out


def with_traffic(roof, name, khash, tile, cells):
    """Adds to a 384^3 kernel roofline entry the HBM bytes per launch that the committed counter
    summary profiles/traffic_<name>_turb384.txt gives (null when it was taken on other kernel
    sources or another tile), and those bytes over the live launch duration: the HBM rate the
    kernel really draws."""
    t = profile_values(f"traffic_{name}_turb384.txt", khash, tile)
    roof["traffic"] = None if t is None else float(t["bytes_per_cell_launch_f32"]) * cells
    roof["traffic_profile"] = None if t is None else "profiles/" + t["profile"]
    roof["traffic_gbs"] = None if t is None else roof["traffic"] / (roof["avg_launch_us"] * 1e-6) / 1e9
    roof["traffic_frac"] = None if t is None else roof["traffic_gbs"] / HBM_PEAK_GBS
    return roof


def kernel_roofline(kind, prec, cells, ms, n):
    """HBM roofline of one stage-kernel class: algorithmic bytes per launch (a quarter of the
    per-cell-step bytes, times the cells) / mean launch duration."""
    avg_s = ms / n / 1e3
    alg = ALG_BYTES[kind][prec] / 4.0 * cells
    return {"bound": "hbm", "achieved": alg / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": alg / avg_s / 1e9 / HBM_PEAK_GBS, "avg_launch_us": avg_s * 1e6, "launches": n,
            "alg_bytes_per_launch": alg, "alg_bytes_per_cell_step": ALG_BYTES[kind][prec]}


def c1_vs_oracle():
    """The 16^3 Taylor-Green window (50 steps, mean pressure over steps 26..50) of every path on
    the GPU against the FP64 oracle's window: relative errors of J, dJ/dw_0 and dJ/ds."""
    import torch

    import oracle
    import paper_1511_06959_amd as adj
    from paper_1511_06959_amd import sweep
    from paper_1511_06959_amd.sweep import RevolveSweep, SegmentSweep
    import workloads as W

    wl = W.tgv_small()
    og = oracle.grid_from(wl.params())
    oobj = oracle.make_obj(wl.obj_kind)
    traj = oracle.primal_window(og, wl.w0, wl.s, wl.nsteps)
    J = oracle.objective_window(og, oobj, traj, wl.weights)
    wh0, gs = oracle.adjoint_window(og, oobj, traj, wl.s, wl.weights)
    ref = adj.reference_state(wl.w0)
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    out = {}
    # slots: None store-all, an int binomial slots, ("seg", L) two-level segments of L steps (the
    # benchmark's own schedule)
    for name, prec, ck, slots in (("f64", adj.F64, adj.CKPT_NATIVE, None), ("f32", adj.F32, adj.CKPT_NATIVE, None),
                                  ("f32_bf16_records", adj.F32, adj.CKPT_BF16, None),
                                  ("f32_bf16_revolve_4_slots", adj.F32, adj.CKPT_BF16, 4),
                                  ("f32_bf16_segments_10", adj.F32, adj.CKPT_BF16, ("seg", 10)),
                                  ("f32_i16_segments_10", adj.F32, adj.CKPT_I16, ("seg", 10)),
                                  ("f64_segments_10", adj.F64, adj.CKPT_NATIVE, ("seg", 10))):
        g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, prec, ck,
                          ref if prec == adj.F32 else None)
        obj = adj.Objective.make(wl.obj_kind)
        ws = adj.workspace(g)
        w0 = torch.from_numpy(g.to_stored(wl.w0)).to("cuda", g.dtype)
        s = torch.from_numpy(wl.s).to("cuda", g.dtype)
        if slots is None:
            tr, _, Jg = sweep.forward(g, w0, s, wl.nsteps, obj, wl.weights, ws)
            whg, gsg, _ = sweep.backward(g, tr, s, obj, wl.weights, 0.0, ws)
        else:
            if isinstance(slots, tuple):
                sw = SegmentSweep(g, wl.nsteps, slots[1], s, obj, wl.weights, 0.0, ws)
            else:
                sw = RevolveSweep(g, wl.nsteps, slots, s, obj, wl.weights, 0.0, ws)
            Jg = sw.forward(w0)
            whg, gsg = sw.backward()
        out[name] = {"J": abs(float(Jg.cpu()[0]) - J) / abs(J), "dJ_dw0": rel(whg.double().cpu().numpy(), wh0),
                     "dJ_ds": rel(gsg.double().cpu().numpy(), gs)}
    out["workload"] = ("Taylor-Green vortex 16^3, Mach 0.3, Re 100, 50 RK4 steps, mean pressure averaged over "
                       "steps 26..50, lambda 0; GPU windows against the FP64 oracle's")
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline_block(wl, n, budget_s, threads=None):
    """The FP64 oracle as it stands on the host cores: primal + reverse steps (lambda and objective
    of the workload) of an n^3 block cut from the workload's initial field and treated as periodic,
    with its cell size, viscosity and dt, repeated for about budget_s seconds.  threads: OpenMP
    threads (None: all)."""
    import oracle

    N = wl.n
    w = wl.w0.reshape(5, N[2], N[1], N[0])[:, :n, :n, :n].copy().reshape(-1)
    p = wl.params()
    p["n"] = (n, n, n)
    p["L"] = tuple(wl.L[d] / wl.n[d] * n for d in range(3))
    og = oracle.grid_from(p)
    obj = oracle.make_obj(wl.obj_kind)
    prev = oracle.num_threads()
    if threads is not None:
        oracle.set_num_threads(threads)
    used = oracle.num_threads()
    a = np.random.default_rng(0).standard_normal(w.size) * 1e-3
    gs = np.zeros_like(w)
    steps, t_pr, t_ad = 0, 0.0, 0.0
    t_start = time.perf_counter()
    try:
        while True:
            t0 = time.perf_counter()
            wn = oracle.primal_step(og, w)
            t1 = time.perf_counter()
            a = oracle.adjoint_step(og, w, None, a, wl.lam, obj, 1.0 / PLAN_STEPS, gs)
            t2 = time.perf_counter()
            t_pr += t1 - t0
            t_ad += t2 - t1
            w = wn
            steps += 1
            if time.perf_counter() - t_start >= budget_s:
                break
    finally:
        oracle.set_num_threads(prev)
    cells = n ** 3
    return {"value": cells * steps / (t_pr + t_ad), "threads": used, "steps": steps, "seconds": t_pr + t_ad,
            "primal_cell_steps_per_s": cells * steps / t_pr, "adjoint_cell_steps_per_s": cells * steps / t_ad}


def schedule_ceiling(r, cells, khash, copy_gbs, K):
    """The schedule's own ceiling: HBM bytes one time step of the plan moves per cell (the stage
    kernels' counter summaries: four reverse-stage launches, four primal-stage launches per
    primal step and the stage recomputations of binomial plans; sigma_1 at its 24 algorithmic
    bytes), and the cell-steps/s that 8 TB/s and the
    device's copy rate would allow at that traffic.  None when a summary was taken on other
    kernel sources or tiles."""
    per = {}
    for name in ("adjoint_stage", "primal_stage"):
        tile = r["tiles"].get(name, {}).get("launched")
        t = profile_values(f"traffic_{name}_turb384.txt", khash, tile)
        if t is None:
            return None
        per[name] = float(t["bytes_per_cell_launch_f32"])
    prim = r["advances"] / K
    # binomial plans also evaluate three stage states inside every reverse step
    rec = r["plan"].get("stage_recomputes_per_step", 0)
    b = 4 * per["adjoint_stage"] + (4 * prim + rec) * per["primal_stage"] + 24.0
    return {"bytes_per_cell_step": b, "reverse_stage_bytes_per_cell_launch": per["adjoint_stage"],
            "primal_stage_bytes_per_cell_launch": per["primal_stage"], "primal_steps_per_time_step": prim,
            "ceiling_at_8tbs": HBM_PEAK_GBS * 1e9 / b, "ceiling_at_copy_rate": copy_gbs * 1e9 / b,
            "value_over_copy_ceiling": r["value"] / (copy_gbs * 1e9 / b)}


def schedule_text(r, K):
    p, w = r["plan"], r["window"]
    if p["schedule"] == "segments":
        return (f"two-level checkpointing: the {PLAN_STEPS}-step plan keeps {p['snapshots']} snapshots, one every "
                f"{p['segment']} steps, and re-advances one segment at a time with its stage states kept "
                f"({p['hbm_gb']:.0f} GB of HBM): 2 primal steps and no stage recomputation per time step; the timed "
                f"{K}-step window is one segment ({w['snapshots']} snapshot) of the same schedule")
    return (f"binomial checkpointing: the {PLAN_STEPS}-step plan fits {p['slots']} snapshot slots ({p['hbm_gb']:.0f} "
            f"GB) and advances {p['advances_per_step']:.3f} primal steps per time step, plus 3 stage evaluations in "
            f"each reverse step; the timed {K}-step window uses {w['slots']} slots and advances "
            f"{r['advances'] / K:.3f}")


def main_c5(args):
    if args.fl or args.ts or args.nw:
        raise SystemExit("--flux, --time-scheme and --nu-weight apply to the store-all window workloads (tgv64, "
                         "turb384_sample, wake, spatial_wake); the 384^3 plan runs the configured RK4 split-flux case")
    import torch

    import paper_1511_06959_amd as adj
    import workloads as W

    K, Wm = args.steps, args.warmup
    print("[bench] generating the 384^3 turbulence field", file=sys.stderr, flush=True)
    wl = W.turb_384(nsteps=PLAN_STEPS, lam_factor=0.1)
    print(f"[bench] workload {wl.name}: {wl.n} cells, plan {PLAN_STEPS} steps, dt {wl.dt:.4e}, lambda {wl.lam:.3e}",
          file=sys.stderr, flush=True)
    copy_gbs = device_copy_gbs()
    r32 = run_plan(wl, adj.F32, K, Wm, not args.no_autotune, bf16=True, rec_fmt=record_format(args))
    print(f"[bench] f32/bf16 window {r32['ms_per_step']:.2f} ms per step, window {r32['window']}, plan "
          f"{r32['plan']}", file=sys.stderr, flush=True)
    r64 = None
    if not args.no_f64:
        r64 = run_plan(wl, adj.F64, K, Wm, not args.no_autotune)
        print(f"[bench] f64 window {r64['ms_per_step']:.2f} ms per step", file=sys.stderr, flush=True)
    cells = wl.ncells

    def rooflines(r, prec):
        out = {}
        for name, kind in (("adjoint_stage", "adjoint"), ("primal_stage", "primal")):
            ms, n = r["prof"][name]
            out[name] = kernel_roofline(kind, prec, cells, ms, n)
        return out

    roofs = rooflines(r32, "f32")
    dom = max(("adjoint_stage", "primal_stage"), key=lambda k: r32["prof"][k][0])
    kname = {"adjoint_stage": "k_adjoint_stage", "primal_stage": "k_primal_stage"}[dom]
    khash = kernel_hash()
    tile = r32["tiles"].get(dom, {}).get("launched")
    valu = profile_values(f"valu_{dom}_turb384.txt", khash, tile)
    for name in roofs:
        with_traffic(roofs[name], name, khash, r32["tiles"].get(name, {}).get("launched"), cells)
    roof = dict(roofs[dom])
    roof["kernel"] = kname
    roof["device_copy_gbs"] = copy_gbs
    roof_valu = valu_roofline(valu, cells, roof["avg_launch_us"])
    if roof_valu is not None:
        roof_valu["profile"] = "profiles/" + valu["profile"]
        roof_valu["kernel"] = kname
    kms = {k: v[0] / K for k, v in r32["prof"].items()}
    line = {
        "metric": METRIC,
        "value": r32["value"],
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS["turb384"],
            "cells": cells,
            "plan_steps": PLAN_STEPS,
            "dt": wl.dt,
            "lambda": wl.lam,
            "step": "one time step of the plan: its primal steps (the forward step with snapshot encoding and "
                    "the re-advance of the segment, or its share of the binomial recomputation) with the objective "
                    "folded in, and the reverse step (sigma_1, four transposed stages with the objective's "
                    "injection, body-force gradient; with binomial plans also the decode and stage recomputation)",
            "schedule": schedule_text(r32, K),
            "plan": r32["plan"],
            "window": r32["window"],
            "checkpoints": ("BF16" if args.ckpt == "bf16" else "16-bit fixed-point") + " snapshot records (per "
                           "4x4x4 block and variable a least-squares plane and the 16-bit code of the residual); the "
                           "segment being reversed in native FP32 states and stage states",
            "source": "body force s = 0 (the base of the gradient), so primal stages skip reading it",
        },
        "roofline": roof,
        "roofline_valu": roof_valu,
        "roofline_by_kernel": roofs,
        "hbm_per_time_step": {"alg_bytes_per_cell_step": ALG_BYTES["adjoint"]["f32"] + ALG_BYTES["primal"]["f32"],
                              "achieved": (ALG_BYTES["adjoint"]["f32"] + ALG_BYTES["primal"]["f32"]) * r32["value"] / 1e9,
                              "unit": "GB/s",
                              "frac": (ALG_BYTES["adjoint"]["f32"] + ALG_BYTES["primal"]["f32"]) * r32["value"] / 1e9
                              / HBM_PEAK_GBS},
        "schedule_ceiling": schedule_ceiling(r32, cells, khash, copy_gbs, K),
        "kernel_ms_per_step": kms,
        "primal_steps_per_time_step": r32["advances"] / K,
        "launch": "eager launches on one stream (each 384^3 launch runs for milliseconds)",
        "tiles": r32["tiles"],
    }
    if r64 is not None:
        r64roofs = rooflines(r64, "f64")
        line["f64"] = {"value": r64["value"], "ms_per_step": r64["ms_per_step"], "plan": r64["plan"],
                       "window": r64["window"], "schedule": schedule_text(r64, K),
                       "primal_steps_per_time_step": r64["advances"] / K,
                       "roofline_by_kernel": r64roofs, "kernel_ms_per_step": {k: v[0] / K for k, v in r64["prof"].items()},
                       "tiles": r64["tiles"]}
        line["f32_speedup_over_f64"] = r32["value"] / r64["value"]
        rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
        line["rel_err_f32_bf16_vs_gpu_f64"] = {
            "J": abs(r32["J"] - r64["J"]) / abs(r64["J"]), "dJ_dw0": rel(r32["wh0"], r64["wh0"]),
            "dJ_ds": rel(r32["grad_s"], r64["grad_s"]),
            "note": f"the timed {K}-step 384^3 window, lambda 0.1 dx^2 sigma_1; the FP64 path is pinned to the FP64 "
                    "oracle (rel_err_vs_oracle and the test suite), which cannot run 384^3 windows"}
    if not args.no_cpu_baseline:
        line["cpu_baseline"], line["rel_err_vs_oracle"] = cpu_baseline_leg(wl, args.cpu_seconds)
    print(json.dumps(line), flush=True)


def cpu_baseline_leg(wl, seconds):
    """The oracle's leg of the benchmark (the only part of it that runs the oracle): the oracle's
    own rate on the host cores, all of them and one, and the 16^3 windows of every GPU path
    checked against the oracle's window."""
    print("[bench] 16^3 windows against the oracle", file=sys.stderr, flush=True)
    rel = c1_vs_oracle()
    print("[bench] oracle on the host cores", file=sys.stderr, flush=True)
    allc = cpu_baseline_block(wl, 48, seconds)
    one = cpu_baseline_block(wl, 24, seconds / 2, threads=1)
    cpu = {
        "value": allc["value"], "unit": "cell-steps/s", "cores": allc["threads"], "kind": "oracle",
        "sample": (f"{allc['steps']} primal + {allc['steps']} reverse FP64 steps (lambda 0.1 dx^2 sigma_1, mean "
                   f"pressure) of a 48^3 block cut from the 384^3 field, periodic, {allc['seconds']:.1f} s on "
                   f"{allc['threads']} OpenMP threads; rate = cells x steps / (primal + reverse time), no "
                   "checkpointing recomputation"),
        "cpu_model": cpu_model(),
        "primal_cell_steps_per_s": allc["primal_cell_steps_per_s"],
        "adjoint_cell_steps_per_s": allc["adjoint_cell_steps_per_s"],
        "single_thread": {"value": one["value"], "threads": 1, "steps": one["steps"],
                          "sample": f"24^3 block, {one['steps']} primal + reverse steps, {one['seconds']:.1f} s",
                          "primal_cell_steps_per_s": one["primal_cell_steps_per_s"],
                          "adjoint_cell_steps_per_s": one["adjoint_cell_steps_per_s"]},
    }
    return cpu, rel


def _oracle_rates(og, obj, w, lam, cn, steps, best_of=3, threads=None):
    """The oracle's own rates on a state w: after one untimed primal and reverse step, best_of
    timings of `steps` primal steps (advancing the state) and `steps` reverse steps (each
    recomputing its stage states, with the objective's injection and lambda)."""
    import oracle

    prev = oracle.num_threads()
    if threads is not None:
        oracle.set_num_threads(threads)
    used = oracle.num_threads()
    cells = w.size // 5
    a = np.random.default_rng(0).standard_normal(w.size) * 1e-3
    gs = np.zeros_like(w)
    best_p = best_a = 0.0
    try:
        w1 = oracle.primal_step(og, w)
        oracle.adjoint_step(og, w, None, a, lam, obj, cn, gs)
        for _ in range(best_of):
            wc = w1
            t0 = time.perf_counter()
            for _ in range(steps):
                wc = oracle.primal_step(og, wc)
            t1 = time.perf_counter()
            for _ in range(steps):
                oracle.adjoint_step(og, w1, None, a, lam, obj, cn, gs)
            t2 = time.perf_counter()
            best_p = max(best_p, cells * steps / (t1 - t0))
            best_a = max(best_a, cells * steps / (t2 - t1))
    finally:
        oracle.set_num_threads(prev)
    return {"threads": used, "steps": steps, "best_of": best_of, "primal_cell_steps_per_s": best_p,
            "adjoint_cell_steps_per_s": best_a, "cell_steps_per_s": 1.0 / (1.0 / best_p + 1.0 / best_a)}


def _block(wl, lo, n, bc_x=None):
    """Block of n cells at lo cut from a workload's initial field, with its cell size, viscosity and
    dt (periodic in y and z; x as given)."""
    import oracle

    N = wl.n
    if any(lo[d] < 0 or lo[d] + n[d] > N[d] for d in range(3)):
        raise ValueError(f"block at {lo} of {n} cells does not fit the {N} grid")
    w = wl.w0.reshape(5, N[2], N[1], N[0])[:, lo[2]:lo[2] + n[2], lo[1]:lo[1] + n[1], lo[0]:lo[0] + n[0]]
    p = wl.params()
    p["n"] = tuple(n)
    p["L"] = tuple(wl.L[d] / wl.n[d] * n[d] for d in range(3))
    if bc_x is not None:
        p["bc_x"] = bc_x
    return oracle.grid_from(p), np.ascontiguousarray(w).reshape(-1)


def main_cpu_baseline(args):
    """The FP64 oracle timed on the host cores for every configuration (nothing runs on the GPU):
    per-cell-step rates of the primal step and of the reverse step (stage recomputation included),
    with lambda = 0 and lambda = 0.1 dx^2 sigma_1, best of three after a warm-up step, on all cores
    and (for the 16^3 window and a 24^3 block) on one.  Large configurations run slices: a few steps,
    or a block cut from the field with the configuration's cell size; only rates are reported."""
    import oracle
    import workloads as W

    rows = []

    def row(name, sample, og, obj, w, lam, cn, steps, threads=None):
        t0 = time.perf_counter()
        r = _oracle_rates(og, obj, w, lam, cn, steps, threads=threads)
        r.update({"config": name, "sample": sample, "lambda": lam, "cells": w.size // 5,
                  "wall_s": time.perf_counter() - t0})
        print(f"[cpu] {name} {sample} lambda {lam:.3g} threads {r['threads']}: primal "
              f"{r['primal_cell_steps_per_s']:.3e}, reverse {r['adjoint_cell_steps_per_s']:.3e} cell-steps/s "
              f"({r['wall_s']:.1f} s)", file=sys.stderr, flush=True)
        rows.append(r)

    # 16^3 Taylor-Green window (50 + 50 steps) in full, all cores and one
    wl = W.tgv_small()
    og = oracle.grid_from(wl.params())
    obj = oracle.make_obj(wl.obj_kind)
    for threads in (None, 1):
        prev = oracle.num_threads()
        if threads:
            oracle.set_num_threads(threads)
        try:
            oracle.primal_window(og, wl.w0, wl.s, 2)
            best = None
            for _ in range(3):
                t0 = time.perf_counter()
                traj = oracle.primal_window(og, wl.w0, wl.s, wl.nsteps)
                t1 = time.perf_counter()
                oracle.adjoint_window(og, obj, traj, wl.s, wl.weights)
                t2 = time.perf_counter()
                best = (t1 - t0, t2 - t1) if best is None else (min(best[0], t1 - t0), min(best[1], t2 - t1))
            used = oracle.num_threads()
        finally:
            oracle.set_num_threads(prev)
        cs = wl.ncells * wl.nsteps
        rows.append({"config": "tgv16", "sample": f"the whole {wl.nsteps}-step window (forward, then reverse)",
                     "lambda": 0.0, "cells": wl.ncells, "threads": used, "steps": wl.nsteps, "best_of": 3,
                     "primal_cell_steps_per_s": cs / best[0], "adjoint_cell_steps_per_s": cs / best[1],
                     "cell_steps_per_s": cs / (best[0] + best[1])})
        print(f"[cpu] tgv16 window threads {used}: {cs / (best[0] + best[1]):.3e} cell-steps/s", file=sys.stderr,
              flush=True)
    # 64^3 Taylor-Green (dissipation objective): two-step slice of the 1000-step window
    wl = W.tgv_64()
    og = oracle.grid_from(wl.params())
    obj = oracle.make_obj(wl.obj_kind)
    dx = wl.L[0] / wl.n[0]
    for lf in (0.0, 0.1):
        row("tgv64", "2-step slice", og, obj, wl.w0, lf * dx * dx, 1.0 / wl.nsteps, 2)
    # the wake: a 128 x 64 x 32 block around the shear layer, slip walls at its x ends
    wl = W.wake(nsteps=4000)
    og, w = _block(wl, (192, 0, 0), (128, 64, 32), bc_x=1)
    obj = oracle.make_obj(wl.obj_kind, 96, wl.pt_ref)
    dx = wl.L[0] / wl.n[0]
    for lf in (0.0, 0.1):
        row("wake", "128x64x32 block from the centre of the 512x256x32 field, 2 steps", og, obj, w, lf * dx * dx,
            1.0 / wl.nsteps, 2)
    del wl, w
    # 384^3 decaying turbulence: 48^3 block (all cores) and 24^3 block (one core)
    wl = W.turb_384()
    dx = wl.L[0] / wl.n[0]
    for n, threads in ((48, None), (24, 1)):
        og, w = _block(wl, (0, 0, 0), (n, n, n))
        obj = oracle.make_obj(wl.obj_kind)
        for lf in (0.0, 0.1):
            row("turb384", f"{n}^3 block of the 384^3 field, {2 if n == 48 else 1} steps", og, obj, w, lf * dx * dx,
                1.0 / PLAN_STEPS, 2 if n == 48 else 1, threads=threads)
    del wl
    # the ensemble's box sizes, one box of each
    for n in (32, 48, 64, 96):
        wl = W.turbulence(n, mach_rms=0.3, nu=0.0175, seed=4, nsteps=2)
        og = oracle.grid_from(wl.params())
        obj = oracle.make_obj(wl.obj_kind)
        dx = wl.L[0] / n
        for lf in (0.0, 0.1):
            row(f"ensemble_box{n}", f"{n}^3 box, 1 step", og, obj, wl.w0, lf * dx * dx, 0.01, 1)
    print(json.dumps({"kind": "oracle_cpu_baseline", "unit": "cell-steps/s", "cpu_model": cpu_model(),
                      "host_cpus": os.cpu_count(), "all_core_threads": max(r["threads"] for r in rows),
                      "rows": rows}), flush=True)


# ---------------------------------------------------------------------------------------------
# The configured windows, run once: the 5000-step 384^3 gradient with finite-difference checks,
# and the 4000-step wake with a lambda sweep over one BF16 trajectory
# ---------------------------------------------------------------------------------------------
def _direction(n5, seed):
    """Seeded N(0, 1) direction of the body force (torch's device generator, FP64)."""
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(int(seed))
    return torch.randn(n5, dtype=torch.float64, device="cuda", generator=gen)


def main_c5_window(args):
    """--parts f32_lam,f32_lam0,f64_lam0: autograd gradients of the whole window (dJ/ds at s = 0,
    checkpointing sized to the free HBM) and their products with the seeded directions;
    --parts fd: central differences of J along the directions (FP64 primal, --fd-eps)."""
    import torch

    import paper_1511_06959_amd as adj
    from paper_1511_06959_amd.autograd import CheckpointedWindow, WindowSpec
    import workloads as W

    T = args.window or PLAN_STEPS
    seeds = [int(x) for x in args.fd_seeds.split(",")]
    print("[window] generating the 384^3 turbulence field", file=sys.stderr, flush=True)
    wl = W.turb_384(nsteps=T, lam_factor=0.1)
    obj = adj.Objective.make(wl.obj_kind)
    out = {"workload": f"decaying turbulence 384^3 (Mach_rms 0.4, nu 2.887e-3), {T} RK4 steps, dt {wl.dt:.6g}, "
                       "time-averaged mean pressure over steps 1..T, gradient wrt the body force at s = 0",
           "steps": T, "dt": wl.dt, "lambda_0.1": wl.lam, "directions": seeds, "parts": {}}
    n5 = 5 * wl.ncells
    for part in args.parts.split(","):
        t0 = time.perf_counter()
        if part == "fd":
            g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, adj.F64)
            ws = adj.workspace(g)
            w0 = torch.from_numpy(wl.w0).to("cuda")
            cur, nxt = torch.empty_like(w0), torch.empty_like(w0)
            J = torch.zeros(1, dtype=torch.float64, device="cuda")
            eps = args.fd_eps
            res = {}
            for seed in seeds:
                d = _direction(n5, seed)
                vals = []
                for sign in (1.0, -1.0):
                    s = sign * eps * d
                    J.zero_()
                    cur.copy_(w0)
                    for n in range(T):
                        adj.primal_step(g, cur, s, nxt, ws)
                        adj.objective_and_grad(g, obj, nxt, ws, weight=float(wl.weights[n + 1]), J_accum=J)
                        cur, nxt = nxt, cur
                        if (n + 1) % 1000 == 0:
                            print(f"[window] fd seed {seed} sign {sign:+.0f}: step {n + 1}", file=sys.stderr,
                                  flush=True)
                    vals.append(float(J.cpu()[0]))
                    del s
                res[str(seed)] = {"J_plus": vals[0], "J_minus": vals[1], "fd": (vals[0] - vals[1]) / (2 * eps)}
                del d
                torch.cuda.empty_cache()
            out["parts"]["fd"] = {"eps": eps, "primal": "FP64", "values": res, "seconds": time.perf_counter() - t0}
            print(json.dumps({"part": "fd", **out["parts"]["fd"]}), flush=True)
            continue
        prec = adj.F64 if part.startswith("f64") else adj.F32
        lam = wl.lam if part.endswith("_lam") else 0.0
        ref = adj.reference_state(wl.w0) if prec == adj.F32 else None
        g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, prec,
                          record_format(args) if prec == adj.F32 else adj.CKPT_NATIVE, ref)
        if not args.no_autotune:
            from paper_1511_06959_amd import autotune
            autotune.tune(g)
        last = [time.perf_counter()]

        def progress(n):
            if time.perf_counter() - last[0] > 30.0:
                last[0] = time.perf_counter()
                print(f"[window] {part}: reverse step {n}", file=sys.stderr, flush=True)

        spec = WindowSpec(g, T, obj, list(wl.weights), lam=lam, energy_every=50 if prec == adj.F32 else 0,
                          progress=progress)
        w0 = torch.from_numpy(g.to_stored(wl.w0)).to("cuda", g.dtype)
        st = torch.zeros(n5, dtype=g.dtype, device="cuda", requires_grad=True)
        print(f"[window] {part}: forward sweep", file=sys.stderr, flush=True)
        J = CheckpointedWindow.apply(w0, st, spec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        print(f"[window] {part}: J = {float(J.detach()):.12g} after {t1 - t0:.1f} s; reverse sweep", file=sys.stderr,
              flush=True)
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        grad = st.grad.double()
        dots = {str(seed): float(torch.dot(grad, _direction(n5, seed))) for seed in seeds}
        rec = {"J": float(J.detach()), "grad_norm": float(grad.norm()), "dots": dots, "plan": dict(spec.last),
               "forward_s": t1 - t0, "reverse_s": t2 - t1,
               "cell_steps_per_s": wl.ncells * T / (t2 - t0), "lambda": lam,
               "precision": "FP32 stencils, BF16 snapshots, FP64 reductions" if prec == adj.F32 else "FP64"}
        rec["plan"].pop("energy", None)
        if spec.last.get("energy"):
            rec["energy"] = spec.last["energy"]
        out["parts"][part] = rec
        print(json.dumps({"part": part, **rec}), flush=True)
        print(f"[window] {part}: done in {t2 - t0:.1f} s", file=sys.stderr, flush=True)
        del st, grad, w0, spec, J
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def main_wake_lambda(args):
    """The 4000-step wake: forward sweep storing BF16 records of every state, then one reverse
    sweep for lambda = (0, 0.1, 1) dx^2 sigma_1 at once over that trajectory, with the adjoint
    energy of every member after every reverse step."""
    import torch

    import paper_1511_06959_amd as adj
    from paper_1511_06959_amd import autotune, sweep
    from paper_1511_06959_amd.ensemble import LambdaSweep
    import workloads as W

    T = args.window or 4000
    wl = W.wake(nsteps=T)
    dx = min(wl.L[d] / wl.n[d] for d in range(3))
    factors = [0.0, 0.1, 1.0]
    lams = [f * dx * dx for f in factors]
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, adj.F32, record_format(args),
                      adj.reference_state(wl.w0))
    if not args.no_autotune:
        autotune.tune(g)
    obj = adj.Objective.make(wl.obj_kind, wl.plane_i, wl.pt_ref)
    ws = adj.workspace(g)
    s = torch.zeros(5 * wl.ncells, dtype=torch.float32, device="cuda")
    print(f"[wake] {wl.n}, {T} steps, dt {wl.dt:.4e}; forward sweep", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    traj, _, J = sweep.forward(g, torch.from_numpy(g.to_stored(wl.w0)).to("cuda", torch.float32), s, T, obj,
                               wl.weights, ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"[wake] J = {float(J.cpu()[0]):.10g} after {t1 - t0:.1f} s; lambda sweep", file=sys.stderr, flush=True)
    ls = LambdaSweep(g, traj, lams, obj, wl.weights, s=s, energy=True)
    last = [time.perf_counter()]

    def progress(n):
        if n % 500 == 0:
            print(f"[wake] reverse step {n}", file=sys.stderr, flush=True)

    wh, gs = ls.backward(progress=progress)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    E = ls.E.cpu().numpy()
    from paper_1511_06959_amd import lamest
    members = []
    g0 = ls.member(gs, 0).double()
    for m, f in enumerate(factors):
        gm = ls.member(gs, m).double()
        wm = ls.member(wh, m).double()
        members.append({"lambda_factor": f, "lambda": lams[m], "grad_s_norm": float(gm.norm()),
                        "w0_adjoint_norm": float(wm.norm()),
                        "grad_s_rel_dev_from_lambda0": float((gm - g0).norm() / g0.norm()),
                        "energy_growth_rate": lamest.growth_rate(E[:, m], wl.dt),
                        "energy_first_last": [float(E[0, m]), float(E[T, m])],
                        "energy_every_500": [float(E[n, m]) for n in range(0, T + 1, 500)]})
    traj_gb = traj.store.numel() / 1e9
    out = {"workload": "temporally developing wake 512x256x32 (slip walls in x, free stream Mach 0.85, centre 0.5, "
                       f"Re 5e4), {T} RK4 steps, stagnation-pressure loss on the face x = 0.75 L_x, BF16 records of "
                       "every state, one reverse sweep for lambda = (0, 0.1, 1) dx^2 sigma_1 at once",
           "steps": T, "J": float(J.cpu()[0]), "trajectory_gb": traj_gb, "forward_s": t1 - t0, "reverse_s": t2 - t1,
           "member_cell_steps_per_s": wl.ncells * T * len(lams) / (t2 - t1), "members": members}
    print(json.dumps(out), flush=True)


WORKLOADS = {
    "tgv64": "Taylor-Green vortex 64^3 periodic, Mach 0.1, Re 1600, {n} RK4 steps forward + full adjoint sweep, "
             "lambda 0, objective time-averaged viscous dissipation, gradient wrt a 5x64^3 body force",
    "turb384": "decaying turbulence 384^3 periodic (k^4 exp(-2k^2/k0^2), k0 4, Mach_rms 0.4, nu 2.887e-3), 5000 "
               "RK4 steps reversed with checkpointing sized to the free HBM (BF16 snapshots), lambda 0.1 dx^2 "
               "sigma_1, time-averaged mean pressure, gradient wrt a 5x384^3 body force",
    "turb384_sample": "decaying turbulence 384^3 periodic (k^4 exp(-2k^2/k0^2), k0 4, Mach_rms 0.4, nu 2.887e-3), "
                      "{n}-step store-all window sample of the 5000-step case, lambda 0.1 dx^2 sigma_1, mean pressure",
    "wake": "temporally developing wake 512x256x32 (slip walls in x, free stream Mach 0.85, centre 0.5, Re 5e4), "
            "{n}-step window sample of the 4000-step case, lambda 0.1 dx^2 sigma_1, stagnation-pressure loss",
    "ensemble": "batched ensemble of 64 periodic decaying-turbulence boxes (sizes from {32,48,64,96}^3, Mach_rms "
                "0.3, nu 0.0175), windows of 50-400 RK4 steps, lambda from {0,0.03,0.1,0.3,1} dx^2 sigma_1, "
                "time-averaged mean pressure per box; one launch per RK stage covers every running box",
    "spatial_wake": "spatially developing wake 512x256x32 (characteristic inlet and outlet in x, uniform free "
                    "stream Mach 0.85, drag strip at 0.1 L_x holding the deficit, Re 5e4), {n}-step window "
                    "sample, lambda 0.1 dx^2 sigma_1, stagnation-pressure loss on the plane x = 0.75 L_x, "
                    "gradient wrt the body force",
    "offload": "decaying turbulence 384^3 periodic (Mach_rms 0.4, nu 2.887e-3), {n}-step window sample, lambda 0.1 "
               "dx^2 sigma_1, mean pressure; the window's BF16 records kept in pinned host memory and streamed "
               "over PCIe (device-to-host after each primal step, host-to-device one step ahead of the reverse "
               "sweep), against the same sweeps with the records in HBM",
    "turb384_window": "the whole 5000-step 384^3 window once: autograd gradients and finite differences",
    "wake_lambda": "the 4000-step wake with a lambda sweep over one BF16 trajectory",
    "cpu_baseline": "the FP64 oracle's rates on the host cores for every configuration (no GPU work)",
    "lamest": "choice of lambda for decaying turbulence 128^3 periodic (Mach_rms 0.4, nu 2.887e-3): {n}-step window, "
              "6 candidate scales {{0,0.01,0.03,0.1,0.3,1}} dx^2 swept backward together as one batched ensemble "
              "from a white-noise terminal adjoint, adjoint energy after every reverse step",
}


def make_workload(name, window):
    import workloads as W
    if name == "tgv64":
        return W.tgv_64(nsteps=window or 1000)
    if name == "turb384_sample":
        return W.turb_384(nsteps=window or 10, lam_factor=0.1)
    if name == "wake":
        return W.wake(nsteps=window or 20, lam_factor=0.1)
    if name == "spatial_wake":
        return W.spatial_wake(nsteps=window or 20, lam_factor=0.1)
    raise SystemExit(f"unknown workload {name}")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="timed steps: time steps of the 384^3 plan (default workload), windows otherwise")
    ap.add_argument("--warmup", type=int, default=5, help="untimed steps (windows) before the timed ones")
    ap.add_argument("--workload", default="turb384", choices=sorted(WORKLOADS))
    ap.add_argument("--window", type=int, default=0, help="RK4 steps per window (default: the workload's)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--parts", default="f32_lam,f32_lam0,f64_lam0",
                    help="turb384_window: f32_lam, f32_lam0, f64_lam0 (gradients), fd (finite differences)")
    ap.add_argument("--fd-seeds", default="10,11,12,13,14,15,16,17", help="turb384_window: direction seeds")
    ap.add_argument("--fd-eps", type=float, default=1e-3, help="turb384_window: finite-difference step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ckpt", default="bf16", choices=("bf16", "i16"),
                    help="record format of the FP32 paths' snapshots: BF16 codes (default) or 16-bit fixed-point "
                         "codes of the same size")
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--schedule", default="stages", choices=("stages", "recompute"),
                    help="stages: the forward sweep keeps the RK4 stage states in HBM; recompute: the reverse "
                         "step recomputes them from w_n")
    ap.add_argument("--time-scheme", default="rk4", choices=("rk4", "ssprk3"),
                    help="time marching: classical RK4, or the strong-stability-preserving RK3 of the paper")
    ap.add_argument("--flux", default="split", choices=("split", "roe"),
                    help="convective flux: split central form, or the paper's Roe upwind flux")
    ap.add_argument("--nu-weight", default=None,
                    help="artificial-viscosity weights of the variable groups rho, rho u, rho E (e.g. 0.3,1,2.5)")
    args = ap.parse_args()
    args.ts = 1 if args.time_scheme == "ssprk3" else 0
    args.fl = 1 if args.flux == "roe" else 0
    args.nw = tuple(float(x) for x in args.nu_weight.split(",")) if args.nu_weight else None
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (sharding over several GPUs "
              "is described in the design notes and not implemented)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "cpu_baseline":
        main_cpu_baseline(args)
        return

    import torch

    import paper_1511_06959_amd as adj

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    adj.lib()
    if args.workload == "turb384":
        main_c5(args)
        return
    if args.workload == "turb384_window":
        main_c5_window(args)
        return
    if args.workload == "wake_lambda":
        main_wake_lambda(args)
        return
    if args.workload == "ensemble":
        main_ensemble(args)
        return
    if args.workload == "lamest":
        main_lamest(args)
        return
    if args.workload == "offload":
        main_offload(args)
        return
    wl = make_workload(args.workload, args.window)
    big = args.workload != "tgv64"
    stages = args.schedule == "stages" and not big
    print(f"[bench] workload {wl.name}: {wl.n} cells, {wl.nsteps} steps, dt {wl.dt:.4e}, lambda {wl.lam:.3e}",
          file=sys.stderr, flush=True)
    # the large configurations keep BF16 checkpoint records on the FP32 path
    r32 = run_gpu(wl, adj.F32, args.steps, args.warmup, not args.no_autotune, stages=stages, ckpt_bf16=big,
                  rec_fmt=record_format(args),
                  time_scheme=args.ts, flux=args.fl, nu_weight=args.nw)
    print(f"[bench] f32 window {r32['ms_per_step']:.1f} ms", file=sys.stderr, flush=True)
    r32b = None
    if stages:
        r32b = run_gpu(wl, adj.F32, args.steps, args.warmup, False, stages=False, time_scheme=args.ts, flux=args.fl,
                       nu_weight=args.nw)
        print(f"[bench] f32 window, recompute schedule {r32b['ms_per_step']:.1f} ms", file=sys.stderr, flush=True)
    r64 = None
    if not args.no_f64:
        r64 = run_gpu(wl, adj.F64, args.steps, args.warmup, not args.no_autotune, stages=stages,
                      time_scheme=args.ts, flux=args.fl, nu_weight=args.nw)
        print(f"[bench] f64 window {r64['ms_per_step']:.1f} ms", file=sys.stderr, flush=True)

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    khash = kernel_hash()
    tile32 = r32["tiles"].get("adjoint_stage", {}).get("launched")
    traffic = profile_values("traffic_adjoint_stage_tgv64.txt", khash, tile32)
    valu = profile_values("valu_adjoint_stage_tgv64.txt", khash, tile32)
    if big:
        traffic = valu = None
    roof = {
        "bound": "hbm",
        "achieved": r32["stage_achieved_gbs"],
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": r32["stage_achieved_gbs"] / HBM_PEAK_GBS,
        "traffic": None if traffic is None else float(traffic["bytes_per_cell_launch_f32"]) * wl.ncells,
        "traffic_profile": None if traffic is None else "profiles/" + traffic["profile"],
        "kernel": "k_adjoint_stage (reverse-stage gather)",
        "avg_launch_us": r32["stage_avg_us"],
        "alg_bytes_per_launch": r32["stage_alg_bytes"],
        "alg_bytes_per_cell_step": ALG_BYTES["adjoint"]["f32"],
        "schedule_bytes_per_launch": r32["stage_schedule_bytes"],
        "schedule_gbs": r32["stage_schedule_gbs"],
        "schedule_frac": r32["stage_schedule_gbs"] / HBM_PEAK_GBS,
    }
    roof_valu = valu_roofline(valu, wl.ncells, r32["stage_avg_us"])
    if roof_valu is not None:
        roof_valu["profile"] = "profiles/" + valu["profile"]
    if "roe" in r32:
        # with the Roe flux the transpose of its flux terms takes the largest share of the window
        rk = r32["roe"]["roe_adjoint"]
        rhash = kernel_hash("roe")
        rtraffic = profile_values("traffic_roe_adjoint_tgv64.txt", rhash, "")
        rvalu = profile_values("valu_roe_adjoint_tgv64.txt", rhash, "")
        if big:
            rtraffic = rvalu = None
        line_stage = dict(roof, traffic=roof["traffic"])
        roof = {
            "bound": "hbm",
            "achieved": rk["achieved_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": rk["frac_hbm"],
            "traffic": None if rtraffic is None else float(rtraffic["bytes_per_cell_launch_f32"]) * wl.ncells,
            "kernel": "k_roe_adjoint (transpose of the Roe convective terms)",
            "avg_launch_us": rk["avg_launch_us"],
            "alg_bytes_per_launch": rk["alg_bytes_per_launch"],
        }
        r32["roe"]["adjoint_stage_roofline"] = line_stage
        r32["roe"]["adjoint_stage_roofline_valu"] = roof_valu
        roof_valu = valu_roofline(rvalu, wl.ncells, rk["avg_launch_us"])
    line = {
        "metric": METRIC,
        "value": r32["value"],
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS[args.workload].format(n=wl.nsteps).replace(
                "RK4 steps", "SSP-RK3 steps" if args.ts == 1 else "RK4 steps"),
            "time_scheme": args.time_scheme,
            "flux": ("Roe upwind flux (linear reconstruction, |lam| smoothed within %g c~)" % ROE_DELTA
                     if args.fl else "split central form (Kennedy-Gruber)"),
            "nu_weight": list(args.nw) if args.nw else "one artificial viscosity for every variable",
            "cells": wl.ncells,
            "window_steps": wl.nsteps,
            "dt": wl.dt,
            "step": "one whole window: forward sweep + reverse sweep",
            "schedule": ("stage states of every step kept in HBM by the forward sweep" if stages else
                         "reverse step recomputes the stage states from the stored w_n"),
            "checkpoints": (("BF16" if args.ckpt == "bf16" else "16-bit fixed-point") + " records (per 4x4x4 block and "
                            "variable a least-squares plane and the 16-bit code of the residual)") if big
                           else "native FP32 / FP64 states",
        },
        "roofline": roof,
        "roofline_valu": roof_valu,
        "adjoint_sweep_cell_steps_per_s": r32["adjoint_sweep_cell_steps_per_s"],
        "primal_cell_steps_per_s": r32["primal_cell_steps_per_s"],
        "kernel_ms_per_window": {k: v[0] / args.steps for k, v in r32["prof"].items()},
        "eager_ms_per_step": r32["eager_ms_per_step"],
        "launch": "each window replayed as two captured HIP graphs (forward sweep, reverse sweep)",
        "tiles": r32["tiles"],
    }
    if "roe" in r32:
        line["roe_kernels"] = r32["roe"]
    if r32b is not None:
        line["f32_recompute_schedule"] = {"value": r32b["value"], "ms_per_step": r32b["ms_per_step"],
                                          "adjoint_sweep_cell_steps_per_s": r32b["adjoint_sweep_cell_steps_per_s"]}
    if r64 is not None:
        line["f64"] = {
            "value": r64["value"],
            "ms_per_step": r64["ms_per_step"],
            "adjoint_sweep_cell_steps_per_s": r64["adjoint_sweep_cell_steps_per_s"],
            "primal_cell_steps_per_s": r64["primal_cell_steps_per_s"],
            "roofline": {"achieved": r64["stage_achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": r64["stage_achieved_gbs"] / HBM_PEAK_GBS, "avg_launch_us": r64["stage_avg_us"]},
            "kernel_ms_per_window": {k: v[0] / args.steps for k, v in r64["prof"].items()},
            "eager_ms_per_step": r64["eager_ms_per_step"],
            "tiles": r64["tiles"],
        }
        line["f32_speedup_over_f64"] = r32["value"] / r64["value"]
        line["rel_err_f32_vs_f64"] = {
            "J": abs(r32["J"] - r64["J"]) / abs(r64["J"]),
            "dJ_dw0": rel(r32["wh0"], r64["wh0"]),
            "dJ_ds": rel(r32["grad_s"], r64["grad_s"]),
            "note": "FP32 states are stored as deviations from the mean initial state (adj_grid.w_ref); the FP64 "
                    "path matches the FP64 oracle to 1e-10 on the 16^3 window in the test suite",
        }
    if not args.no_cpu_baseline and not big:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds, args.fl)
    print(json.dumps(line), flush=True)


def main_ensemble(args):
    import paper_1511_06959_amd as adj
    boxes = make_ensemble()
    print(f"[bench] ensemble: {len(boxes)} boxes, {sum(w.ncells for w in boxes)} cells, windows "
          f"{boxes[-1].nsteps}-{boxes[0].nsteps}", file=sys.stderr, flush=True)
    r = run_ensemble(boxes, adj.F32, args.steps, args.warmup, not args.no_autotune)
    print(f"[bench] ensemble f32 window {r['ms_per_step']:.1f} ms", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS["ensemble"],
            "cells": r["cells"],
            "cell_steps_per_window": r["cell_steps"],
            "step": "one whole ensemble window: forward sweep + reverse sweep of every box",
            "schedule": "every state of every box kept in HBM (native FP32); the reverse step recomputes the "
                        "stage states",
            "trajectory_gb": r["trajectory_gb"],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": r["stage_achieved_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": r["stage_achieved_gbs"] / HBM_PEAK_GBS,
            "alg_bytes_per_cell_step": ALG_BYTES["adjoint"]["f32"],
            "schedule_gbs": r["stage_schedule_gbs"],
            "schedule_frac": r["stage_schedule_gbs"] / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "k_adjoint_stage_batch (reverse-stage gather over all running members)",
            "avg_launch_us": r["stage_avg_us"],
            "launches": r["stage_launches"],
        },
        "adjoint_sweep_cell_steps_per_s": r["adjoint_sweep_cell_steps_per_s"],
        "primal_cell_steps_per_s": r["primal_cell_steps_per_s"],
        "kernel_ms_per_window": {k: v[0] for k, v in r["prof"].items()},
        "eager_ms_per_step": r["eager_ms_per_step"],
        "launch": "the ensemble window replayed as two captured HIP graphs (forward sweep, reverse sweep)",
        "tiles": r["tiles"],
    }
    print(json.dumps(line), flush=True)


def main_lamest(args):
    """The batched reverse sweeps of the lambda estimate (paper_1511_06959_amd.lamest): one
    ensemble of 6 members over one stored 128^3 window, timed per sweep; value = member
    cell-steps per second of the sweep."""
    import torch

    import paper_1511_06959_amd as adj
    import workloads as W
    from paper_1511_06959_amd import autotune, lamest

    T = args.window or 50
    wl = W.turbulence(128, mach_rms=0.4, nu=2.887e-3, seed=4, nsteps=T)
    ref = adj.reference_state(wl.w0)
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, adj.F32, w_ref=ref)
    tiles = {}
    if not args.no_autotune:
        tiles = _tile_report(autotune.tune(g), g, True)
    factors = [0.0, 0.01, 0.03, 0.1, 0.3, 1.0]
    dx2 = (wl.L[0] / 128) ** 2
    lams = [f * dx2 for f in factors]
    aT = np.random.default_rng(0).standard_normal(5 * g.ncells)
    print(f"[bench] lamest: 128^3, {T} steps, {len(factors)} candidates", file=sys.stderr, flush=True)
    sw = lamest.EnergySweeps(g, g.to_stored(wl.w0), None, T, "cuda")
    for _ in range(args.warmup):
        sw.energies(lams, aT)
    adj.profile_enable(True)
    Es = sw.energies(lams, aT)
    torch.cuda.synchronize()
    adj.profile_enable(False)
    ms, n = adj.profile_read(adj.PROF_ADJOINT_STAGE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Es = sw.energies(lams, aT)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    rates = [lamest.growth_rate(E, g.dt) for E in Es]
    k = lamest.choose(factors, rates, [True] * len(factors), 0.0)
    cells = g.ncells * len(factors) * T
    avg_s = ms / n / 1e3
    alg = ALG_BYTES["adjoint"]["f32"] / 4 * g.ncells * len(factors)
    sched = VALUES_PER_STAGE_LAUNCH * 4 * g.ncells * len(factors)
    print(f"[bench] lamest sweep {sec * 1e3:.1f} ms, chosen factor {factors[k] if k is not None else None}",
          file=sys.stderr, flush=True)
    line = {
        "metric": METRIC,
        "value": cells / sec,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["lamest"].format(n=T), "cells": g.ncells, "members": len(factors),
                   "window_steps": T, "step": "the batched homogeneous reverse sweep of all candidates over the "
                   "stored window (one estimate without refinement)"},
        "roofline": {"bound": "hbm", "achieved": alg / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg / avg_s / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_adjoint_stage_batch (reverse-stage gather over all members)",
                     "avg_launch_us": avg_s * 1e6, "alg_bytes_per_cell_step": ALG_BYTES["adjoint"]["f32"],
                     "schedule_gbs": sched / avg_s / 1e9, "schedule_frac": sched / avg_s / 1e9 / HBM_PEAK_GBS},
        "estimate": {"factors": factors, "growth_rates": rates,
                     "chosen_factor": factors[k] if k is not None else None},
        "tiles": tiles,
    }
    print(json.dumps(line), flush=True)


def main_offload(args):
    """Eager windows with the trajectory in pinned host memory (offload) and in HBM (sweep);
    value = cell-steps/s of the host-memory window, PCIe transfers included."""
    import torch

    import paper_1511_06959_amd as adj
    import workloads as W
    from paper_1511_06959_amd import autotune, offload, sweep

    wl = make_workload("turb384_sample", args.window)
    T = wl.nsteps
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, adj.F32, adj.CKPT_BF16,
                      adj.reference_state(wl.w0))
    tiles = _tile_report(autotune.tune(g), g, True) if not args.no_autotune else {}
    obj = adj.Objective.make(wl.obj_kind, wl.plane_i, wl.pt_ref)
    w0 = torch.from_numpy(g.to_stored(wl.w0)).to("cuda", torch.float32)
    s = torch.from_numpy(wl.s).to("cuda", torch.float32)
    ws = adj.workspace(g)
    ht = offload.HostTrajectory(g, T)
    hh = offload.HostTrajectory(g, T, device_tail=(T + 1) // 2)
    import tempfile
    fd, fpath = tempfile.mkstemp(prefix="adjns_traj_", suffix=".bin")
    os.close(fd)
    hf = offload.HostTrajectory(g, T, path=fpath)
    traj = sweep.Trajectory(g, T)

    def timed(fwd, bwd):
        out = []
        for k in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fwd()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            bwd()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if k >= args.warmup:
                out.append((t1 - t0, t2 - t1))
        f = sum(x for x, _ in out) / len(out)
        b = sum(y for _, y in out) / len(out)
        return f, b

    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    fh, bh = timed(lambda: offload.forward(g, w0, s, T, obj, wl.weights, ws, traj=ht, J=J.zero_()),
                   lambda: offload.backward(g, ht, s, obj, wl.weights, wl.lam, ws))
    ft, bt = timed(lambda: offload.forward(g, w0, s, T, obj, wl.weights, ws, traj=hh, J=J.zero_()),
                   lambda: offload.backward(g, hh, s, obj, wl.weights, wl.lam, ws))
    ff, bf = timed(lambda: offload.forward(g, w0, s, T, obj, wl.weights, ws, traj=hf, J=J.zero_()),
                   lambda: offload.backward(g, hf, s, obj, wl.weights, wl.lam, ws))
    hf.close()
    fd, bd = timed(lambda: sweep.forward(g, w0, s, T, obj, wl.weights, ws, traj=traj, J=J.zero_()),
                   lambda: sweep.backward(g, traj, s, obj, wl.weights, wl.lam, ws))
    cells = g.ncells * T
    rec_gb = ht.rec_len / 1e9
    print(f"[bench] offload window {1e3 * (fh + bh):.1f} ms (HBM {1e3 * (fd + bd):.1f} ms)", file=sys.stderr,
          flush=True)
    line = {
        "metric": METRIC,
        "value": cells / (fh + bh),
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * (fh + bh),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["offload"].format(n=T), "cells": g.ncells, "window_steps": T,
                   "step": "one whole eager window: forward sweep + reverse sweep",
                   "record_gb": rec_gb, "host_trajectory_gb": ht.nbytes / 1e9},
        "pcie_inclusive": True,
        "forward_ms": 1e3 * fh, "reverse_ms": 1e3 * bh,
        "file": {"path_dir": os.path.dirname(fpath), "value": cells / (ff + bf), "ms_per_step": 1e3 * (ff + bf),
                 "forward_ms": 1e3 * ff, "reverse_ms": 1e3 * bf},
        "half_in_hbm": {"device_tail": hh.tail, "value": cells / (ft + bt), "ms_per_step": 1e3 * (ft + bt),
                        "forward_ms": 1e3 * ft, "reverse_ms": 1e3 * bt},
        "hbm_trajectory": {"value": cells / (fd + bd), "ms_per_step": 1e3 * (fd + bd), "forward_ms": 1e3 * fd,
                           "reverse_ms": 1e3 * bd},
        "host_copy_gbs": {"device_to_host": (T + 1) * rec_gb / fh, "host_to_device": (T + 1) * rec_gb / bh},
        "tiles": tiles,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
