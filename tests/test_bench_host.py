"""Host parts of bench.py: the oracle's timing leg on a tiny grid, the algorithmic-byte roofline
arithmetic and the schedule ceiling (no GPU)."""
import numpy as np
import pytest

import bench
import workloads as W


def test_oracle_rates_tiny_grid(orc):
    wl = W.turbulence(8, mach_rms=0.3, nu=0.0175, seed=4, nsteps=2)
    og = orc.grid_from(wl.params())
    r = bench._oracle_rates(og, orc.make_obj(wl.obj_kind), wl.w0, 0.0, 0.5, 1, best_of=2, threads=1)
    assert r["threads"] == 1 and r["steps"] == 1 and r["best_of"] == 2
    assert r["primal_cell_steps_per_s"] > 0 and r["adjoint_cell_steps_per_s"] > 0
    # one primal plus one reverse step per cell-step
    hm = 1.0 / (1.0 / r["primal_cell_steps_per_s"] + 1.0 / r["adjoint_cell_steps_per_s"])
    assert r["cell_steps_per_s"] == pytest.approx(hm)


def test_block_cut_keeps_cell_size(orc):
    wl = W.turbulence(16, mach_rms=0.3, nu=0.0175, seed=4, nsteps=1)
    og, w = bench._block(wl, (10, 3, 9), (6, 5, 4))
    assert w.size == 5 * 6 * 5 * 4
    full = wl.w0.reshape(5, 16, 16, 16)
    assert np.array_equal(w.reshape(5, 4, 5, 6), full[:, 9:13, 3:8, 10:16])
    assert og.n[0] == 6 and og.n[1] == 5 and og.n[2] == 4
    assert og.L[0] / og.n[0] == pytest.approx(wl.L[0] / 16)
    with pytest.raises(ValueError):
        bench._block(wl, (12, 3, 9), (6, 5, 4))


def test_kernel_roofline_uses_per_unit_bytes():
    # 90 B per adjoint cell-step, a quarter per stage launch; 80 launches of 2.5 ms each
    cells = 384 ** 3
    r = bench.kernel_roofline("adjoint", "f32", cells, 80 * 2.5, 80)
    assert r["alg_bytes_per_launch"] == pytest.approx(22.5 * cells)
    assert r["achieved"] == pytest.approx(22.5 * cells / 2.5e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    r64 = bench.kernel_roofline("primal", "f64", cells, 10.0, 4)
    assert r64["alg_bytes_per_launch"] == pytest.approx(30.0 * cells)


def test_schedule_ceiling_counts_every_launch(monkeypatch):
    per = {"adjoint_stage": 100.0, "primal_stage": 60.0}

    def fake(name, khash, tile):
        kind = "adjoint_stage" if "adjoint" in name else "primal_stage"
        return {"bytes_per_cell_launch_f32": str(per[kind]), "profile": name}

    monkeypatch.setattr(bench, "profile_values", fake)
    tiles = {"adjoint_stage": {"launched": "32x4x4"}, "primal_stage": {"launched": "32x4x4"}}
    seg = {"tiles": tiles, "advances": 40, "plan": {"schedule": "segments"}, "value": 1e9}
    c = bench.schedule_ceiling(seg, 1000, "h", 4000.0, 20)
    assert c["bytes_per_cell_step"] == pytest.approx(4 * 100 + 8 * 60 + 24)
    assert c["ceiling_at_8tbs"] == pytest.approx(8e12 / c["bytes_per_cell_step"])
    binom = dict(seg, plan={"schedule": "binomial", "stage_recomputes_per_step": 3})
    c2 = bench.schedule_ceiling(binom, 1000, "h", 4000.0, 20)
    assert c2["bytes_per_cell_step"] == pytest.approx(c["bytes_per_cell_step"] + 3 * 60)


def _counter_csv(path, rows):
    import csv
    import os
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(("Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"), r)))


def test_profile_summaries_from_counter_files(tmp_path, capsys):
    from paper_1511_06959_amd import profile_run as pr
    k = "void adjns::k_adjoint_stage<float, 0, 0, 1, 1, 32, 4, 4>(adjns::Consts<float>, float const*)"
    # stall fractions: two dispatches, averaged, then divided by the summed wave cycles
    rows = []
    for d, scale in ((1, 1.0), (2, 3.0)):
        for c, v in (("SQ_WAVE_CYCLES", 1000.0), ("SQ_ACTIVE_INST_VALU", 200.0), ("SQ_WAIT_INST_ANY", 400.0),
                     ("SQ_WAIT_INST_LDS", 100.0), ("SQ_INSTS_LDS", 50.0), ("SQ_LDS_BANK_CONFLICT", 25.0)):
            rows.append((d, k, c, v * scale))
    _counter_csv(str(tmp_path / "stall" / "run_counter_collection.csv"), rows)
    pr.stall(str(tmp_path / "stall"), 64, "_stage", ["cmd"])
    out = capsys.readouterr().out
    assert "2 dispatches" in out and "SQ_WAVE_CYCLES 2000" in out
    assert "valu_active_frac = 0.200, wait_issue_frac = 0.400, wait_lds_frac = 0.100" in out
    assert "lds_conflict_per_lds_inst = 0.500" in out
    # a second run with other counters: each counter averaged over the dispatches of its own run
    rows2 = [(d, k, c, v) for d in (7, 8, 9) for c, v in (("SQ_WAVE_CYCLES", 2000.0), ("SQ_WAIT_ANY", 600.0),
                                                          ("SQ_ACTIVE_INST_LDS", 100.0))]
    _counter_csv(str(tmp_path / "stall2" / "run_counter_collection.csv"), rows2)
    pr.stall([str(tmp_path / "stall"), str(tmp_path / "stall2")], 64, "_stage", [])
    out = capsys.readouterr().out
    assert "5 dispatches" in out and "wait_any_frac = 0.300" in out and "lds_active_frac = 0.050" in out
    assert "valu_active_frac = 0.200" in out and "lds_conflict_per_lds_active_cycle = 0.500" in out
    # traffic: counters scaled by what a copy of known size reads (here fetch x2, write x1)
    copyk = "__amd_rocclr_copyBuffer"
    _counter_csv(str(tmp_path / "cf" / "a_counter_collection.csv"), [(1, copyk, "FETCH_SIZE", 512.0)])
    _counter_csv(str(tmp_path / "cw" / "a_counter_collection.csv"), [(1, copyk, "WRITE_SIZE", 1024.0)])
    _counter_csv(str(tmp_path / "f" / "a_counter_collection.csv"), [(1, k, "FETCH_SIZE", 10.0), (2, k, "FETCH_SIZE", 30.0)])
    _counter_csv(str(tmp_path / "w" / "a_counter_collection.csv"), [(1, k, "WRITE_SIZE", 5.0), (2, k, "WRITE_SIZE", 5.0)])
    pr.traffic(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"), str(tmp_path / "cw"), 1, 1024,
               "k_adjoint_stage", [])
    vals = dict(l.split(" = ") for l in capsys.readouterr().out.splitlines() if " = " in l and not l.startswith("#"))
    assert float(vals["fetch_bytes_per_launch"]) == pytest.approx(2 * 20.0 * 1024)
    assert float(vals["write_bytes_per_launch"]) == pytest.approx(5.0 * 1024)
    assert float(vals["bytes_per_cell_launch_f32"]) == pytest.approx((40.0 + 5.0) * 1024 / 1024)
    assert vals["tile_f32"] == "32x4x4" and vals["kernel_source_sha256"] == pr._src_hash("k_adjoint_stage")
    # trace table with a note paragraph before it
    import csv
    os_dir = tmp_path / "tr"
    os_dir.mkdir()
    with open(os_dir / "x_kernel_stats.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": k, "Calls": 4, "TotalDurationNs": 4e6, "AverageNs": 1e6, "Percentage": 100.0})
    pr.trace_summary(str(os_dir), "T", "C", ["a note"])
    out = capsys.readouterr().out
    assert out.index("a note") < out.index("| kernel |")
    assert "| `k_adjoint_stage<float, 0, 0, 1, 1, 32, 4, 4>` | 4 | 4.00 | 1000.00 | 100.0 |" in out


def test_more_than_one_gpu_is_refused():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True, timeout=120,
                       cwd=str(__import__("pathlib").Path(bench.__file__).parent))
    assert r.returncode == 2 and "one GPU only" in r.stderr and r.stdout == ""


def test_valu_summary_per_cell(tmp_path, capsys):
    from paper_1511_06959_amd import profile_run as pr
    k = "void adjns::k_primal_stage<float, 1, 1, 32, 4, 4>(adjns::Consts<float>, float const*)"
    vals = {"SQ_WAVES": 8.0, "SQ_INSTS_VALU": 6400.0, "SQ_INSTS_VALU_ADD_F32": 100.0, "SQ_INSTS_VALU_MUL_F32": 50.0,
            "SQ_INSTS_VALU_FMA_F32": 200.0, "SQ_INSTS_VALU_TRANS_F32": 10.0}
    _counter_csv(str(tmp_path / "v" / "run_counter_collection.csv"),
                 [(d, k, c, v) for d in (1, 2) for c, v in vals.items()])
    pr.valu(str(tmp_path / "v"), 512, "k_primal_stage", [])
    out = dict(l.split(" = ") for l in capsys.readouterr().out.splitlines() if " = " in l and not l.startswith("#"))
    assert float(out["valu_insts_per_cell_launch_f32"]) == pytest.approx(6400.0 / 512)
    # 64 lanes per wave instruction, an FMA counts two operations
    assert float(out["fp32_ops_per_cell_launch_f32"]) == pytest.approx(64.0 * (100 + 50 + 10 + 2 * 200) / 512)
    assert out["tile_f32"] == "32x4x4"


def test_with_traffic_fills_or_nulls(monkeypatch):
    cells = 1000
    roof = bench.kernel_roofline("primal", "f32", cells, 8 * 2.0, 8)   # 2 ms per launch
    monkeypatch.setattr(bench, "profile_values",
                        lambda name, h, tile: {"bytes_per_cell_launch_f32": "60", "profile": name}
                        if tile == "32x4x4" else None)
    r = bench.with_traffic(dict(roof), "primal_stage", "h", "32x4x4", cells)
    assert r["traffic"] == pytest.approx(60.0 * cells)
    assert r["traffic_gbs"] == pytest.approx(60.0 * cells / 2e-3 / 1e9)
    assert r["traffic_frac"] == pytest.approx(r["traffic_gbs"] / 8000.0)
    assert r["traffic_profile"] == "profiles/traffic_primal_stage_turb384.txt"
    r2 = bench.with_traffic(dict(roof), "primal_stage", "h", "32x8x2", cells)
    assert r2["traffic"] is None and r2["traffic_gbs"] is None and r2["traffic_frac"] is None
