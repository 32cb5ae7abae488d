"""CPU checks of the benchmark's host logic: the one-GPU guard and the
cpu_baseline sample (the oracle's step time, cycled over the given states
until the requested oracle time has passed or the step cap is reached)."""
import os
import subprocess
import sys

import numpy as np

import bench
from paper_1702_01106_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_oracle_throughput_counts_box_steps(oracle_mod):
    wl = W.workload("emhd3d_kerr_192")
    P0 = W.initial_state(wl, seed=0)
    box = bench.kerr_box(wl)
    Pin = bench.cut(P0, box, True)
    dt = 1e-3
    # a zero time budget still runs one pass over the states
    zu, t, n = bench.oracle_throughput(oracle_mod, wl, [Pin, Pin], dt, 2, box, min_seconds=0.0)
    assert n == 2 and zu == 2 * bench.BOX_N ** 3 and t > 0.0
    # the step cap bounds the sample
    zu, t, n = bench.oracle_throughput(oracle_mod, wl, [Pin], dt, 2, box, min_seconds=1e9, max_steps=3)
    assert n == 3 and zu == 3 * bench.BOX_N ** 3


def test_oracle_throughput_whole_grid(oracle_mod):
    wl = W.small("emhd2d_modes_256", [32, 16])
    P0 = np.ascontiguousarray(W.initial_state(wl, seed=0))
    zu, t, n = bench.oracle_throughput(oracle_mod, wl, [P0], 1e-3, 2, None, min_seconds=0.0)
    assert n == 1 and zu == 32 * 16 and t > 0.0


def test_kernel_table_bytes():
    wl = W.workload("emhd3d_kerr_192")
    zones = 192 * 192 * 96
    t = bench.kernel_table(wl, 10, 20, {"kernel_ms_per_step": {"face_flux": 1.0, "stage_rhs": 1.0, "newton": 1.0}})
    # per zone-stage: faces 10 + 30 doubles, rhs 50 read + 10 + 13 written, Newton 10 + 13 + 10 read + 10 written
    assert t["face_flux"]["alg_bytes_per_step"] == 2 * zones * 8 * 40
    assert t["stage_rhs"]["alg_bytes_per_step"] == 2 * zones * 8 * 73
    assert t["newton"]["alg_bytes_per_step"] == 2 * zones * 8 * 43
    assert abs(t["newton"]["hbm_frac"] - 2 * zones * 8 * 43 / 1e-3 / 8e12) < 1e-12
    # the one-kernel stage has no split to report
    assert bench.kernel_table(W.workload("emhd2d_modes_256"), 10, 20, {"kernel_ms_per_step": {"newton": 1.0}}) is None


def test_end_to_end_reports_per_primitive(oracle_mod):
    wl = W.small("grmhd3d_kerr_128", [16, 16, 8])
    P0 = W.initial_state(wl, seed=0)
    o = oracle_mod.Oracle(dict(wl, nthreads=2))
    dt = o.cfl_dt(P0, wl["cfl"])
    ref, _ = o.step(P0, dt, 2)
    r = bench.end_to_end(oracle_mod, wl, P0, dt, 2, ref, 2)
    assert r["steps"] == 2 and r["zones"] == 16 * 16 * 8
    assert set(r["max_rel_diff"]) == set(bench.PRIM_NAMES[:8])
    assert all(v == 0.0 for v in r["max_rel_diff"].values())
    bad = ref.copy()
    bad[1, 3, 4, 5] *= 1.0 + 1e-3
    r2 = bench.end_to_end(oracle_mod, wl, P0, dt, 2, bad, 2)
    assert r2["max_rel_diff"]["u"] > 0.0 and r2["max_rel_diff"]["rho"] == 0.0


def test_step_roofline_sums_kernel_bounds():
    wl = W.workload("emhd3d_kerr_192")
    zones = 192 * 192 * 96
    form = {"kernel_ms_per_step": {"face_flux": 1.0, "stage_rhs": 1.0, "newton": 2.0}}
    r = bench.step_roofline(wl, 10, 20, form, {"flops_per_launch": 15.0e9})
    faces = zones * 8 * 40 / 8e12 * 1e3          # HBM bound: 400 B a zone-stage
    rhs = zones * 8 * 73 / 8e12 * 1e3
    newton = max(zones * 8 * 43 / 8e12, 15.0e9 / 78.6e12) * 1e3
    assert abs(r["t_roofline_ms_per_step"] - 2 * (faces + rhs + newton)) < 1e-12
    assert r["per_kernel"]["newton"]["bound"] == "alu" and r["per_kernel"]["stage_rhs"]["bound"] == "hbm"
    assert abs(r["frac"] - r["t_roofline_ms_per_step"] / 4.0) < 1e-12
