#!/usr/bin/env python3
"""Benchmark of the grim per-zone Newton method on one MI355X.

Metric: zone-updates per second at Newton residual 1e-10 (one zone-update =
one interior zone advanced one full two-stage step), with the mean Newton
iterations per zone and stage, on the 2D EMHD workload (256 x 256 zones, 10
FP64 primitives, 16 seeded Fourier modes in rho and u, 50 steps, plain FP64
Newton).  Inputs are synthetic and resident in HBM before the timed region.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

One "step" is one full time step (both stages: ghost fill, PLM/LLF fluxes,
flux-CT, stage right-hand side, Newton solve) over the whole grid, replayed
from a captured HIP graph.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector, dense
HBM_PEAK_GBS = 8000.0

# FP64 operations (fma = 2, sqrt = div = 1) of one residual evaluation R(P)
# in Minkowski coordinates, counted on the specialised register code: derive
# the state, T^0_nu, U(P), and for EMHD the rescaled q, DP and the implicit
# relaxation terms.  The Newton system has N = nvar - 3 unknowns (5 ideal,
# 7 EMHD: B is fixed at its explicit update).  Norm over the system rows:
# 2N + 2.  Jacobian column: perturbation (4), the reciprocal of h (1), N
# subtractions and N multiplications.  Dense solve with partial pivoting and
# one right-hand side, counted as LU: 2N^3/3 + 2N^2 (rounded, below).
RESID_FLOPS = {8: 66, 10: 157}
LU_FLOPS = {5: 133, 7: 327}

# FP64 operations of one face flux in Minkowski coordinates (same counting):
# PLM of every variable (15 per variable: three differences, two
# generalized-minmod slopes, two half-slope updates), and per state derive
# (41 EMHD / 31 ideal), wave speed (41 / 33), U (76 / 20) and F (73 / 26),
# then LLF (5 per non-normal variable).
FACE_FLOPS = {8: 376, 10: 658}
# FP64 operations of one zone's stage right-hand side on a 2-D grid: flux
# divergence with the flux-CT EMFs (~100 EMHD), U(P_n) and the derived
# states of P_n and P^E (158), and for EMHD the limited slopes of Theta, u_mu
# and u^i from the four neighbours and the folded relaxation coefficients
# (434); ideal MHD ~180 in all.
RHS_FLOPS_2D = {8: 180, 10: 712}


def newton_flops(nvar: int, zone_stages: int, iters: float, resid_calls: int) -> float:
    """Algorithmic FP64 flops of the Newton solves summed over a run (the
    learned-guess candidate check counts as one more residual call)."""
    n = nvar - 3
    ls_trials = resid_calls - zone_stages - n * iters
    norm = 2 * n + 2
    return (resid_calls * RESID_FLOPS[nvar]
            + (zone_stages + ls_trials) * norm
            + iters * (n * (2 * n + 5) + LU_FLOPS[n])
            + ls_trials * 2 * n)


STAGE_SOURCES = ["newton.hip", "grim_zone.h", "grim_device.h", "grim_internal.h", "grim_rhs.h"]


def stage_source_hash() -> str:
    """Hash of the sources the stage (and Newton) kernels are compiled from."""
    h = hashlib.sha256()
    for f in STAGE_SOURCES:
        with open(os.path.join(ROOT, "paper_1702_01106_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles():
    """HBM bytes per launch of the dominant kernel from committed rocprofv3
    counters, if they were taken on the current kernel sources; otherwise None."""
    p = os.path.join(ROOT, "profiles", "stage_emhd2d_256_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except (OSError, ValueError):
        return None
    if d.get("source_sha256_16") != stage_source_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(wl: dict, P0, dt: float, steps: int) -> dict:
    import oracle

    threads = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        threads = min(threads, int(env))
    o = oracle.Oracle(dict(wl, nthreads=threads))
    t0 = time.perf_counter()
    _, st = o.step(P0, dt, steps)
    t = time.perf_counter() - t0
    zones = P0[0].size
    return {
        "value": zones * steps / t,
        "unit": "zone-updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {steps} of the {wl['steps']} steps of the same workload, full grid",
        "seconds": t,
        "mean_iters": st["mean_iters"],
    }


def stream_probe(grim, wl, n: int = 1 << 26, reps: int = 20) -> dict:
    """STREAM c = a + b over n doubles per array (Sec. 7.2's yardstick),
    through the library's own kernel; bytes = 3 * 8 * n per launch."""
    import torch

    ctx = grim.Context(wl)
    a = torch.rand(n, dtype=torch.float64, device="cuda")
    b = torch.rand(n, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    torch.cuda.synchronize()
    grim.grim_stream_add(ctx.ctx, a, b, c, n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        grim.grim_stream_add(ctx.ctx, a, b, c, n)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ok = bool(torch.equal(c, a + b))
    ctx.close()
    return {"gbs": 3 * 8 * n * reps / t / 1e9, "bytes_per_launch": 3 * 8 * n, "exact": ok}


def timed_run(grim, W, wl, P0, steps, warmup, weights=None):
    """Graph-replayed timed run, then an instrumented eager pass over the same
    steps (per-kernel device time).  Returns dt, seconds, stats of both runs,
    kernel times and the final primitives of the timed run."""
    import torch

    # the library runs on torch's current stream, so that torch's events
    # bracket the graph-replayed steps on the stream they run on
    stream = torch.cuda.current_stream()
    ctx = grim.Context(wl, stream=stream)
    if weights is not None:
        grim.grim_mlp_set_weights(ctx.ctx, weights)
    ctx.set_prims(P0)
    dt = ctx.cfl_dt(wl["cfl"])
    if warmup > 0:
        ctx.run(dt, warmup, use_graph=True)
    ctx.set_prims(P0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    st = ctx.run(dt, steps, use_graph=True, want_stats=True)
    e1.record(stream)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    st["event_seconds"] = e0.elapsed_time(e1) * 1e-3
    P_end = ctx.get_prims()
    # instrumented eager pass over the same steps: per-kernel device time
    ctx.set_prims(P0)
    ctx.profile(True)
    st_p = ctx.run(dt, steps, use_graph=False, want_stats=True)
    times = ctx.kernel_times()
    ctx.profile(False)
    ctx.close()
    return dt, t, st, st_p, times, P_end


FAMILIES = [[0], [1], [2, 3, 4], [5, 6, 7], [8], [9]]


def max_rel_diff(A, B):
    """Largest |A - B| per primitive over max(|B_v|, RMS of B over v's family)."""
    import numpy as np

    worst = 0.0
    for fam in FAMILIES:
        fam = [v for v in fam if v < B.shape[0]]
        if not fam:
            continue
        rms = float(np.sqrt(np.mean(np.stack([B[v] ** 2 for v in fam]))))
        for v in fam:
            den = np.maximum(np.abs(B[v]), rms)
            den = np.where(den > 0, den, 1.0)
            worst = max(worst, float((np.abs(A[v] - B[v]) / den).max()))
    return worst


def variant_line(zones, steps, t, st, times, P_end, P_ref, value_ref):
    v = zones * steps / t
    return {
        "value": v,
        "ms_per_step": t / steps * 1e3,
        "mean_newton_iters": st["mean_iters"],
        "max_resid": st["max_resid"],
        "n_fail": st["n_fail"],
        "n_fallback": st.get("n_fallback", 0),
        "n_f64_retry": st.get("n_f64_retry", 0),
        "newton_avg_launch_us": times["newton"][0] / max(times["newton"][1], 1) * 1e3,
        "kernel_ms": {k: x[0] for k, x in times.items()},
        "max_rel_diff_vs_f64_gpu": max_rel_diff(P_end, P_ref),
        "speedup_vs_f64": v / value_ref,
    }


def forms(grim, W, wl, P0, args, plain=None):
    """Plain FP64, FP32 Jacobian, and both with the learned guess.  The
    network is trained once (untimed) on pairs from FP64 runs of the same
    workload on seeds 1-4 and evaluated on seed 0."""
    import torch

    from paper_1702_01106_amd import learned

    zones = int(P0[0].size)
    res = {}
    if plain is None:
        r = timed_run(grim, W, wl, P0, args.steps, args.warmup)
        value_ref, P_ref = zones * args.steps / r[1], r[5]
        res["f64"] = variant_line(zones, args.steps, r[1], r[2], r[4], r[5], P_ref, value_ref)
    else:
        value_ref, P_ref = plain
    r = timed_run(grim, W, dict(wl, jac="f32"), P0, args.steps, args.warmup)
    res["f32_jacobian"] = variant_line(zones, args.steps, r[1], r[2], r[4], r[5], P_ref, value_ref)
    t0 = time.perf_counter()
    w, info = learned.train_guess(wl, seeds=(1, 2, 3, 4), steps=wl["steps"], pairs=args.pairs, epochs=args.epochs,
                                  batch=4096)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    for name, jac in (("f64_learned_guess", "f64"), ("f32_jacobian_learned_guess", "f32")):
        r = timed_run(grim, W, dict(wl, jac=jac, guess="mlp"), P0, args.steps, args.warmup, weights=w)
        res[name] = variant_line(zones, args.steps, r[1], r[2], r[4], r[5], P_ref, value_ref)
    res["training"] = {"pairs": info["pairs"], "epochs": args.epochs, "seconds": t_train,
                       "loss_first_last": [info["loss"][0], info["loss"][-1]], "seeds": [1, 2, 3, 4]}
    return res


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="emhd2d_modes_256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=50)
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--pairs", type=int, default=1_000_000, help="training pairs of the learned guess")
    ap.add_argument("--epochs", type=int, default=8, help="training epochs of the learned guess")
    ap.add_argument("--variant-workloads", default="emhd2d_modes_512",
                    help="comma-separated extra workloads for the four forms")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU halo exchange is not built",
              file=sys.stderr)
        return 2

    import torch

    from paper_1702_01106_amd import grim
    from paper_1702_01106_amd import workloads as W

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 2
    grim.load()  # raises if the HIP library is missing: no fallback
    wl = W.workload(args.workload)
    P0 = W.initial_state(wl, seed=0)
    zones = int(P0[0].size)
    nvar = wl["nvar"]

    dt, t, st, st_p, times, P_f64 = timed_run(grim, W, wl, P0, args.steps, args.warmup)
    value = zones * args.steps / t
    ms_newton, n_newton = times["newton"]
    flops = newton_flops(nvar, st_p["zone_stages"], (st_p["mean_iters"][0] + st_p["mean_iters"][1]) * zones
                         * args.steps, st_p["n_resid_calls"])
    per_launch_flops = flops / max(n_newton, 1)
    # on a 1- or 2-D Minkowski grid without the network the stage is one
    # kernel (faces, right-hand side and Newton); its algorithmic flops
    # count every face once and every zone's right-hand side once
    tiled = times.get("face_flux", (0.0, 0))[1] == 0 and wl["ndim"] == 2 and wl["metric"] == "minkowski"
    if tiled:
        n = list(wl["n"])
        faces = (n[0] + 1) * n[1] + n[0] * (n[1] + 1)
        per_launch_flops += faces * FACE_FLOPS[nvar] + zones * RHS_FLOPS_2D[nvar]
    avg_s = ms_newton / max(n_newton, 1) * 1e-3
    if tiled:
        # the timed region runs this kernel, two launches a step, plus one
        # statistics reset and read-back: its average duration from the
        # events around that region
        avg_s = st["event_seconds"] / (2 * args.steps)
    achieved = per_launch_flops / avg_s / 1e12
    roofline = {
        "bound": "alu",
        "achieved": achieved,
        "peak": FP64_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / FP64_PEAK_TFLOPS,
        "traffic": traffic_from_profiles(),
        "kernel": (f"k_stage<{nvar}, 2> (tile face fluxes + stage right-hand side + Newton, f64)" if tiled
                   else f"k_newton<{nvar}, Minkowski, f64>"),
        "avg_launch_us": avg_s * 1e6,
        "flops_per_launch": per_launch_flops,
    }
    out = {
        "metric": "zone-updates/sec at Newton residual 1e-10; mean Newton iters/zone; vs FP64 GPU",
        "value": value,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "zones": zones, "nvar": nvar, "steps_in_workload": wl["steps"],
                   "tol": wl["tol"], "jacobian": "f64", "guess": "P_n", "dt": dt},
        "mean_newton_iters": st["mean_iters"],
        "max_resid": st["max_resid"],
        "n_fail": st["n_fail"],
        "kernel_ms": {k: v[0] for k, v in times.items()},
        "roofline": roofline,
    }
    out["stream"] = stream_probe(grim, wl)
    if not args.no_variants:
        # the four forms (FP64 or FP32 Jacobian, P_n or learned guess) on this
        # workload and on the learned-guess configuration (512^2), each against
        # the plain FP64 form of the same workload
        variants = {}
        for vname in [args.workload] + [v for v in args.variant_workloads.split(",") if v and v != args.workload]:
            vwl = W.workload(vname)
            vP0 = P0 if vname == args.workload else W.initial_state(vwl, seed=0)
            variants[vname] = forms(grim, W, vwl, vP0, args, None if vname != args.workload else (value, P_f64))
        out["variants"] = variants
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, P0, dt, args.cpu_steps)
        out["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
