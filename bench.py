#!/usr/bin/env python3
"""Benchmark of the grim per-zone Newton method on one MI355X.

Metric: zone-updates per second at Newton residual 1e-10 (one zone-update =
one interior zone advanced one full two-stage step), with the mean Newton
iterations per zone and stage, against the plain FP64 form on the same GPU.
Headline workload: 3-D EMHD in Kerr spacetime (a = 0.9375, modified
Kerr-Schild), 192 x 192 x 96 zones, 10 FP64 primitives, Fishbone-Moncrief
torus with 4% seeded noise in u and a weak poloidal field, chi = nu = 0.01,
20 steps, plain FP64 Newton.  Inputs are synthetic and resident in HBM
before the timed region.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload NAME]

One "step" is one full time step (both stages: PLM/LLF fluxes, flux-CT,
stage right-hand side with the geometric and EMHD sources, Newton solve)
over the whole grid, replayed from captured HIP graphs.  Prints one JSON
line.  Besides the headline it reports the other forms of the method on the
same workload (FP32 Jacobian, learned initial guess, both), the 2-D EMHD
workloads at 256^2 and 512^2 as variants, the per-primitive error of every
form against the CPU oracle, the roofline of the dominant kernel and the
oracle's own throughput on the host (the cpu_baseline leg).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector, dense
HBM_PEAK_GBS = 8000.0

# FP64 operations (fma = 2, sqrt = div = 1) of one residual evaluation R(P),
# counted on the specialised register code: derive the state, T^0_nu, U(P),
# and for EMHD the rescaled q, DP and the implicit relaxation terms.
# Minkowski: 66 (ideal) / 157 (EMHD).  Modified Kerr-Schild adds, per
# derived state: g_ij ut^i ut^j over the five non-zero spatial entries (+9),
# u^0 = gamma/alpha and the shift terms u^i = ut^i - gamma alpha g^{0i}
# (+10), and lowering u^mu and b^mu with the seven non-zero entries of
# g_{mu nu} (+16 each), plus sqrt(-g)/dt' (+1): +52.
RESID_FLOPS = {("minkowski", 8): 66, ("minkowski", 10): 157, ("mks", 8): 118, ("mks", 10): 209}
# The Newton system has N = nvar - 3 unknowns (5 ideal, 7 EMHD: B is fixed at
# its explicit update).  Norm over the system rows: 2N + 2.  Jacobian column:
# perturbation (4), the reciprocal of h (1), N subtractions and N
# multiplications.  Dense solve with partial pivoting and one right-hand
# side, counted as LU: 2N^3/3 + 2N^2 (rounded).
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

def newton_flops(nvar: int, metric: str, zone_stages: int, iters: float, resid_calls: int) -> float:
    """Algorithmic FP64 flops of the Newton solves summed over a run (the
    learned-guess candidate check counts as one more residual call)."""
    n = nvar - 3
    ls_trials = resid_calls - zone_stages - n * iters
    norm = 2 * n + 2
    return (resid_calls * RESID_FLOPS[(metric, nvar)]
            + (zone_stages + ls_trials) * norm
            + iters * (n * (2 * n + 5) + LU_FLOPS[n])
            + ls_trials * 2 * n)


KERNEL_SOURCES = ["newton.hip", "kernels.hip", "grim_zone.h", "grim_device.h", "grim_internal.h", "grim_rhs.h"]


def kernel_source_hash() -> str:
    """Hash of the sources the stage, flux, rhs and Newton kernels are compiled from."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1702_01106_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` on `workload` from committed rocprofv3
    counters, if they were taken on the current kernel sources; else None."""
    p = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except (OSError, ValueError):
        return None
    if d.get("source_sha256_16") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch", {}).get(kernel)


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
    del a, b, c
    return {"gbs": 3 * 8 * n * reps / t / 1e9, "bytes_per_launch": 3 * 8 * n, "exact": ok}


def log(msg: str) -> None:
    """Progress of the benchmark's phases on stderr (the JSON line is stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ------------------------------------------------------------------ GPU runs

def timed_run(grim, wl, P0, steps, warmup, weights=None):
    """Graph-replayed timed run of `steps` steps from P0, then an instrumented
    eager pass over the same steps (per-kernel device time from HIP events
    around each launch group, on the context's stream).  Returns dt, seconds,
    stats of both runs, kernel times and the final primitives."""
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
    ctx.set_prims(P0)
    ctx.profile(True)
    st_p = ctx.run(dt, steps, use_graph=False, want_stats=True)
    times = ctx.kernel_times()
    ctx.profile(False)
    ctx.close()
    return dt, t, st, st_p, times, P_end


def check_states(grim, wl, P0, dt, steps, weights=None, box=None):
    """States for the oracle check, from an untimed run of the same form:
    for each check step s, P_{s-1} (the input of step s) and P_s, both cut to
    `box` (a subdomain with its halo) or whole."""
    ctx = grim.Context(wl)
    if weights is not None:
        grim.grim_mlp_set_weights(ctx.ctx, weights)
    ctx.set_prims(P0)
    out = []
    done = 0
    for s in check_steps(wl, steps):
        if s - 1 > done:
            ctx.run(dt, s - 1 - done, use_graph=True, want_stats=False)
            done = s - 1
        Pin = ctx.get_prims()
        ctx.run(dt, 1, use_graph=True, want_stats=False)
        done = s
        Pout = ctx.get_prims()
        if box is not None:
            Pin, Pout = cut(Pin, box, halo=True), cut(Pout, box, halo=False)
        out.append((s, Pin, Pout))
    ctx.close()
    return out


def final_state(grim, wl, P0, dt, steps):
    """The GPU's state after `steps` graph-replayed steps from P0."""
    ctx = grim.Context(wl)
    ctx.set_prims(P0)
    ctx.run(dt, steps, use_graph=True, want_stats=False)
    P = ctx.get_prims()
    ctx.close()
    return P


# a full-grid oracle run of a whole workload is made when the oracle's
# measured rate puts it under this many seconds (the 192x192x96 torus: ~90 s
# on 16 threads)
E2E_MAX_SECONDS = 180.0


def end_to_end(O, wl, P0, dt, steps, Pgpu, threads):
    """The oracle's full-grid run of the workload from P0 against the GPU's
    state after the same steps: per primitive, the largest difference over
    max |P_v| of the oracle's state.  Reported, not bounded: after several
    steps the two runs also differ by the tolerance each Newton solve leaves
    open, carried forward."""
    o = O.Oracle(dict(wl, nthreads=threads))
    t0 = time.perf_counter()
    ref, _ = o.step(P0, dt, steps)
    seconds = time.perf_counter() - t0
    nv = wl["nvar"]
    rel = {PRIM_NAMES[v] if nv == 10 or v < 8 else str(v):
           float(np.abs(Pgpu[v] - ref[v]).max() / max(np.abs(ref[v]).max(), 1e-300)) for v in range(nv)}
    return {"steps": steps, "zones": int(ref[0].size), "oracle_seconds": seconds, "threads": threads,
            "max_rel_diff": rel}


def check_steps(wl, steps):
    return sorted({1, max(1, steps // 2), steps}) if wl.get("metric") == "mks" else [steps]


# The Kerr check subdomain: 32^3 zones in the torus body (r ~ 6.5..11.5,
# within 15 degrees of the equator) with a halo of 2 Ng = 4 zones; X3 is
# periodic, so the box wraps in k.
BOX_N, BOX_HALO = 32, 4
CPU_SAMPLE_S = 10.0  # oracle time the cpu_baseline sample runs for


def kerr_box(wl):
    n = wl["n"]
    i0 = int(round((np.log(6.5) - wl["x_start"][0]) / ((wl["x_end"][0] - wl["x_start"][0]) / n[0])))
    j0 = n[1] // 2 - BOX_N // 2
    assert BOX_HALO <= i0 and i0 + BOX_N + BOX_HALO <= n[0] and BOX_HALO <= j0 and j0 + BOX_N + BOX_HALO <= n[1]
    return (i0, j0, 0)


def cut(P, box, halo):
    """P[:, k, j, i] on the box (with its halo if asked), wrapping in k."""
    h = BOX_HALO if halo else 0
    i0, j0, k0 = box
    ks = np.arange(k0 - h, k0 + BOX_N + h) % P.shape[1]
    return np.ascontiguousarray(P[:, ks][:, :, j0 - h:j0 + BOX_N + h][:, :, :, i0 - h:i0 + BOX_N + h])


def form_line(zones, steps, t, st, times, value_ref):
    v = zones * steps / t
    return {
        "value": v,
        "ms_per_step": t / steps * 1e3,
        "mean_newton_iters": st["mean_iters"],
        "max_resid": st["max_resid"],
        "n_fail": st["n_fail"],
        "n_backtracks": st.get("n_backtracks", 0),
        "n_fallback": st.get("n_fallback", 0),
        "n_f64_retry": st.get("n_f64_retry", 0),
        "kernel_ms_per_step": {k: x[0] / steps for k, x in times.items() if x[1]},
        "speedup_vs_f64": v / value_ref,
    }


def run_forms(grim, W, wl, P0, args, names):
    """The forms `names` of the method on one workload, each timed and with
    its states for the oracle check.  The network of the learned forms is
    trained once (untimed) on pairs from FP64 runs of the same workload on
    seeds 1-4 and evaluated on seed 0."""
    import torch

    from paper_1702_01106_amd import learned

    zones = int(P0[0].size)
    box = kerr_box(wl) if wl.get("metric") == "mks" else None
    res, checks, weights = {}, {}, None
    value_ref = None
    for name in names:
        jac = "f32" if name.startswith("f32") else "f64"
        learned_guess = name.endswith("learned_guess")
        if learned_guess and weights is None:
            t0 = time.perf_counter()
            weights, info = learned.train_guess(wl, seeds=(1, 2, 3, 4), steps=wl["steps"], pairs=args.pairs,
                                                epochs=args.epochs, batch=4096)
            torch.cuda.synchronize()
            res["training"] = {"pairs": info["pairs"], "epochs": args.epochs, "seconds": time.perf_counter() - t0,
                               "loss_first_last": [info["loss"][0], info["loss"][-1]], "seeds": [1, 2, 3, 4]}
            log(f"{wl['name']}: trained the guess network on {info['pairs']} pairs in "
                f"{res['training']['seconds']:.1f} s")
        fwl = dict(wl, jac=jac, guess="mlp" if learned_guess else "pn",
                   system="full" if "full_system" in name else "reduced")
        w = weights if learned_guess else None
        dt, t, st, st_p, times, _ = timed_run(grim, fwl, P0, args.steps, args.warmup, weights=w)
        if value_ref is None:
            value_ref = zones * args.steps / t
        line = form_line(zones, args.steps, t, st, times, value_ref)
        line["stats_eager_pass"] = st_p
        line["dt"] = dt
        res[name] = line
        log(f"{wl['name']} {name}: {line['value']:.4g} zone-updates/s, {line['ms_per_step']:.3f} ms/step, "
            f"iters {line['mean_newton_iters']}")
        checks[name] = check_states(grim, fwl, P0, dt, args.steps, weights=w, box=box)
    return res, checks


def roofline(wl, nvar, steps, form):
    """Roofline of the step's dominant kernel from the instrumented pass:
    algorithmic FP64 flops per launch over its average launch time."""
    st = form["stats_eager_pass"]
    kms = {k: v for k, v in form["kernel_ms_per_step"].items()}
    metric = wl.get("metric", "minkowski")
    zones = int(np.prod(wl["n"]))
    iters = (st["mean_iters"][0] + st["mean_iters"][1]) * zones * steps
    flops = newton_flops(nvar, metric, st["zone_stages"], iters, st["n_resid_calls"])
    launches = 2 * steps
    tiled = metric == "minkowski" and wl["ndim"] == 2 and "face_flux" not in kms
    per_launch = flops / launches
    if tiled:
        n = list(wl["n"])
        faces = (n[0] + 1) * n[1] + n[0] * (n[1] + 1)
        per_launch += faces * FACE_FLOPS[nvar] + zones * RHS_FLOPS_2D[nvar]
        name = f"k_stage<{nvar}, 2> (tile face fluxes + stage right-hand side + Newton, f64)"
    else:
        geo = "GeoKS" if metric == "mks" else "GeoMink"
        name = f"k_newton<{nvar}, {geo}, double, {0 if metric == 'mks' else wl['ndim']}>"
    avg_s = kms["newton"] * steps / launches * 1e-3
    achieved = per_launch / avg_s / 1e12
    dominant = max(kms, key=kms.get)
    return {
        "bound": "alu",
        "achieved": achieved,
        "peak": FP64_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / FP64_PEAK_TFLOPS,
        "traffic": traffic_from_profiles(wl["name"], name),
        "kernel": name,
        "dominant_group": dominant,
        "avg_launch_us": avg_s * 1e6,
        "flops_per_launch": per_launch,
        "launches": launches,
    }


# bytes a zone-stage must move through each kernel of the three-kernel path
# (faces, stored right-hand side, Newton), the interior counted once and the
# 2-D metric tables, shared by every plane, left out: faces read P^E and
# write a face per direction; the right-hand side reads the three faces, P^E
# and P_n and writes rhs and (EMHD) the 13-double bundle; the Newton kernel
# reads rhs, the bundle and P_n and writes P
def kernel_alg_bytes(nvar):
    w = 8 * nvar
    bundle = 8 * 13 if nvar == 10 else 0
    return {"face_flux": w + 3 * w, "stage_rhs": 5 * w + w + bundle, "newton": w + bundle + w + w}


def measured_traffic(workload):
    """Measured HBM bytes per launch of each kernel group from the committed
    counters, if they were taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    try:
        d = json.load(open(p))
    except (OSError, ValueError):
        return {}
    if d.get("source_sha256_16") != kernel_source_hash():
        return {}
    out = {}
    for name, (rd, wr) in d.get("read_write_bytes", {}).items():
        for group, key in (("face_flux", "k_fluxes"), ("stage_rhs", "k_rhs"), ("newton", "k_newton<")):
            if key in name:
                out[group] = rd + wr
    return out


def kernel_table(wl, nvar, steps, form):
    """Per kernel group of the three-kernel path: time per step, the
    algorithmic bytes per step and their rate against the HBM peak, and the
    measured bytes per launch where counters exist (None otherwise)."""
    kms = form["kernel_ms_per_step"]
    if "face_flux" not in kms:
        return None
    zones = int(np.prod(wl["n"]))
    alg = kernel_alg_bytes(nvar)
    meas = measured_traffic(wl["name"])
    table = {}
    for group in ("face_flux", "stage_rhs", "newton"):
        if group not in kms:
            continue
        b = alg[group] * zones * 2  # two stages a step
        gbs = b / (kms[group] * 1e-3) / 1e9
        table[group] = {"ms_per_step": kms[group], "alg_bytes_per_step": b, "alg_GBps": gbs,
                        "hbm_frac": gbs / HBM_PEAK_GBS, "measured_bytes_per_launch": meas.get(group)}
    return table


def step_roofline(wl, nvar, steps, form, roof):
    """The step's roofline over the three-kernel path: each kernel's lower
    bound is the larger of its algorithmic bytes at the HBM peak and its
    algorithmic flops at the FP64 peak (faces and right-hand side counted
    with the Minkowski operation counts, so a lower bound in Kerr; the Newton
    kernel with its counted flops), summed over the kernels of a step and
    divided by their measured time."""
    table = kernel_table(wl, nvar, steps, form)
    if table is None:
        return None
    zones = int(np.prod(wl["n"]))
    alg = kernel_alg_bytes(nvar)
    flops = {"face_flux": wl["ndim"] * zones * FACE_FLOPS[nvar], "stage_rhs": zones * RHS_FLOPS_2D[nvar],
             "newton": roof["flops_per_launch"]}
    per = {}
    for group in ("face_flux", "stage_rhs", "newton"):
        tb = alg[group] * zones / (HBM_PEAK_GBS * 1e9)
        tf = flops[group] / (FP64_PEAK_TFLOPS * 1e12)
        per[group] = {"bound": "hbm" if tb >= tf else "alu", "t_roofline_ms_per_launch": max(tb, tf) * 1e3}
    t_roof = 2 * sum(v["t_roofline_ms_per_launch"] for v in per.values())
    t_meas = sum(table[g]["ms_per_step"] for g in per)
    return {"t_roofline_ms_per_step": t_roof, "t_measured_ms_per_step": t_meas, "frac": t_roof / t_meas,
            "per_kernel": per}


# ------------------------------------------------------------------ CPU leg

FAMILY = [[0], [1], [2, 3, 4], [5, 6, 7], [8], [9]]
PRIM_NAMES = ["rho", "u", "u1", "u2", "u3", "B1", "B2", "B3", "q", "dP"]


def box_workload(wl, box, n):
    """The workload's physics on a box of n^3 zones starting at zone `box`
    of the full grid (same zone width)."""
    dx = [(wl["x_end"][d] - wl["x_start"][d]) / wl["n"][d] for d in range(3)]
    xs = [wl["x_start"][d] + box[d] * dx[d] for d in range(3)]
    return dict(wl, n=[n, n, n], x_start=xs, x_end=[xs[d] + n * dx[d] for d in range(3)])


def oracle_box_step(O, wl, box, Pin, dt, threads):
    """One full step of the oracle on the box from the GPU's P_n on the box
    and a 2 Ng halo: stage 1 on the box grown by Ng (its outer ring is then
    exact, being computed from the true P_n), stage 2 on the box with that
    ring as the halo of P_{n+1/2}."""
    ref, info, _ = oracle_step_checked(O, wl, Pin, dt, threads, box=box)
    return ref, info


def oracle_step_checked(O, wl, Pin, dt, threads, box=None, Pgpu=None):
    """The oracle's step from Pin (the box with its halo, or the whole grid),
    and with Pgpu (the GPU's result) the per-primitive comparison.

    Both solvers stop once the scaled residual norm is below tol, so their
    answers may differ by what that leaves open: with J the oracle's Newton
    Jacobian at its root, P_a - P_b = J^-1 (R_a - R_b) to first order, and
    |(P_a - P_b)_v| <= ||row v of J^-1|| (||R_a|| + ||R_b||), where
    ||R|| = ||R||_s U_rho / dt'.  ||R_a||_s is taken at the bar the GPU's
    answer must meet in the oracle's equations (2 tol, checked separately:
    a wrong answer would otherwise widen its own bound), ||R_b||_s is the
    oracle's own final norm.  The comparison allows, per zone and primitive,
    the larger of 1e-6 of max(|P_v|, family RMS) and twice that bound; an
    answer is within if every primitive is inside its allowance and the
    oracle's residual at it is below 2 tol (zones on the atmosphere floor,
    not roots by construction, excepted from the residual test)."""
    g = BOX_HALO // 2
    wl2 = wl
    if box is not None:
        big = (box[0] - g, box[1] - g, box[2] - g)
        wl2 = box_workload(wl, box, BOX_N)
        o1 = O.Oracle(dict(box_workload(wl, big, BOX_N + 2 * g), nthreads=threads))
        o2 = O.Oracle(dict(wl2, nthreads=threads))
        Pn1 = np.ascontiguousarray(Pin[:, g:-g, g:-g, g:-g])
        Pn2 = np.ascontiguousarray(Pin[:, 2 * g:-2 * g, 2 * g:-2 * g, 2 * g:-2 * g])
        PEg1 = Pin
    else:
        o1 = o2 = O.Oracle(dict(wl, nthreads=threads))
        Pn1 = Pn2 = Pin
        PEg1 = o1.fill_ghosts(Pin)
    t0 = time.perf_counter()
    Ph, _, _, fl1, _ = o1.stage_ghosted(Pn1, PEg1, 0.5 * dt)
    PEg2 = Ph if box is not None else o2.fill_ghosts(Ph)
    ref, it, rr, fl2, bt = o2.stage_ghosted(Pn2, PEg2, dt)
    seconds = time.perf_counter() - t0
    info = {"fail_stage1": int(np.sum((fl1 & 21) != 0)), "fail_stage2": int(np.sum((fl2 & 21) != 0)),
            "mean_iters_stage2": float(it.mean()), "oracle_seconds": seconds}
    if Pgpu is None:
        return ref, info, None
    return ref, info, compare_stage(o2, wl2, Pn2, PEg2, dt, Pgpu, ref, rr)


def oracle_throughput(O, wl, states, dt, threads, box, min_seconds=CPU_SAMPLE_S, max_steps=400):
    """Oracle step-time over the states (box with halo, or whole grid),
    cycling through them, one pass at least, until min_seconds of oracle
    time have passed or max_steps steps have run: (zone-updates, seconds,
    steps)."""
    g = BOX_HALO // 2
    if box is not None:
        big = (box[0] - g, box[1] - g, box[2] - g)
        o1 = O.Oracle(dict(box_workload(wl, big, BOX_N + 2 * g), nthreads=threads))
        o2 = O.Oracle(dict(box_workload(wl, box, BOX_N), nthreads=threads))
    else:
        o1 = o2 = O.Oracle(dict(wl, nthreads=threads))
    if not states or max_steps < 1:
        raise ValueError("oracle_throughput needs a state and a step")
    t_all, zu, steps = 0.0, 0, 0
    while steps == 0 or (t_all < min_seconds and steps < max_steps):
        for Pin in states:
            if steps >= max_steps:
                break
            if box is not None:
                Pn1 = np.ascontiguousarray(Pin[:, g:-g, g:-g, g:-g])
                Pn2 = np.ascontiguousarray(Pin[:, 2 * g:-2 * g, 2 * g:-2 * g, 2 * g:-2 * g])
                PEg1 = Pin
            else:
                Pn1 = Pn2 = Pin
                PEg1 = o1.fill_ghosts(Pin)
            t0 = time.perf_counter()
            Ph, _, _, _, _ = o1.stage_ghosted(Pn1, PEg1, 0.5 * dt)
            PEg2 = Ph if box is not None else o2.fill_ghosts(Ph)
            o2.stage_ghosted(Pn2, PEg2, dt)
            t_all += time.perf_counter() - t0
            zu += Pn2[0].size
            steps += 1
    return zu, t_all, steps


def compare_stage(o, wl, Pn, PEg, dtp, Pgpu, ref, rr):
    """Per-primitive comparison of the GPU's stage answer Pgpu with the
    oracle's ref (final norms rr) for a stage with P_n, ghost-filled P^E and
    dtp on the grid of wl and oracle instance o (see oracle_step_checked)."""
    nv, tol = wl["nvar"], wl["tol"]
    _, rn = o.residual_ghosted(Pn, PEg, dtp, Pgpu)
    floored = floored_zones(wl, ref) | floored_zones(wl, Pgpu)
    J, ur = o.system_jacobians_ghosted(Pn, PEg, dtp, ref)
    rows = np.linalg.norm(np.linalg.inv(J), axis=2)  # [nz][m]
    bound = rows * ((2 * tol + rr) * ur / dtp)[:, None]
    unk = [0, 1, 2, 3, 4] + ([8, 9] if nv == 10 else [])
    scale = family_scale(ref).reshape(nv, -1)
    err = np.abs(Pgpu - ref).reshape(nv, -1)
    allowed = 1e-6 * scale
    for i, v in enumerate(unk):
        allowed[v] = np.maximum(allowed[v], 2.0 * bound[:, i])
    rel = (err / scale).max(axis=1)
    ratio = (err / allowed).max(axis=1)
    resid = float(rn[~floored].max()) if np.any(~floored) else 0.0
    return {
        "rel": {PRIM_NAMES[v]: float(rel[v]) for v in range(nv)},
        "worst_over_allowed": {PRIM_NAMES[v]: float(ratio[v]) for v in range(nv)},
        "tol_bound_rel": {PRIM_NAMES[v]: float((2 * bound[:, i] / scale[v]).max()) for i, v in enumerate(unk)},
        "max_oracle_resid_at_gpu": resid,
        "within": bool(ratio.max() <= 1.0 and resid < 2 * tol),
    }


def family_scale(P):
    """max(|P_v|, RMS over the grid of v's family of P), per element."""
    nv = P.shape[0]
    out = np.empty_like(P)
    for fam in FAMILY:
        fam = [v for v in fam if v < nv]
        if not fam:
            continue
        rms = float(np.sqrt(np.mean(np.stack([P[v] ** 2 for v in fam]))))
        for v in fam:
            out[v] = np.maximum(np.abs(P[v]), rms)
    return np.where(out > 0, out, 1.0)


def floored_zones(wl, P):
    """Zones of the grid of wl whose rho or u sits on the Kerr atmosphere
    floor (not roots of the stage equations)."""
    if not wl.get("floors"):
        return np.zeros(P[0].size, dtype=bool)
    n = wl["n"]
    X1 = wl["x_start"][0] + (np.arange(n[0]) + 0.5) * (wl["x_end"][0] - wl["x_start"][0]) / n[0]
    r = np.broadcast_to(np.exp(X1), P[0].shape)
    rf, uf = wl["rho_floor"] * r ** -1.5, wl["u_floor"] * r ** -2.5
    return ((np.abs(P[0] - rf) <= 1e-12 * rf) | (np.abs(P[1] - uf) <= 1e-12 * uf)).ravel()


def cpu_leg(W, wl, forms, checks, variant_checks, finals=None):
    """The oracle (test infrastructure, plain C) on the host: its throughput
    on a bounded sample of the workload, and the per-primitive error of every
    GPU form against it on the same inputs."""
    import oracle as O

    threads = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        threads = min(threads, int(env))
    kerr = wl.get("metric") == "mks"
    box = kerr_box(wl) if kerr else None
    errors = {}
    for name, states in checks.items():
        errs = {}
        for s, Pin, Pout in states:
            _, info, rep = oracle_step_checked(O, wl, Pin, forms[name]["dt"], threads, box=box, Pgpu=Pout)
            log(f"oracle check {name} step {s}: within {rep['within']}")
            errs[f"step_{s}"] = dict(rep, oracle=info)
        errors[name] = errs
    zone_updates, t_all, nsteps = oracle_throughput(O, wl, [x[1] for x in checks["f64"]], forms["f64"]["dt"],
                                                    threads, box)
    log(f"oracle throughput: {nsteps} steps in {t_all:.1f} s")
    one_core = None
    if kerr:
        s, Pin, _ = checks["f64"][0]
        _, info, _ = oracle_step_checked(O, wl, Pin, forms["f64"]["dt"], 1, box=box)
        one_core = BOX_N ** 3 / info["oracle_seconds"]
        sample = (f"{nsteps} steps, each one step of a {BOX_N}^3 subdomain in the torus body with a "
                  f"{BOX_HALO}-zone halo from one of the GPU's states before steps {[x[0] for x in checks['f64']]} "
                  f"in turn; stage 1 runs on the {BOX_N + BOX_HALO}^3 box around it, counted as {BOX_N}^3 "
                  f"zone-updates")
    else:
        sample = f"{nsteps} repetitions of the last step of the workload on the full grid, from the GPU's state before it"
    verrors = {}
    for vname, vchecks in variant_checks.items():
        vwl = W.workload(vname)
        verrors[vname] = {}
        for name, (vdt, states) in vchecks.items():
            vbox = kerr_box(vwl) if vwl.get("metric") == "mks" else None
            verrors[vname][name] = {
                f"step_{s}": oracle_step_checked(O, vwl, Pin, vdt, threads, box=vbox, Pgpu=Pout)[2]
                for s, Pin, Pout in states}
    e2e = {}
    rate = zone_updates / t_all
    for fname, (fwl, fP0, fdt, fsteps, Pf) in (finals or {}).items():
        est = fP0[0].size * fsteps / rate
        if est > E2E_MAX_SECONDS:
            e2e[fname] = {"skipped": f"the oracle would take ~{est:.0f} s"}
            continue
        e2e[fname] = end_to_end(O, fwl, fP0, fdt, fsteps, Pf, threads)
        log(f"oracle end-to-end {fname}: {e2e[fname]['oracle_seconds']:.1f} s")
    model = platform.processor()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    base = {
        "value": zone_updates / t_all,
        "unit": "zone-updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": sample,
        "seconds": t_all,
        "cpu_model": model,
    }
    if one_core is not None:
        base["value_one_core"] = one_core
    return base, errors, verrors, e2e


# ------------------------------------------------------------------ probes

def residual_probe(grim, W):
    """Residual hook on four 64 x 64 x 16 grids (every lane active), for the
    FP64 instruction counters that cross-check the residual flop counts."""
    import torch

    for name, nv in (("emhd2d_modes_256", 8), ("emhd2d_modes_256", 10), ("grmhd3d_kerr_128", 8),
                     ("emhd3d_kerr_192", 10)):
        if name.startswith("emhd2d"):
            wl = dict(W._BASE, ndim=3, n=[64, 64, 16], x_start=[0, 0, 0], x_end=[1, 1, 1], nvar=nv, gamma=4 / 3,
                      tau_R=1.0, chi=0.01, nu=0.01, name="mink3d")
            rng = np.random.default_rng(0)
            P = np.zeros((nv, 16, 64, 64))
            P[0] = 1 + 0.1 * rng.uniform(-1, 1, P[0].shape)
            P[1] = 1 + 0.1 * rng.uniform(-1, 1, P[0].shape)
            P[2:5] = 0.1 * rng.uniform(-1, 1, P[2:5].shape)
            P[5:8] = 0.1
        else:
            wl = W.small(name, [64, 64, 16])
            P = W.kerr_torus(wl, seed=0)
        ctx = grim.Context(wl)
        Pd = torch.from_numpy(P).cuda()
        R = torch.empty_like(Pd)
        for _ in range(3):
            grim.grim_residual(ctx.ctx, Pd, Pd, 1e-3, Pd, R, None)
        torch.cuda.synchronize()
        print(f"residual probe {wl['name']} nvar={nv} zones={P[0].size}", flush=True)
        ctx.close()


# ------------------------------------------------------------------ main

# the plain method and its three faster forms; then the 8x8 / 10x10 system
# (B among the unknowns), the comparison form of the paper's reduced system
FORMS = ["f64", "f32_jacobian", "f64_learned_guess", "f32_jacobian_learned_guess", "f64_full_system"]


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="emhd3d_kerr_192")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle (throughput and errors)")
    ap.add_argument("--no-variants", action="store_true", help="only the plain FP64 form of the workload")
    ap.add_argument("--pairs", type=int, default=1_000_000, help="training pairs of the learned guess")
    ap.add_argument("--epochs", type=int, default=8, help="training epochs of the learned guess")
    ap.add_argument("--variant-workloads", default="emhd2d_modes_256,emhd2d_modes_512,grmhd3d_kerr_128",
                    help="comma-separated other workloads for the forms (the ideal-MHD torus runs the FP64, "
                         "FP32-Jacobian and full-system forms its configuration compares)")
    ap.add_argument("--residual-probe", action="store_true", help="run the residual hook for counters and exit")
    ap.add_argument("--stream", action="store_true", help="run the STREAM probe also with --no-variants")
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
    if args.residual_probe:
        residual_probe(grim, W)
        return 0
    wl = W.workload(args.workload)
    P0 = W.initial_state(wl, seed=0)
    zones = int(P0[0].size)
    nvar = wl["nvar"]

    names = FORMS[:1] if args.no_variants else FORMS
    forms, checks = run_forms(grim, W, wl, P0, args, names)
    head = forms["f64"]
    value = head["value"]
    out = {
        "metric": "zone-updates/sec at Newton residual 1e-10; mean Newton iters/zone; vs FP64 GPU",
        "value": value,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "zones": zones, "grid": wl["n"], "nvar": nvar,
                   "metric": wl.get("metric", "minkowski"), "steps_in_workload": wl["steps"], "tol": wl["tol"],
                   "jacobian": "f64", "guess": "P_n", "dt": head["dt"]},
        "mean_newton_iters": head["mean_newton_iters"],
        "max_resid": head["max_resid"],
        "n_fail": head["n_fail"],
        "kernel_ms_per_step": head["kernel_ms_per_step"],
        "roofline": roofline(wl, nvar, args.steps, head),
        "kernels": kernel_table(wl, nvar, args.steps, head),
        "step_roofline": step_roofline(wl, nvar, args.steps, head, roofline(wl, nvar, args.steps, head)),
        "forms": {k: v for k, v in forms.items() if k != "f64"},
    }
    if "f64_full_system" in forms:
        full = forms["f64_full_system"]
        out["system_ab"] = {
            "reduced_zone_updates_per_s": value, "full_zone_updates_per_s": full["value"],
            "reduced_over_full": value / full["value"],
            "mean_iters_reduced": head["mean_newton_iters"], "mean_iters_full": full["mean_newton_iters"],
            "newton_ms_per_step_reduced": head["kernel_ms_per_step"].get("newton"),
            "newton_ms_per_step_full": full["kernel_ms_per_step"].get("newton"),
        }
    variant_checks, finals = {}, {}
    if not args.no_cpu_baseline:
        finals[args.workload] = (wl, P0, forms["f64"]["dt"], args.steps,
                                 final_state(grim, dict(wl, jac="f64"), P0, forms["f64"]["dt"], args.steps))
    if args.stream or not args.no_variants:
        out["stream"] = stream_probe(grim, wl)
    if not args.no_variants:
        variants = {}
        for vname in [v for v in args.variant_workloads.split(",") if v and v != args.workload]:
            vwl = W.workload(vname)
            vP0 = W.initial_state(vwl, seed=0)
            names = FORMS if vwl["nvar"] == 10 else ["f64", "f32_jacobian", "f64_full_system"]
            vforms, vchecks = run_forms(grim, W, vwl, vP0, args, names)
            vforms["roofline"] = roofline(vwl, vwl["nvar"], args.steps, vforms["f64"])
            vforms["system_ab"] = {"reduced_over_full": vforms["f64"]["value"] / vforms["f64_full_system"]["value"],
                                   "mean_iters_full": vforms["f64_full_system"]["mean_newton_iters"]}
            variants[vname] = vforms
            variant_checks[vname] = {k: (vforms[k]["dt"], v) for k, v in vchecks.items()}
            if not args.no_cpu_baseline:
                vdt = vforms["f64"]["dt"]
                finals[vname] = (vwl, vP0, vdt, args.steps, final_state(grim, dict(vwl, jac="f64"), vP0, vdt,
                                                                         args.steps))
        out["variants"] = variants
    if not args.no_cpu_baseline:
        base, errors, verrors, e2e = cpu_leg(W, wl, forms, checks, variant_checks, finals)
        out["cpu_baseline"] = base
        out["error_vs_oracle"] = errors
        for vname, e in verrors.items():
            out["variants"][vname]["error_vs_oracle"] = e
        for fname, e in e2e.items():
            if fname == args.workload:
                out["end_to_end_vs_oracle"] = e
            else:
                out["variants"][fname]["end_to_end_vs_oracle"] = e
        out["gpu_over_cpu"] = value / base["value"]
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
