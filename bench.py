#!/usr/bin/env python3
"""Benchmark of one full ADER-DG step with the a-posteriori subcell limiter on one MI355X.

Workload: the smooth isentropic vortex of Sec. 5 (beta = 5, rho = p = 1, u = v = 1
background, periodic [0,10]^2) with N = 9 on 64 x 64 cells, limiter active (detection
runs every step; the resolved vortex triggers no troubled cell).  One step = Delta t
reduction (eq. (cfl)) + old-time bounds + space-time predictor + face fluxes + corrector
+ scatter/detection + compaction (+ subcell recompute and flux correction when cells are
flagged).  Metric: space-time degrees of freedom updated per second, counted per
conserved variable as the paper does ((N+1)^(d+1) per cell and step).

Prints one JSON line.  With --gpus above 1 it exits: the benchmark runs on one GPU.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks used for the roofline fraction
PEAK_FP64_VALU_TFLOPS = 78.6
# FP32 vector work compiled without packed-FP32 instructions issues at the FP64 vector
# rate (one FMA per lane per cycle); the 157.3 TFLOP/s FP32 figure needs packed FP32.
PEAK_FP32_VALU_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of k_predictor<2, 9, true, float> on the N=9, 64x64 vortex: rocprofv3
# FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 (the factors that make a plain 256 MiB copy read its
# own size), taken on the predictor source (the files below, concatenated) whose SHA-256 starts
# with the prefix below; reported as null once that source has changed.
PREDICTOR_SOURCES = ("adg_internal.h", "adg_physics.h", "adg_predictor.h")
PREDICTOR_TRAFFIC_BYTES = 74257524
PREDICTOR_TRAFFIC_SOURCE = "19eedc28bf47549f"


def predictor_flops_per_cell(d: int, N: int) -> float:
    """Algorithmic flops of the local space-time predictor per cell: n Picard sweeps,
    each with d + 1 length-n contractions (d spatial, one in time) of nu * n^(d+1)
    values and one flux evaluation per axis and space-time node ((10 + 8 d) flops per
    node for the d fluxes).  The first sweep starts from a state constant in time, so its
    fluxes and spatial contractions are counted on one time slice (its time contraction
    in full)."""
    n, nv = N + 1, d + 2
    sweep = 2.0 * (d + 1) * nv * n ** (d + 2) + (10 + 8 * d) * n ** (d + 1)
    first = 2.0 * d * nv * n ** (d + 1) + 2.0 * nv * n ** (d + 2) + (10 + 8 * d) * n ** d
    return (n - 1) * sweep + first


def vortex_convergence(N: int = 9, grids=(16, 32, 64), t_end: float = 10.0) -> dict:
    """L1 density error against the exact isentropic vortex at t_end (10: the vortex crosses
    the periodic box once and is back at its start), per grid and precision form, and the
    observed orders between successive grids.  Initial data by nodal interpolation; CFL
    time steps, the last one shortened to land on t_end."""
    import numpy as np
    from paper_1406_7416_amd import adg
    from paper_1406_7416_amd import workloads as W
    out = {"workload": f"isentropic vortex, N={N}, t_end={t_end}", "grids": list(grids)}
    for form, prec in (("fp64", adg.ADG_FP64), ("mixed", adg.ADG_MIXED)):
        errs, nsteps = [], []
        for g in grids:
            wl = W.vortex(g, N)
            prob = adg.Problem(wl, precision=prec)
            u0, _ = prob.project(wl.ic, 0)
            prob.set_state(u0)
            steps = 0
            while prob.time < t_end * (1 - 1e-14):
                prob.step(min(prob.cfl_dt(), t_end - prob.time))
                steps += 1
            ue, _ = prob.project(lambda x, t: wl.ic(x, t_end), 0)
            errs.append(l1_norm(prob.state()[0] - ue[0], wl))
            nsteps.append(steps)
            prob.close()
            print(f"# convergence {form} {g}^2: L1(rho) {errs[-1]:.3e} after {steps} steps", file=sys.stderr,
                  flush=True)
        orders = [float(np.log2(errs[i] / errs[i + 1]) / np.log2(grids[i + 1] / grids[i]))
                  for i in range(len(grids) - 1)]
        out[form] = {"l1_rho": errs, "steps": nsteps, "orders": orders}
    return out


def l1_norm(f, wl):
    """L1 norm over the domain of a nodal field f[cell][node] (tensor Gauss-Legendre
    quadrature of the cells' nodes)."""
    import numpy as np
    n = wl.N + 1
    w1 = np.polynomial.legendre.leggauss(n)[1] / 2.0
    w = w1
    for _ in range(wl.dim - 1):
        w = np.multiply.outer(w1, w).reshape(-1)
    vol = 1.0
    for k in range(wl.dim):
        vol *= (wl.hi[k] - wl.lo[k]) / wl.ncell[k]
    return float((np.abs(f) * w[None, :]).sum() * vol)


def traffic_bytes(N, grid):
    """Measured HBM traffic of the dominant kernel, if it was measured on this workload and
    on the kernel source as it stands."""
    import hashlib
    h = hashlib.sha256()
    for name in PREDICTOR_SOURCES:
        with open(os.path.join(ROOT, "paper_1406_7416_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    h = h.hexdigest()
    if N != 9 or grid != 64 or not h.startswith(PREDICTOR_TRAFFIC_SOURCE):
        return None
    return PREDICTOR_TRAFFIC_BYTES


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--grid", type=int, default=64)
    ap.add_argument("--N", type=int, default=9)
    ap.add_argument("--breakdown-steps", type=int, default=10,
                    help="untimed steps with events around every kernel group (per-kernel breakdown)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="bounded CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the four-quadrant batch measurement")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D explosion measurement (128^3, N=3)")
    ap.add_argument("--steps-3d", type=int, default=6)
    ap.add_argument("--no-small", action="store_true", help="skip the 2D explosion, double Mach and shock-vortex measurements")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device-to-device copy of this size (counter calibration)")
    ap.add_argument("--convergence", action="store_true",
                    help="only measure the vortex's L1 error at t = 10 on 16^2, 32^2, 64^2 cells (degree --N)")
    args = ap.parse_args()

    if args.convergence:
        print(json.dumps(vortex_convergence(args.N)))
        return

    if args.copy_bytes:
        import torch
        src = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes, "launches": 3}))
        return

    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1406_7416_amd import adg
    from paper_1406_7416_amd import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)

    wl = W.vortex(args.grid, args.N)
    d, N = wl.dim, wl.N
    st_dof_step = wl.st_dof_per_step()
    print(f"# workload vortex N={N} grid={args.grid}^2 cells={wl.num_cells} cfl={wl.cfl}", file=sys.stderr,
          flush=True)

    forms = {}
    finals = {}
    u0 = None
    # the Osher-type flux (the paper's flux for its vortex runs) alongside Rusanov
    for form, prec, flux in (("fp64", adg.ADG_FP64, 0), ("mixed", adg.ADG_MIXED, 0),
                             ("fp64_osher", adg.ADG_FP64, 1), ("mixed_osher", adg.ADG_MIXED, 1)):
        prob = adg.Problem(wl, precision=prec, flux=flux)
        if u0 is None:
            u0, _ = prob.project(wl.ic, 0)      # nodal values of the initial condition
        prob.set_state(u0)
        for _ in range(args.warmup):
            prob.step_cfl()
        torch.cuda.synchronize()
        # timed region: HIP events around the dominant kernel only (two event records per
        # step on the problem's stream)
        prob.profile(True, groups=["predictor"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            prob.step_cfl()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pred_ms, pred_n = prob.profile_read()["predictor"]
        prob.profile(False)
        elapsed = t1 - t0
        # per-kernel-group breakdown from a separate, untimed pass with events around
        # every group
        prob.profile(True)
        for _ in range(args.breakdown_steps):
            prob.step_cfl()
        prof = prob.profile_read()
        prob.profile(False)
        t_sim = prob.time
        u = prob.state()
        ue, _ = prob.project(lambda x, t: wl.ic(x, t_sim), 0)
        forms[form] = {
            "value": st_dof_step * args.steps / elapsed,
            "ms_per_step": 1e3 * elapsed / args.steps,
            "predictor_avg_us": 1e3 * pred_ms / max(1, pred_n),
            "kernels": {g: {"ms_total": round(ms, 4), "launches": n, "avg_us": round(1e3 * ms / n, 3) if n else None}
                        for g, (ms, n) in prof.items()},
            "troubled_last_step": prob.stats()["troubled"],
            "t_simulated": t_sim,
            "linf_rho_vs_exact": float(np.abs(u[0] - ue[0]).max()),
            "l1_rho_vs_exact": l1_norm(u[0] - ue[0], wl),
        }
        finals[form] = u
        prob.close()
        print(f"# {form}: {forms[form]['value']:.3e} st-dof/s, predictor {forms[form]['predictor_avg_us']:.1f} us",
              file=sys.stderr, flush=True)
    # the two forms after the same number of steps: density difference (max and mean)
    drho = np.abs(finals["mixed"][0] - finals["fp64"][0])
    head = "mixed"
    h = forms[head]
    pred_avg_s = h["predictor_avg_us"] * 1e-6
    flops_launch = predictor_flops_per_cell(d, N) * wl.num_cells
    achieved_tflops = flops_launch / pred_avg_s / 1e12

    out = {
        "metric": "space-time dof-updates/s",
        "value": h["value"],
        "unit": "st-dof/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 predictor and face fluxes, f64 state/detection",
        "data": "synthetic (analytic initial condition)",
        "config": {
            "workload": f"isentropic vortex (Sec. 5), N={N}, {args.grid}x{args.grid} cells, periodic [0,10]^2, "
                        f"limiter on, CFL factor {wl.cfl}, Ns={2 * N + 1}",
            "cells": wl.num_cells,
            "st_dof_per_step": st_dof_step,
            "form": "mixed (headline); FP64 GPU form alongside",
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_predictor (FP32 space-time predictor + volume term + face traces)",
            "achieved": achieved_tflops,
            "peak": PEAK_FP32_VALU_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / PEAK_FP32_VALU_TFLOPS,
            "traffic": traffic_bytes(args.N, args.grid),
            "traffic_unit": "bytes per launch (HBM, calibrated rocprofv3 counters)",
            "flops_per_launch": flops_launch,
            "avg_launch_us": h["predictor_avg_us"],
        },
        "forms": forms,
        # memory-bound kernel of the step against a measured copy bandwidth: the face fluxes
        # read every cell's face traces once and write one time-integrated flux per face node
        # and adjacent cell (FP32 in the mixed form)
        "memory_bound": face_bandwidth(wl, forms["mixed"]["kernels"]["faces"]["avg_us"]),
        "speedup_mixed_vs_fp64": forms["mixed"]["value"] / forms["fp64"]["value"],
        "speedup_mixed_vs_fp64_osher": forms["mixed_osher"]["value"] / forms["fp64_osher"]["value"],
        "rho_mixed_minus_fp64": {"max": float(drho.max()), "mean": float(drho.mean())},
        # both forms after the same steps, against the exact (advected) vortex
        "matched_l1_rho": {"fp64": forms["fp64"]["l1_rho_vs_exact"], "mixed": forms["mixed"]["l1_rho_vs_exact"],
                           "mixed_over_fp64": forms["mixed"]["l1_rho_vs_exact"] / forms["fp64"]["l1_rho_vs_exact"]},
    }

    if not args.no_batch:
        out["batch"] = batch_measurement(args.batch_count, args.batch_steps)

    if not args.no_3d:
        out["explosion3d"] = explosion3d_measurement(args.steps_3d)

    if not args.no_small:
        # the other 2D workloads: the 2D explosion (40 x 40, N = 3), the double Mach reflection
        # at its full size (400 x 100, N = 5) and the shock-vortex interaction (200 x 100, N = 5)
        out["explosion2d"] = form_pair_measurement(W.explosion_2d(40, 3), 4, steps=50)
        out["double_mach"] = form_pair_measurement(W.double_mach(400, 100, 5), 1, steps=20)
        out["shock_vortex"] = form_pair_measurement(W.shock_vortex(200, 100, 5), 3, steps=20)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, u0, args.cpu_seconds)
        out["cpu_baseline_single_thread"] = cpu_baseline(wl, u0, args.cpu_seconds / 2, threads=1)

    print(json.dumps(out), flush=True)


def form_pair_measurement(wl, m, steps, warmup=3):
    """Both precision forms on one workload at the CFL time step: initial data by the
    m-point rule per subcell with the initial detection, `warmup` untimed steps, then
    `steps` timed steps."""
    import torch
    from paper_1406_7416_amd import adg
    u0, v0 = adg.project(wl, m)
    res = {"workload": f"{wl.name}, N={wl.N}, {wl.ncell[0]}x{wl.ncell[1]} cells", "cells": wl.num_cells,
           "st_dof_per_step": wl.st_dof_per_step(), "steps": steps}
    for form, prec in (("fp64", adg.ADG_FP64), ("mixed", adg.ADG_MIXED)):
        prob = adg.Problem(wl, precision=prec)
        prob.set_state(u0, v0)
        for _ in range(warmup):
            prob.step_cfl()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            prob.step_cfl()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res[form] = {"value": wl.st_dof_per_step() * steps / el, "ms_per_step": 1e3 * el / steps,
                     "troubled_last_step": prob.stats()["troubled"]}
        prob.close()
    res["speedup_mixed_vs_fp64"] = res["mixed"]["value"] / res["fp64"]["value"]
    print(f"# {wl.name}: fp64 {res['fp64']['value']:.3e}, mixed {res['mixed']['value']:.3e} st-dof/s, "
          f"troubled {res['mixed']['troubled_last_step']}", file=sys.stderr, flush=True)
    return res


def explosion3d_measurement(steps, warmup=2, breakdown=2, ncell=128, N=3):
    """The 3D explosion at its full size (128^3 cells on [-1,1]^3, N = 3): both precision
    forms stepped at the CFL time step from the initial data (nodal interpolant, initial
    detection against the subcell-centre values), `warmup` untimed steps, then `steps`
    timed steps."""
    import torch
    from paper_1406_7416_amd import adg
    from paper_1406_7416_amd import workloads as W
    wl = W.explosion_3d(ncell, N)
    t0 = time.perf_counter()
    u0 = adg.project(wl, 0)[0]
    v0 = adg.project(wl, 1)[1]
    t_init = time.perf_counter() - t0
    print(f"# explosion3d {ncell}^3 N={N}: initial data {t_init:.1f} s", file=sys.stderr, flush=True)
    st_dof = wl.st_dof_per_step()
    res = {"workload": f"3D explosion (Sec. 5), N={N}, {ncell}^3 cells on [-1,1]^3, transmissive, "
                       f"CFL factor {wl.cfl}, Ns={2 * N + 1}",
           "cells": wl.num_cells, "st_dof_per_step": st_dof, "steps": steps, "warmup": warmup}
    for form, prec in (("fp64", adg.ADG_FP64), ("mixed", adg.ADG_MIXED)):
        prob = adg.Problem(wl, precision=prec, pool_capacity=wl.num_cells // 8)
        prob.set_state(u0, v0)
        troubled0 = int(prob.troubled().sum())
        for _ in range(warmup):
            prob.step_cfl()
        torch.cuda.synchronize()
        prob.profile(True, groups=["predictor"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            prob.step_cfl()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        pred_ms, pred_n = prob.profile_read()["predictor"]
        prob.profile(True)
        for _ in range(breakdown):
            prob.step_cfl()
        prof = prob.profile_read()
        prob.profile(False)
        pred_s = pred_ms * 1e-3 / max(1, pred_n)
        res[form] = {
            "value": st_dof * steps / elapsed,
            "unit": "st-dof/s",
            "ms_per_step": 1e3 * elapsed / steps,
            "predictor_avg_us": 1e6 * pred_s,
            "predictor_tflops": predictor_flops_per_cell(3, N) * wl.num_cells / pred_s / 1e12,
            "kernels": {g: {"ms_total": round(ms, 4), "launches": n, "avg_us": round(1e3 * ms / n, 3) if n else None}
                        for g, (ms, n) in prof.items()},
            "face_kernel_gbs": (wl.num_cells * 2 * 3 * 5 * ((N + 1) ** 3 + (N + 1) ** 2) * (4 if prec == adg.ADG_MIXED else 8)
                                / (prof["faces"][0] * 1e-3 / max(1, prof["faces"][1])) / 1e9) if prof["faces"][1] else None,
            "troubled_initial": troubled0,
            "troubled_last_step": prob.stats()["troubled"],
            "t_simulated": prob.time,
        }
        prob.close()
        del prob
        torch.cuda.empty_cache()
        print(f"# explosion3d {form}: {res[form]['value']:.3e} st-dof/s, {res[form]['ms_per_step']:.2f} ms/step, "
              f"troubled {res[form]['troubled_last_step']}", file=sys.stderr, flush=True)
    res["speedup_mixed_vs_fp64"] = res["mixed"]["value"] / res["fp64"]["value"]
    return res


def copy_bandwidth_gbs(nbytes=1 << 30, reps=5):
    """Device-to-device copy of nbytes (read + write counted), HIP events around `reps`
    copies: the achievable HBM bandwidth the memory-bound kernels are compared with."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def face_bandwidth(wl, avg_us):
    d, n, nv = wl.dim, wl.N + 1, wl.dim + 2
    nbytes = wl.num_cells * 2 * d * nv * (n ** d + n ** (d - 1)) * 4
    copy = copy_bandwidth_gbs()
    gbs = nbytes / (avg_us * 1e-6) / 1e9
    return {"kernel": "k_face (mixed form)", "algorithmic_bytes": nbytes, "avg_launch_us": avg_us,
            "achieved_gbs": gbs, "copy_gbs_measured": copy, "frac_of_copy": gbs / copy,
            "frac_of_peak": gbs / PEAK_HBM_GBS}


def batch_measurement(count, steps):
    """Independent four-quadrant Riemann problems (random states, grids from
    {32,64,128,256}^2, N from {3,4,5}): the mixed form advanced as one batch (one hipGraph
    launch per batch step) against the plain FP64 form stepped problem by problem."""
    import gc
    import torch
    from paper_1406_7416_amd import adg
    from paper_1406_7416_amd import workloads as W
    wls = W.quadrant_batch(count)
    cfl = min(wl.cfl for wl in wls)
    st_dof = sum(wl.st_dof_per_step() for wl in wls)
    res = {"problems": count, "cells": sum(wl.num_cells for wl in wls), "st_dof_per_step": st_dof,
           "steps": steps, "cfl": cfl}

    def build(prec, mood=False):
        ps = []
        for wl in wls:
            cap = wl.num_cells if wl.num_cells <= 4096 else wl.num_cells // 3
            p = adg.Problem(wl, precision=prec, pool_capacity=cap, mood=mood)
            u, _ = p.project(wl.ic, 0)
            p.set_state(u)
            ps.append(p)
        return ps

    # mixed form, batched
    ps = build(adg.ADG_MIXED)
    b = adg.Batch(ps)
    b.step_cfl(cfl, 3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step_cfl(cfl, steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res["mixed_batched"] = {"value": st_dof * steps / el, "ms_per_batch_step": 1e3 * el / steps,
                            "troubled_last_step": int(sum(int(p.troubled().sum()) for p in ps))}
    b.close()
    for p in ps:
        p.close()
    del ps, b
    gc.collect()
    torch.cuda.empty_cache()
    # plain FP64 form, one problem after the other, per-problem launches
    ps = build(adg.ADG_FP64)
    for p in ps:
        for _ in range(3):
            p.step_cfl(cfl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p in ps:
        for _ in range(steps):
            p.step_cfl(cfl)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res["fp64_per_problem"] = {"value": st_dof * steps / el, "ms_per_batch_step": 1e3 * el / steps}
    res["speedup"] = res["mixed_batched"]["value"] / res["fp64_per_problem"]["value"]
    for p in ps:
        p.close()
    del ps
    gc.collect()
    torch.cuda.empty_cache()
    # the same batch with the MOOD layer after the subcell scheme (Sec. 6, Fig. algo2)
    ps = build(adg.ADG_MIXED, mood=True)
    b = adg.Batch(ps)
    b.step_cfl(cfl, 3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step_cfl(cfl, steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    fl = [p.mood_stats() for p in ps]
    res["mixed_batched_mood"] = {"value": st_dof * steps / el, "ms_per_batch_step": 1e3 * el / steps,
                                 "flagged_subcells_last_step": int(sum(f for f, _ in fl)),
                                 "recomputed_cells_last_step": int(sum(r for _, r in fl)),
                                 "troubled_last_step": int(sum(int(p.troubled().sum()) for p in ps))}
    b.close()
    for p in ps:
        p.close()
    del ps, b
    gc.collect()
    torch.cuda.empty_cache()
    print(f"# batch: mixed batched {res['mixed_batched']['value']:.3e}, fp64 per problem "
          f"{res['fp64_per_problem']['value']:.3e} st-dof/s", file=sys.stderr, flush=True)
    return res


def cpu_baseline(wl, u0, budget_s, threads=None):
    """The FP64 CPU oracle, as it stands, on the same workload: whole steps until the
    time budget is used (at least one); all host threads, or the number given."""
    from oracle import oracle as O
    o = O.Oracle(wl)
    o.set_state(u0)
    saved = O.get_threads()
    if threads:
        O.set_threads(threads)
    threads = O.get_threads()
    steps, t0 = 0, time.perf_counter()
    while True:
        o.step(o.cfl_dt())
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 50:
            break
    O.set_threads(saved)
    return {
        "value": wl.st_dof_per_step() * steps / el,
        "unit": "st-dof/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{steps} full steps of the same workload ({wl.num_cells} cells, N={wl.N}), {el:.1f} s, "
                  f"OpenMP threads={threads}",
    }


if __name__ == "__main__":
    main()
