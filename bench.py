#!/usr/bin/env python3
"""Benchmark of the ADER-DG step with the a-posteriori subcell limiter on one MI355X.

Headline workload: a batch of 256 independent four-quadrant Riemann problems (Sec. 5, 2D
Riemann problems; random quadrant states rho, p ~ U[0.1, 2], u, v ~ U[-1, 1], seed
20140627), grids drawn from {32, 64, 128, 256}^2 and degrees from N = 3, 4, 5 (6.1M cells),
transmissive boundaries, every problem at the batch's smallest CFL factor.  One step of the
batch = one step of every problem: Delta t (eq. (cfl)), old-time bounds, space-time
predictor, face fluxes, corrector + scatter + detection, compaction, subcell ADER-WENO3
recompute of the troubled cells, flux correction.  The mixed form runs batched (one launch
per stage and (d, N) class, the step captured in a hipGraph); the plain FP64 form is
stepped problem by problem.  Metric: space-time degrees of freedom updated per second,
counted per conserved variable as the paper does ((N+1)^(d+1) per cell and step).

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
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
# FP32 vector work compiled without packed-FP32 instructions issues one FMA per lane and
# clock: 256 CUs x 2.4 GHz x 128 flop per clock = 78.6 TFLOP/s, the FP64 vector rate (a
# secondary ceiling, reported beside the published FP32 figure)
PEAK_FP32_NONPACKED_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# HBM traffic per launch of the batch step's dominant kernels, from rocprofv3 counter runs
# (FETCH_SIZE x the factor that makes a plain copy read its own size, plus WRITE_SIZE, in
# bytes; mean over the steady launches of the run), keyed to the SHA-256 prefix of the
# kernel sources it was measured on (null once they change).
# (launch "stage:N<degree>" -> (bytes per launch, source hash prefix)); copy calibration: a 256 MiB
# copy reads FETCH_SIZE = 131,084 KiB (factor 2.0) and writes WRITE_SIZE = 262,144 KiB (factor 1.0)
TRAFFIC = {
    "predictor:N5": (10796879296, "7856a18f536122a0"),
    "subcell:N5": (22236328917, "7856a18f536122a0"),
    "corrector_detect:N5": (6559405568, "7856a18f536122a0"),
}
# the kernel sources and the tile-parameter table the build compiles them with
KERNEL_SOURCES = ("csrc/adg_internal.h", "csrc/adg_tune.h", "csrc/adg_physics.h", "csrc/adg_device.h",
                  "csrc/adg_predictor.h", "csrc/adg_kernels_impl.h", "tuning.json")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1406_7416_amd", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


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
    for form, prec in (("fp64", adg.ADG_FP64), ("mixed", adg.ADG_MIXED), ("mixed_dev", adg.ADG_MIXED_DEV)):
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


def subcell_flops_per_cell(d: int, N: int) -> float:
    """Algorithmic flops of the subcell ADER-WENO3 recompute of one troubled cell (Ns = 2N+1
    subcells per axis, nu = d+2 variables).  Positions: the Ns^d subcells and the 2d Ns^(d-1)
    face-adjacent subcells of the neighbours.  Per position: the dimension-by-dimension WENO3
    reconstruction (2D: 5 + 3 one-dimensional reconstructions per variable, 3D: 25 + 15 + 9;
    148 flops each: three stencil polynomials, indicators, weights, evaluation at 3 points),
    the degree-2 space-time predictor (the predictor count with n = 3) and its face traces
    (2d faces x nu x 3^(d-1) x 3 nodes, a length-3 contraction each).  Per sub-face: the
    numerical flux at 3^(d-1) x 3 points (70 flops each).  The FV update and the gather R
    (sum-factorised) are counted in full."""
    Ns, nv, n = 2 * N + 1, d + 2, N + 1
    pos = Ns ** d + 2 * d * Ns ** (d - 1)
    weno_1d = {2: 8, 3: 49}[d] * nv * 148
    pred = 3 * (2.0 * (d + 1) * nv * 3 ** (d + 2) + (10 + 8 * d) * 3 ** (d + 1))   # 3 full sweeps, n = 3
    traces = 2 * d * nv * 3 ** (d - 1) * 3 * 3 * 2
    subfaces = d * (Ns + 1) * Ns ** (d - 1) * 3 ** d * 70
    update = Ns ** d * nv * d * 3
    gather = 2 * nv * sum(n ** (j + 1) * Ns ** (d - j) for j in range(d))
    return pos * (weno_1d + pred + traces) + subfaces + update + gather


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed batch steps")
    ap.add_argument("--warmup", type=int, default=3, help="untimed batch steps before the timed region")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="bounded CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline batch (no vortex, 3D explosion, double Mach, 2D explosion, shock-vortex)")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D explosion measurement (128^3, N=3)")
    ap.add_argument("--steps-3d", type=int, default=6)
    ap.add_argument("--grid", type=int, default=64, help="vortex grid (extra measurement)")
    ap.add_argument("--N", type=int, default=9, help="vortex degree (extra measurement)")
    ap.add_argument("--vortex-steps", type=int, default=100)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device-to-device copy of this size (counter calibration)")
    ap.add_argument("--convergence", action="store_true",
                    help="only measure the vortex's L1 error at t = 10 on 16^2, 32^2, 64^2 cells (degree --N)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the mixed batched form of the batch: no FP64 forms, MOOD run, CPU leg or extras "
                         "(profiling runs)")
    ap.add_argument("--explosion3d-only", action="store_true",
                    help="only the 3D explosion at its full size, both forms (profiling runs)")
    ap.add_argument("--explosion3d-p9-only", action="store_true",
                    help="only the 3D explosion at N = 9 on 50^3 cells, both forms (profiling runs)")
    ap.add_argument("--no-p9", action="store_true", help="skip the 3D explosion at N = 9 (50^3 cells)")
    ap.add_argument("--vortex-only", action="store_true",
                    help="only the vortex measurement (degree --N on --grid^2 cells), every form (profiling runs)")
    args = ap.parse_args()

    if args.explosion3d_only:
        print(json.dumps(explosion3d_measurement(args.steps_3d, warmup=2)))
        return
    if args.vortex_only:
        print(json.dumps(vortex_measurement(args.grid, args.N, args.vortex_steps)))
        return
    if args.explosion3d_p9_only:
        print(json.dumps(explosion3d_p9_measurement()))
        return

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

    import torch
    from paper_1406_7416_amd import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)

    wls = W.quadrant_batch(args.batch_count)
    bres = batch_measurement(wls, args.steps, args.warmup, fp64_forms=not args.batch_only)
    head = bres["mixed_batched"]
    out = {
        "metric": "space-time dof-updates/s",
        "value": head["value"],
        "unit": "st-dof/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 predictor, face fluxes and subcell reconstruction/predictor/fluxes; f64 state, detection, "
                 "projection/gather, subcell halo and update",
        "data": "synthetic (seeded random four-quadrant states, analytic initial data)",
        "config": {
            "workload": f"batch of {len(wls)} four-quadrant Riemann problems (Sec. 5), grids 32^2..256^2, "
                        f"N = 3..5, {bres['cells']} cells, transmissive, CFL factor {bres['cfl']}, Ns = 2N+1, "
                        f"limiter on",
            "problems": len(wls),
            "cells": bres["cells"],
            "st_dof_per_step": bres["st_dof_per_step"],
            "form": "mixed precision, batched (one launch per stage and (d, N) class, hipGraph); "
                    "the plain FP64 form stepped problem by problem alongside",
        },
        "roofline": bres["roofline"],
        "batch": bres,
        "speedup_mixed_batched_vs_fp64_per_problem": bres.get("speedup"),
    }
    del bres

    if not args.batch_only and not args.no_extra:
        out["vortex"] = vortex_measurement(args.grid, args.N, args.vortex_steps)
        if not args.no_3d:
            out["explosion3d"] = explosion3d_measurement(args.steps_3d)
        if not args.no_p9:
            out["explosion3d_p9"] = explosion3d_p9_measurement(cpu=not args.no_cpu_baseline)
        # the other 2D workloads: the 2D explosion (40 x 40, N = 3), the double Mach reflection
        # at its full size (400 x 100, N = 5) and the shock-vortex interaction (200 x 100, N = 5)
        out["explosion2d"] = form_pair_measurement(W.explosion_2d(40, 3), 4, steps=50)
        out["double_mach"] = form_pair_measurement(W.double_mach(400, 100, 5), 1, steps=20)
        out["shock_vortex"] = form_pair_measurement(W.shock_vortex(200, 100, 5), 3, steps=20)

    if not args.batch_only and not args.no_cpu_baseline:
        cpu = cpu_baseline_leg(wls, min(wl.cfl for wl in wls), args.cpu_seconds)
        out["cpu_baseline"] = cpu["cpu_baseline"]
        out["l1_rho_vs_oracle"] = cpu["l1_rho_vs_oracle"]

    print(json.dumps(out), flush=True)


def vortex_measurement(grid, N, steps, warmup=10, breakdown_steps=10):
    """The isentropic vortex (Sec. 5, beta = 5, periodic [0,10]^2), degree N on grid^2 cells, in
    both precision forms with both fluxes: throughput, the predictor's rate (its algorithmic
    flops over its average launch time from HIP events around every predictor launch on the
    problem's stream in the timed region), the face kernel's bandwidth, and the L1 density
    error against the exact (translated) vortex after the steps taken."""
    import numpy as np
    import torch
    from paper_1406_7416_amd import adg
    from paper_1406_7416_amd import workloads as W
    wl = W.vortex(grid, N)
    d = wl.dim
    st_dof_step = wl.st_dof_per_step()
    forms, finals, u0 = {}, {}, None
    for form, prec, flux in (("fp64", adg.ADG_FP64, 0), ("mixed", adg.ADG_MIXED, 0), ("mixed_dev", adg.ADG_MIXED_DEV, 0),
                             ("fp64_osher", adg.ADG_FP64, 1), ("mixed_osher", adg.ADG_MIXED, 1)):
        prob = adg.Problem(wl, precision=prec, flux=flux)
        if u0 is None:
            u0, _ = prob.project(wl.ic, 0)      # nodal values of the initial condition
        prob.set_state(u0)
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
        prob.profile(False)
        prob.profile(True)
        for _ in range(breakdown_steps):
            prob.step_cfl()
        prof = prob.profile_read()
        prob.profile(False)
        t_sim = prob.time
        u = prob.state()
        ue, _ = prob.project(lambda x, t: wl.ic(x, t_sim), 0)
        pred_avg_s = 1e-3 * pred_ms / max(1, pred_n)
        tflops = predictor_flops_per_cell(d, N) * wl.num_cells / pred_avg_s / 1e12
        forms[form] = {
            "value": st_dof_step * steps / elapsed,
            "ms_per_step": 1e3 * elapsed / steps,
            "predictor_avg_us": 1e6 * pred_avg_s,
            "predictor_tflops": tflops,
            "predictor_frac": tflops / (PEAK_FP64_TFLOPS if prec == adg.ADG_FP64 else PEAK_FP32_TFLOPS),
            "kernels": {g: {"ms_total": round(ms, 4), "launches": n, "avg_us": round(1e3 * ms / n, 3) if n else None}
                        for g, (ms, n) in prof.items()},
            "troubled_last_step": prob.stats()["troubled"],
            "t_simulated": t_sim,
            "l1_rho_vs_exact": l1_norm(u[0] - ue[0], wl),
        }
        finals[form] = u
        prob.close()
        print(f"# vortex {form}: {forms[form]['value']:.3e} st-dof/s, predictor {forms[form]['predictor_avg_us']:.1f} us",
              file=sys.stderr, flush=True)
    drho = np.abs(finals["mixed"][0] - finals["fp64"][0])
    return {
        "workload": f"isentropic vortex (Sec. 5), N={N}, {grid}x{grid} cells, periodic [0,10]^2, limiter on, "
                    f"CFL factor {wl.cfl}",
        "cells": wl.num_cells, "st_dof_per_step": st_dof_step, "steps": steps, "forms": forms,
        "speedup_mixed_vs_fp64": forms["mixed"]["value"] / forms["fp64"]["value"],
        "speedup_mixed_dev_vs_fp64": forms["mixed_dev"]["value"] / forms["fp64"]["value"],
        "speedup_mixed_vs_fp64_osher": forms["mixed_osher"]["value"] / forms["fp64_osher"]["value"],
        "rho_mixed_minus_fp64": {"max": float(drho.max()), "mean": float(drho.mean())},
        "l1_rho_vs_exact": {f: forms[f]["l1_rho_vs_exact"] for f in ("fp64", "mixed", "mixed_dev")},
        "memory_bound": face_bandwidth(wl, forms["mixed"]["kernels"]["faces"]["avg_us"]),
    }


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


def explosion3d_measurement(steps, warmup=2, breakdown=2, ncell=128, N=3, detect=True, pool_div=8, note=""):
    """The 3D explosion (cube [-1,1]^3, ncell^3 cells, degree N; by default its full size
    128^3 at N = 3): both precision forms stepped at the CFL time step from the initial data
    (nodal interpolant; with detect, the initial detection against the subcell-centre values,
    else the first step's detection finds the cells the sphere cuts), `warmup` untimed steps,
    then `steps` timed steps."""
    import torch
    from paper_1406_7416_amd import adg
    from paper_1406_7416_amd import workloads as W
    wl = W.explosion_3d(ncell, N)
    t0 = time.perf_counter()
    u0 = adg.project(wl, 0)[0]
    v0 = adg.project(wl, 1)[1] if detect else None
    t_init = time.perf_counter() - t0
    print(f"# explosion3d {ncell}^3 N={N}: initial data {t_init:.1f} s", file=sys.stderr, flush=True)
    st_dof = wl.st_dof_per_step()
    res = {"workload": f"3D explosion (Sec. 5), N={N}, {ncell}^3 cells on [-1,1]^3, transmissive, "
                       f"CFL factor {wl.cfl}, Ns={2 * N + 1}{note}",
           "cells": wl.num_cells, "st_dof_per_step": st_dof, "steps": steps, "warmup": warmup}
    for form, prec in (("fp64", adg.ADG_FP64), ("mixed", adg.ADG_MIXED)):
        prob = adg.Problem(wl, precision=prec, pool_capacity=wl.num_cells // pool_div)
        res["workspace_gb"] = prob.workspace_bytes / 1e9
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
            # against the published peak of the form's working precision (FP32 157.3, FP64 78.6 TFLOP/s)
            "predictor_frac": predictor_flops_per_cell(3, N) * wl.num_cells / pred_s / 1e12
                              / (157.3 if prec == adg.ADG_MIXED else 78.6),
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
        print(f"# explosion3d {ncell}^3 N={N} {form}: {res[form]['value']:.3e} st-dof/s, "
              f"{res[form]['ms_per_step']:.2f} ms/step, "
              f"troubled {res[form]['troubled_last_step']}", file=sys.stderr, flush=True)
    res["speedup_mixed_vs_fp64"] = res["mixed"]["value"] / res["fp64"]["value"]
    return res


def explosion3d_p9_measurement(steps=2, warmup=1, breakdown=1, cpu=False):
    """The 3D explosion at N = 9 (Sec. 5's P9 run: 10^4 space-time nodes per cell and
    variable, N_s = 19) on 50^3 cells: one eighth of the paper's 100^3-cell run, the share of
    one GPU of eight under a Cartesian split.  Both precision forms, from the nodal initial
    data with the initial detection against the subcell-centre values (at degree 9 the nodal
    interpolant of the discontinuity oscillates too strongly for P(u) to be a usable start of
    the subcell scheme in the cells the sphere cuts)."""
    res = explosion3d_measurement(steps, warmup=warmup, breakdown=breakdown, ncell=50, N=9, pool_div=4,
                                  note="; one eighth of the 100^3-cell P9 run (one GPU's share of eight)")
    if cpu:
        res["cpu_oracle"] = p9_oracle_sample()
    return res


def p9_oracle_sample(nw=5, origin=(35, 22, 22)):
    """The FP64 CPU oracle on a sample of the 50^3, N = 9 explosion: one step of an nw^3-cell
    window of the same grid cut on the sphere (same h and initial data, initial detection,
    transmissive sides), all host threads."""
    from oracle import oracle as O
    from paper_1406_7416_amd import workloads as W
    h = 2.0 / 50
    lo = tuple(-1.0 + i * h for i in origin)
    hi = tuple(l + nw * h for l in lo)
    bc = (W.BC.simple(W.TRANSMISSIVE), W.BC.simple(W.TRANSMISSIVE))
    ww = W.Workload("explosion3d-window", 3, 9, (nw,) * 3, lo, hi, [bc] * 3, W.explosion_ic(3))
    o = O.Oracle(ww)
    u, v = o.project(ww.ic, 0)[0], o.project(ww.ic, 1)[1]
    o.set_state(u, v)
    t0 = time.perf_counter()
    o.step(o.cfl_dt())
    el = time.perf_counter() - t0
    threads = O.get_threads()
    return {"value": ww.st_dof_per_step() / el, "unit": "st-dof/s", "cores": threads, "kind": "oracle",
            "sample": f"one step of a {nw}^3-cell window of the 50^3 grid on the sphere (cells {origin} on), "
                      f"{int(o.troubled().sum())} of {nw ** 3} cells troubled after it; {el:.1f} s, "
                      f"OpenMP threads={threads}"}


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


def _make_batch_problems(wls, prec, mood=False):
    from paper_1406_7416_amd import adg
    ps = []
    for wl in wls:
        cap = wl.num_cells if wl.num_cells <= 4096 else wl.num_cells // 3
        p = adg.Problem(wl, precision=prec, pool_capacity=cap, mood=mood)
        u, _ = p.project(wl.ic, 0)
        p.set_state(u)
        ps.append(p)
    return ps


def _free(*objs):
    import gc
    import torch
    for o in objs:
        if isinstance(o, list):
            for p in o:
                p.close()
        elif o is not None:
            o.close()
    gc.collect()
    torch.cuda.empty_cache()


def batch_measurement(wls, steps, warmup, fp64_forms=True):
    """The batch in the mixed form, batched: `warmup` untimed batch steps, then `steps` timed
    graph replays (the first call also takes one ordinary step per problem and captures).
    Then the same number of steps with the stages timed (HIP events at every stage boundary
    on the batch stream, the same launches enqueued directly): the per-stage times and the
    roofline of the dominant stage.  Then the plain FP64 form problem after problem
    (per-problem launches, no graph) and the FP64 form batched, and the mixed form batched
    with the MOOD layer of Sec. 6."""
    import numpy as np
    import torch
    from paper_1406_7416_amd import adg
    cfl = min(wl.cfl for wl in wls)
    st_dof = sum(wl.st_dof_per_step() for wl in wls)
    res = {"problems": len(wls), "cells": sum(wl.num_cells for wl in wls), "st_dof_per_step": st_dof,
           "steps": steps, "warmup": warmup, "cfl": cfl}

    def timed_batch(prec, mood=False, stages=True):
        ps = _make_batch_problems(wls, prec, mood)
        b = adg.Batch(ps)
        b.step_cfl(cfl, max(1, warmup))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step_cfl(cfl, steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        r = {"value": st_dof * steps / el, "ms_per_step": 1e3 * el / steps,
             "troubled_last_step": int(sum(int(p.troubled().sum()) for p in ps))}
        if stages:
            b.profile(True)
            b.step_cfl(cfl, steps)
            pr = b.profile_read()
            b.profile(False)
            launches = pr.pop("launches")
            nst = max(1, next(iter(pr.values()))[1])
            r["stages_ms_per_step"] = {g: ms / max(1, n) for g, (ms, n) in pr.items()}
            r["launch_ms"] = {f"{g}:N{cl[1]}": ms / nst for (g, cl), ms in launches.items()
                              if g in ("predictor", "subcell", "corrector_detect", "faces")}
            r["troubled_per_class"] = {}
            for p, wl in zip(ps, wls):
                key = f"N{wl.N}"
                r["troubled_per_class"][key] = r["troubled_per_class"].get(key, 0) + int(p.troubled().sum())
        if mood:
            fl = [p.mood_stats() for p in ps]
            r["flagged_subcells_last_step"] = int(sum(f for f, _ in fl))
            r["recomputed_cells_last_step"] = int(sum(x for _, x in fl))
        r["workspace_bytes"] = int(b.workspace_bytes + sum(p.workspace_bytes for p in ps))
        _free(b, ps)
        return r

    res["mixed_batched"] = timed_batch(adg.ADG_MIXED)
    res["roofline"] = batch_roofline(wls, res["mixed_batched"])
    print(f"# batch mixed: {res['mixed_batched']['value']:.3e} st-dof/s, "
          f"{res['mixed_batched']['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
    if fp64_forms:
        # the plain FP64 GPU form: per-problem launches, one problem after the other
        ps = _make_batch_problems(wls, adg.ADG_FP64)
        for p in ps:
            for _ in range(max(1, warmup)):
                p.step_cfl(cfl)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for p in ps:
            for _ in range(steps):
                p.step_cfl(cfl)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res["fp64_per_problem"] = {"value": st_dof * steps / el, "ms_per_step": 1e3 * el / steps}
        _free(ps)
        res["fp64_batched"] = timed_batch(adg.ADG_FP64)
        res["speedup"] = res["mixed_batched"]["value"] / res["fp64_per_problem"]["value"]
        res["speedup_vs_fp64_batched"] = res["mixed_batched"]["value"] / res["fp64_batched"]["value"]
        res["mixed_batched_mood"] = timed_batch(adg.ADG_MIXED, mood=True, stages=False)
        # the deviation form (FP32 carried as deviations from each cell's reference state)
        res["mixed_dev_batched"] = timed_batch(adg.ADG_MIXED_DEV, stages=False)
        print(f"# batch fp64 per problem {res['fp64_per_problem']['value']:.3e}, fp64 batched "
              f"{res['fp64_batched']['value']:.3e} st-dof/s", file=sys.stderr, flush=True)
    return res


def batch_roofline(wls, m):
    """Roofline of the dominant kernel of the mixed batched step: the launch (stage, degree
    class) with the largest time per step among the predictor and the subcell recompute,
    its algorithmic flops (predictor_flops_per_cell x the class's cells, or
    subcell_flops_per_cell x the class's troubled cells) over its average launch duration
    (HIP events around that launch on the batch stream, the timed steps of the profiled
    pass).  The other stage's rate is reported beside it."""
    lm = m["launch_ms"]
    cells = {}
    for wl in wls:
        cells[wl.N] = cells.get(wl.N, 0) + wl.num_cells
    troubled = {int(k[1:]): v for k, v in m["troubled_per_class"].items()}
    def flops(stage, N):
        if stage == "predictor":
            return predictor_flops_per_cell(2, N) * cells[N]
        return subcell_flops_per_cell(2, N) * troubled.get(N, 0)
    cand = [(k.split(":")[0], int(k.split(":N")[1])) for k in lm if k.startswith(("predictor:", "subcell:"))]
    stage, N = max(cand, key=lambda x: lm[f"{x[0]}:N{x[1]}"])
    dur_ms = lm[f"{stage}:N{N}"]
    f = flops(stage, N)
    achieved = f / (dur_ms * 1e-3) / 1e12
    tr = TRAFFIC.get(f"{stage}:N{N}")
    traffic = tr[0] if tr and tr[1] == kernel_source_hash() else None
    kern = {"predictor": f"kb_predictor<2, {N}, float> (FP32 space-time predictor + volume term + face traces, "
                         f"all {cells[N]} cells of degree {N})",
            "subcell": f"kb_subcell<2, {N}, float, false> (subcell ADER-WENO3 over the global worklist of the "
                       f"{troubled.get(N, 0)} troubled cells of degree {N})"}[stage]
    st = m["stages_ms_per_step"]
    pred_all = sum(flops("predictor", n) for n in cells)
    sub_all = sum(flops("subcell", n) for n in cells)
    return {
        "bound": "alu",
        "kernel": kern,
        "achieved": achieved,
        "peak": PEAK_FP32_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP32_TFLOPS,
        "frac_of_nonpacked_fp32": achieved / PEAK_FP32_NONPACKED_TFLOPS,
        "traffic": traffic,
        "traffic_unit": "HBM bytes per launch (calibrated rocprofv3 counters)",
        "flops_per_launch": f,
        "avg_launch_ms": dur_ms,
        "stage_rates_tflops": {"predictor": pred_all / (st["predictor"] * 1e-3) / 1e12,
                               "subcell": sub_all / (st["subcell"] * 1e-3) / 1e12},
    }


def cpu_baseline_leg(wls, cfl, budget_s, l1_steps=10):
    """The FP64 CPU oracle on the headline workload.

    Timing: the oracle as it stands, all host threads, whole steps of the batch's problems in
    order (one step per problem, from its initial data) until the time budget is used; the
    rate is the space-time dofs of those steps over their time.

    L1 density error against the oracle: a sample of the batch (up to three 32^2 problems of
    every degree and one 64^2 problem) stepped `l1_steps` times by the oracle and by both GPU
    forms with the oracle's time steps; L1(rho_gpu - rho_oracle) relative to L1(rho_oracle)
    per problem, worst over the sample."""
    import numpy as np
    from oracle import oracle as O
    from paper_1406_7416_amd import adg
    threads = O.get_threads()
    done, st_dof, el, t0 = 0, 0, 0.0, time.perf_counter()
    for wl in wls:
        o = O.Oracle(wl)
        u, _ = o.project(wl.ic, 0)
        o.set_state(u)
        t1 = time.perf_counter()
        o.step(o.cfl_dt(cfl))
        el += time.perf_counter() - t1
        st_dof += wl.st_dof_per_step()
        done += 1
        del o
        if el >= budget_s or time.perf_counter() - t0 >= 3 * budget_s:
            break
    cpu = {"value": st_dof / el, "unit": "st-dof/s", "cores": threads, "kind": "oracle",
           "sample": f"one step (time step + step, timed) of each of the first {done} problems of the batch, "
                     f"from their initial data; {el:.1f} s of stepping, OpenMP threads={threads}"}
    # L1 against the oracle on a sample
    idx, per_n = [], {}
    for i, wl in enumerate(wls):
        if wl.ncell[0] == 32 and per_n.get(wl.N, 0) < 3:
            per_n[wl.N] = per_n.get(wl.N, 0) + 1
            idx.append(i)
    idx.append(next(i for i, wl in enumerate(wls) if wl.ncell[0] == 64))
    worst = {"fp64": 0.0, "mixed": 0.0}
    per = []
    for i in idx:
        wl = wls[i]
        o = O.Oracle(wl)
        u, _ = o.project(wl.ic, 0)
        o.set_state(u)
        gs = {}
        for form, prec in (("fp64", adg.ADG_FP64), ("mixed", adg.ADG_MIXED)):
            g = adg.Problem(wl, precision=prec)
            g.set_state(u)
            gs[form] = g
        for _ in range(l1_steps):
            dt = o.cfl_dt(cfl)
            o.step(dt)
            for g in gs.values():
                g.step(dt)
        ro = o.state()[0]
        norm = l1_norm(ro, wl)
        row = {"problem": i, "grid": wl.ncell[0], "N": wl.N}
        for form, g in gs.items():
            e = l1_norm(g.state()[0] - ro, wl) / norm
            row[form] = e
            worst[form] = max(worst[form], e)
            g.close()
        per.append(row)
    l1 = {"steps": l1_steps, "sample": idx, "relative_l1_worst": worst, "per_problem": per,
          "tolerance_mixed": 1e-5, "tolerance_fp64": 1e-12,
          "within_tolerance": worst["mixed"] <= 1e-5 and worst["fp64"] <= 1e-12}
    print(f"# cpu oracle {cpu['value']:.3e} st-dof/s on {threads} threads; L1 vs oracle: fp64 {worst['fp64']:.2e}, "
          f"mixed {worst['mixed']:.2e}", file=sys.stderr, flush=True)
    return {"cpu_baseline": cpu, "l1_rho_vs_oracle": l1}


if __name__ == "__main__":
    main()
