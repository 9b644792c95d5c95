"""Offline sweep of the compile-time tile parameters (csrc/adg_tune.h) on the batch of
four-quadrant Riemann problems, writing the fastest values into tuning.json, which the
build turns into the header <adg_tuning.h>.

    python -m paper_1406_7416_amd.tune build   [--dir D]   # CPU: builds one library per variant
    python -m paper_1406_7416_amd.tune measure [--dir D]   # GPU: times every variant, writes tuning.json
    python -m paper_1406_7416_amd.tune choose              # re-derive the choice from the stored times

The parameters act on different stages of the step (predictor: pred_tb, pred_wps;
corrector + detection: corr_cpb; subcell recompute: sub_wps), every variant computes the
same step, and the batch's stage timing gives each (stage, class) launch its own time.  So
variant i takes option i of every parameter's list for every class at once, and each
parameter is then chosen per class from its own stage's times: five builds sweep five
options of every parameter.  A variant replaces the defaults only when it is faster by more
than the run-to-run spread of the stage times.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
DEFAULT_DIR = os.path.join(PKG, "_tune")          # the variant libraries (carried to the GPU)
OBJ_DIR = os.path.join(PKG, "_build", "tune")        # their objects (not)

# the classes of the benchmark's batch: d = 2, N = 3, 4, 5, both working precisions
CLASSES = [(2, N, prec) for N in (3, 4, 5) for prec in ("fp32", "fp64")]

# option i of every list goes into variant i (option 0: csrc/adg_tune.h's defaults)
PRED = {"fp32": [(256, 4), (128, 4), (512, 4), (256, 3), (256, 5)],
        "fp64": [(256, 2), (128, 2), (512, 2), (256, 1), (256, 3)]}
CORR_CPB = [4, 2, 1, 8, 4]          # 8 only where the workgroup's LDS allows it (N = 3)
SUB_WPS = {"fp32": [3, 2, 4, 3, 3], "fp64": [3, 2, 2, 3, 3]}
NVAR = 5
# a variant replaces the defaults (option 0) only when it is faster by more than the
# run-to-run spread of the stage times (about 2 %)
MARGIN = 1.03


def variant_table(i: int) -> dict:
    classes = {}
    for d, N, prec in CLASSES:
        tb, wps = PRED[prec][i]
        cpb = CORR_CPB[i] if (CORR_CPB[i] <= 4 or N <= 3) else 4
        classes[f"{d},{N},{prec}"] = {"pred_tb": tb, "pred_wps": wps, "corr_cpb": cpb, "sub_wps": SUB_WPS[prec][i]}
    return {"classes": classes}


def cmd_build(dirname: str) -> None:
    from paper_1406_7416_amd import build as B
    for i in range(NVAR):
        vd = os.path.join(dirname, f"v{i}")
        os.makedirs(vd, exist_ok=True)
        table = variant_table(i)
        with open(os.path.join(vd, "tuning.json"), "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        t0 = time.time()
        B.build_hip(tuning=table, out=os.path.join(vd, "libadg.so"), objdir=os.path.join(OBJ_DIR, f"v{i}"))
        print(f"variant {i} built in {time.time() - t0:.0f} s", flush=True)


def measure_variant(lib: str, steps: int = 5) -> dict:
    """Runs in a child process (one library per process): the batch in both forms, the
    stage timing of `steps` batch steps; returns {form: {"stage:N": ms per step}}."""
    import torch
    from paper_1406_7416_amd import adg
    from paper_1406_7416_amd import workloads as W
    adg.LIB_PATH = lib
    wls = W.quadrant_batch(256)
    cfl = min(wl.cfl for wl in wls)
    out = {}
    for form, prec in (("fp32", adg.ADG_MIXED), ("fp64", adg.ADG_FP64)):
        ps = []
        for wl in wls:
            p = adg.Problem(wl, precision=prec, pool_capacity=max(1024, wl.num_cells // 4))
            u, _ = p.project(wl.ic, 0)
            p.set_state(u)
            ps.append(p)
        b = adg.Batch(ps)
        b.step_cfl(cfl, 3)
        b.profile(True)
        b.step_cfl(cfl, steps)
        pr = b.profile_read()
        b.profile(False)
        out[form] = {f"{g}:N{cl[1]}": ms / steps for (g, cl), ms in pr["launches"].items()}
        b.close()
        for p in ps:
            p.close()
        del ps, b
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


def cmd_measure(dirname: str) -> None:
    times = []
    for i in range(NVAR):
        lib = os.path.join(dirname, f"v{i}", "libadg.so")
        print(f"variant {i}: {lib}", flush=True)
        r = subprocess.run([sys.executable, "-u", "-m", "paper_1406_7416_amd.tune", "_child", lib],
                           cwd=ROOT, capture_output=True, text=True, timeout=600)
        if r.returncode != 0:
            print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
            raise SystemExit(r.returncode)
        times.append(json.loads(r.stdout.strip().splitlines()[-1]))
        print("  " + " ".join(f"{k}={v:.2f}" for k, v in sorted(times[-1]["fp32"].items())
                               if k.split(":")[0] in ("predictor", "corrector_detect", "subcell")), flush=True)
    measured = {}
    for d, N, prec in CLASSES:
        key = f"{d},{N},{prec}"
        tables = [variant_table(i)["classes"][key] for i in range(NVAR)]
        for group, names in GROUPS:
            ms = [times[i][prec].get(f"{group}:N{N}", float("inf")) for i in range(NVAR)]
            measured[f"{key}:{group}"] = {"ms_per_step": [round(x, 4) for x in ms],
                                         "options": [[tables[i][n] for n in names] for i in range(NVAR)]}
    write_table(measured)


GROUPS = (("predictor", ("pred_tb", "pred_wps")), ("corrector_detect", ("corr_cpb",)), ("subcell", ("sub_wps",)))


def choose(measured: dict) -> dict:
    """Per class and parameter group: the fastest option, unless the defaults (option 0)
    are within MARGIN of it."""
    chosen = {}
    for key, m in measured.items():
        cls, group = key.rsplit(":", 1)
        ms = m["ms_per_step"]
        best = min(range(len(ms)), key=lambda i: ms[i])
        if ms[0] <= MARGIN * ms[best]:
            best = 0
        names = dict(GROUPS)[group]
        for name, val in zip(names, m["options"][best]):
            chosen.setdefault(cls, {})[name] = val
    return chosen


def write_table(measured: dict) -> None:
    table = {"classes": choose(measured),
             "measured": measured,
             "workload": "batch of 256 four-quadrant problems (d = 2, N = 3..5), stage times per batch step",
             "variants": NVAR, "margin": MARGIN}
    path = os.path.join(PKG, "tuning.json")
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(f"wrote {path}", flush=True)


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["build", "measure", "choose", "_child"])
    ap.add_argument("lib", nargs="?")
    ap.add_argument("--dir", default=DEFAULT_DIR)
    a = ap.parse_args()
    if a.cmd == "build":
        cmd_build(a.dir)
    elif a.cmd == "measure":
        cmd_measure(a.dir)
    elif a.cmd == "choose":
        # re-derive the chosen values from the times already in tuning.json
        with open(os.path.join(PKG, "tuning.json")) as f:
            write_table(json.load(f)["measured"])
    else:
        print(json.dumps(measure_variant(a.lib)), flush=True)


if __name__ == "__main__":
    main()
