"""Benchmark: Euler-Maruyama path-steps per second of the Monte Carlo assembly
of G and b on one MI355X.

Workload (default): the variable-coefficient problem on [0,1]^2 with 8 x 8
subdomains, knot spacing 1/128 (1729 knots, 229,405 structural nonzeros),
N = 1e4 paths per knot, h = 1e-4, Gobet-Menozzi exits, float32 paths with
float64 accumulation of G and b.  One step = one full assembly (all paths of
all knots, CSR values and b written).  Inputs are formula-defined and resident
on the device before timing.

Prints one JSON line.  ``roofline`` reports the assembly kernel against the
VALU issue peak (the path is bound by plain ALU work: integer multiplies of
the counter-based generator, transcendentals, float32 arithmetic; HBM traffic
is a few MB per launch).  ``cpu_baseline`` is the float64 CPU oracle timed on
a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU issue peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one
# full-rate 32-bit lane operation per lane per clock).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# Algorithmic VALU work of one float32 path-step of each coefficient family,
# in full-rate lane-operation equivalents (quarter-rate transcendentals and
# 32x32->64-bit integer multiplies count 4).  Derivation in the design doc.
ALG_OPS_PER_STEP = {"varcoef": 149, "poisson": 108, "amplitude": 125, "lut": 132}
FP32_FLOP_PER_STEP = {"varcoef": 60, "poisson": 25, "amplitude": 40, "lut": 70}
FP32_PEAK_TFLOPS = 157.3


def _oracle_sample(args):
    """Worker: run the oracle on one knot and return its path-step count."""
    w, k = args
    from oracle.geometry import Geometry
    from oracle.coeffs import Coefficients
    from oracle.assemble import integrate_knot, exit_points, knot_row
    g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
    c = Coefficients(w["kind"], w.get("param", ()))
    rec = integrate_knot(g, c, k, w["n_paths"], w["h"], w["seed"], 0, w["exit_rule"])
    ex = exit_points(g, c, k, rec)
    knot_row(g, c, k, rec, ex)
    return int(rec["K"].sum())


def cpu_baseline(w, n_knots, workers):
    import multiprocessing as mp
    import numpy as np
    from paper_2301_05780_amd import pdd
    n = pdd.pattern(w)[0]
    knots = np.linspace(0, n - 1, n_knots).round().astype(int).tolist()
    t0 = time.perf_counter()
    if workers > 1:
        with mp.get_context("spawn").Pool(workers) as pool:
            steps = pool.map(_oracle_sample, [(w, k) for k in knots])
    else:
        steps = [_oracle_sample((w, k)) for k in knots]
    dt = time.perf_counter() - t0
    return dict(value=sum(steps) / dt, unit="path-steps/s", cores=workers, kind="oracle",
                sample=f"{n_knots} of {n} knots (evenly spaced), all {w['n_paths']} paths each, "
                       f"{sum(steps)} path-steps in {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="varcoef", choices=["varcoef", "poisson_small"])
    ap.add_argument("--exit-rule", default="gm", choices=["gm", "naive"])
    ap.add_argument("--cpu-knots", type=int, default=32)
    ap.add_argument("--cpu-workers", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the assembly shards by knot rows and "
              "this build runs on a single MI355X (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2301_05780_amd import pdd, workloads

    w = workloads.varcoef(args.exit_rule) if args.workload == "varcoef" else workloads.poisson_small(args.exit_rule)
    if args.workload == "poisson_small":
        w["precision"] = "fp32"
    ctx = pdd.Context(0)
    out = ctx.assemble(w)                     # allocates outputs, builds caches
    ctx.sync()
    for _ in range(args.warmup):
        ctx.assemble(w, out=out)
    ctx.sync()

    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.assemble(w, out=out)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern_ms, launches = ctx.kernel_ms()
    ctx.set_timing(False)

    diag = out["diag"].view(-1, pdd.DIAG_WIDTH)
    steps_per_launch = float(diag[:, 0].sum().item())
    paths = float(diag[:, 1].sum().item())
    value = steps_per_launch * args.steps / elapsed
    kavg = kern_ms / max(launches, 1) / 1e3
    ops = ALG_OPS_PER_STEP[w["kind"]]
    achieved = ops * steps_per_launch / kavg / 1e12
    grid, block, tickets = ctx.last_launch()

    rec = {
        "metric": "Euler-Maruyama path-steps/s building G,b",
        "value": value,
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 paths / f64 accumulation",
        "data": "synthetic (formula-defined manufactured BVP)",
        "config": {"workload": f"{w['name']}: {w['kind']} coefficients, {w['H']}x{w['H']} subdomains, "
                               f"knot spacing 1/{w['H'] * w['m']}, N={w['n_paths']}, h={w['h']}, "
                               f"{w['exit_rule']} exits",
                   "knots": int(out["n"]), "nnz": int(out["nnz"]), "paths": int(paths),
                   "path_steps_per_step": int(steps_per_launch),
                   "mean_steps_per_path": steps_per_launch / paths,
                   "launch": {"grid": grid, "block": block, "tickets": tickets}},
        "kernel_ms_avg": kavg * 1e3,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                     "ops_per_path_step": ops,
                     "fp32_flop_frac": FP32_FLOP_PER_STEP[w["kind"]] * steps_per_launch / kavg / 1e12
                     / FP32_PEAK_TFLOPS},
    }
    ctx.close()
    if not args.no_cpu_baseline:
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        rec["cpu_baseline"] = cpu_baseline(w, args.cpu_knots, workers)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
