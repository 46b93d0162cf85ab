"""Benchmark of the CCZ4 FD4 hot path on one MI355X.

A step is one classical RK4 step of the whole hot path over the single-puncture workload of
16^3 patches of 9^3 cells (144^3 = 2,985,984 cells on [-9,9]^3, Sommerfeld boundaries, 1+log
slicing, Gamma-driver): four times (halo fill, RHS = FD4 + CCZ4 algebra + KO, RK4 stage
combine), the last stage with the algebraic projection.  The metric is cell-updates per second
per RK4 stage: cells x 4 stages x steps / wall time, inputs resident in HBM.

Prints one JSON line.  --gpus N > 1 is not supported (the path runs on one GPU).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
RHS_BYTES_PER_CELL = 1888   # 2187 cell-vectors read (interior + face halos) / 729 + 1 written, 59 x 8 B each
STAGE_BYTES_PER_CELL = 2360  # RK4 stage: read Qn, k, acc; write acc, Q_next
FILL_BYTES_PER_CELL = 1888   # face halos: 1458 read + 1458 written per 729 cells


def run_gpu(args, w, precision):
    import torch
    from paper_2406_11626_amd import ccz4
    ctx = ccz4.Context(w.n0, w.origin, w.extent, w.bc, w.params(), w.refined)
    Q = ctx.new_state(0.0)
    ctx.init_patches(Q, w.scenario, w.scen)
    Qs, k, acc = ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0)
    dt = w.dt()
    stream = torch.cuda.current_stream()
    ev = {}

    def step(timed):
        cur = Q
        for s in range(4):
            ctx.fill_halos(cur)
            if timed:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            ctx.rhs(cur, k, precision)
            if timed:
                e1.record(stream)
                ev.setdefault("rhs", []).append((e0, e1))
            nxt = Q if s == 3 else Qs
            ctx.rk4_stage(s, dt, Q, k, acc, nxt)
            cur = nxt

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
        if args.progress:
            print(f"# step {i + 1}/{args.steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rhs_ms = sum(a.elapsed_time(b) for a, b in ev["rhs"]) / len(ev["rhs"])
    norms, st = ctx.constraints(Q, r_excise=1.0)
    cells = ctx.n_patches * 729
    out = dict(wall=wall, cells=cells, patches=ctx.n_patches, rhs_ms=rhs_ms, norms=norms, status=st)
    del Q, Qs, k, acc
    ctx.close()
    torch.cuda.empty_cache()
    return out


def cpu_baseline(w, target_s):
    """The oracle (single-threaded C, as it stands) on a bounded sample of the same workload:
    the full mesh is initialised and filled once (untimed), then one RK4 stage is timed on a
    sample of patches -- fill of the whole mesh and stage combine pro-rated to the sample."""
    import numpy as np
    import oracle as orc
    from paper_2406_11626_amd import ccz4
    m = orc.Mesh(w.n0, w.origin, w.extent, w.bc, w.refined)
    Q = m.zeros()
    m.init(Q, w.scenario, w.scen)
    pr = orc.Params(**{f: getattr(w.params(), f) for f, _ in ccz4.Params._fields_})
    t = time.perf_counter()
    m.fill_halos(Q)
    t_fill = time.perf_counter() - t
    # probe the RHS cost on 8 patches, then size the sample to ~target_s of work
    rng = np.random.default_rng(0)
    probe = sorted(rng.choice(m.np, 8, replace=False).tolist())
    k = np.zeros_like(Q)
    t = time.perf_counter()
    m.rhs(pr, Q, k, subset=probe)
    per_patch = (time.perf_counter() - t) / len(probe)
    n = int(min(m.np, max(8, target_s / max(per_patch, 1e-9))))
    sel = sorted(rng.choice(m.np, n, replace=False).tolist())
    t = time.perf_counter()
    m.rhs(pr, Q, k, subset=sel)
    t_rhs = time.perf_counter() - t
    acc, Qnext = np.zeros_like(Q), np.zeros_like(Q)
    t = time.perf_counter()
    m.rk4_stage(0, w.dt(), Q, k, acc, Qnext)
    t_stage = time.perf_counter() - t
    frac = n / m.np
    t_total = t_rhs + (t_fill + t_stage) * frac
    cells = n * 729
    return dict(value=cells / t_total, unit="cell-updates/s", cores=1, kind="oracle",
                sample=f"one RK4 stage (fill + RHS + stage) on {n} of {m.np} patches ({cells} cells) "
                       f"of the same workload; fill and stage pro-rated; {t_total:.1f} s of CPU work")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision run")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--progress", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs the hot path on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2406_11626_amd import scenarios
    assert torch.cuda.is_available(), "no GPU"
    w = scenarios.config(args.config)
    r64 = run_gpu(args, w, 0)
    stages = 4 * args.steps
    value = r64["cells"] * stages / r64["wall"]
    achieved = RHS_BYTES_PER_CELL * r64["cells"] / (r64["rhs_ms"] * 1e-3) / 1e9
    line = {
        "metric": "CCZ4 cell-updates/s per RK4 stage (FP64 vs mixed), % of FP64/HBM roofline",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["wall"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (analytic puncture initial data)",
        "config": {"workload": w.name, "patches": r64["patches"], "cells": r64["cells"],
                   "stages_per_step": 4, "dt": w.dt(), "precision": "fp64"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_rhs<double>",
                     "avg_ms": r64["rhs_ms"], "algorithmic_bytes_per_cell": RHS_BYTES_PER_CELL},
        "constraints_after": {"L2_H": r64["norms"][0], "L2_M": r64["norms"][1], "nonfinite": r64["norms"][2]},
    }
    if not args.no_mixed:
        rm = run_gpu(args, w, 1)
        line["mixed"] = {"value": rm["cells"] * stages / rm["wall"], "rhs_avg_ms": rm["rhs_ms"],
                         "speedup_vs_fp64": (rm["cells"] * stages / rm["wall"]) / value,
                         "L2_H": rm["norms"][0], "L2_M": rm["norms"][1]}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
