"""Benchmark of the CCZ4 FD4 hot path on one MI355X.

A step is one classical RK4 step of the whole hot path over the largest single-GPU workload by
default: the single puncture on 24^3 patches of 9^3 cells (216^3 = 10,077,696 cells on [-9,9]^3,
Sommerfeld boundaries, 1+log slicing, Gamma-driver; six state-sized buffers of 23.5 GB).  The
step is four fused stages (FD4 derivatives + CCZ4 algebra + Kreiss-Oliger + RK4 stage combine,
the last stage with the algebraic projection) captured in one HIP graph; each stage also writes
the same-level face halos its successor needs, so on a uniform mesh no fill kernel runs between
stages.  The metric is cell-updates per second per RK4 stage: cells x 4 stages x steps / wall
time, with the state resident in HBM.

Beside the FP64 graph step (the headline `value`) the line carries: the mixed-precision step and
its state error against the FP64 step after the same number of steps (the FP64 GPU step is held
to the oracle by the parity tests), the constraint norms of both after at least 50 steps (every leg
runs the same number), the plain unfused path (halo fill, right-hand side, RK4 stage as three
calls per stage) timed on the same workload, the standalone right-hand-side kernel, and the oracle
on the host cores.

The roofline object is the fused stage kernel's: 3304 algorithmic bytes per cell-stage (every
evolved slot with its three-cell face halos read once, Q^n and the accumulator read, the
accumulator and Q_next written) over its average launch time, taken with events on the launch
stream; the halo copies and Sommerfeld ghost updates the launch also does are reported apart.

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
FP64_PEAK_TFLOPS = 78.6
NV = 59
# Algorithmic bytes per interior cell: fused stage (the evolved slots over interior and face halos,
# 3 x 472, plus Q^n and the accumulator read, 2 x 472, plus the accumulator and Q_next written,
# 2 x 472) and standalone right-hand side (3 x 472 read, 472 written).
FUSED_BYTES_PER_CELL = 3304
RHS_BYTES_PER_CELL_MODEL = 1888
METRIC = "CCZ4 cell-updates/s per RK4 stage (FP64 vs mixed), % of FP64/HBM roofline"
# Fused stage, bytes per interior cell.  Q_s: the 58 evolved slots with interior + face halos
# (2187 cell-vectors per 729 cells) and K_0 pointwise.  Streamed, per stage s:
#   s = 0: read Q_n, write acc, write Q_next;  s = 1, 2: read/write acc, read Q_n, write Q_next;
#   s = 3: read acc, write Q_next.
QS_BYTES_PER_CELL = 8 * (58 * 3 + 1)
STREAM_BYTES_PER_CELL = {0: 3 * 8 * NV, 1: 4 * 8 * NV, 2: 4 * 8 * NV, 3: 2 * 8 * NV}


HALO_BYTES_PER_FACE = 243 * NV * 8   # a same-level face halo written by the stage
# Sommerfeld ghost update of the stage, cell-vectors per ghost cell (243 per boundary face): the
# three ghost layers and the interior layer beside them (4 per 3 ghost cells) and the background
# read; Q_n read (s < 3), acc read (s > 0), acc written (s < 3), Q_next written.
GHOST_VECTORS = {0: 4.0 / 3 + 4, 1: 4.0 / 3 + 5, 2: 4.0 / 3 + 5, 3: 4.0 / 3 + 3}


def stage_bytes_per_cell(s):
    return QS_BYTES_PER_CELL + STREAM_BYTES_PER_CELL[s]


# Standalone right-hand side with every cell-vector read once (no halo duplication) and k written:
# the ideal lower bound beside the 1888 B per cell of its roofline (the Sommerfeld ghosts' right-hand
# side, which its slab work-groups also compute, is counted in neither)
RHS_IDEAL_BYTES_PER_CELL = 2 * 8 * NV


def stage_bytes(s, cells, pushed_faces, ghost_faces=0):
    """Algorithmic bytes of one fused stage call with pushed_faces same-level face halos written
    (a stage that reads some same-level halos from the neighbours reads the same cell-vectors as
    one that reads its own halos) and ghost_faces Sommerfeld faces updated."""
    return (stage_bytes_per_cell(s) * cells + HALO_BYTES_PER_FACE * pushed_faces +
            GHOST_VECTORS[s] * 8 * NV * 243 * ghost_faces)


def same_level_faces_per_axis(ctx):
    """Number of leaf faces per axis whose neighbour across the face is a leaf of the same level
    (each counted from both sides), from the context's leaf table (level, i, j, k)."""
    from paper_2406_11626_amd import ccz4
    ids = [tuple(int(v) for v in r) for r in ctx.ids]
    leaves = set(ids)
    count = [0, 0, 0]
    for lev, *c in ids:
        n = [v * 3 ** lev for v in ctx.n0]
        for a in range(3):
            for d in (-1, 1):
                q = list(c)
                q[a] += d
                if ctx.bc == ccz4.BC_PERIODIC:
                    q[a] %= n[a]
                elif not 0 <= q[a] < n[a]:
                    continue
                count[a] += (lev, *q) in leaves
    return count


# workload tags of the committed counter summaries (profiles/<kernel>_<tag>_<what>.md)
WORKLOAD_TAG = {2: "puncture16", 3: "puncture_static3", 4: "puncture24", 5: "bbh_amr4"}


def traffic_file(config):
    return os.path.join(ROOT, "profiles", f"k_stage_lds_{WORKLOAD_TAG.get(config, config)}_hbm_traffic.md")


def flops_file(config):
    return os.path.join(ROOT, "profiles", f"k_stage_lds_{WORKLOAD_TAG.get(config, config)}_fp64_ops.md")


def kernel_source_digest():
    """sha256 over the HIP sources that the stencil kernels and their launches are built from (the
    traffic figure is void once they change); the learned indicator's sources (ccz4_mlp.*) take no
    part in them."""
    import hashlib
    d = os.path.join(ROOT, "paper_2406_11626_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".hpp", ".cpp")) and not name.startswith("ccz4_mlp"):
            with open(os.path.join(d, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def _profile_record(path, config):
    """The "- key: value" lines of a committed counter summary, or None when there is none, when it
covers another workload, or when the kernel sources have changed since the counters were taken."""
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for ln in f:
            if ln.startswith("- ") and ":" in ln:
                k, v = ln[2:].split(":", 1)
                rec[k.strip()] = v.strip().strip("`")
    if rec.get("source_sha256") != kernel_source_digest() or rec.get("workload_config") != str(config):
        return None
    return rec


def _record_float(rec, key):
    try:
        return float(rec[key]) if rec is not None else None
    except (KeyError, ValueError):
        return None


def measured_traffic(config, key="hbm_bytes_per_launch"):
    """HBM bytes per launch of the fused stage kernel (or, with key hbm_bytes_per_rhs_launch, of the
    standalone right-hand side) from the committed counter summary."""
    return _record_float(_profile_record(traffic_file(config), config), key)


def measured_fp64_ops(config):
    """FP64 operations per launch of the fused stage kernel and of the standalone right-hand side
    (64 lanes x (ADD + MUL + 2 FMA + TRANS) wave instructions) from the committed counter summary."""
    rec = _profile_record(flops_file(config), config)
    return _record_float(rec, "fp64_ops_per_stage_launch"), _record_float(rec, "fp64_ops_per_rhs_launch")


def fp64_rate(ops, avg_ms):
    """Achieved FP64 rate of a kernel from its counted operations per launch and its live average
    launch duration, against the FP64 vector peak; None without a valid counter summary."""
    if ops is None or not avg_ms:
        return None
    t = ops / (avg_ms * 1e-3) / 1e12
    return {"ops_per_launch": ops, "achieved": t, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": t / FP64_PEAK_TFLOPS}


def copy_bandwidth(nbytes=2**30, reps=10):
    """Measured device-to-device copy rate in GB/s (read + write bytes per second) of a plain torch
    copy of nbytes, the practical reference beside the spec peak."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def _say(msg):
    print("# " + msg, file=sys.stderr, flush=True)


def run_gpu(args, w, precision, formulation=0, advection=0, total_steps=0, keep=False, rhs=True):
    """One leg of the benchmark: the fused step on workload w, eager (events per stage launch)
    and as the captured graph (the timed value), then untimed graph steps up to total_steps steps
    since the initial data; constraint norms at t = 0 and at the end.  keep: also return the final
    state (the caller frees it)."""
    import torch
    from paper_2406_11626_amd import ccz4
    prm = ccz4.params(**{**w.prm, "formulation": formulation, "advection": advection})
    ctx = ccz4.Context(w.n0, w.origin, w.extent, w.bc, prm, w.refined)
    so = ctx.second_order
    Q = ctx.new_state(0.0)
    ctx.init_patches(Q, w.scenario, w.scen)
    dt = w.dt()
    stream = torch.cuda.current_stream()
    rest = ccz4.FILL_NEUMANN | ccz4.FILL_LEVELS
    events, recon_events = [], []
    ctx.fill_halos(Q, stream)
    if so:  # the auxiliaries of the initial data from its primaries
        ctx.reconstruct(Q, True, stream)
        ctx.fill_halos(Q, stream)
    norms0, _ = ctx.constraints(Q, r_excise=1.0)
    tune_ms = None
    if args.autotune:
        ms = ctx.autotune(Q, precision, reps=2)
        tune_ms = {"chosen": ccz4.kernel_config_name(ctx.get_kernel(precision)),
                   "ms": {ccz4.kernel_config_name(k): t for k, t in enumerate(ms)}}
    ctx.fill_halos(Q, stream)
    # the work buffers: a pool of five, the rotation with the fastest steps kept (the placement of
    # the buffers in physical memory moves a step by up to 8%); the trial steps advance Q
    done = 0
    place = None
    if args.place:
        (Q1, Q2, acc), pms = ctx.tune_step_buffers(Q, dt, precision, pool=5, steps=2, stream=stream)
        done += 10
        place = {"pool": 5, "steps_per_trial": 2, "ms_per_step": [round(x, 2) for x in pms],
                 "chosen": int(min(range(5), key=lambda i: pms[i]))}
    else:
        Q1, Q2, acc = ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0)
    order = ((Q, Q1), (Q1, Q2), (Q2, Q1), (Q1, Q))

    def step(timed):
        for s, (src, dst) in enumerate(order):
            if s > 0:
                ctx.fill_halos_kinds(src, rest, stream)
            if timed:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            fl = ctx.step_stage_flags(s, precision)
            ctx.rhs_rk4_stage(s, dt, src, Q, acc, dst, precision, fl, stream)
            if timed:
                e1.record(stream)
                events.append((s, e0, e1, fl))
            if so:
                ctx.fill_halos_kinds(dst, rest, stream)
                if timed:
                    r0 = torch.cuda.Event(enable_timing=True)
                    r1 = torch.cuda.Event(enable_timing=True)
                    r0.record(stream)
                ctx.reconstruct(dst, stream=stream, flags=fl)
                if timed:
                    r1.record(stream)
                    recon_events.append((r0, r1))
        ctx.fill_halos_kinds(Q, rest, stream)

    for _ in range(args.warmup):
        step(False)
        done += 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
        done += 1
        if args.progress:
            _say(f"step {i + 1}/{args.steps}")
    torch.cuda.synchronize()
    wall_eager = time.perf_counter() - t0
    # the same step captured once as a HIP graph and replayed (the production path)
    graph = ctx.step_graph(Q, (Q1, Q2, acc), dt, precision)
    for _ in range(args.warmup):
        graph.launch(stream)
        done += 1
    torch.cuda.synchronize()
    # the timed steps in up to five equal repetitions, each bracketed by events on the launch stream
    nrep = min(5, args.steps)
    bounds = [round(r * args.steps / nrep) for r in range(nrep + 1)]
    marks = {b: torch.cuda.Event(enable_timing=True) for b in bounds}
    t0 = time.perf_counter()
    marks[0].record(stream)
    for i in range(args.steps):
        graph.launch(stream)
        done += 1
        if i + 1 in marks:
            marks[i + 1].record(stream)
        if args.progress:
            _say(f"graph step {i + 1}/{args.steps}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rep_ms = [marks[b0].elapsed_time(marks[b1]) / (b1 - b0) for b0, b1 in zip(bounds, bounds[1:]) if b1 > b0]
    while done < total_steps:  # untimed, up to the drift horizon
        graph.launch(stream)
        done += 1
        if done % 10 == 0:
            torch.cuda.synchronize()
            _say(f"step {done}/{total_steps}")
    torch.cuda.synchronize()
    graph.close()
    cells = ctx.n_patches * 729
    faces = same_level_faces_per_axis(ctx)
    assert sum(faces) == ctx.plan_counts()["same_level"]

    def pushed(fl):
        return sum(faces) if fl & ccz4.STAGE_FILL_SAME_LEVEL else (
            faces[0] if fl & ccz4.STAGE_FILL_SAME_LEVEL_X else 0)
    # the standalone right-hand side on the final state (its own kernel, same launch configuration)
    rhs_ms = None
    if rhs and precision == ccz4.PREC_FP64 and not so:
        del Q1
        kbuf = ctx.new_state(0.0)
        ctx.rhs(Q, kbuf, precision, stream)
        r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        r0.record(stream)
        for _ in range(5):
            ctx.rhs(Q, kbuf, precision, stream)
        r1.record(stream)
        torch.cuda.synchronize()
        rhs_ms = r0.elapsed_time(r1) / 5
        del kbuf
        Q1 = None
    stage_ms = [a.elapsed_time(b) for _, a, b, _ in events]
    nbf = ctx.plan_counts()["sommerfeld"]
    launch_bytes = [stage_bytes(s, cells, pushed(fl), nbf) for s, _, _, fl in events]
    halo_bytes = [HALO_BYTES_PER_FACE * pushed(fl) for s, _, _, fl in events]
    ghost_bytes = [GHOST_VECTORS[s] * 8 * NV * 243 * nbf for s, _, _, fl in events]
    norms, st = ctx.constraints(Q, r_excise=1.0)
    monitor = None
    if rhs and precision == ccz4.PREC_FP64 and not so:
        # the other calls of the path on the final state, each timed with events on the stream:
        # the constraint monitor (norms only), the plain refinement criterion (its indicator
        # evaluates the constraints too) and the initial data (into the spent Q2)
        tags = torch.empty(ctx.n_patches, dtype=torch.int8, device="cuda")

        def timed(fn, reps=5):
            fn()
            ts = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                fn()
                b.record(stream)
                torch.cuda.synchronize()
                ts.append(a.elapsed_time(b))
            return sorted(ts)[len(ts) // 2]
        monitor = {"constraints_ms": timed(lambda: ctx.constraints(Q, None, 1.0, stream)),
                   "tag_refine_ms": timed(lambda: ctx.tag_refine(Q, 1e300, -1.0, 2, tags, stream=stream)),
                   "init_patches_ms": timed(lambda: ctx.init_patches(Q2, w.scenario, w.scen, stream)),
                   "cells": ctx.n_patches * 729, "timing": "median of 5 calls, HIP events on the stream"}
        del tags
    kc = ctx.get_kernel(precision)
    targs = ("<double, " if precision == ccz4.PREC_FP64 else "<float, ") + ("1>" if advection else "0>")
    border = " (" + ccz4.kernel_config_name(kc).split("/", 1)[1] + ")"
    # the kernels one stage call (one right-hand-side call) launches
    kname = ("k_stage_lds" if kc & ccz4.KERNEL_LDS else "k_stage") + targs + border
    rname = ("k_rhs_lds" if kc & ccz4.KERNEL_LDS else "k_rhs") + targs + border + \
        (" + k_rhs_sommerfeld" if nbf and not kc & ccz4.KERNEL_LDS else "")
    recon_ms = [a.elapsed_time(b) for a, b in recon_events]
    avg = lambda v: sum(v) / len(v)  # noqa: E731
    out = dict(wall=wall, wall_eager=wall_eager, rep_ms=rep_ms, tune_ms=tune_ms, monitor=monitor, place=place, cells=cells, patches=ctx.n_patches, rhs_ms=rhs_ms,
               reconstruct_ms=avg(recon_ms) if recon_ms else None, stage_ms=avg(stage_ms),
               stage_ms_by_s=[avg([t for (s, _, _, _), t in zip(events, stage_ms) if s == q]) for q in range(4)],
               stage_bytes=avg(launch_bytes), halo_bytes=avg(halo_bytes), ghost_bytes=avg(ghost_bytes),
               stage_gbs=sum(launch_bytes) / (sum(stage_ms) * 1e-3) / 1e9, norms=norms, norms0=norms0, status=st,
               kernel=kname, rhs_kernel=rname, ghost_faces=nbf, steps_total=done, dt=dt)
    if keep:
        out["Q"] = Q
    del Q, Q2, acc
    ctx.close()
    torch.cuda.empty_cache()
    return out


def run_plain(args, w, total_steps=0, keep=False):
    """The plain, unfused FP64 path on workload w: per stage a full halo fill, the right-hand side
    into a state-sized k, and the RK4 stage combine (three calls, each its own launch), with
    events per call; total_steps as in run_gpu."""
    import torch
    from paper_2406_11626_amd import ccz4
    ctx = ccz4.Context(w.n0, w.origin, w.extent, w.bc, w.params(), w.refined)
    Q = ctx.new_state(0.0)
    ctx.init_patches(Q, w.scenario, w.scen)
    dt = w.dt()
    stream = torch.cuda.current_stream()
    ev = {"fill": [], "rhs": [], "rk4_stage": []}
    done = 0

    def plain_step(Qs, k, acc):
        cur = Q
        for s in range(4):
            nxt = Q if s == 3 else Qs
            ctx.fill_halos(cur, stream)
            ctx.rhs(cur, k, ccz4.PREC_FP64, stream)
            ctx.rk4_stage(s, dt, Q, k, acc, nxt, stream)
            cur = nxt
    # the work buffers chosen from a pool of five as for the fused path (same rule, same cost)
    place = None
    if args.place:
        pool = [ctx.new_state(0.0) for _ in range(5)]
        pms = []
        for i in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(2):
                plain_step(pool[i], pool[(i + 1) % 5], pool[(i + 2) % 5])
            e1.record(stream)
            e1.synchronize()
            pms.append(e0.elapsed_time(e1) / 2)
        done += 10
        b = min(range(5), key=lambda i: pms[i])
        Qs, k, acc = pool[b], pool[(b + 1) % 5], pool[(b + 2) % 5]
        del pool
        place = {"pool": 5, "steps_per_trial": 2, "ms_per_step": [round(x, 2) for x in pms], "chosen": b}
    else:
        Qs, k, acc = ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0)

    def timed(name, fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        ev[name].append((e0, e1))

    def step(with_events):
        cur = Q
        for s in range(4):
            nxt = Q if s == 3 else Qs
            if with_events:
                timed("fill", lambda: ctx.fill_halos(cur, stream))
                timed("rhs", lambda: ctx.rhs(cur, k, ccz4.PREC_FP64, stream))
                timed("rk4_stage", lambda: ctx.rk4_stage(s, dt, Q, k, acc, nxt, stream))
            else:
                ctx.fill_halos(cur, stream)
                ctx.rhs(cur, k, ccz4.PREC_FP64, stream)
                ctx.rk4_stage(s, dt, Q, k, acc, nxt, stream)
            cur = nxt

    for _ in range(args.warmup):
        step(False)
        done += 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(False)
        done += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step(True)  # one more step with events per call
    done += 1
    while done < total_steps:
        step(False)
        done += 1
        if done % 10 == 0:
            torch.cuda.synchronize()
            _say(f"plain step {done}/{total_steps}")
    torch.cuda.synchronize()
    ctx.fill_halos(Q, stream)
    norms, _ = ctx.constraints(Q, r_excise=1.0)
    ms = {n: sum(a.elapsed_time(b) for a, b in v) / len(v) for n, v in ev.items()}
    out = dict(wall=wall, cells=ctx.n_patches * 729, norms=norms, steps_total=done, call_ms=ms, place=place)
    if keep:
        out["Q"] = Q
    del Q, Qs, k, acc
    ctx.close()
    torch.cuda.empty_cache()
    return out


def state_error(Qa, Qb, chunk=256):
    """Per-slot error of state Qa against Qb over the interior cells: max|a - b| / max|b| for slots
    above 1e-10 of the largest slot, max|a - b| / (largest slot) for the others (the parity
    measure of the tests).  Returns (per-slot list, largest value, its slot)."""
    import torch
    n = Qa.shape[0]
    diff = torch.zeros(NV, dtype=torch.float64, device=Qa.device)
    scale = torch.zeros(NV, dtype=torch.float64, device=Qa.device)
    for p0 in range(0, n, chunk):
        a = Qa[p0:p0 + chunk, :, 3:12, 3:12, 3:12]
        b = Qb[p0:p0 + chunk, :, 3:12, 3:12, 3:12]
        diff = torch.maximum(diff, (a - b).abs().amax(dim=(0, 2, 3, 4)))
        scale = torch.maximum(scale, b.abs().amax(dim=(0, 2, 3, 4)))
    diff, scale = diff.cpu().tolist(), scale.cpu().tolist()
    top = max(max(scale), 1e-300)
    e = [d / (sc if sc > 1e-10 * top else top) for d, sc in zip(diff, scale)]
    k = max(range(NV), key=lambda i: e[i])
    return e, e[k], k


def run_stability(args, w):
    """First- against second-order formulation on the same workload (or, with
    --stability-transfer, the second-order formulation with the App. E against the higher-order
    coarse-fine operators), graph-launched steps until t_end or the first non-finite value: L2
    norms of the constraints (cells with r >= 1) every sample_dt."""
    import torch
    from paper_2406_11626_amd import ccz4
    dt = w.dt()
    nsteps = int(round(args.t_end / dt))
    every = max(1, int(round(args.sample_dt / dt)))
    out = {}
    if args.stability_transfer:  # second order with the App. E and the higher-order operators
        variants = ((dict(formulation=1, transfer=0), "second_order_app_e_transfer"),
                    (dict(formulation=1, transfer=1), "second_order_higher_order_transfer"))
    else:
        variants = ((dict(formulation=0), "first_order"), (dict(formulation=1), "second_order"))
    for over, name in variants:
        form = over["formulation"]
        prm = ccz4.params(**{**w.prm, **over})
        ctx = ccz4.Context(w.n0, w.origin, w.extent, w.bc, prm, w.refined)
        Q = ctx.new_state(0.0)
        ctx.init_patches(Q, w.scenario, w.scen)
        ctx.fill_halos(Q)
        if form:
            ctx.reconstruct(Q)
            ctx.fill_halos(Q)
        bufs = (ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0))
        graph = ctx.step_graph(Q, bufs, dt)
        hist = []
        n0, _ = ctx.constraints(Q, r_excise=1.0)
        hist.append((0.0, n0[0], n0[1], n0[2]))
        t0 = time.perf_counter()
        for i in range(1, nsteps + 1):
            graph.launch()
            if i % every == 0 or i == nsteps:
                norms, _ = ctx.constraints(Q, r_excise=1.0)
                hist.append((i * dt, norms[0], norms[1], norms[2]))
                print(f"# {name} t = {i * dt:.3f}: L2(H) = {norms[0]:.3e}, L2(M) = {norms[1]:.3e}, "
                      f"non-finite = {norms[2]:.0f}", file=sys.stderr, flush=True)
                if norms[2] > 0 or not all(map(lambda v: v == v, norms[:2])):
                    break
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        graph.close()
        out[name] = dict(history=[dict(t=t, L2_H=h, L2_M=m, nonfinite=nf) for t, h, m, nf in hist],
                         t_reached=hist[-1][0], finite=hist[-1][3] == 0, wall_s=wall)
        del Q, bufs
        ctx.close()
        torch.cuda.empty_cache()
    return out


def run_tracker(args):
    """Puncture trackers (tracers moved by -beta with explicit Euler, one step per RK4 step) in the
    binary-puncture data, second-order formulation, graph-launched steps up to t_end; the tracker
    positions and the count of non-finite cells every sample_dt."""
    import torch
    from paper_2406_11626_amd import ccz4, scenarios
    w = scenarios.binary_tracking()
    prm = ccz4.params(**{**w.prm, "formulation": ccz4.FORMULATION_SO})
    ctx = ccz4.Context(w.n0, w.origin, w.extent, w.bc, prm, w.refined)
    Q = ctx.new_state(0.0)
    ctx.init_patches(Q, w.scenario, w.scen)
    ctx.fill_halos(Q)
    ctx.reconstruct(Q)
    ctx.fill_halos(Q)
    bufs = (ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0))
    dt = w.dt()
    graph = ctx.step_graph(Q, bufs, dt)
    pos = torch.tensor([[3.0, 0.0, 0.0], [-3.0, 0.0, 0.0]], dtype=torch.float64, device="cuda")
    nsteps = int(round(args.t_end / dt))
    every = max(1, int(round(args.sample_dt / dt)))
    track = [dict(t=0.0, pos=pos.cpu().numpy().tolist(), nonfinite=0.0)]
    t0 = time.perf_counter()
    for i in range(1, nsteps + 1):
        graph.launch()
        ctx.tracers_advance(Q, pos, dt)
        if i % every == 0 or i == nsteps:
            norms, _ = ctx.constraints(Q)
            p = pos.cpu().numpy()
            track.append(dict(t=i * dt, pos=p.tolist(), nonfinite=norms[2]))
            print(f"# t = {i * dt:.2f}: trackers {p[0].round(4).tolist()} {p[1].round(4).tolist()}, "
                  f"non-finite = {norms[2]:.0f}", file=sys.stderr, flush=True)
            if norms[2] > 0:
                break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    graph.close()
    return dict(workload=w.name, leaves=ctx.n_patches, dt=dt, formulation="second order", t_end=args.t_end,
                wall_s=wall, ms_per_step=wall * 1e3 / max(1, i), track=track)


def _bbh_training_runs(args, names, theta=None, max_level=2):
    """Second-order binary-puncture runs on the static r = 2 refinement (the tracker workload) to
    t_end, with snapshots of the leaf features and the plain tags every sample_dt; the Bowen-York
    momenta scaled per run.  The plain tags use the thresholds theta (default: the 99th and 30th
    percentiles of the first run's indicator at t = 0) and max_level.  Returns {name: (ctx,
    snapshots, norms)} and the thresholds."""
    import numpy as np
    import torch
    from paper_2406_11626_amd import ccz4, learned, scenarios
    w = scenarios.binary_tracking()
    prm = ccz4.params(**{**w.prm, "formulation": ccz4.FORMULATION_SO})
    dt = w.dt()
    steps = int(round(args.t_end / dt))
    every = max(1, int(round(args.sample_dt / dt)))
    theta = None
    runs = {}
    for name, scale in names:
        scen = list(w.scen)
        scen[5] *= scale   # y momentum of the puncture at +x
        scen[12] *= scale  # and of the one at -x
        ctx = ccz4.Context(w.n0, w.origin, w.extent, w.bc, prm, w.refined)
        Q = ctx.new_state(0.0)
        ctx.init_patches(Q, w.scenario, scen)
        ctx.fill_halos(Q)
        ctx.reconstruct(Q)
        ctx.fill_halos(Q)
        if theta is None:  # thresholds from the first run's indicator at t = 0, kept for all runs
            ind = torch.empty((ctx.n_patches, 3), dtype=torch.float64, device="cuda")
            tags = torch.empty(ctx.n_patches, dtype=torch.int8, device="cuda")
            ctx.tag_refine(Q, 1e300, -1.0, max_level, tags, ind)
            e = ind.max(dim=1).values.cpu().numpy()
            theta = (float(np.percentile(e, 99.0)), float(np.percentile(e, 30.0)))
        snaps = learned.snapshots(ctx, Q, dt, steps, every, theta[0], theta[1], max_level)
        norms, _ = ctx.constraints(Q)
        del Q
        runs[name] = (ctx, snaps, norms)
        _say(f"{name}: {len(snaps)} snapshots, REFINE per snapshot {[int((t == 1).sum()) for _, t in snaps]}, "
             f"non-finite {norms[2]:.0f}")
    return runs, theta, w, dt, every


def _train_on(runs, names, args):
    import torch
    from paper_2406_11626_amd import learned
    feats, targets = [], []
    for name in names:
        snaps = runs[name][1]
        for k in range(len(snaps) - 1):
            feats.append(snaps[k][0])
            targets.append(snaps[k + 1][1])
    feat = torch.cat(feats)
    target = torch.cat(targets)
    ind = learned.LearnedIndicator(seed=0)
    ind.fit_normalisation(feat)
    t1 = time.perf_counter()
    loss0 = ind.train(feat, target, 0)
    loss = ind.train(feat, target, args.train_iters)
    torch.cuda.synchronize()
    return ind, dict(training_rows=int(feat.shape[0]), train_iters=args.train_iters, loss_before=loss0,
                     loss_after=loss, train_s=time.perf_counter() - t1)


def train_bbh_indicator(args, theta=None, max_level=2):
    """The indicator trained on two second-order binary-puncture runs (momenta x0.9 and x1.1),
    features of snapshot k against the plain tags of snapshot k + 1 (thresholds theta, max_level
    as the workload it will serve uses them)."""
    names = (("train_0.9", 0.9), ("train_1.1", 1.1))
    t0 = time.perf_counter()
    runs, theta, w, dt, every = _bbh_training_runs(args, names, theta, max_level)
    sim_s = time.perf_counter() - t0
    ind, info = _train_on(runs, [n for n, _ in names], args)
    for ctx, _, _ in runs.values():
        ctx.close()
    return ind, dict(info, workload=w.name + ", second-order formulation", t_end=args.t_end,
                     sample_dt=every * dt, simulation_s=sim_s)


def train_mesh_indicator(args, w, theta, max_level, scales=(0.9, 1.1), steps=60, every=10):
    """The indicator trained on runs of workload w's own mesh and formulation with the Bowen-York
    momenta scaled (the workload's own momenta held out): features every `every` steps (the regrid
    interval) against the plain tags (thresholds theta) `every` steps later."""
    import torch
    from paper_2406_11626_amd import ccz4, learned
    t0 = time.perf_counter()
    runs = {}
    for scale in scales:
        scen = list(w.scen)
        scen[5] *= scale   # y momentum of the puncture at +x
        scen[12] *= scale  # and of the one at -x
        ctx = ccz4.Context(w.n0, w.origin, w.extent, w.bc, w.params(), w.refined)
        Q = ctx.new_state(0.0)
        ctx.init_patches(Q, w.scenario, scen)
        ctx.fill_halos(Q)
        snaps = learned.snapshots(ctx, Q, w.dt(), steps, every, theta[0], theta[1], max_level)
        del Q
        ctx.close()
        torch.cuda.empty_cache()
        name = f"momenta_x{scale}"
        runs[name] = (None, snaps, None)
        _say(f"{name}: {len(snaps)} snapshots, REFINE per snapshot {[int((t == 1).sum()) for _, t in snaps]}")
    sim_s = time.perf_counter() - t0
    ind, info = _train_on(runs, list(runs), args)
    return ind, dict(info, workload=w.name + f", Bowen-York momenta x{list(scales)}, {steps} steps, a snapshot "
                     f"every {every}", simulation_s=sim_s)


def run_learned_bbh(args):
    """The learned refinement indicator trained on the solver's own binary-puncture runs in the
    second-order formulation (stable, and the punctures orbit, so the refinement pattern moves).
    Two training runs with Bowen-York momenta scaled to 0.9 and 1.1 of the standard 0.095 and one
    held-out run at the standard momenta, each on the static r = 2 refinement around the punctures
    to t_end.  Snapshots of the leaf features and the plain tags every sample_dt; the network learns
    the plain tag of the next snapshot from the features of the current one, and is scored on the
    held-out run by the REFINE miss rate against the next snapshot's plain tags."""
    from paper_2406_11626_amd import learned
    names = (("train_0.9", 0.9), ("train_1.1", 1.1), ("heldout_1.0", 1.0))
    t0 = time.perf_counter()
    runs, theta, w, dt, every = _bbh_training_runs(args, names)
    sim_s = time.perf_counter() - t0
    ind, info = _train_on(runs, ("train_0.9", "train_1.1"), args)
    ctx_h, snaps_h, norms_h = runs["heldout_1.0"]
    score = learned.anticipation(ind, ctx_h, snaps_h, conf=0.6, max_level=2)
    return dict(workload=w.name + ", second-order formulation", leaves=ctx_h.n_patches, dt=dt, t_end=args.t_end,
                sample_dt=every * dt, theta_refine_coarsen=theta, simulation_s=sim_s, **info,
                heldout_nonfinite=norms_h[2],
                heldout_refine_per_snapshot=[int((t == 1).sum()) for _, t in snaps_h],
                heldout_score={k: {"miss_rate": v[0], "extra_refine": v[1]} for k, v in score.items()})


def run_dynamic(args, w):
    """Binary puncture with dynamic AMR: a regrid every 10 steps, first by the plain criterion
    alone, then with the learned indicator trained as in run_learned_bbh (the plain criterion's
    REFINE tags kept, the network adding confident REFINE tags and vetoing COARSEN).  The
    thresholds are fixed once from the indicator at t = 0 (its 99.5th and 30th percentiles over
    the leaves, which keeps the mesh near its initial 20k leaves).  Per regrid: the REFINE tags of
    the plain criterion and of the combination, and the network's own miss rate against the
    plain criterion (the share of plain-REFINE leaves its arg-max does not tag REFINE).  Returns
    the stepping throughput of both runs (graph-launched fused steps, regrids excluded)."""
    import numpy as np
    import torch
    from paper_2406_11626_amd import ccz4, dynamic, learned

    def start():
        ctx = ccz4.Context(w.n0, w.origin, w.extent, w.bc, w.params(), w.refined)
        Q = ctx.new_state(0.0)
        ctx.init_patches(Q, w.scenario, w.scen)
        ctx.fill_halos(Q)
        return ctx, Q

    ctx, Q = start()
    ind = torch.empty((ctx.n_patches, 3), dtype=torch.float64, device="cuda")
    tags = torch.empty(ctx.n_patches, dtype=torch.int8, device="cuda")
    ctx.tag_refine(Q, 1e300, -1.0, 3, tags, ind)
    e = ind.max(dim=1).values.cpu().numpy()
    theta_r, theta_c = float(np.percentile(e, 99.5)), float(np.percentile(e, 30))
    leaves0 = dynamic.levels(ctx)
    _say("config 5, plain criterion")
    ctx, Q, log = dynamic.evolve(ctx, Q, w, args.steps, 10, theta_r, theta_c, 3)
    plain = dict(value=log["cell_stages"] / log["step_seconds"], ms_per_step=log["step_seconds"] * 1e3 / args.steps,
                 leaves_final=dynamic.levels(ctx), regrids=log["regrids"])
    norms, _ = ctx.constraints(Q, r_excise=0.5)
    plain["constraints_after"] = {"L2_H": norms[0], "L2_M": norms[1], "nonfinite": norms[2]}
    del Q
    ctx.close()
    torch.cuda.empty_cache()
    _say("training the learned indicator on runs of the same mesh with other momenta")
    net, train = train_mesh_indicator(args, w, (theta_r, theta_c), 3)
    torch.cuda.empty_cache()
    ctx, Q = start()

    def score_against_plain(rec, ctx_, Q_, plain_tags, feat):
        logits = net.forward(feat)
        own = (torch.argmax(logits, dim=1) - 1).to(torch.int8)
        miss, extra = learned.miss_rate(own, plain_tags)
        rec["network_miss_rate_vs_plain"] = miss
        rec["network_extra_refine"] = extra

    _say("config 5, plain criterion with the learned indicator")
    ctx, Q, logl = dynamic.evolve(ctx, Q, w, args.steps, 10, theta_r, theta_c, 3, indicator=net, conf=0.6,
                                  on_tags=score_against_plain)
    norms, _ = ctx.constraints(Q, r_excise=0.5)
    lrn = dict(value=logl["cell_stages"] / logl["step_seconds"], ms_per_step=logl["step_seconds"] * 1e3 / args.steps,
               leaves_final=dynamic.levels(ctx), regrids=logl["regrids"],
               constraints_after={"L2_H": norms[0], "L2_M": norms[1], "nonfinite": norms[2]})
    del Q
    ctx.close()
    torch.cuda.empty_cache()
    return dict(value=plain["value"], steps=args.steps, ms_per_step=plain["ms_per_step"], leaves_initial=leaves0,
                theta=(theta_r, theta_c), plain=plain, learned=lrn, training=train)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, target_s):
    """The oracle (plain C, as it stands; OpenMP over patches changes no arithmetic) on a bounded
    piece of the workload: the whole mesh up to 16^3 leaves, else the 8^3-patch sub-box around the
    puncture at the workload's spacing (512 patches, 373,248 cells).  All host threads: whole RK4 steps (per stage a fill of the
    sub-box, the right-hand side of every patch and the stage combine) until target_s / 2 has
    passed.  One thread: one stage on a sample of patches sized to target_s / 2, the fill and
    combine pro-rated."""
    import numpy as np
    import oracle as orc
    from paper_2406_11626_amd import ccz4, scenarios
    # workloads of up to 16^3 leaves whole; larger uniform ones by the 8^3-leaf sub-box
    sw = scenarios.subbox(w) if not w.refined and w.n0[0] * w.n0[1] * w.n0[2] > 4096 else w
    m = orc.Mesh(sw.n0, sw.origin, sw.extent, sw.bc, sw.refined)
    Q = m.zeros()
    m.init(Q, sw.scenario, sw.scen)
    m.set_background(Q)
    pr = orc.Params(**{f: getattr(sw.params(), f) for f, _ in ccz4.Params._fields_})
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    orc.set_threads(threads)
    used = orc.max_threads()
    cells = m.np * 729
    t0 = time.perf_counter()
    steps = 0
    while True:
        Q = m.rk4_step(pr, Q, sw.dt())
        steps += 1
        if time.perf_counter() - t0 >= 0.5 * target_s:
            break
    t_all = time.perf_counter() - t0
    all_rate = cells * 4 * steps / t_all
    # one thread
    orc.set_threads(1)
    t = time.perf_counter()
    m.fill_halos(Q)
    t_fill = time.perf_counter() - t
    rng = np.random.default_rng(0)
    probe = sorted(rng.choice(m.np, 4, replace=False).tolist())
    k = np.zeros_like(Q)
    t = time.perf_counter()
    m.rhs(pr, Q, k, subset=probe)
    per_patch = (time.perf_counter() - t) / len(probe)
    n = int(min(m.np, max(4, 0.5 * target_s / max(per_patch, 1e-9))))
    sel = sorted(rng.choice(m.np, n, replace=False).tolist())
    t = time.perf_counter()
    m.rhs(pr, Q, k, subset=sel)
    t_rhs = time.perf_counter() - t
    acc, Qnext = np.zeros_like(Q), np.zeros_like(Q)
    t = time.perf_counter()
    m.rk4_stage(0, sw.dt(), Q, k, acc, Qnext)
    t_stage = time.perf_counter() - t
    t_one = t_rhs + (t_fill + t_stage) * n / m.np
    orc.set_threads(threads)
    return dict(value=all_rate, unit="cell-updates/s", cores=used, kind="oracle",
                sample=f"{steps} RK4 steps (4 stages of fill + RHS + stage combine) of the "
                       f"{'whole ' + str(m.np) + '-patch mesh' if sw is w else str(m.np) + '-patch sub-box'} "
                       f"({cells} cells) {sw.name}, on {used} host threads: {t_all:.1f} s",
                nproc=os.cpu_count(), cpu_model=_cpu_model(),
                single_thread={"value": n * 729 / t_one, "unit": "cell-updates/s", "cores": 1,
                               "sample": f"one stage on {n} of the {m.np} patches, fill and combine pro-rated: "
                                         f"{t_one:.1f} s"})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--drift-steps", type=int, default=50,
                    help="steps since the initial data after which the constraint norms are compared")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision run")
    ap.add_argument("--no-so", action="store_true", help="skip the second-order-formulation run")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain unfused FP64 path")
    ap.add_argument("--no-lopsided", action="store_true", help="skip the lopsided-advection run")
    ap.add_argument("--stability", action="store_true",
                    help="instead of timing: evolve the workload in both formulations up to --t-end and "
                         "print the constraint norms")
    ap.add_argument("--tracker", action="store_true",
                    help="instead of timing: puncture trackers in the binary-puncture data up to --t-end")
    ap.add_argument("--stability-transfer", action="store_true",
                    help="with --stability: second order with the App. E against the higher-order coarse-fine "
                         "operators")
    ap.add_argument("--learned-bbh", action="store_true",
                    help="train the learned refinement indicator on second-order binary-puncture runs and score "
                         "it on a held-out run")
    ap.add_argument("--train-iters", type=int, default=2000)
    ap.add_argument("--t-end", type=float, default=10.0)
    ap.add_argument("--sample-dt", type=float, default=0.5)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (reference kernel for the HBM byte counters)")
    ap.add_argument("--no-place", dest="place", action="store_false",
                    help="allocate the step's work buffers once instead of choosing among a pool")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the default launch configuration instead of timing the candidates first")
    ap.add_argument("--progress", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs the hot path on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2406_11626_amd import scenarios
    assert torch.cuda.is_available(), "no GPU"
    w = scenarios.config(args.config)
    if args.tracker:
        print(json.dumps(run_tracker(args)), flush=True)
        return
    if args.learned_bbh:
        print(json.dumps(run_learned_bbh(args)), flush=True)
        return
    if args.stability:
        r = run_stability(args, w)
        print(json.dumps({"workload": w.name, "dt": w.dt(), "t_end": args.t_end, "r_excise": 1.0, **r}), flush=True)
        return
    if args.config == 5:
        r = run_dynamic(args, w)
        print(json.dumps({
            "metric": METRIC,
            "value": r["value"], "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": 0,
            "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic (analytic binary-puncture initial data)",
            "config": {"workload": w.name, "leaves_initial_per_level": r["leaves_initial"], "regrid_every": 10,
                       "theta_refine_coarsen": r["theta"], "precision": "fp64"},
            "plain_criterion": r["plain"], "learned_indicator": r["learned"], "training": r["training"],
            "learned_over_plain_throughput": r["learned"]["value"] / r["plain"]["value"],
        }), flush=True)
        return
    if args.copy_calibration:
        a = torch.ones(2**27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()
    horizon = max(args.drift_steps, 0)
    _say(f"FP64 fused step on {w.name}")
    r64 = run_gpu(args, w, 0, total_steps=horizon, keep=not args.no_mixed or not args.no_plain)
    stages = 4 * args.steps
    value = r64["cells"] * stages / r64["wall"]
    traffic = measured_traffic(args.config)
    traffic_rhs = measured_traffic(args.config, "hbm_bytes_per_rhs_launch")
    ops_stage, ops_rhs = measured_fp64_ops(args.config)
    copy_gbs = copy_bandwidth()
    alg = FUSED_BYTES_PER_CELL * r64["cells"]
    ach = alg / (r64["stage_ms"] * 1e-3) / 1e9
    l2h = r64["norms"][0]
    line = {
        "metric": METRIC,
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
                   "stages_per_step": 4, "dt": w.dt(), "precision": "fp64",
                   "step": "HIP graph of 4 fused stages (y/z halos read from the neighbours, x-face halos "
                           "copied; every halo copied at the last stage)",
                   "launch_config": r64["kernel"], "autotune": r64["tune_ms"], "placement": r64["place"]},
        "eager_ms_per_step": r64["wall_eager"] * 1e3 / args.steps,
        "repetitions_ms_per_step": [round(x, 3) for x in r64["rep_ms"]],
        "median_ms_per_step": float(sorted(r64["rep_ms"])[len(r64["rep_ms"]) // 2]),
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": r64["kernel"], "avg_ms": r64["stage_ms"], "avg_ms_by_stage": r64["stage_ms_by_s"],
                     "bytes_per_cell_stage": FUSED_BYTES_PER_CELL, "algorithmic_bytes_per_launch": alg,
                     "extra_bytes_per_launch": {"same_level_halo_copies": r64["halo_bytes"],
                                                "sommerfeld_ghost_update": r64["ghost_bytes"],
                                                "stage_dependent_stream": r64["stage_bytes"] - alg - r64["halo_bytes"] -
                                                r64["ghost_bytes"]},
                     "achieved_with_extra": r64["stage_gbs"],
                     "copy_gbs": copy_gbs, "frac_of_copy": ach / copy_gbs,
                     "fp64": fp64_rate(ops_stage, r64["stage_ms"])},
        "constraints": {"steps": r64["steps_total"], "t": r64["steps_total"] * r64["dt"], "r_excise": 1.0,
                        "L2_H_t0": r64["norms0"][0], "L2_M_t0": r64["norms0"][1],
                        "L2_H": l2h, "L2_M": r64["norms"][1], "nonfinite": r64["norms"][2]},
    }
    if r64["rhs_ms"]:
        rb = RHS_BYTES_PER_CELL_MODEL * r64["cells"]
        gbs = rb / (r64["rhs_ms"] * 1e-3) / 1e9
        line["rhs_kernel"] = {"kernel": r64["rhs_kernel"], "avg_ms": r64["rhs_ms"], "bytes_per_cell": RHS_BYTES_PER_CELL_MODEL,
                              "algorithmic_bytes_per_launch": rb, "achieved": gbs, "unit": "GB/s",
                              "frac": gbs / HBM_PEAK_GBS, "frac_of_copy": gbs / copy_gbs, "traffic": traffic_rhs,
                              "frac_ideal_bytes": RHS_IDEAL_BYTES_PER_CELL * r64["cells"] /
                              (r64["rhs_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "fp64": fp64_rate(ops_rhs, r64["rhs_ms"])}
    if r64.get("monitor"):
        line["monitor_calls"] = r64["monitor"]
    Q64 = r64.pop("Q", None)
    if not args.no_mixed:
        _say("mixed-precision fused step")
        rm = run_gpu(args, w, 1, total_steps=max(horizon, r64["steps_total"]), keep=True)
        vm = rm["cells"] * stages / rm["wall"]
        Qm = rm.pop("Q")
        per_slot, emax, kmax = state_error(Qm, Q64)
        del Qm
        torch.cuda.empty_cache()
        line["mixed"] = {"value": vm, "ms_per_step": rm["wall"] * 1e3 / args.steps, "stage_avg_ms": rm["stage_ms"],
                         "kernel": rm["kernel"], "speedup_vs_fp64": vm / value, "placement": rm["place"],
                         "L2_H": rm["norms"][0], "L2_M": rm["norms"][1], "steps": rm["steps_total"],
                         "dL2_H_rel": abs(rm["norms"][0] - l2h) / l2h if l2h else None,
                         "equal_constraint_violation": abs(rm["norms"][0] - l2h) <= 0.01 * l2h,
                         "state_error_vs_fp64": {"max": emax, "slot": kmax, "per_slot": per_slot,
                                                 "measure": "max|Q_mixed - Q_fp64| / max|Q_fp64| per slot over "
                                                            "interior cells (slots below 1e-10 of the largest: "
                                                            "relative to the largest)"},
                         # the parity tests' bounds for one or two mixed steps against the FP64 oracle, per
                         # slot relative to the slot's size on the mesh
                         "stated_bound_vs_oracle": {"per_slot": 1e-6,
                                                    "leaves_touching_the_puncture_at_dx_1_12": 1e-4}}
    if not args.no_plain:
        _say("plain unfused FP64 path")
        rp = run_plain(args, w, total_steps=max(horizon, r64["steps_total"]), keep=True)
        vp = rp["cells"] * stages / rp["wall"]
        Qp = rp.pop("Q")
        per_slot, emax, kmax = state_error(Qp, Q64)
        del Qp
        torch.cuda.empty_cache()
        lp = rp["norms"][0]
        line["plain_fp64"] = {"value": vp, "ms_per_step": rp["wall"] * 1e3 / args.steps,
                              "call_ms": rp["call_ms"], "L2_H": lp, "L2_M": rp["norms"][1], "steps": rp["steps_total"],
                              "path": "per stage: ccz4_fill_halos, ccz4_rhs, ccz4_rk4_stage (eager launches)",
                              "placement": rp["place"],
                              "state_error_vs_fused": {"max": emax, "slot": kmax},
                              "speedup_fused_fp64_over_plain": value / vp,
                              "speedup_mixed_over_plain": line["mixed"]["value"] / vp if "mixed" in line else None,
                              "dL2_H_rel_fused_fp64": abs(l2h - lp) / lp if lp else None,
                              "dL2_H_rel_mixed": abs(line["mixed"]["L2_H"] - lp) / lp if lp and "mixed" in line
                              else None}
    del Q64
    torch.cuda.empty_cache()
    if not args.no_so:
        _say("second-order formulation")
        rs = run_gpu(args, w, 0, formulation=1, rhs=False)
        vs = rs["cells"] * stages / rs["wall"]
        line["second_order"] = {"value": vs, "ms_per_step": rs["wall"] * 1e3 / args.steps,
                                "stage_avg_ms": rs["stage_ms"], "reconstruct_avg_ms": rs["reconstruct_ms"],
                                "speedup_vs_first_order": vs / value,
                                "L2_H": rs["norms"][0], "L2_M": rs["norms"][1]}
    if not args.no_lopsided:
        _say("lopsided advection")
        rl = run_gpu(args, w, 0, advection=1, rhs=False)
        vl = rl["cells"] * stages / rl["wall"]
        line["lopsided_advection"] = {"value": vl, "ms_per_step": rl["wall"] * 1e3 / args.steps,
                                      "stage_avg_ms": rl["stage_ms"], "speedup_vs_central": vl / value,
                                      "L2_H": rl["norms"][0], "L2_M": rl["norms"][1]}
    if not args.no_cpu:
        _say("oracle on the host")
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
