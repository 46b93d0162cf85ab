"""Benchmark of the CCZ4 FD4 hot path on one MI355X.

A step is one classical RK4 step of the whole hot path over the single-puncture workload of
16^3 patches of 9^3 cells (144^3 = 2,985,984 cells on [-9,9]^3, Sommerfeld boundaries, 1+log
slicing, Gamma-driver): four fused stages (FD4 derivatives + CCZ4 algebra + Kreiss-Oliger + RK4
stage combine, the last stage with the algebraic projection), each of which also writes the
same-level face halos of its output; the Neumann and coarse-fine halo fill between stages has
no faces on this uniform mesh.  The metric is cell-updates per second per RK4 stage: cells x 4
stages x steps / wall time, with the state resident in HBM.

The roofline object is the fused stage kernel's: algorithmic bytes per launch (per cell: every
evolved slot with its three-cell face halos read once, the step state and accumulator streamed
as the stage requires; plus the same-level halo cells written) over its average launch time,
taken with events on the launch stream.

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


# Standalone right-hand side, bytes per interior cell: the 58 evolved slots over the interior and
# face halos (2187 cell-vectors per 729 cells) plus K_0 pointwise, and the 59 slots of k written.
RHS_BYTES_PER_CELL = QS_BYTES_PER_CELL + 8 * NV
# the same with every cell-vector read once (no halo duplication): the ideal lower bound
RHS_IDEAL_BYTES_PER_CELL = 2 * 8 * NV
# its Sommerfeld ghost right-hand side, cell-vectors per ghost cell: ghost and interior layers
# (4 per 3 ghost cells), the background, k written
RHS_GHOST_VECTORS = 4.0 / 3 + 2


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


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_stage_lds_puncture16_hbm_traffic.md")
FLOPS_FILE = os.path.join(ROOT, "profiles", "k_stage_lds_puncture16_fp64_ops.md")


def kernel_source_digest():
    """sha256 over the HIP sources of the library (the traffic figure is void once they change)."""
    import hashlib
    d = os.path.join(ROOT, "paper_2406_11626_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".hpp", ".cpp")):
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


def measured_traffic(config):
    """HBM bytes per launch of the fused stage kernel from the committed counter summary."""
    return _record_float(_profile_record(TRAFFIC_FILE, config), "hbm_bytes_per_launch")


def measured_fp64_ops(config):
    """FP64 operations per launch of the fused stage kernel and of the standalone right-hand side
    (64 lanes x (ADD + MUL + 2 FMA + TRANS) wave instructions) from the committed counter summary."""
    rec = _profile_record(FLOPS_FILE, config)
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


def run_gpu(args, w, precision, formulation=0, advection=0):
    import torch
    from paper_2406_11626_amd import ccz4
    prm = ccz4.params(**{**w.prm, "formulation": formulation, "advection": advection})
    ctx = ccz4.Context(w.n0, w.origin, w.extent, w.bc, prm, w.refined)
    so = ctx.second_order
    Q = ctx.new_state(0.0)
    ctx.init_patches(Q, w.scenario, w.scen)
    Q1, Q2, acc = ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0)
    dt = w.dt()
    stream = torch.cuda.current_stream()
    order = ((Q, Q1), (Q1, Q2), (Q2, Q1), (Q1, Q))
    rest = ccz4.FILL_NEUMANN | ccz4.FILL_LEVELS
    events, recon_events = [], []
    ctx.fill_halos(Q, stream)
    if so:  # the auxiliaries of the initial data from its primaries
        ctx.reconstruct(Q, True, stream)
        ctx.fill_halos(Q, stream)
    tune_ms = ctx.autotune(Q, precision, reps=2) if args.autotune else None
    ctx.fill_halos(Q, stream)

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
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
        if args.progress:
            print(f"# step {i + 1}/{args.steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall_eager = time.perf_counter() - t0
    # the same step captured once as a HIP graph and replayed (the production path)
    graph = ctx.step_graph(Q, (Q1, Q2, acc), dt, precision)
    for _ in range(args.warmup):
        graph.launch(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        graph.launch(stream)
        if args.progress:
            print(f"# graph step {i + 1}/{args.steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    graph.close()
    cells = ctx.n_patches * 729
    faces = same_level_faces_per_axis(ctx)
    assert sum(faces) == ctx.plan_counts()["same_level"]

    def pushed(fl):
        return sum(faces) if fl & ccz4.STAGE_FILL_SAME_LEVEL else (
            faces[0] if fl & ccz4.STAGE_FILL_SAME_LEVEL_X else 0)
    # the standalone right-hand side on the final state (its own kernel, same launch configuration)
    rhs_ms = None
    if precision == ccz4.PREC_FP64 and not so:
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
    stage_ms = [a.elapsed_time(b) for _, a, b, _ in events]
    nbf = ctx.plan_counts()["sommerfeld"]
    launch_bytes = [stage_bytes(s, cells, pushed(fl), nbf) for s, _, _, fl in events]
    norms, st = ctx.constraints(Q, r_excise=1.0)
    kc = ctx.get_kernel(precision)
    targs = ("<double, " if precision == ccz4.PREC_FP64 else "<float, ") + ("1>" if advection else "0>")
    order = " (plain block order)" if kc & ccz4.KERNEL_LINEAR_ORDER else ""
    # the kernels one stage call (one right-hand-side call) launches
    kname = ("k_stage_lds" if kc & ccz4.KERNEL_LDS else "k_stage") + targs + order
    rname = ("k_rhs_lds" if kc & ccz4.KERNEL_LDS else "k_rhs") + targs + order + \
        (" + k_rhs_sommerfeld" if nbf and not kc & ccz4.KERNEL_LDS else "")
    recon_ms = [a.elapsed_time(b) for a, b in recon_events]
    out = dict(wall=wall, wall_eager=wall_eager, tune_ms=tune_ms, cells=cells, patches=ctx.n_patches, rhs_ms=rhs_ms,
               reconstruct_ms=sum(recon_ms) / len(recon_ms) if recon_ms else None,
               stage_ms=sum(stage_ms) / len(stage_ms),
               stage_bytes=sum(launch_bytes) / len(launch_bytes),
               stage_gbs=sum(launch_bytes) / (sum(stage_ms) * 1e-3) / 1e9, norms=norms, status=st,
               kernel=kname, rhs_kernel=rname, ghost_faces=nbf)
    del Q, Q1, Q2, acc
    ctx.close()
    torch.cuda.empty_cache()
    return out


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


def run_learned_bbh(args):
    """The learned refinement indicator trained on the solver's own binary-puncture runs in the
    second-order formulation (stable, and the punctures orbit, so the refinement pattern moves).
    Two training runs with Bowen-York momenta scaled to 0.9 and 1.1 of the standard 0.095 and one
    held-out run at the standard momenta, each on the static r = 2 refinement around the punctures
    to t_end.  Snapshots of the leaf features and the plain tags every sample_dt; the network learns
    the plain tag of the next snapshot from the features of the current one, and is scored on the
    held-out run by the REFINE miss rate against the next snapshot's plain tags."""
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
    t0 = time.perf_counter()
    for name, scale in (("train_0.9", 0.9), ("train_1.1", 1.1), ("heldout_1.0", 1.0)):
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
            ctx.tag_refine(Q, 1e300, -1.0, 2, tags, ind)
            e = ind.max(dim=1).values.cpu().numpy()
            theta = (float(np.percentile(e, 99.0)), float(np.percentile(e, 30.0)))
        snaps = learned.snapshots(ctx, Q, dt, steps, every, theta[0], theta[1], 2)
        norms, _ = ctx.constraints(Q)
        runs[name] = (ctx, snaps, norms)
        print(f"# {name}: {len(snaps)} snapshots, REFINE per snapshot "
              f"{[int((t == 1).sum()) for _, t in snaps]}, non-finite {norms[2]:.0f}", file=sys.stderr, flush=True)
    sim_s = time.perf_counter() - t0
    feats, targets = [], []
    for name in ("train_0.9", "train_1.1"):
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
    train_s = time.perf_counter() - t1
    ctx_h, snaps_h, norms_h = runs["heldout_1.0"]
    score = learned.anticipation(ind, ctx_h, snaps_h, conf=0.6, max_level=2)
    return dict(workload=w.name + ", second-order formulation", leaves=ctx_h.n_patches, dt=dt, t_end=args.t_end,
                sample_dt=every * dt, theta_refine_coarsen=theta, training_rows=int(feat.shape[0]),
                train_iters=args.train_iters, loss_before=loss0, loss_after=loss, train_s=train_s,
                simulation_s=sim_s, heldout_nonfinite=norms_h[2],
                heldout_refine_per_snapshot=[int((t == 1).sum()) for _, t in snaps_h],
                heldout_score={k: {"miss_rate": v[0], "extra_refine": v[1]} for k, v in score.items()})


def run_dynamic(args, w):
    """Binary puncture with dynamic AMR: a regrid by the plain criterion every 10 steps.  The
    thresholds are fixed once from the indicator at t = 0 (its 99.5th and 30th percentiles over
    the leaves, which keeps the mesh near its initial 20k leaves).  Returns the stepping throughput (graph-launched fused steps, regrids excluded), the
    regrid records and the cost of the learned indicator's inference on the final mesh."""
    import numpy as np
    import torch
    from paper_2406_11626_amd import ccz4, dynamic
    from paper_2406_11626_amd.learned import LearnedIndicator
    ctx = ccz4.Context(w.n0, w.origin, w.extent, w.bc, w.params(), w.refined)
    Q = ctx.new_state(0.0)
    ctx.init_patches(Q, w.scenario, w.scen)
    ctx.fill_halos(Q)
    ind = torch.empty((ctx.n_patches, 3), dtype=torch.float64, device="cuda")
    tags = torch.empty(ctx.n_patches, dtype=torch.int8, device="cuda")
    ctx.tag_refine(Q, 1e300, -1.0, 3, tags, ind)
    e = ind.max(dim=1).values.cpu().numpy()
    theta_r, theta_c = float(np.percentile(e, 99.5)), float(np.percentile(e, 30))
    leaves0 = dynamic.levels(ctx)
    ctx, Q, log = dynamic.evolve(ctx, Q, w, args.steps, 10, theta_r, theta_c, 3)
    # learned indicator inference on the final mesh (features from the constraint fields)
    net = LearnedIndicator(seed=0)
    HM = torch.empty((ctx.n_patches, 4, 729), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.constraints(Q, HM)
    feat = ctx.features(Q, HM)
    logits = net.forward(feat)
    torch.cuda.synchronize()
    t_learned = time.perf_counter() - t0
    norms, _ = ctx.constraints(Q, r_excise=0.5)
    return dict(value=log["cell_stages"] / log["step_seconds"], steps=args.steps,
                ms_per_step=log["step_seconds"] * 1e3 / args.steps, leaves_initial=leaves0,
                leaves_final=dynamic.levels(ctx), regrids=log["regrids"], theta=(theta_r, theta_c),
                learned_inference_ms=t_learned * 1e3, norms=norms, logits_shape=list(logits.shape))


def cpu_baseline(w, target_s):
    """The oracle (single-threaded C, as it stands) on a bounded sample of the same workload:
    the full mesh is initialised and filled once, then one RK4 stage's RHS is timed on a sample
    of patches; the fill of the whole mesh and the stage combine are pro-rated to the sample."""
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
                sample=f"one RK4 stage (fill + RHS + stage combine) on {n} of {m.np} patches ({cells} cells) "
                       f"of the same workload; fill and combine pro-rated; {t_total:.1f} s of CPU work")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision run")
    ap.add_argument("--no-so", action="store_true", help="skip the second-order-formulation run")
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
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (reference kernel for the HBM byte counters)")
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
            "metric": "CCZ4 cell-updates/s per RK4 stage (FP64 vs mixed), % of FP64/HBM roofline",
            "value": r["value"], "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": 0,
            "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic (analytic binary-puncture initial data)",
            "config": {"workload": w.name, "leaves_initial_per_level": r["leaves_initial"],
                       "leaves_final_per_level": r["leaves_final"], "regrid_every": 10,
                       "theta_refine_coarsen": r["theta"], "precision": "fp64"},
            "regrids": r["regrids"], "learned_indicator_inference_ms": r["learned_inference_ms"],
            "constraints_after": {"L2_H": r["norms"][0], "L2_M": r["norms"][1], "nonfinite": r["norms"][2]},
        }), flush=True)
        return
    if args.copy_calibration:
        a = torch.ones(2**27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()
    r64 = run_gpu(args, w, 0)
    stages = 4 * args.steps
    value = r64["cells"] * stages / r64["wall"]
    traffic = measured_traffic(args.config)
    ops_stage, ops_rhs = measured_fp64_ops(args.config)
    copy_gbs = copy_bandwidth()
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
                   "stages_per_step": 4, "dt": w.dt(), "precision": "fp64",
                   "step": "HIP graph of 4 fused stages (y/z halos read from the neighbours, x-face halos "
                           "copied; every halo copied at the last stage)",
                   "launch_config": r64["kernel"], "autotune_ms": r64["tune_ms"]},
        "eager_ms_per_step": r64["wall_eager"] * 1e3 / args.steps,
        "roofline": {"bound": "hbm", "achieved": r64["stage_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": r64["stage_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": r64["kernel"], "avg_ms": r64["stage_ms"],
                     "copy_gbs": copy_gbs, "frac_of_copy": r64["stage_gbs"] / copy_gbs,
                     "algorithmic_bytes_per_launch": r64["stage_bytes"],
                     "fp64": fp64_rate(ops_stage, r64["stage_ms"])},
        "constraints_after": {"L2_H": r64["norms"][0], "L2_M": r64["norms"][1], "nonfinite": r64["norms"][2]},
    }
    if r64["rhs_ms"]:
        rb = RHS_BYTES_PER_CELL * r64["cells"] + RHS_GHOST_VECTORS * 8 * NV * 243 * r64["ghost_faces"]
        gbs = rb / (r64["rhs_ms"] * 1e-3) / 1e9
        line["rhs_kernel"] = {"kernel": r64["rhs_kernel"], "avg_ms": r64["rhs_ms"],
                              "algorithmic_bytes_per_launch": rb, "achieved": gbs, "unit": "GB/s",
                              "frac": gbs / HBM_PEAK_GBS, "frac_of_copy": gbs / copy_gbs,
                              "frac_ideal_bytes": RHS_IDEAL_BYTES_PER_CELL * r64["cells"] /
                              (r64["rhs_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "fp64": fp64_rate(ops_rhs, r64["rhs_ms"])}
    if not args.no_mixed:
        rm = run_gpu(args, w, 1)
        vm = rm["cells"] * stages / rm["wall"]
        line["mixed"] = {"value": vm, "stage_avg_ms": rm["stage_ms"], "speedup_vs_fp64": vm / value,
                         "L2_H": rm["norms"][0], "L2_M": rm["norms"][1]}
    if not args.no_so:
        rs = run_gpu(args, w, 0, formulation=1)
        vs = rs["cells"] * stages / rs["wall"]
        line["second_order"] = {"value": vs, "ms_per_step": rs["wall"] * 1e3 / args.steps,
                                "stage_avg_ms": rs["stage_ms"], "reconstruct_avg_ms": rs["reconstruct_ms"],
                                "speedup_vs_first_order": vs / value,
                                "L2_H": rs["norms"][0], "L2_M": rs["norms"][1]}
    if not args.no_lopsided:
        rl = run_gpu(args, w, 0, advection=1)
        vl = rl["cells"] * stages / rl["wall"]
        line["lopsided_advection"] = {"value": vl, "ms_per_step": rl["wall"] * 1e3 / args.steps,
                                      "stage_avg_ms": rl["stage_ms"], "speedup_vs_central": vl / value,
                                      "L2_H": rl["norms"][0], "L2_M": rl["norms"][1]}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
