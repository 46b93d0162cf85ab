"""Evolution with dynamic AMR: fused RK4 steps on the current mesh and, every `regrid_every`
steps, the plain criterion's tags (optionally combined with the learned indicator), a regrid
plan, a new mesh and the transfer of the state onto it.  Every step runs in the library's
kernels; this module only sequences the calls and records what happened."""
import time

import numpy as np

from . import ccz4


def evolve(ctx, Q, w, steps, regrid_every, theta_r, theta_c, max_level, indicator=None, conf=0.6,
           precision=ccz4.PREC_FP64, on_regrid=None, on_tags=None):
    """Returns (ctx, Q, log): the final context and state, and per-regrid records (step, leaves
    before and after, REFINE tags of the plain criterion and of the combination, time of the
    regrid) plus the stepping time.  Q enters with filled halos.  With an indicator,
    on_tags(rec, ctx, Q, plain_tags, feat) is called at each regrid before the combination replaces
    the plain tags (to score the network against them)."""
    import torch
    dt = w.dt_for(ctx) if hasattr(w, "dt_for") else w.dt()
    log = {"regrids": [], "step_seconds": 0.0, "cell_stages": 0}
    bufs = tuple(ctx.new_state(0.0) for _ in range(3))
    graph = ctx.step_graph(Q, bufs, dt, precision)
    tags = torch.empty(ctx.n_patches, dtype=torch.int8, device="cuda")
    for s in range(steps):
        if regrid_every and s > 0 and s % regrid_every == 0:
            t0 = time.perf_counter()
            tags = torch.empty(ctx.n_patches, dtype=torch.int8, device="cuda")
            ctx.tag_refine(Q, theta_r, theta_c, max_level, tags)
            rec = {"step": s, "leaves_before": ctx.n_patches, "plain_refine": int((tags == 1).sum().item())}
            if indicator is not None:
                HM = torch.empty((ctx.n_patches, 4, 729), dtype=torch.float64, device="cuda")
                ctx.constraints(Q, HM)
                feat = ctx.features(Q, HM)
                if on_tags:
                    on_tags(rec, ctx, Q, tags, feat)
                combined = ctx.tag_learned(indicator.forward(feat), tags, conf, max_level)
                rec["learned_refine"] = int((combined == 1).sum().item())
                tags = combined
            graph.close()
            del bufs
            ctx, Q = ctx.regrid(Q, tags, max_level, w.scenario, w.scen)
            dt = w.dt_for(ctx) if hasattr(w, "dt_for") else w.dt()
            bufs = tuple(ctx.new_state(0.0) for _ in range(3))
            graph = ctx.step_graph(Q, bufs, dt, precision)
            torch.cuda.synchronize()
            rec["leaves_after"] = ctx.n_patches
            rec["seconds"] = time.perf_counter() - t0
            log["regrids"].append(rec)
            if on_regrid:
                on_regrid(rec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        graph.launch()
        torch.cuda.synchronize()
        log["step_seconds"] += time.perf_counter() - t0
        log["cell_stages"] += 4 * ctx.n_patches * 729
    graph.close()
    return ctx, Q, log


def levels(ctx):
    return np.bincount(ctx.ids[:, 0]).tolist()
