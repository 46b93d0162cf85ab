"""Tuning cache: the launch configuration chosen by ``ccz4_autotune`` for a mesh, kept in a JSON
file keyed by the device and a signature of the mesh (leaf count per level, boundary kind), so
that a later run on the same kind of mesh applies it without timing again."""
import json
import os

from . import ccz4

DEFAULT_PATH = os.path.join(os.path.expanduser("~"), ".cache", "ccz4_mi355x", "tuning.json")


def signature(ctx, precision):
    import numpy as np
    import torch
    levels = np.bincount(ctx.ids[:, 0]).tolist() if ctx.n_patches else []
    name = torch.cuda.get_device_name() if torch.cuda.is_available() else "none"
    return f"{name}|levels={levels}|bc={ctx.bc}|prec={precision}"


def load(path=DEFAULT_PATH):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(ctx, Q, precision=ccz4.PREC_FP64, path=DEFAULT_PATH, reps=3, force=False):
    """Apply the cached configuration for this mesh, or time the candidates (ccz4_autotune),
    apply the fastest and record it.  Returns (configuration, timings or None)."""
    key = signature(ctx, precision)
    cache = load(path)
    if key in cache and not force:
        ctx.set_kernel(precision, cache[key]["kernel"])
        return cache[key]["kernel"], None
    ms = ctx.autotune(Q, precision, reps)
    k = ctx.get_kernel(precision)
    cache[key] = {"kernel": k, "ms": ms}
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return k, ms
