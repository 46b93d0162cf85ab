"""Helpers of the GPU parity tests: moving states between the oracle and the device layout,
and the per-component error measure of the parity bar."""
import numpy as np

from seeded_inputs import from_device_layout, to_device_layout

FACE_MASK = None


def face_slab_mask():
    m = np.zeros((15, 15, 15), bool)
    inner = slice(3, 12)
    for a in range(3):
        for sl in (slice(0, 3), slice(12, 15)):
            idx = [inner, inner, inner]
            idx[2 - a] = sl
            m[tuple(idx)] = True
    return m


SLABS = face_slab_mask()
INTERIOR = np.zeros((15, 15, 15), bool)
INTERIOR[3:12, 3:12, 3:12] = True


def to_gpu(Qo):
    import torch
    return torch.from_numpy(to_device_layout(Qo)).cuda()


def to_host(Qd, patches=None):
    t = Qd if patches is None else Qd[patches]
    return from_device_layout(t.cpu().numpy())


FLOOR = 1e-10
# A slot whose oracle value moves by more than the parity bar when the oracle's own inputs move by
# one unit in the last place (a cancellation residual of much larger terms) is held to KAPPA times
# that measured sensitivity instead: below it the oracle does not determine the value.
KAPPA = 4.0


def parity_error(gpu, ref, mask=INTERIOR, nslots=59, sens=None, tol=None):
    """Per-slot error of the parity bar over the masked cells:
        e_c = max|gpu_c - ref_c| / max|ref_c|   where max|ref_c| > FLOOR * top,
        e_c = max|gpu_c - ref_c| / top          otherwise,
    with top = max_c' max|ref_c'|.  Slots within ten orders of magnitude of the largest one are
    measured relative to their own size; the others (slots that vanish, or cancellation
    residuals far below the rounding of the terms that form them) are held to an absolute bound
    relative to the largest slot.  With sens (per-slot sensitivity of the oracle result, from
    oracle_sensitivity) and the test's bar tol, e_c <= tol also holds where
    max|gpu_c - ref_c| <= KAPPA * sens_c."""
    g = gpu[:, mask][..., :nslots]
    r = ref[:, mask][..., :nslots]
    diff = np.abs(g - r).reshape(-1, nslots).max(0)
    scale = np.abs(r).reshape(-1, nslots).max(0)
    top = max(scale.max(), 1e-300)
    e = diff / np.where(scale > FLOOR * top, scale, top)
    if sens is not None:
        e = np.minimum(e, tol * diff / np.maximum(KAPPA * np.asarray(sens)[:nslots], 1e-300))
    return e


def ulp_perturbed(Q, seed):
    """Q with every value moved by one unit in the last place, up or down at random."""
    up = np.random.default_rng(seed).random(Q.shape) < 0.5
    return np.where(up, np.nextafter(Q, np.inf), np.nextafter(Q, -np.inf))


def perturbed_runs(fn, Q, trials=2, seed=1234):
    """fn of `trials` copies of Q whose every value moved by one unit in the last place."""
    return [fn(ulp_perturbed(Q, seed + t)) for t in range(trials)]


def sensitivity(ref, runs, mask=INTERIOR, nslots=59):
    """Per-slot rounding sensitivity of an oracle result ref: the largest change over the masked
    cells among the results `runs` of one-ulp perturbed inputs."""
    out = np.zeros(nslots)
    for r in runs:
        d = np.abs(r[:, mask][..., :nslots] - ref[:, mask][..., :nslots]).reshape(-1, nslots).max(0)
        out = np.maximum(out, d)
    return out


def oracle_sensitivity(fn, Q, mask=INTERIOR, trials=2, nslots=59, ref=None):
    """sensitivity of fn(Q) under one-ulp perturbations of every input value (trials draws)."""
    if ref is None:
        ref = fn(Q.copy())
    return sensitivity(ref, perturbed_runs(fn, Q, trials), mask, nslots)


def same_level_halo_mask(ctx, Q, axes=(0, 1, 2)):
    """Device boolean mask of the halo cells of the faces normal to `axes` that a same-level leaf
    covers: the cells that a full fill restores but a Neumann + coarse-fine fill leaves alone."""
    import torch

    from paper_2406_11626_amd import ccz4

    def refilled(kinds):
        H = torch.full_like(Q, float("nan"))
        H[:, :, 3:12, 3:12, 3:12] = Q[:, :, 3:12, 3:12, 3:12]
        ctx.fill_halos_kinds(H, kinds)
        return ~torch.isnan(H)

    m = refilled(ccz4.FILL_ALL) & ~refilled(ccz4.FILL_NEUMANN | ccz4.FILL_LEVELS)
    face = torch.zeros_like(m)
    for a in axes:  # device layout [patch][slot][z][y][x]
        idx = [slice(None), slice(None), slice(3, 12), slice(3, 12), slice(3, 12)]
        for h in (slice(0, 3), slice(12, 15)):
            idx[4 - a] = h
            face[tuple(idx)] = True
    return m & face
