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


def parity_error(gpu, ref, mask=INTERIOR, nslots=59):
    """Per-slot error of the parity bar over the masked cells:
        e_c = max|gpu_c - ref_c| / max|ref_c|   where max|ref_c| > FLOOR * top,
        e_c = max|gpu_c - ref_c| / top          otherwise,
    with top = max_c' max|ref_c'|.  Slots within ten orders of magnitude of the largest one are
    measured relative to their own size; the others (slots that vanish, or cancellation
    residuals far below the rounding of the terms that form them) are held to an absolute bound
    relative to the largest slot."""
    g = gpu[:, mask][..., :nslots]
    r = ref[:, mask][..., :nslots]
    diff = np.abs(g - r).reshape(-1, nslots).max(0)
    scale = np.abs(r).reshape(-1, nslots).max(0)
    top = max(scale.max(), 1e-300)
    return diff / np.where(scale > FLOOR * top, scale, top)


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
