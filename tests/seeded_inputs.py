"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

This module only draws numbers: smooth random fields on patch boxes and helpers to move
arrays between the two storage layouts.  It holds none of the method's arithmetic.
"""
import numpy as np

NV, NB = 59, 15

# slot groups (order of the paper's first-order variables, then K_0)
METRIC = [0, 1, 2, 3, 4, 5]
DIAG = [0, 3, 5]


def smooth_state(centers, seed, amp=0.1, alpha_range=(0.6, 1.4), phi_range=(0.6, 1.0),
                 k_max=2.0, frozen_shift=False):
    """Smooth random values at points `centers` (..., 3): every slot is a constant plus three
    random low Fourier modes.  gt = delta + amp * modes (symmetric positive definite for
    amp <= 0.1), alpha and phi stay inside the given ranges, K_0 = 0."""
    rng = np.random.default_rng(seed)
    x = np.asarray(centers, dtype=np.float64)
    out = np.zeros(x.shape[:-1] + (NV,))
    for v in range(58):
        base = rng.uniform(-0.2, 0.2)
        val = np.full(x.shape[:-1], base)
        for _ in range(3):
            kv = rng.uniform(-k_max, k_max, 3)
            ph = rng.uniform(0, 2 * np.pi)
            val = val + rng.uniform(-1, 1) * np.sin(x @ kv + ph)
        out[..., v] = val
    # metric: delta + amp * (bounded modes)
    for v in METRIC:
        out[..., v] = (1.0 if v in DIAG else 0.0) + amp * out[..., v] / 3.5
    # lapse and conformal factor strictly positive
    lo, hi = alpha_range
    out[..., 6] = lo + (hi - lo) * 0.5 * (1 + np.tanh(out[..., 6]))
    lo, hi = phi_range
    out[..., 10] = lo + (hi - lo) * 0.5 * (1 + np.tanh(out[..., 10]))
    if frozen_shift:
        out[..., 7:10] = 0.0
        out[..., 22:25] = 0.0
        out[..., 28:37] = 0.0
    out[..., 58] = 0.0
    return out


def box_centers(origin, dx):
    """(15,15,15,3) cell centres [z,y,x,axis] of a box whose interior starts at `origin`."""
    c = np.arange(NB) - 3 + 0.5
    out = np.zeros((NB, NB, NB, 3))
    out[..., 0] = origin[0] + c[None, None, :] * dx[0]
    out[..., 1] = origin[1] + c[None, :, None] * dx[1]
    out[..., 2] = origin[2] + c[:, None, None] * dx[2]
    return out


def box_points(center, h):
    """(15,15,15,3) points of a box of spacing h centred on `center`, [z,y,x,axis]."""
    c = (np.arange(NB) - 7.0) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    return np.stack([X + center[0], Y + center[1], Z + center[2]], -1)


# ---- layout conversion between the oracle (cell-major) and the device (slot-major) ----

XPAD = 16  # the device pads x to 16 doubles per row


def to_device_layout(Qo):
    """oracle [n, z, y, x, slot] -> device [n, slot, z, y, 16] (x padded with zeros)."""
    n = Qo.shape[0]
    out = np.zeros((n, NV, NB, NB, XPAD))
    out[..., :NB] = np.transpose(Qo, (0, 4, 1, 2, 3))
    return out


def from_device_layout(Qd):
    """device [n, slot, z, y, 16] -> oracle [n, z, y, x, slot]."""
    return np.ascontiguousarray(np.transpose(Qd[..., :NB], (0, 2, 3, 4, 1)))
