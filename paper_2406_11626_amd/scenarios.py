"""Workload presets: grids, parameters and initial data of the five benchmark configurations.

Parameter values follow the paper's experiment sections (gauge wave: kappa1 = 1,
kappa2 = kappa3 = 0, e = c = tau = 1, mu = 0.2; black holes: kappa1 = 0.1, kappa2 = 0,
kappa3 = 0.5, e = c = tau = 1, mu = 0.2, f = 0.75) with KO strength 0.1, the Gamma-driver
eta = 2 of these workloads, and dt = CFL * (smallest dx) with CFL = 0.1.
"""
import math

import numpy as np
from dataclasses import dataclass, field

from . import ccz4


@dataclass
class Workload:
    name: str
    n0: tuple
    origin: tuple
    extent: tuple
    bc: int
    prm: dict
    scenario: int
    scen: list
    steps: int
    refined: list = field(default_factory=list)
    cfl: float = 0.1

    def params(self):
        return ccz4.params(**self.prm)

    def dx_min(self):
        maxlev = max([r[0] + 1 for r in self.refined], default=0)
        return self.extent[0] / (self.n0[0] * 9 * 3 ** maxlev)

    def dt(self):
        return self.cfl * self.dx_min()

    def dt_for(self, ctx):
        """CFL * the finest spacing of the context's current mesh (global time step)."""
        maxlev = int(ctx.ids[:, 0].max()) if ctx.n_patches else 0
        return self.cfl * self.extent[0] / (self.n0[0] * 9 * 3 ** maxlev)


GAUGE = dict(kappa1=1.0, kappa2=0.0, kappa3=0.0, tau=1.0, e=1.0, c=1.0, mu=0.2, f=0.75, eta=2.0,
             ko_eps=0.1, slicing=0, shift=0)
BLACK_HOLE = dict(kappa1=0.1, kappa2=0.0, kappa3=0.5, tau=1.0, e=1.0, c=1.0, mu=0.2, f=0.75, eta=2.0,
                  ko_eps=0.1, slicing=1, shift=1)


def sphere_refinement(n0, origin, extent, center, radii):
    """Static refinement by concentric spheres: every cube of level l whose nearest point to
    `center` (one point, or a list of points: the nearest of them) lies within radii[l] is
    refined (levels 0..len(radii)-1), keeping only cubes whose parents are refined."""
    centers = [center] if np.ndim(center) == 1 else list(center)
    refined = []
    current = [(0, i, j, k) for k in range(n0[2]) for j in range(n0[1]) for i in range(n0[0])]
    for lev, R in enumerate(radii):
        n = [n0[a] * 3 ** lev for a in range(3)]
        L = [extent[a] / n[a] for a in range(3)]
        nxt = []
        for (l, i, j, k) in current:
            lo = [origin[a] + L[a] * idx for a, idx in enumerate((i, j, k))]
            dmin = math.inf
            for cen in centers:
                d2 = 0.0
                for a in range(3):
                    c = min(max(cen[a], lo[a]), lo[a] + L[a])
                    d2 += (c - cen[a]) ** 2
                dmin = min(dmin, math.sqrt(d2))
            if dmin <= R:
                refined.append((lev, i, j, k))
                nxt += [(lev + 1, 3 * i + u, 3 * j + v, 3 * k + w)
                        for w in range(3) for v in range(3) for u in range(3)]
        current = nxt
    return refined


def config(n):
    """Configurations 1..5 of the benchmark list."""
    if n == 1:
        return Workload("gauge-wave 27^3 (3^3 patches of 9^3, periodic)", (3, 3, 3), (-0.5,) * 3, (1.0,) * 3,
                        ccz4.BC_PERIODIC, GAUGE, ccz4.SCEN_GAUGE_WAVE, [0.01, 2.0], 10)
    if n == 2:
        return Workload("single puncture 144^3 (16^3 patches of 9^3 on [-9,9]^3)", (16, 16, 16), (-9.0,) * 3,
                        (18.0,) * 3, ccz4.BC_SOMMERFELD, BLACK_HOLE, ccz4.SCEN_PUNCTURE, [1.0, 0.0, 0.0, 0.0, 0], 20)
    if n == 3:
        ref = sphere_refinement((16, 16, 16), (-9.0,) * 3, (18.0,) * 3, (0.0, 0.0, 0.0), [1.5, 0.5])
        return Workload("single puncture, static 3-level AMR (spheres r = 1.5, 0.5)", (16, 16, 16), (-9.0,) * 3,
                        (18.0,) * 3, ccz4.BC_SOMMERFELD, BLACK_HOLE, ccz4.SCEN_PUNCTURE, [1.0, 0.0, 0.0, 0.0, 0], 20,
                        refined=ref)
    if n == 4:
        return Workload("single puncture 216^3 (24^3 patches of 9^3 on [-9,9]^3)", (24, 24, 24), (-9.0,) * 3,
                        (18.0,) * 3, ccz4.BC_SOMMERFELD, BLACK_HOLE, ccz4.SCEN_PUNCTURE, [1.0, 0.0, 0.0, 0.0, 0], 50)
    if n == 5:
        scen = [0.5, 3.0, 0.0, 0.0, 0.0, 0.095, 0.0, 0.5, -3.0, 0.0, 0.0, 0.0, -0.095, 0.0]
        ref = sphere_refinement((16, 16, 16), (-12.0,) * 3, (24.0,) * 3, [(3.0, 0.0, 0.0), (-3.0, 0.0, 0.0)],
                                [3.0, 1.0, 0.4])
        return Workload("binary puncture (Brill-Lindquist + Bowen-York) on [-12,12]^3, 4 levels, dynamic regrid",
                        (16, 16, 16), (-12.0,) * 3, (24.0,) * 3, ccz4.BC_SOMMERFELD, BLACK_HOLE, ccz4.SCEN_BL_BY, scen,
                        20, refined=ref)
    raise ValueError(n)


def binary_tracking(radii=(2.0,)):
    """The binary-puncture data of configuration 5 (masses 0.5 at (+-3, 0, 0), Bowen-York momenta
    (0, +-0.095, 0)) on [-12, 12]^3 with a static refinement of the given radii around the two
    punctures: the workload of the puncture-tracker run."""
    w = config(5)
    ref = sphere_refinement(w.n0, w.origin, w.extent, [(3.0, 0.0, 0.0), (-3.0, 0.0, 0.0)], list(radii))
    return Workload(f"binary puncture on [-12,12]^3, static refinement r = {list(radii)} around the punctures",
                    w.n0, w.origin, w.extent, w.bc, BLACK_HOLE, w.scenario, w.scen, 20, refined=ref)


def subbox(w, n=8):
    """An n^3-patch box of workload w's level-0 spacing centred on the origin (same puncture, same
    parameters and boundary condition): a bounded piece of a uniform workload of the same per-cell
    arithmetic, for timing the host oracle."""
    assert not w.refined
    L = w.extent[0] / w.n0[0]  # edge of one patch
    return Workload(f"{n}^3-patch sub-box of: {w.name}", (n, n, n), (-0.5 * n * L,) * 3, (n * L,) * 3, w.bc, w.prm,
                    w.scenario, w.scen, w.steps, cfl=w.cfl)
