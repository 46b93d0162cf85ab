"""Exact CCZ4 states built from closed-form spacetimes, independent of the oracle and the GPU.

A spacetime is given either as a 4-metric g_{mu nu}(t, x, y, z) or as 3+1 data
(gamma_ij, K_ij, alpha, beta^i) as functions of (t, x, y, z).  Everything else follows from
the definitions of App. B of the paper (conformal decomposition, Ghat = Gt for Z = 0, and
the first-order auxiliaries A = d alpha, B = d beta, D = d gt / 2, P = d phi), evaluated with
forward-mode automatic differentiation in float64.  Time derivatives of the whole state come
from one more differentiation, so exact d_t Q is available wherever the spacetime is known
for all t.
"""
import math

import numpy as np
import torch
from torch.func import jacfwd, vmap

torch.set_default_dtype(torch.float64)

SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def det3(m):
    return (m[0, 0] * (m[1, 1] * m[2, 2] - m[1, 2] * m[2, 1])
            - m[0, 1] * (m[1, 0] * m[2, 2] - m[1, 2] * m[2, 0])
            + m[0, 2] * (m[1, 0] * m[2, 1] - m[1, 1] * m[2, 0]))


def inv3(m):
    """Adjugate inverse (explicit, so that nested forward-mode differentiation under vmap
    never goes through a batched LU)."""
    c = [[m[(j + 1) % 3, (i + 1) % 3] * m[(j + 2) % 3, (i + 2) % 3]
          - m[(j + 1) % 3, (i + 2) % 3] * m[(j + 2) % 3, (i + 1) % 3] for j in range(3)]
         for i in range(3)]
    return torch.stack([torch.stack(r) for r in c]) / det3(m)


def adm_from_g4(g4):
    """g4(X) -> (gamma, K, alpha, beta) as functions of X = (t, x, y, z)."""

    def parts(X):
        g = g4(X)
        dg = jacfwd(g4)(X)  # [mu, nu, rho] = d_rho g_mu nu
        gam = g[1:, 1:]
        igam = inv3(gam)
        bl = g[0, 1:]
        beta = igam @ bl
        alpha = torch.sqrt(bl @ beta - g[0, 0])
        dgam = dg[1:, 1:, 1:]          # [i, j, k] = d_k gamma_ij
        dtgam = dg[1:, 1:, 0]
        dbl = dg[0, 1:, 1:]            # [i, k] = d_k beta_i
        # Christoffel of the first kind G1[k,i,j] = (d_i g_kj + d_j g_ki - d_k g_ij)/2
        G1 = 0.5 * (torch.einsum("kji->kij", dgam) + dgam - torch.einsum("ijk->kij", dgam))
        Gam = torch.einsum("kl,lij->kij", igam, G1)
        Dbeta = dbl.T - torch.einsum("kij,k->ij", Gam, bl)  # D_i beta_j = d_i beta_j - Gamma^k_ij beta_k
        K = (Dbeta + Dbeta.T - dtgam) / (2.0 * alpha)
        return gam, K, alpha, beta

    return parts


def ccz4_from_adm(adm, b_fun=None):
    """Return Q(X) -> 59-vector (slot order of the paper's first-order variables + K_0)."""

    def prim(X):
        gam, K, alpha, beta = adm(X)
        det = det3(gam)
        phi = det ** (-1.0 / 6.0)
        gt = phi ** 2 * gam
        igam = inv3(gam)
        trK = torch.sum(igam * K)
        At = phi ** 2 * (K - trK * gam / 3.0)
        return gt, alpha, beta, phi, At, trK

    def gt_of(X):
        return prim(X)[0]

    def Q(X):
        gt, alpha, beta, phi, At, trK = prim(X)
        dgt = jacfwd(gt_of)(X)[..., 1:]          # [i, j, k] = d_k gt_ij
        igt = inv3(gt)
        # Gt^i = gt^jk Gt^i_jk, Gt^i_jk = gt^il (d_j gt_lk + d_k gt_lj - d_l gt_jk)/2
        t1 = torch.einsum("lkj->ljk", dgt)   # d_j gt_lk  -> [l, j, k]
        t2 = torch.einsum("ljk->ljk", dgt)   # d_k gt_lj  -> [l, j, k]
        t3 = torch.einsum("jkl->ljk", dgt)   # d_l gt_jk  -> [l, j, k]
        Gt1 = 0.5 * (t1 + t2 - t3)
        Gt = torch.einsum("il,ljk->ijk", igt, Gt1)
        Gtv = torch.einsum("jk,ijk->i", igt, Gt)
        A = jacfwd(lambda Y: prim(Y)[1])(X)[1:]
        B = jacfwd(lambda Y: prim(Y)[2])(X)[:, 1:].T   # B[k, i] = d_k beta^i
        D = 0.5 * dgt.permute(2, 0, 1)                  # D[k, i, j]
        P = jacfwd(lambda Y: prim(Y)[3])(X)[1:]
        b = b_fun(X) if b_fun is not None else torch.zeros(3, dtype=X.dtype)
        out = [gt[i, j] for (i, j) in SYM]
        out += [alpha]
        out += [beta[i] for i in range(3)]
        out += [phi]
        out += [At[i, j] for (i, j) in SYM]
        out += [trK, torch.zeros((), dtype=X.dtype)]
        out += [Gtv[i] for i in range(3)]
        out += [b[i] for i in range(3)]
        out += [A[k] for k in range(3)]
        out += [B[k, i] for k in range(3) for i in range(3)]
        out += [D[k, i, j] for k in range(3) for (i, j) in SYM]
        out += [P[k] for k in range(3)]
        out += [torch.zeros((), dtype=X.dtype)]
        return torch.stack(out)

    return Q


def evaluate(Qfun, pts, t=0.0, with_dt=False, with_dx=False):
    """pts: (..., 3) numpy -> Q (..., 59) [, dQ/dt (..., 59)] [, dQ/dx_k (..., 3, 59)]."""
    shp = pts.shape[:-1]
    X = torch.zeros((int(np.prod(shp)), 4))
    X[:, 0] = t
    X[:, 1:] = torch.from_numpy(np.ascontiguousarray(pts.reshape(-1, 3)))
    outs = [vmap(Qfun)(X).detach().numpy().reshape(shp + (59,))]
    if with_dt or with_dx:
        J = vmap(jacfwd(Qfun))(X).detach().numpy()  # (n, 59, 4)
        if with_dt:
            outs.append(J[:, :, 0].reshape(shp + (59,)))
        if with_dx:
            outs.append(np.transpose(J[:, :, 1:], (0, 2, 1)).reshape(shp + (3, 59)))
    return outs if len(outs) > 1 else outs[0]


# ---------------------------------------------------------------- closed-form spacetimes

def _assemble(g00, g0i, gij):
    """4x4 metric from its blocks, out of place (vmap-friendly)."""
    top = torch.cat([g00.reshape(1), g0i])
    rest = torch.cat([g0i.reshape(3, 1), gij], dim=1)
    return torch.cat([top.reshape(1, 4), rest], dim=0)


def g4_gauge_wave(A=0.01, k=2.0, n=(1.0, 0.0, 0.0)):
    """Gauge wave (paper's gauge-wave section) propagating along the unit vector n:
    ds^2 = -H dt^2 + H (n.dx)^2 + |dx_perp|^2, H = 1 - A sin(k pi (n.x - t))."""
    nn = torch.tensor(n, dtype=torch.float64)
    nn = nn / torch.linalg.norm(nn)

    def g4(X):
        t, x = X[0], X[1:]
        Hh = 1.0 - A * torch.sin(k * math.pi * (nn @ x - t))
        gij = torch.eye(3, dtype=X.dtype) + (Hh - 1.0) * torch.outer(nn, nn)
        return _assemble(-Hh, torch.zeros(3, dtype=X.dtype) * Hh, gij)

    return g4


def g4_distorted_minkowski(eps=0.04):
    """Minkowski space in smoothly distorted coordinates Y^a = X^a + eps f^a(X): generic
    lapse, shift, metric and extrinsic curvature with all components non-zero."""
    eta = torch.diag(torch.tensor([-1.0, 1.0, 1.0, 1.0]))

    def Ymap(X):
        t, x, y, z = X[0], X[1], X[2], X[3]
        f0 = torch.sin(0.7 * x + 1.1 * y - 0.5 * z + 0.9 * t) + 0.5 * torch.cos(1.3 * z - 0.4 * x)
        f1 = torch.sin(1.2 * y + 0.8 * z - 0.6 * t) + 0.3 * torch.cos(0.9 * x + 0.5 * y)
        f2 = torch.cos(0.9 * x - 0.7 * z + 0.4 * t) + 0.4 * torch.sin(1.4 * y - 0.3 * x)
        f3 = torch.sin(1.0 * x + 0.6 * y + 0.5 * t) + 0.6 * torch.cos(0.8 * z + 0.2 * y)
        return X + eps * torch.stack([f0, f1, f2, f3])

    def g4(X):
        J = jacfwd(Ymap)(X)  # [a, mu] = d Y^a / d X^mu
        return J.T @ eta @ J

    return g4


def g4_schwarzschild_isotropic(M=1.0, center=(0.0, 0.0, 0.0)):
    """Static Schwarzschild in isotropic coordinates, alpha = (1 - M/2r)/(1 + M/2r)."""
    c = torch.tensor(center, dtype=torch.float64)

    def g4(X):
        d = X[1:] - c
        r = torch.sqrt(d @ d)
        psi = 1.0 + M / (2.0 * r)
        al = (1.0 - M / (2.0 * r)) / psi
        return _assemble(-al * al, torch.zeros(3, dtype=X.dtype) * al,
                         psi ** 4 * torch.eye(3, dtype=X.dtype))

    return g4


def adm_puncture(M=1.0, center=(0.0, 0.0, 0.0), lapse="psi-2"):
    """Time-symmetric puncture: gamma = psi^4 delta, K_ij = 0, beta = 0."""
    c = torch.tensor(center, dtype=torch.float64)

    def adm(X):
        d = X[1:] - c
        r = torch.sqrt(d @ d)
        psi = 1.0 + M / (2.0 * r)
        gam = psi ** 4 * torch.eye(3, dtype=X.dtype)
        if lapse == "psi-2":
            al = psi ** -2
        elif lapse == "static":
            al = (1.0 - M / (2.0 * r)) / psi
        else:
            al = 0.5 * ((1.0 - M / (2.0 * r)) / psi + 1.0)
        return gam, torch.zeros((3, 3), dtype=X.dtype), al, torch.zeros(3, dtype=X.dtype)

    return adm


def bowen_york_Ahat(X, holes):
    """Flat-space Bowen-York extrinsic curvature (no spin): sum over holes of
    3/(2 r^2) [P_i n_j + P_j n_i - (delta_ij - n_i n_j) P.n]."""
    Ah = torch.zeros((3, 3), dtype=X.dtype)
    I = torch.eye(3, dtype=X.dtype)
    for (m, pos, Pm) in holes:
        d = X[1:] - torch.tensor(pos, dtype=X.dtype)
        r = torch.sqrt(d @ d)
        n = d / r
        Pv = torch.tensor(Pm, dtype=X.dtype)
        Pn = Pv @ n
        Ah = Ah + 3.0 / (2.0 * r * r) * (torch.outer(Pv, n) + torch.outer(n, Pv) - (I - torch.outer(n, n)) * Pn)
    return Ah


def adm_brill_lindquist_bowen_york(holes):
    """holes: [(m, (x,y,z), (Px,Py,Pz)), ...].  psi = 1 + sum m/(2 r_a), gamma = psi^4 delta,
    K_ij = psi^-2 Ahat_ij (conformally flat, maximal), alpha = psi^-2, beta = 0."""

    def adm(X):
        psi = 1.0
        for (m, pos, _) in holes:
            d = X[1:] - torch.tensor(pos, dtype=X.dtype)
            psi = psi + m / (2.0 * torch.sqrt(d @ d))
        gam = psi ** 4 * torch.eye(3, dtype=X.dtype)
        K = psi ** -2 * bowen_york_Ahat(X, holes)
        return gam, K, psi ** -2, torch.zeros(3, dtype=X.dtype)

    return adm


def brill_lindquist_psi(X, holes):
    psi = 1.0
    for (m, pos, _) in holes:
        d = X[1:] - torch.tensor(pos, dtype=X.dtype)
        psi = psi + m / (2.0 * torch.sqrt(d @ d))
    return psi
