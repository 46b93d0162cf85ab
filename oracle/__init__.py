"""ctypes binding of the plain FP64 CPU oracle (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  The product library never loads it.

Arrays use the oracle's own layout: one patch box of 15^3 cells (9^3 interior + 3 halo layers
per face), cell-major with the 59 slots innermost: ``Q[patch, z, y, x, slot]``.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libccz4_oracle.so")

NV, NB, P, H = 59, 15, 9, 3


def build():
    subprocess.check_call(["sh", os.path.join(_HERE, "build.sh")])


def _load():
    if not os.path.exists(_LIB):
        build()
    return ctypes.CDLL(_LIB)


_lib = _load()

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i8p = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")


class Params(ctypes.Structure):
    _fields_ = [
        ("kappa1", ctypes.c_double), ("kappa2", ctypes.c_double), ("kappa3", ctypes.c_double),
        ("tau", ctypes.c_double), ("e", ctypes.c_double), ("c", ctypes.c_double),
        ("mu", ctypes.c_double), ("f", ctypes.c_double), ("eta", ctypes.c_double),
        ("ko_eps", ctypes.c_double), ("slicing", ctypes.c_int), ("shift", ctypes.c_int),
        ("formulation", ctypes.c_int), ("advection", ctypes.c_int),
    ]


def params(**kw):
    d = dict(kappa1=0.1, kappa2=0.0, kappa3=0.5, tau=1.0, e=1.0, c=1.0, mu=0.2, f=0.75,
             eta=2.0, ko_eps=0.1, slicing=1, shift=1, formulation=0, advection=0)
    d.update(kw)
    return Params(**d)


def _sig(name, res, args):
    fn = getattr(_lib, name)
    fn.restype = res
    fn.argtypes = args
    return fn


_PP = ctypes.POINTER(Params)
_rhs_point = _sig("orc_rhs_point", None, [_PP, _dp, _dp, _dp])
_cons_point = _sig("orc_constraints_point", None, [_dp, _dp, _dp])
_fd4 = _sig("orc_fd4", ctypes.c_double, [_dp, ctypes.c_double])
_ko = _sig("orc_ko", ctypes.c_double, [_dp, ctypes.c_double, ctypes.c_double])
_fd4_lop = _sig("orc_fd4_lop", ctypes.c_double, [_dp, ctypes.c_double, ctypes.c_int])
_rhs_box = _sig("orc_rhs_box", None, [_PP, _dp, _dp, _dp])
_cons_box = _sig("orc_constraints_box", None, [_dp, _dp, _dp])
_mesh_create = _sig("orc_mesh_create", ctypes.c_void_p,
                    [_ip, _dp, _dp, ctypes.c_int, ctypes.c_int, _ip])
_mesh_destroy = _sig("orc_mesh_destroy", None, [ctypes.c_void_p])
_mesh_np = _sig("orc_mesh_npatches", ctypes.c_int64, [ctypes.c_void_p])
_mesh_ids = _sig("orc_mesh_patch_ids", None, [ctypes.c_void_p, _ip])
_mesh_geom = _sig("orc_mesh_patch_geom", None, [ctypes.c_void_p, _dp])
_init_point = _sig("orc_init_point", ctypes.c_int, [ctypes.c_int, _dp, _dp, _dp])
_init = _sig("orc_init", ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.c_int, _dp])
_set_bg = _sig("orc_set_background", None, [ctypes.c_void_p, _dp])
_fill = _sig("orc_fill_halos", None, [ctypes.c_void_p, _dp])
_rhs = _sig("orc_rhs", None, [ctypes.c_void_p, _PP, _dp, _dp])
_recon = _sig("orc_reconstruct_aux", None, [ctypes.c_void_p, _dp])
_set_transfer = _sig("orc_mesh_set_transfer", None, [ctypes.c_void_p, ctypes.c_int])
_find_leaf = _sig("orc_find_leaf", ctypes.c_int64, [ctypes.c_void_p, _dp])
_tr_sample = _sig("orc_tracer_sample", ctypes.c_int64,
                  [ctypes.c_void_p, _dp, ctypes.c_int64, _dp, ctypes.c_int, _ip, _dp])
_tag_tracers = _sig("orc_tag_tracers", None, [ctypes.c_void_p, ctypes.c_int64, _dp, ctypes.c_int, _dp, ctypes.c_int,
                                              _i8p])
_tr_advance = _sig("orc_tracer_advance", ctypes.c_int64, [ctypes.c_void_p, _dp, ctypes.c_int64, _dp, ctypes.c_double])
_rhs_subset = _sig("orc_rhs_subset", None,
                   [ctypes.c_void_p, _PP, _dp, _dp, ctypes.c_int64, _i64p])
_rk4 = _sig("orc_rk4_stage", ctypes.c_int,
            [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp])
_project = _sig("orc_project_point", None, [_dp])
_cons = _sig("orc_constraints", ctypes.c_int64,
             [ctypes.c_void_p, _dp, ctypes.c_void_p, ctypes.c_double, _dp])
_tag_ind = _sig("orc_tag_indicator", None, [ctypes.c_void_p, _dp, _dp])
_tag = _sig("orc_tag_refine", None,
            [ctypes.c_void_p, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, _i8p])


def _c(a, dt=np.float64):
    return np.ascontiguousarray(a, dtype=dt)


_feat = _sig("orc_features", None, [ctypes.c_void_p, _dp, _dp])
_set_threads = _sig("orc_set_threads", None, [ctypes.c_int])
_max_threads = _sig("orc_max_threads", ctypes.c_int, [])


def set_threads(n):
    """Host threads of the oracle's patch loops (RHS and RK4 stage); the arithmetic of each
    patch is the same for any number."""
    _set_threads(int(n))


def max_threads():
    return int(_max_threads())

_rg_plan = _sig("orc_regrid_plan", ctypes.c_int64, [ctypes.c_void_p, _i8p, ctypes.c_int, _ip, ctypes.c_int64])
_rg_transfer = _sig("orc_regrid_transfer", None, [ctypes.c_void_p, _dp, ctypes.c_void_p, _dp])
_bf16 = _sig("orc_bf16_round", ctypes.c_double, [ctypes.c_double])
_tag_learned = _sig("orc_tag_learned", None, [ctypes.c_void_p, np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS"),
                                              _i8p, ctypes.c_float, ctypes.c_int, _i8p])
_fp = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_stdz = _sig("orc_mlp_standardize", None, [ctypes.c_int64, _fp, _fp, _dp])
_mlp_fwd = _sig("orc_mlp_forward", None, [ctypes.c_int64, _dp, _dp, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p])
_mlp_grad = _sig("orc_mlp_loss_grad", ctypes.c_double, [ctypes.c_int64, _dp, _i32p, _dp, ctypes.c_int, _dp])
_adam = _sig("orc_adam_step", None, [ctypes.c_int64, _dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double])

MLP_NIN, MLP_NH, MLP_NOUT, MLP_NPARAM = 81, 64, 3, 9603


def bf16_round(x):
    """Nearest BF16 (ties to even) of the FP32 value nearest to x."""
    return float(_bf16(float(x)))


def mlp_standardize(feat, norm):
    feat = np.ascontiguousarray(feat, dtype=np.float32)
    out = np.zeros(feat.shape, dtype=np.float64)
    _stdz(feat.shape[0], feat, np.ascontiguousarray(norm, dtype=np.float32), out)
    return out


def mlp_forward(x, prm, bf16=True):
    """(a1, a2, logits) of the perceptron on standardised inputs x[n][81]."""
    x = _c(x)
    n = x.shape[0]
    a1, a2, z3 = np.zeros((n, MLP_NH)), np.zeros((n, MLP_NH)), np.zeros((n, MLP_NOUT))
    _mlp_fwd(n, x, _c(prm), int(bf16), a1.ctypes.data, a2.ctypes.data, z3.ctypes.data)
    return a1, a2, z3


def mlp_loss_grad(x, labels, prm, bf16=True):
    x = _c(x)
    g = np.zeros(MLP_NPARAM)
    loss = _mlp_grad(x.shape[0], x, np.ascontiguousarray(labels, dtype=np.int32), _c(prm), int(bf16), g)
    return loss, g


def _mlp_split(prm):
    """(W1, b1, W2, b2, W3, b3) views of a parameter vector (row-major, out x in)."""
    prm = np.asarray(prm, dtype=np.float64)
    o = np.cumsum([0, MLP_NH * MLP_NIN, MLP_NH, MLP_NH * MLP_NH, MLP_NH, MLP_NOUT * MLP_NH, MLP_NOUT])
    shp = [(MLP_NH, MLP_NIN), (MLP_NH,), (MLP_NH, MLP_NH), (MLP_NH,), (MLP_NOUT, MLP_NH), (MLP_NOUT,)]
    return [prm[o[i]:o[i + 1]].reshape(shp[i]) for i in range(6)]


def bf16_array(x):
    """bf16_round of every element."""
    return np.vectorize(bf16_round, otypes=[np.float64])(np.asarray(x, dtype=np.float64))


def mlp_layers(prm, x, a1, a2, labels, d3, d2, d1, bf16=True):
    """The perceptron layer by layer in FP64, each layer from the given operands of the layer
    before it rather than from this function's own previous layer: x, a1, a2 (rows of layer
    inputs, BF16 values) and d3, d2, d1 (pre-activation gradients, rounded here to BF16 where
    they enter a matrix product, as the forward activations are).  Returns a dict with
      z1, z2, z3: pre-activations x W1b^T + b1, a1 W2b^T + b2, a2 W3b^T + b3 (Wb = BF16 weights);
      d3: (softmax(z3) - onehot(labels)) / n;
      d2, d1: (bf16(d3) W3b) * [a2 > 0], (bf16(d2) W2b) * [a1 > 0];
      gW3, gb3, gW2, gb2, gW1, gb1: bf16(d3)^T a2, sum d3, bf16(d2)^T a1, sum d2, bf16(d1)^T x,
      sum d1 (the loss gradient of the mean cross-entropy).
    bf16=False skips every BF16 rounding; chained on its own outputs this is then the gradient
    of mlp_loss_grad."""
    W1, b1, W2, b2, W3, b3 = _mlp_split(prm)
    rnd = bf16_array if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    W1b, W2b, W3b = rnd(W1), rnd(W2), rnd(W3)
    n = x.shape[0]
    out = {"z1": x @ W1b.T + b1, "z2": a1 @ W2b.T + b2, "z3": a2 @ W3b.T + b3}
    z3 = out["z3"]
    e = np.exp(z3 - z3.max(axis=1, keepdims=True))
    onehot = np.zeros_like(z3)
    onehot[np.arange(n), np.asarray(labels)] = 1.0
    out["d3"] = (e / e.sum(axis=1, keepdims=True) - onehot) / n
    d3b, d2b, d1b = rnd(d3), rnd(d2), rnd(d1)
    out["d2"] = (d3b @ W3b) * (a2 > 0)
    out["d1"] = (d2b @ W2b) * (a1 > 0)
    out["gW3"], out["gb3"] = d3b.T @ a2, d3.sum(axis=0)
    out["gW2"], out["gb2"] = d2b.T @ a1, d2.sum(axis=0)
    out["gW1"], out["gb1"] = d1b.T @ x, d1.sum(axis=0)
    return out


def adam_step(p, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """In place on float64 arrays p, m, v."""
    _adam(p.size, p, m, v, _c(g), int(t), lr, b1, b2, eps)




def rhs_point(pr, q, dq):
    out = np.zeros(NV)
    _rhs_point(ctypes.byref(pr), _c(q), _c(dq).reshape(-1), out)
    return out


def constraints_point(q, dq):
    out = np.zeros(4)
    _cons_point(_c(q), _c(dq).reshape(-1), out)
    return out


def fd4(v5, dx):
    return _fd4(_c(v5), dx)


def ko(v7, dx, eps):
    return _ko(_c(v7), dx, eps)


def fd4_lop(v7, dx, right):
    return _fd4_lop(_c(v7), dx, int(right))


def rhs_box(pr, dx, box):
    box = _c(box)
    out = np.zeros_like(box)
    _rhs_box(ctypes.byref(pr), _c(dx), box, out)
    return out


def constraints_box(dx, box):
    out = np.zeros((729, 4))
    _cons_box(_c(dx), _c(box), out)
    return out


def init_point(scenario, sp, x):
    q = np.zeros(NV)
    if _init_point(scenario, _c(sp), _c(x), q):
        raise ValueError("unknown scenario")
    return q


def project_point(q):
    q = _c(q).copy()
    _project(q)
    return q


class Mesh:
    """Forest of 9^3-cell patches (oracle side).  bc: 0 periodic, 1 Neumann, 2 Sommerfeld."""

    def __init__(self, n0, origin, extent, bc=0, refined=()):
        ref = np.asarray(refined, dtype=np.int32).reshape(-1, 4)
        self.n_refined = ref.shape[0]
        ref = _c(ref if ref.size else np.zeros((1, 4)), np.int32)
        self._h = _mesh_create(_c(n0, np.int32), _c(origin), _c(extent), bc, self.n_refined, ref)
        self.np = int(_mesh_np(self._h))
        self.ids = np.zeros((self.np, 4), dtype=np.int32)
        _mesh_ids(self._h, self.ids)
        self.geom = np.zeros((self.np, 6))
        _mesh_geom(self._h, self.geom)

    def __del__(self):
        # at interpreter shutdown the module's globals may already be gone: the process frees all
        if getattr(self, "_h", None) and _mesh_destroy is not None:
            _mesh_destroy(self._h)
            self._h = None

    def zeros(self):
        return np.zeros((self.np, NB, NB, NB, NV))

    def cell_centers(self, p):
        """(15,15,15,3) centres of box cells of leaf p, [z,y,x,axis]."""
        org, dx = self.geom[p, :3], self.geom[p, 3:]
        c = (np.arange(NB) - H + 0.5)
        X = org[0] + c[None, None, :] * dx[0]
        Y = org[1] + c[None, :, None] * dx[1]
        Z = org[2] + c[:, None, None] * dx[2]
        out = np.zeros((NB, NB, NB, 3))
        out[..., 0], out[..., 1], out[..., 2] = np.broadcast_arrays(X, Y, Z)
        return out

    def init(self, Q, scenario, sp):
        if _init(self._h, Q, scenario, _c(sp)):
            raise ValueError("init failed")

    def set_background(self, Q):
        _set_bg(self._h, Q)

    def fill_halos(self, Q):
        _fill(self._h, Q)

    def rhs(self, pr, Q, k=None, subset=None):
        if k is None:
            k = np.zeros_like(Q)
        if subset is None:
            _rhs(self._h, ctypes.byref(pr), Q, k)
        else:
            sel = _c(subset, np.int64)
            _rhs_subset(self._h, ctypes.byref(pr), Q, k, sel.size, sel)
        return k

    def find_leaf(self, x):
        return int(_find_leaf(self._h, _c(x)))

    def tracer_sample(self, Q, pos, slots):
        """(n, len(slots)) trilinear samples at the points pos (n, 3); NaN outside the mesh."""
        pos = _c(pos).reshape(-1, 3)
        sl = np.ascontiguousarray(slots, dtype=np.int32)
        out = np.zeros((pos.shape[0], sl.size))
        _tr_sample(self._h, Q, pos.shape[0], pos, sl.size, sl, out)
        return out

    def tracer_advance(self, Q, pos, dt):
        """One explicit Euler step of puncture trackers, in place on pos (n, 3) float64."""
        assert pos.dtype == np.float64 and pos.flags.c_contiguous
        return int(_tr_advance(self._h, Q, pos.shape[0], pos, dt))

    def tag_tracers(self, pos, radii, max_level):
        pos = _c(pos).reshape(-1, 3)
        r = _c(radii)
        tags = np.zeros(self.np, dtype=np.int8)
        _tag_tracers(self._h, pos.shape[0], pos, r.size, r, int(max_level), tags)
        return tags

    def set_transfer(self, transfer):
        """0: the App. E coarse-fine operators as printed; 1: injection restriction and quadratic
        prolongation."""
        _set_transfer(self._h, int(transfer))

    def reconstruct(self, Q):
        """Second-order formulation: the auxiliaries of every interior cell from FD4
        differences of the primaries (halos of Q must be filled); in place."""
        _recon(self._h, Q)

    def rk4_stage(self, s, dt, Qn, k, acc, Qnext):
        if _rk4(self._h, s, dt, Qn, k, acc, Qnext):
            raise ValueError("bad stage")

    def constraints(self, Q, r_excise=0.0, want_fields=False):
        norms = np.zeros(3)
        HM = np.zeros((self.np, 729, 4)) if want_fields else None
        _cons(self._h, Q, HM.ctypes.data if want_fields else None, r_excise, norms)
        return (norms, HM) if want_fields else norms

    def tag_indicator(self, Q):
        ind = np.zeros((self.np, 3))
        _tag_ind(self._h, Q, ind)
        return ind

    def regrid_plan(self, tags, max_level):
        """Refined cubes (n, 4) of the mesh after the tags."""
        cap = 4 * (len(self.ids) + 64) * 27
        out = np.zeros((cap, 4), dtype=np.int32)
        n = _rg_plan(self._h, np.ascontiguousarray(tags, dtype=np.int8), int(max_level), out, cap)
        assert n >= 0
        return out[:n]

    def regrid_transfer(self, Q, new, Qnew):
        """In place on Qnew (a state of the Mesh `new`)."""
        _rg_transfer(self._h, Q, new._h, Qnew)

    def features(self, Q):
        f = np.zeros((self.np, MLP_NIN))
        _feat(self._h, Q, f)
        return f

    def tag_learned(self, logits, plain, conf, max_level):
        tags = np.zeros(self.np, dtype=np.int8)
        _tag_learned(self._h, np.ascontiguousarray(logits, dtype=np.float32),
                     np.ascontiguousarray(plain, dtype=np.int8), conf, max_level, tags)
        return tags

    def tag_refine(self, Q, theta_r, theta_c, max_level):
        tags = np.zeros(self.np, dtype=np.int8)
        _tag(self._h, Q, theta_r, theta_c, max_level, tags)
        return tags

    def rk4_step(self, pr, Q, dt):
        """One classical RK4 step: four (fill, rhs, stage) sweeps.  In the second-order
        formulation every stage result (the final one after its projection) gets its halos
        filled and its auxiliaries reconstructed before it is used (Algorithm 2)."""
        acc = np.zeros_like(Q)
        Qs = Q.copy()
        Qnew = Q.copy()
        for s in range(4):
            self.fill_halos(Qs)
            k = self.rhs(pr, Qs)
            Qnext = Q.copy() if s < 3 else Qnew
            self.rk4_stage(s, dt, Q, k, acc, Qnext)
            if pr.formulation:
                self.fill_halos(Qnext)
                self.reconstruct(Qnext)
            Qs = Qnext
        return Qnew
