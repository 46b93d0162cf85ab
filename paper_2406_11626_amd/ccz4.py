"""ctypes binding of libccz4.so (include/ccz4.h).  Argument marshalling only: every step of
the path runs in the HIP kernels of the library.  Device buffers are torch tensors (float64,
CUDA/HIP device) or raw device addresses; streams are torch streams or raw hipStream_t.

The module-level functions carry the C names; ``Context`` bundles them around one handle.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccz4.so")

PATCH_DOUBLES = 212400
NV = 59

CCZ4_OK, CCZ4_EINVAL, CCZ4_ENOMEM, CCZ4_ELAYOUT, CCZ4_EHIP, CCZ4_ENONFINITE, CCZ4_ESTATE = range(7)
BC_PERIODIC, BC_NEUMANN, BC_SOMMERFELD = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1
FORMULATION_FO, FORMULATION_SO = 0, 1
ADVECTION_CENTRAL, ADVECTION_LOPSIDED_UPWIND, ADVECTION_LOPSIDED_PRINTED = 0, 1, 2
TRANSFER_APP_E, TRANSFER_HIGHER_ORDER = 0, 1
KERNEL_PHASED, KERNEL_LDS, KERNEL_LINEAR_ORDER = 0, 1, 2
KERNEL_ORDER_CANONICAL, KERNEL_ORDER_Z_PENCILS, KERNEL_ORDER_BRICKS, KERNEL_ORDER_MORTON = 0, 4, 8, 12
KERNEL_CONFIGS = 16  # launch configurations: kernel | block order | leaf order


def kernel_config_name(k):
    """Readable name of launch configuration k."""
    order = ("canonical", "z-pencils", "bricks", "morton")[(k >> 2) & 3]
    return (("lds" if k & KERNEL_LDS else "phased") + ("/linear" if k & KERNEL_LINEAR_ORDER else "/xcd") +
            "/" + order)
FILL_SAME_LEVEL, FILL_NEUMANN, FILL_LEVELS, FILL_ALL = 1, 2, 4, 7
STAGE_FILL_SAME_LEVEL, STAGE_GATHER_SAME_LEVEL, STAGE_FILL_SAME_LEVEL_X = 1, 2, 4
MLP_NIN, MLP_NH, MLP_NOUT, MLP_NPARAM = 81, 64, 3, 9603
MLP_TRACE = 340  # floats per row of the optional gradient trace
SCEN_GAUGE_WAVE, SCEN_PUNCTURE, SCEN_BL_BY = 0, 1, 2


class CCZ4Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ccz4 status {status}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("kappa1", ctypes.c_double), ("kappa2", ctypes.c_double), ("kappa3", ctypes.c_double),
        ("tau", ctypes.c_double), ("e", ctypes.c_double), ("c", ctypes.c_double),
        ("mu", ctypes.c_double), ("f", ctypes.c_double), ("eta", ctypes.c_double),
        ("ko_eps", ctypes.c_double), ("slicing", ctypes.c_int32), ("shift", ctypes.c_int32),
        ("formulation", ctypes.c_int32), ("advection", ctypes.c_int32), ("transfer", ctypes.c_int32),
    ]


class GridDesc(ctypes.Structure):
    _fields_ = [
        ("n0", ctypes.c_int32 * 3), ("origin", ctypes.c_double * 3), ("extent", ctypes.c_double * 3),
        ("bc", ctypes.c_int32), ("n_refined", ctypes.c_int32), ("refined", ctypes.POINTER(ctypes.c_int32)),
    ]


def params(**kw):
    """Black-hole defaults of the paper (kappa1 = 0.1, kappa3 = 0.5, e = c = tau = 1, mu = 0.2,
    f = 0.75), eta = 2, KO 0.1, 1+log slicing, Gamma-driver shift, first-order formulation
    (formulation=FORMULATION_SO for the second-order one), central advection (advection=
    ADVECTION_LOPSIDED_UPWIND or ADVECTION_LOPSIDED_PRINTED for App. D's lopsided stencils), the
    App. E coarse-fine operators (transfer=TRANSFER_HIGHER_ORDER for injection and quadratics)."""
    d = dict(kappa1=0.1, kappa2=0.0, kappa3=0.5, tau=1.0, e=1.0, c=1.0, mu=0.2, f=0.75,
             eta=2.0, ko_eps=0.1, slicing=1, shift=1, formulation=0, advection=0, transfer=0)
    d.update(kw)
    return Params(**d)


_lib = None


def lib():
    """Load libccz4.so; raise if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2406_11626_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "ccz4_create": (i32, [ctypes.POINTER(P), ctypes.POINTER(GridDesc), ctypes.POINTER(Params)]),
            "ccz4_destroy": (None, [P]),
            "ccz4_set_params": (i32, [P, ctypes.POINTER(Params)]),
            "ccz4_layout": (i32, [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]),
            "ccz4_patch_table": (i32, [P, P, P]),
            "ccz4_init_patches": (i32, [P, P, i32, P, i32, P]),
            "ccz4_set_background": (i32, [P, P, P]),
            "ccz4_fill_halos": (i32, [P, P, P]),
            "ccz4_rhs": (i32, [P, P, P, i32, P]),
            "ccz4_rk4_stage": (i32, [P, i32, f64, P, P, P, P, P]),
            "ccz4_rhs_rk4_stage": (i32, [P, i32, f64, P, P, P, P, i32, i32, P]),
            "ccz4_step_stage_flags": (i32, [P, i32, i32, ctypes.POINTER(i32)]),
            "ccz4_reconstruct_aux": (i32, [P, P, i32, P]),
            "ccz4_tracers_sample": (i32, [P, P, i64, P, i32, P, P, P]),
            "ccz4_tracers_advance": (i32, [P, P, i64, P, f64, P]),
            "ccz4_tag_tracers": (i32, [P, i64, P, i32, P, i32, P, P]),
            "ccz4_fill_halos_kinds": (i32, [P, P, i32, P]),
            "ccz4_plan_counts": (i32, [P, ctypes.POINTER(i64)]),
            "ccz4_constraints": (i32, [P, P, P, f64, P, P]),
            "ccz4_tag_refine": (i32, [P, P, f64, f64, i32, P, P, P]),
            "ccz4_set_kernel": (i32, [P, i32, i32]),
            "ccz4_get_kernel": (i32, [P, i32, ctypes.POINTER(i32)]),
            "ccz4_autotune": (i32, [P, P, P, P, i32, i32, ctypes.POINTER(f64), P]),
            "ccz4_step_graph_create": (i32, [P, P, P, P, P, f64, i32, ctypes.POINTER(P)]),
            "ccz4_step_graph_launch": (i32, [P, P]),
            "ccz4_step_graph_destroy": (None, [P]),
            "ccz4_regrid_plan": (i32, [P, P, i32, P, i64, ctypes.POINTER(i64)]),
            "ccz4_regrid_transfer": (i32, [P, P, P, P, P]),
            "ccz4_features": (i32, [P, P, P, P, P]),
            "ccz4_mlp_forward": (i32, [P, P, P, i64, P, P]),
            "ccz4_mlp_workspace": (i32, [i64, ctypes.POINTER(i64)]),
            "ccz4_mlp_grad": (i32, [P, P, P, P, i64, P, i64, P, P, P]),
            "ccz4_mlp_grad_noalloc": (i32, [P, P, P, P, i64, P, P, P]),
            "ccz4_mlp_adam": (i32, [P, P, P, P, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, P]),
            "ccz4_tag_learned": (i32, [P, P, P, ctypes.c_float, i32, P, P]),
            "ccz4_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        if not x.is_cuda:
            raise ValueError("device tensor expected")
        if not x.is_contiguous():
            raise ValueError("contiguous tensor expected")
        return x.data_ptr()
    return ctypes.cast(x, ctypes.c_void_p).value


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _check(status):
    if status != CCZ4_OK:
        raise CCZ4Error(status, lib().ccz4_last_error().decode())
    return status


# ---------------------------------------------------------------- C names

def ccz4_create(n0, origin, extent, bc, prm, refined=()):
    ref = [int(v) for r in refined for v in r]
    arr = (ctypes.c_int32 * max(len(ref), 1))(*ref)
    g = GridDesc()
    g.n0[:] = [int(v) for v in n0]
    g.origin[:] = [float(v) for v in origin]
    g.extent[:] = [float(v) for v in extent]
    g.bc = int(bc)
    g.n_refined = len(ref) // 4
    g.refined = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
    h = ctypes.c_void_p()
    _check(lib().ccz4_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(prm)))
    return h


def ccz4_destroy(h):
    lib().ccz4_destroy(h)


def ccz4_set_params(h, prm):
    return _check(lib().ccz4_set_params(h, ctypes.byref(prm)))


def ccz4_layout(h):
    n, pd, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().ccz4_layout(h, ctypes.byref(n), ctypes.byref(pd), ctypes.byref(b)))
    return n.value, pd.value, b.value


def ccz4_patch_table(h):
    import numpy as np
    n = ccz4_layout(h)[0]
    ids = np.zeros((n, 4), dtype=np.int32)
    geom = np.zeros((n, 6))
    _check(lib().ccz4_patch_table(h, ids.ctypes.data, geom.ctypes.data))
    return ids, geom


def ccz4_init_patches(h, Q, scenario, scen, stream=None):
    arr = (ctypes.c_double * max(len(scen), 1))(*[float(v) for v in scen])
    return _check(lib().ccz4_init_patches(h, _ptr(Q), int(scenario), ctypes.cast(arr, ctypes.c_void_p),
                                          len(scen), _stream(stream)))


def ccz4_set_background(h, Q, stream=None):
    return _check(lib().ccz4_set_background(h, _ptr(Q), _stream(stream)))


def ccz4_fill_halos(h, Q, stream=None):
    return _check(lib().ccz4_fill_halos(h, _ptr(Q), _stream(stream)))


def ccz4_fill_halos_kinds(h, Q, kinds, stream=None):
    return _check(lib().ccz4_fill_halos_kinds(h, _ptr(Q), int(kinds), _stream(stream)))


def ccz4_plan_counts(h):
    out = (ctypes.c_int64 * 5)()
    _check(lib().ccz4_plan_counts(h, out))
    return dict(zip(("same_level", "neumann", "restrict", "prolong", "sommerfeld"), list(out)))


def ccz4_rhs(h, Q, k, precision=PREC_FP64, stream=None):
    return _check(lib().ccz4_rhs(h, _ptr(Q), _ptr(k), int(precision), _stream(stream)))


def ccz4_rk4_stage(h, s, dt, Qn, k, acc, Qnext, stream=None):
    return _check(lib().ccz4_rk4_stage(h, int(s), float(dt), _ptr(Qn), _ptr(k), _ptr(acc), _ptr(Qnext),
                                       _stream(stream)))


def ccz4_reconstruct_aux(h, Q, flags=0, stream=None):
    return _check(lib().ccz4_reconstruct_aux(h, _ptr(Q), int(flags), _stream(stream)))


def ccz4_tracers_sample(h, Q, pos, slots, out, stream=None):
    sl = (ctypes.c_int32 * len(slots))(*[int(v) for v in slots])
    return _check(lib().ccz4_tracers_sample(h, _ptr(Q), int(pos.shape[0]) if pos is not None else 0, _ptr(pos),
                                            len(slots), ctypes.cast(sl, ctypes.c_void_p), _ptr(out), _stream(stream)))


def ccz4_tracers_advance(h, Q, pos, dt, stream=None):
    return _check(lib().ccz4_tracers_advance(h, _ptr(Q), int(pos.shape[0]), _ptr(pos), float(dt), _stream(stream)))


def ccz4_tag_tracers(h, pos, radii, max_level, tags, stream=None):
    r = (ctypes.c_double * max(1, len(radii)))(*[float(v) for v in radii])
    return _check(lib().ccz4_tag_tracers(h, int(pos.shape[0]), _ptr(pos), len(radii), ctypes.cast(r, ctypes.c_void_p),
                                         int(max_level), _ptr(tags), _stream(stream)))


def ccz4_rhs_rk4_stage(h, s, dt, Qs, Qn, acc, Qnext, precision=PREC_FP64, flags=0, stream=None):
    return _check(lib().ccz4_rhs_rk4_stage(h, int(s), float(dt), _ptr(Qs), _ptr(Qn), _ptr(acc), _ptr(Qnext),
                                           int(precision), int(flags), _stream(stream)))


def ccz4_set_kernel(h, precision, kernel):
    return _check(lib().ccz4_set_kernel(h, int(precision), int(kernel)))


def ccz4_get_kernel(h, precision):
    out = ctypes.c_int32(-1)
    _check(lib().ccz4_get_kernel(h, int(precision), ctypes.byref(out)))
    return out.value


def ccz4_step_stage_flags(h, precision, s):
    out = ctypes.c_int32(0)
    _check(lib().ccz4_step_stage_flags(h, int(precision), int(s), ctypes.byref(out)))
    return out.value


def ccz4_autotune(h, Q, acc, Qx, precision=PREC_FP64, reps=3, stream=None):
    ms = (ctypes.c_double * KERNEL_CONFIGS)()
    _check(lib().ccz4_autotune(h, _ptr(Q), _ptr(acc), _ptr(Qx), int(precision), int(reps), ms, _stream(stream)))
    return list(ms)


def ccz4_step_graph_create(h, Qn, Q1, Q2, acc, dt, precision=PREC_FP64):
    g = ctypes.c_void_p()
    _check(lib().ccz4_step_graph_create(h, _ptr(Qn), _ptr(Q1), _ptr(Q2), _ptr(acc), float(dt), int(precision),
                                        ctypes.byref(g)))
    return g


def ccz4_step_graph_launch(g, stream=None):
    return _check(lib().ccz4_step_graph_launch(g, _stream(stream)))


def ccz4_step_graph_destroy(g):
    lib().ccz4_step_graph_destroy(g)


def ccz4_regrid_plan(h, tags_host, max_level):
    """Refined cubes (n, 4) int32 of the mesh after the tags (host array or tensor)."""
    import numpy as np
    if hasattr(tags_host, "cpu"):
        tags_host = tags_host.cpu().numpy()
    tags = np.ascontiguousarray(tags_host, dtype=np.int8)
    n = ctypes.c_int64(0)
    lib().ccz4_regrid_plan(h, tags.ctypes.data, int(max_level), None, 0, ctypes.byref(n))
    buf = np.zeros((max(n.value, 1), 4), dtype=np.int32)
    _check(lib().ccz4_regrid_plan(h, tags.ctypes.data, int(max_level), buf.ctypes.data, n.value, ctypes.byref(n)))
    return buf[:n.value]


def ccz4_regrid_transfer(h_old, Qold, h_new, Qnew, stream=None):
    return _check(lib().ccz4_regrid_transfer(h_old, _ptr(Qold), h_new, _ptr(Qnew), _stream(stream)))


def ccz4_features(h, Q, HM, feat, stream=None):
    return _check(lib().ccz4_features(h, _ptr(Q), _ptr(HM), _ptr(feat), _stream(stream)))


def ccz4_mlp_forward(params, norm, feat, n, logits, stream=None):
    return _check(lib().ccz4_mlp_forward(_ptr(params), _ptr(norm), _ptr(feat), int(n), _ptr(logits),
                                         _stream(stream)))


def ccz4_mlp_workspace(n):
    out = ctypes.c_int64(0)
    _check(lib().ccz4_mlp_workspace(int(n), ctypes.byref(out)))
    return out.value


def ccz4_mlp_grad(params, norm, feat, tags, n, work, grad, loss=None, stream=None):
    return _check(lib().ccz4_mlp_grad(_ptr(params), _ptr(norm), _ptr(feat), _ptr(tags), int(n), _ptr(work),
                                      int(work.numel()), _ptr(grad), _ptr(loss), _stream(stream)))


MLP_NOALLOC_MAX_ROWS = 4096


def ccz4_mlp_grad_noalloc(params, norm, feat, tags, n, grad, loss=None, stream=None):
    return _check(lib().ccz4_mlp_grad_noalloc(_ptr(params), _ptr(norm), _ptr(feat), _ptr(tags), int(n), _ptr(grad),
                                              _ptr(loss), _stream(stream)))


def ccz4_mlp_adam(params, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    return _check(lib().ccz4_mlp_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), int(step), float(lr),
                                      float(beta1), float(beta2), float(eps), _stream(stream)))


def ccz4_tag_learned(h, logits, plain_tags, conf, max_level, tags, stream=None):
    return _check(lib().ccz4_tag_learned(h, _ptr(logits), _ptr(plain_tags), float(conf), int(max_level),
                                         _ptr(tags), _stream(stream)))


def ccz4_constraints(h, Q, HM=None, r_excise=0.0, want_norms=True, stream=None):
    norms = (ctypes.c_double * 3)()
    st = lib().ccz4_constraints(h, _ptr(Q), _ptr(HM), float(r_excise),
                                ctypes.cast(norms, ctypes.c_void_p) if want_norms else None, _stream(stream))
    if st not in (CCZ4_OK, CCZ4_ENONFINITE):
        _check(st)
    return (list(norms), st) if want_norms else (None, st)


def ccz4_tag_refine(h, Q, theta_r, theta_c, max_level, tags, indicator=None, stream=None):
    return _check(lib().ccz4_tag_refine(h, _ptr(Q), float(theta_r), float(theta_c), int(max_level), _ptr(tags),
                                        _ptr(indicator), _stream(stream)))


def ccz4_last_error():
    return lib().ccz4_last_error().decode()


# ---------------------------------------------------------------- convenience wrapper

class Context:
    """One mesh of patches on the current device; state buffers are caller-owned tensors."""

    def __init__(self, n0, origin, extent, bc=BC_PERIODIC, prm=None, refined=()):
        self.prm = prm if prm is not None else params()
        self.bc = bc
        self.n0, self.origin, self.extent = tuple(n0), tuple(origin), tuple(extent)
        self.h = ccz4_create(n0, origin, extent, bc, self.prm, refined)
        self.n_patches, self.patch_doubles, self.bytes_per_state = ccz4_layout(self.h)
        self.ids, self.geom = ccz4_patch_table(self.h)

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            try:
                _lib.ccz4_destroy(self.h)
            except Exception:
                pass
            self.h = None

    __del__ = close

    def new_state(self, fill=0.0):
        import torch
        t = torch.empty((self.n_patches, NV, 15, 15, 16), dtype=torch.float64, device="cuda")
        t.fill_(fill)
        return t

    def set_params(self, prm):
        self.prm = prm
        ccz4_set_params(self.h, prm)

    def init_patches(self, Q, scenario, scen, stream=None):
        ccz4_init_patches(self.h, Q, scenario, scen, stream)

    def set_background(self, Q, stream=None):
        ccz4_set_background(self.h, Q, stream)

    def fill_halos(self, Q, stream=None):
        ccz4_fill_halos(self.h, Q, stream)

    def rhs(self, Q, k, precision=PREC_FP64, stream=None):
        ccz4_rhs(self.h, Q, k, precision, stream)

    def rk4_stage(self, s, dt, Qn, k, acc, Qnext, stream=None):
        ccz4_rk4_stage(self.h, s, dt, Qn, k, acc, Qnext, stream)

    def constraints(self, Q, HM=None, r_excise=0.0, stream=None):
        return ccz4_constraints(self.h, Q, HM, r_excise, True, stream)

    def tag_refine(self, Q, theta_r, theta_c, max_level, tags, indicator=None, stream=None):
        ccz4_tag_refine(self.h, Q, theta_r, theta_c, max_level, tags, indicator, stream)

    def rhs_rk4_stage(self, s, dt, Qs, Qn, acc, Qnext, precision=PREC_FP64, flags=0, stream=None):
        ccz4_rhs_rk4_stage(self.h, s, dt, Qs, Qn, acc, Qnext, precision, flags, stream)

    def reconstruct(self, Q, push=True, stream=None, flags=None):
        """Second-order formulation: the auxiliaries A, B, D, P of every interior cell from FD4
        differences of the primaries (whose halos must be filled); with push, also into the
        same-level neighbours' face halos.  flags, if given, replaces push (the STAGE_* flags, as
        ccz4_step_stage_flags gives them for a step)."""
        if flags is None:
            flags = STAGE_FILL_SAME_LEVEL if push else 0
        ccz4_reconstruct_aux(self.h, Q, flags, stream)

    def tracers_sample(self, Q, pos, slots, stream=None):
        """(n, len(slots)) float64 device tensor: trilinear samples at the points pos (n, 3) float64
        device tensor; NaN outside the mesh."""
        import torch
        out = torch.empty((pos.shape[0], len(slots)), dtype=torch.float64, device=pos.device)
        ccz4_tracers_sample(self.h, Q, pos, slots, out, stream)
        return out

    def tracers_advance(self, Q, pos, dt, stream=None):
        """Puncture trackers: one explicit Euler step with velocity -beta, in place on pos."""
        ccz4_tracers_advance(self.h, Q, pos, dt, stream)

    def tag_tracers(self, pos, radii, max_level, tags=None, stream=None):
        """int8 device tensor of refinement tags by coordinates (REFINE near the tracers, COARSEN
        where the parent cube is far from all of them)."""
        import torch
        if tags is None:
            tags = torch.empty(self.n_patches, dtype=torch.int8, device="cuda")
        ccz4_tag_tracers(self.h, pos, radii, max_level, tags, stream)
        return tags

    @property
    def second_order(self):
        return self.prm.formulation == FORMULATION_SO

    def fill_halos_kinds(self, Q, kinds, stream=None):
        ccz4_fill_halos_kinds(self.h, Q, kinds, stream)

    def plan_counts(self):
        return ccz4_plan_counts(self.h)

    def regrid(self, Q, tags, max_level, scenario, scen, stream=None):
        """(new context, new state) after the tags: plan, new mesh, the analytic initial data for
        its background and new ghost slabs, the transfer of Q, and a full halo fill."""
        refined = [tuple(int(v) for v in r) for r in ccz4_regrid_plan(self.h, tags, max_level)]
        new = Context(self.n0, self.origin, self.extent, self.bc, self.prm, refined)
        for prec in (PREC_FP64, PREC_MIXED):
            new.set_kernel(prec, self.get_kernel(prec))
        Qn = new.new_state(0.0)
        new.init_patches(Qn, scenario, scen, stream)
        ccz4_regrid_transfer(self.h, Q, new.h, Qn, stream)
        new.fill_halos(Qn, stream)
        return new, Qn

    def autotune(self, Q, precision=PREC_FP64, reps=3, stream=None):
        """Time the four launch configurations on this mesh and keep the fastest; returns the
        average stage times in ms (index = configuration)."""
        acc, Qx = self.new_state(0.0), self.new_state(0.0)
        ms = ccz4_autotune(self.h, Q, acc, Qx, precision, reps, stream)
        del acc, Qx
        return ms

    def step_graph(self, Qn, bufs, dt, precision=PREC_FP64):
        """A captured fused RK4 step on (Qn, Q1, Q2, acc) = (Qn,) + bufs; see StepGraph."""
        return StepGraph(self, Qn, bufs, dt, precision)

    def features(self, Q, HM, feat=None, stream=None):
        import torch
        if feat is None:
            feat = torch.empty((self.n_patches, MLP_NIN), dtype=torch.float32, device="cuda")
        ccz4_features(self.h, Q, HM, feat, stream)
        return feat

    def tag_learned(self, logits, plain_tags, conf, max_level, tags=None, stream=None):
        import torch
        if tags is None:
            tags = torch.empty(self.n_patches, dtype=torch.int8, device="cuda")
        ccz4_tag_learned(self.h, logits, plain_tags, conf, max_level, tags, stream)
        return tags

    def set_kernel(self, precision, kernel):
        ccz4_set_kernel(self.h, precision, kernel)

    def get_kernel(self, precision):
        return ccz4_get_kernel(self.h, precision)

    def step_stage_flags(self, s, precision=PREC_FP64):
        return ccz4_step_stage_flags(self.h, precision, s)

    def rk4_step_fused(self, Qn, dt, bufs, precision=PREC_FP64, stream=None, push=True):
        """One RK4 step in place on Qn with the fused stage kernel; bufs = (Q1, Q2, acc).
        With push (default) the stages handle the same-level halos themselves, with the flags of
        ccz4_step_stage_flags (read from the neighbours, or written into them), so only Neumann
        and coarse-fine faces are filled between stages; Qn must enter with all halos filled
        (ccz4_fill_halos once after the initial data) and leaves with them filled.  Without push
        every halo is filled before each stage."""
        Q1, Q2, acc = bufs
        order = ((Qn, Q1), (Q1, Q2), (Q2, Q1), (Q1, Qn))
        rest = FILL_NEUMANN | FILL_LEVELS
        for s, (src, dst) in enumerate(order):
            if push:
                if s > 0:
                    self.fill_halos_kinds(src, rest, stream)
                fl = self.step_stage_flags(s, precision)
                self.rhs_rk4_stage(s, dt, src, Qn, acc, dst, precision, fl, stream)
                if self.second_order:  # Algorithm 2: the auxiliaries of the new state
                    self.fill_halos_kinds(dst, rest, stream)
                    self.reconstruct(dst, stream=stream, flags=fl)
            else:
                self.fill_halos(src, stream)
                self.rhs_rk4_stage(s, dt, src, Qn, acc, dst, precision, 0, stream)
                if self.second_order:
                    self.fill_halos(dst, stream)
                    self.reconstruct(dst, False, stream)
        if push:
            self.fill_halos_kinds(Qn, rest, stream)

    def tune_step_buffers(self, Qn, dt, precision=PREC_FP64, pool=5, steps=2, stream=None):
        """Work buffers (Q1, Q2, acc) for fused steps on Qn, chosen for their place in memory.
        The same step runs up to about 8% faster or slower depending on where the driver places
        the state buffers in physical memory, and on which buffer plays which role.  This allocates
        `pool` state buffers, times `steps` fused steps on Qn with each of the `pool` rotations
        (i, i+1, i+2) of them in the three roles, keeps the fastest and frees the others.  Qn is
        advanced by pool * steps RK4 steps: it must enter with its halos filled, and leaves with
        them filled.  Returns ((Q1, Q2, acc), step times in ms per rotation)."""
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        bufs = [self.new_state(0.0) for _ in range(pool)]
        ms = []
        for i in range(pool):
            trio = (bufs[i], bufs[(i + 1) % pool], bufs[(i + 2) % pool])
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(steps):
                self.rk4_step_fused(Qn, dt, trio, precision, st)
            e1.record(st)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1) / steps)
        best = min(range(pool), key=lambda i: ms[i])
        keep = (bufs[best], bufs[(best + 1) % pool], bufs[(best + 2) % pool])
        del bufs
        return keep, ms

    def rk4_step(self, Qn, dt, bufs, precision=PREC_FP64, stream=None):
        """One RK4 step in place on Qn; bufs = (Qs, k, acc) work tensors of the state shape."""
        Qs, k, acc = bufs
        cur = Qn
        for s in range(4):
            self.fill_halos(cur, stream)
            self.rhs(cur, k, precision, stream)
            nxt = Qn if s == 3 else Qs
            self.rk4_stage(s, dt, Qn, k, acc, nxt, stream)
            if self.second_order:  # Algorithm 2: the auxiliaries of the new state
                self.fill_halos(nxt, stream)
                self.reconstruct(nxt, False, stream)
            cur = nxt



class StepGraph:
    """ccz4_step_graph_*: one fused RK4 step (push fill) captured once and replayed."""

    def __init__(self, ctx, Qn, bufs, dt, precision=PREC_FP64):
        Q1, Q2, acc = bufs
        self._keep = (ctx, Qn, Q1, Q2, acc)  # the graph holds raw pointers to these
        self.g = ccz4_step_graph_create(ctx.h, Qn, Q1, Q2, acc, dt, precision)

    def launch(self, stream=None):
        ccz4_step_graph_launch(self.g, stream)

    def close(self):
        if self.g is not None and _lib is not None:
            ccz4_step_graph_destroy(self.g)
        self.g = None
        self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
