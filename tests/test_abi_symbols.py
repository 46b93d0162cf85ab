"""The C-ABI library loads on a machine without a GPU and exports every function that
include/ccz4.h declares; argument errors are reported before any HIP call."""
import ctypes
import os
import re

import pytest

from paper_2406_11626_amd import ccz4

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "ccz4.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ccz4_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for n in ("ccz4_init_patches", "ccz4_fill_halos", "ccz4_rhs", "ccz4_rk4_stage",
              "ccz4_constraints", "ccz4_tag_refine", "ccz4_create", "ccz4_destroy", "ccz4_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = ccz4.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_argument_errors_without_gpu():
    L = ccz4.lib()
    assert L.ccz4_create(None, None, None) == ccz4.CCZ4_EINVAL
    h = ctypes.c_void_p()
    assert L.ccz4_create(ctypes.byref(h), None, None) == ccz4.CCZ4_EINVAL
    assert b"NULL" in L.ccz4_last_error()
    for fn, args in (("ccz4_fill_halos", (None, None, None)), ("ccz4_rhs", (None, None, None, 0, None)),
                     ("ccz4_rk4_stage", (None, 0, 0.1, None, None, None, None, None)),
                     ("ccz4_constraints", (None, None, None, 0.0, None, None)),
                     ("ccz4_set_kernel", (None, 0, 1)), ("ccz4_get_kernel", (None, 0, None)),
                     ("ccz4_reconstruct_aux", (None, None, 0, None)),
                     ("ccz4_mlp_grad_noalloc", (None, None, None, None, 1, None, None, None))):
        assert getattr(L, fn)(*args) == ccz4.CCZ4_EINVAL
    # the no-allocation gradient: row counts outside 1..CCZ4_MLP_NOALLOC_MAX_ROWS before any launch
    buf = (ctypes.c_float * 4)()
    for n in (0, -1, ccz4.MLP_NOALLOC_MAX_ROWS + 1):
        assert L.ccz4_mlp_grad_noalloc(buf, buf, buf, buf, n, buf, None, None) == ccz4.CCZ4_EINVAL
    g = ccz4.GridDesc()
    g.n0[:] = [0, 1, 1]
    g.extent[:] = [1.0, 1.0, 1.0]
    prm = ccz4.params()
    assert L.ccz4_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(prm)) == ccz4.CCZ4_EINVAL
    g.n0[:] = [1, 1, 1]
    bad = ccz4.params(slicing=7)
    assert L.ccz4_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(bad)) == ccz4.CCZ4_EINVAL
    bad = ccz4.params(formulation=2)
    assert L.ccz4_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(bad)) == ccz4.CCZ4_EINVAL
    assert b"formulation" in L.ccz4_last_error()
    for bad, word in ((ccz4.params(advection=3), b"advection"), (ccz4.params(transfer=2), b"transfer")):
        assert L.ccz4_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(bad)) == ccz4.CCZ4_EINVAL
        assert word in L.ccz4_last_error()
    ccz4.ccz4_destroy(None)
