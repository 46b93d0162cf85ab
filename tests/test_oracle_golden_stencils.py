"""The oracle's one-dimensional stencils against the weights printed in App. D
(tests/golden/app_d_stencils.txt): each stencil applied to the unit impulses at offsets -3..+3
must return the printed weight times the printed factor over dx (times eps for KO)."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as orc

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "app_d_stencils.txt")


def load():
    out, cur = {}, None
    with open(GOLDEN) as fh:
        lines = fh.read().splitlines()
    for ln in lines:
        ln = ln.strip()
        if not ln or ln.startswith("#"):
            continue
        if ln.startswith("["):
            name, _, fac = ln[1:].partition("]")
            cur = name
            out[cur] = [float(Fraction(fac.split()[1]))]
        else:
            out[cur] = np.array([float(Fraction(t)) for t in ln.split()]) * out[cur][0]
    return out


S = load()
DX = 0.37


def impulses(fn, width):
    """fn applied to the unit impulse at each offset of a stencil of the given width."""
    return np.array([fn(np.eye(width)[j]) for j in range(width)])


def test_central_fd4_is_the_printed_stencil():
    got = impulses(lambda v: orc.fd4(v, DX), 5)
    np.testing.assert_allclose(got * DX, S["fd4_central"][1:6], rtol=0, atol=1e-15)


def test_ko_is_the_printed_sum():
    eps = 0.1
    got = impulses(lambda v: orc.ko(v, DX, eps), 7)
    np.testing.assert_allclose(got * DX / eps, S["ko"], rtol=0, atol=1e-14)


@pytest.mark.parametrize("right,name", [(0, "fd4_lopsided_left"), (1, "fd4_lopsided_right")])
def test_lopsided_pair_is_the_printed_pair(right, name):
    """The right-biased member reads Q+++ and not Q---, the left-biased one the reverse."""
    got = impulses(lambda v: orc.fd4_lop(v, DX, right), 7)
    np.testing.assert_allclose(got * DX, S[name], rtol=0, atol=1e-14)
