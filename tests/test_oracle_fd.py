"""Pins of the oracle's finite-difference primitives (no GPU).

Each check fixes the primitives against something other than their own code:
two independent derivations of the weights, textbook values, polynomial
exactness, dense-matrix transposition and the truncation identities
D^T = -D and (D+)^T = -D- that make the rotated TTI operators self-adjoint.
"""
from fractions import Fraction

import numpy as np
import pytest


@pytest.mark.parametrize("so", [2, 4, 6, 8, 10, 12, 14, 16])
def test_centered_closed_form_equals_fornberg(orc, so):
    r = so // 2
    w = orc.fornberg(1, 0, list(range(-r, r + 1)))
    assert w[r] == 0
    assert w[r + 1:] == orc.fd_centered(so)
    assert [-x for x in reversed(w[:r])] == orc.fd_centered(so)


def test_textbook_weights(orc):
    # classical 4th-order centred and staggered first-derivative stencils
    assert orc.fd_centered(4) == [Fraction(2, 3), Fraction(-1, 12)]
    assert orc.fd_centered(2) == [Fraction(1, 2)]
    assert orc.fd_staggered(4) == [Fraction(9, 8), Fraction(-1, 24)]
    assert orc.fd_staggered(2) == [Fraction(1)]


@pytest.mark.parametrize("so", [4, 8, 12, 16])
def test_polynomial_exactness(orc, so):
    """D x^p is exact for p <= so (centred) and p <= so (staggered, at half nodes)."""
    r = so // 2
    a, c = orc.fd_centered(so), orc.fd_staggered(so)
    for p in range(0, so + 1):
        # centred at x = 0 on unit spacing: sum_j a_j (j^p - (-j)^p) == d/dx x^p at 0
        val = sum(a[j - 1] * (Fraction(j) ** p - Fraction(-j) ** p) for j in range(1, r + 1))
        assert val == (1 if p == 1 else 0)
        # staggered at x = 0 with nodes +-(j-1/2)
        val = sum(c[j - 1] * (Fraction(2 * j - 1, 2) ** p - Fraction(-(2 * j - 1), 2) ** p)
                  for j in range(1, r + 1))
        assert val == (1 if p == 1 else 0)


def _dense(orc, g, fn):
    n = g.shape[0]
    M = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(g.arr_shape)
        e[0, 0, i] = 1.0
        M[:, i] = fn(e).reshape(-1)
    return M


@pytest.mark.parametrize("so", [4, 8, 12])
def test_dense_truncation_identities(orc, so):
    g = orc.Grid((16, 1, 1), (0.7, 1.0, 1.0), space_order=so)
    D = _dense(orc, g, lambda f: orc.dcen(g, 0, f))
    DT = _dense(orc, g, lambda f: orc.dcen(g, 0, f, transpose=True))
    Dp = _dense(orc, g, lambda f: orc.dstag(g, 0, True, f))
    Dm = _dense(orc, g, lambda f: orc.dstag(g, 0, False, f))
    DpT = _dense(orc, g, lambda f: orc.dstag(g, 0, True, f, transpose=True))
    DmT = _dense(orc, g, lambda f: orc.dstag(g, 0, False, f, transpose=True))
    assert np.abs(DT - D.T).max() < 1e-15
    assert np.abs(DpT - Dp.T).max() < 1e-15
    assert np.abs(DmT - Dm.T).max() < 1e-15
    assert np.abs(D + D.T).max() < 1e-15          # D^T = -D under truncation
    assert np.abs(Dp.T + Dm).max() < 1e-15        # (D+)^T = -D-
    # interior rows are the textbook stencil divided by h
    r = so // 2
    a = [float(x) for x in orc.fd_centered(so)]
    row = D[8]
    for j in range(1, r + 1):
        assert abs(row[8 + j] - a[j - 1] / 0.7) < 1e-14 and abs(row[8 - j] + a[j - 1] / 0.7) < 1e-14


@pytest.mark.parametrize("so", [4, 8])
def test_derivative_convergence_order(orc, so):
    """Centred and staggered derivatives of sin converge at the stencil order under refinement."""
    errs_c, errs_s = [], []
    for n in (40, 80):
        L = 1.0
        h = L / (n - 1)
        x = np.arange(n) * h
        g = orc.Grid((n, 1, 1), (h, 1.0, 1.0), space_order=so)
        f = np.sin(10 * x).reshape(g.arr_shape)
        r = so // 2
        inner = slice(2 * r, n - 2 * r)
        dc = orc.dcen(g, 0, f).reshape(-1)
        errs_c.append(np.abs(dc[inner] - 10 * np.cos(10 * x[inner])).max())
        ds = orc.dstag(g, 0, True, f).reshape(-1)
        errs_s.append(np.abs(ds[inner] - 10 * np.cos(10 * (x[inner] + h / 2))).max())
    rate_c = np.log2(errs_c[0] / errs_c[1]) * np.log(2) / np.log(79 / 39)
    rate_s = np.log2(errs_s[0] / errs_s[1]) * np.log(2) / np.log(79 / 39)
    assert rate_c > so - 0.5
    assert rate_s > so - 0.5
