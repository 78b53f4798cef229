"""Pins of the oracle's cubature rules against exact monomial moments.

A cubature rule of degree d integrates every monomial x^n y^m with n + m <= d exactly
and fails for some monomial of degree d + 1 (Sec. 3).  The weights sum to one
(Eq. 3.1).  Exact moments:
  reference triangle (x = lambda_B, y = lambda_C):  mean of x^n y^m = 2 n! m! / (n+m+2)!
  square [-1, 1]^2:                                 mean = prod_k 1/(k+1) for even k, else 0
A mistyped digit, a wrong orbit expansion (e.g. full permutations instead of the cyclic
ones of the 12-point rule) or a swapped weight breaks exactness at the stated degree.
"""
import json
import math
import os

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "dr_limits_sec4.json")))
DEG = GOLD["degree"]


def tri_moment(n, m):
    return 2.0 * math.factorial(n) * math.factorial(m) / math.factorial(n + m + 2)


def sq_moment(n, m):
    f = lambda k: 0.0 if k % 2 else 1.0 / (k + 1)
    return f(n) * f(m)


def max_tri_err(lam, w, deg):
    x, y = lam[:, 1], lam[:, 2]
    return max(abs(np.sum(w * x ** n * y ** (d - n)) - tri_moment(n, d - n)) for d in [deg] for n in range(d + 1))


def max_sq_err(xy, w, deg):
    x, y = xy[:, 0], xy[:, 1]
    return max(abs(np.sum(w * x ** n * y ** (deg - n)) - sq_moment(n, deg - n)) for n in range(deg + 1))


@pytest.mark.parametrize("n", [4, 7, 12, 19, 33])
def test_triangle_rule_degree(orc, n):
    lam, w = orc.tri_rule(n)
    d = DEG[f"tri{n}"]
    assert lam.shape == (n, 3)
    assert abs(w.sum() - 1.0) < 4e-16
    assert np.all(np.abs(lam.sum(axis=1) - 1.0) < 4e-16)
    for k in range(d + 1):
        assert max_tri_err(lam, w, k) < 1e-15, (n, k)
    assert max_tri_err(lam, w, d + 1) > 1e-9, "rule is more exact than its stated degree"


@pytest.mark.parametrize("n", [4, 7, 12, 17, 33])
def test_rectangle_table_degree(orc, n):
    xy, w = orc.rect_rule(0, n)
    d = DEG[f"rect{n}"]
    assert xy.shape == (n, 2)
    assert abs(w.sum() - 1.0) < 4e-16
    assert np.all(np.abs(xy) <= 1.0)
    for k in range(d + 1):
        assert max_sq_err(xy, w, k) < 1e-15, (n, k)
    assert max_sq_err(xy, w, d + 1) > 1e-7


def test_positive_weights_and_interior_nodes(orc):
    """All rules except the 4-point triangle rule have positive weights and interior nodes
    (Sec. 3 prefers both; Table A1 has the negative centroid weight -9/16)."""
    for n in (7, 12, 19, 33):
        lam, w = orc.tri_rule(n)
        assert np.all(w > 0) and np.all(lam > 0)
    lam, w = orc.tri_rule(4)
    assert w[0] == -9.0 / 16.0
    for n in (4, 7, 12, 17, 33):
        xy, w = orc.rect_rule(0, n)
        assert np.all(w > 0)


def test_twelve_point_rule_is_cyclic_not_symmetric(orc):
    """Table A3 expands each row by cyclic shifts only: reflecting the rule (swap B, C)
    gives a different node set."""
    lam, _ = orc.tri_rule(12)
    refl = lam[:, [0, 2, 1]]
    same = [np.min(np.linalg.norm(lam - r, axis=1)) < 1e-15 for r in refl]
    assert not all(same)


@pytest.mark.parametrize("n", list(range(1, 17)) + [24, 32, 48, 64])
def test_gauss_legendre_matches_library(orc, n):
    """Newton-iteration nodes vs numpy's Golub-Welsch-based leggauss (a library routine)."""
    x, w = orc.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.max(np.abs(x - xr)) < 4e-15
    assert np.max(np.abs(w - wr)) < 4e-15
    # exact for polynomials of degree 2n - 1
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-14


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 10, 16])
def test_tensor_gauss_rectangle_rule(orc, n):
    xy, w = orc.rect_rule(n, 0)
    assert xy.shape == (n * n, 2)
    assert abs(w.sum() - 1.0) < 1e-15
    for a in range(2 * n):
        for b in range(2 * n):
            assert abs(np.sum(w * xy[:, 0] ** a * xy[:, 1] ** b) - sq_moment(a, b)) < 4e-15
    # not exact at degree 2n in x alone
    assert abs(np.sum(w * xy[:, 0] ** (2 * n)) - sq_moment(2 * n, 0)) > 1e-11


def test_seven_point_closed_forms(orc):
    """Table A2 written with t, s, r: the coordinates are t+2ts, t-ts etc.  Check the
    oracle's expansion against the same numbers written as decimals of the closed forms
    evaluated independently here with mpmath."""
    import mpmath as mp

    mp.mp.dps = 40
    q = mp.sqrt(15)
    t = mp.mpf(1) / 3
    s, r = (1 - q) / 7, (1 + q) / 7
    a1, b1 = t + 2 * t * s, t - t * s
    a2, b2 = t + 2 * t * r, t - t * r
    lam, w = orc.tri_rule(7)
    got = sorted((round(float(l[0]), 15), round(float(wi), 15)) for l, wi in zip(lam, w))
    exp = sorted([(round(float(t), 15), round(float(mp.mpf(9) / 40), 15))]
                 + [(round(float(a1), 15), round(float((155 + q) / 1200), 15))]
                 + [(round(float(b1), 15), round(float((155 + q) / 1200), 15))] * 2
                 + [(round(float(a2), 15), round(float((155 - q) / 1200), 15))]
                 + [(round(float(b2), 15), round(float((155 - q) / 1200), 15))] * 2)
    assert got == exp
