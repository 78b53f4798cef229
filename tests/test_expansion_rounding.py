"""Rounding of the expanded squared distance used by the far-field kernels (host check).

The far-field kernels form, in each element's frame, r^2 = |p|^2 + (a^2 + b^2) - 2 (p1 a + p2 b)
instead of (p1 - a)^2 + (p2 - b)^2 + p3^2.  For a field point at distance ratio >= 3 the
expansion cancels at most a factor (D + L)^2 / (D - L)^2 ~ 4, and after the square root the
error of 1/r stays close to that of the difference form.  This test measures both forms in
IEEE double (numpy) against long double on points at distance ratios 3..100 and checks the
statement made in the kernels' comments: about a tenth of an ulp more, nothing more.
"""
import numpy as np
import pytest


def _errors(n=100_000, seed=5):
    if np.finfo(np.longdouble).nmant < 60:
        pytest.skip("long double is not wider than double on this platform")
    rng = np.random.default_rng(seed)
    a = rng.uniform(-0.6, 0.6, n)
    b = rng.uniform(-0.6, 0.6, n)
    dr = np.exp(rng.uniform(np.log(3.0), np.log(100.0), n))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    p = d * dr[:, None]
    p1, p2, p3 = p[:, 0], p[:, 1], p[:, 2]
    h = p3 * p3
    L = np.longdouble
    exact = 1 / np.sqrt((p1.astype(L) - a) ** 2 + (p2.astype(L) - b) ** 2 + p3.astype(L) ** 2)
    diff = (p1 - a) * (p1 - a) + ((p2 - b) * (p2 - b) + h)
    H = p1 * p1 + (p2 * p2 + h)
    expd = (-2 * p1) * a + ((-2 * p2) * b + (H + (a * a + b * b)))
    ulp = np.finfo(np.float64).eps
    out = []
    for r2 in (diff, expd):
        ri = 1 / np.sqrt(r2.astype(L))
        out.append(np.abs((ri - exact) / exact).astype(np.float64) / ulp)
    return out


def test_expanded_distance_rounds_like_the_differences():
    e_diff, e_exp = _errors()
    assert e_exp.max() < 1.5 and e_diff.max() < 1.5
    assert e_exp.max() - e_diff.max() < 0.3
    assert np.median(e_exp) < 1.3 * np.median(e_diff) + 0.02
