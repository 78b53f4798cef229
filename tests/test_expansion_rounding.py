"""Rounding of the squared distances the far-field kernels form (host model of their
arithmetic, FP64 and FP32, against long double).

Expanded form (triangles, Table B rectangles, short distance-ratio levels): with d = P - c
(FP64), D^2 = dx^2 + dy^2 + dz^2 by FMAs, q1 = -2 f1.d and q2 = -2 f2.d from the element's
orthonormal frame (in the precision of the sums: the mixed path rounds d to FP32 first) and
the node staged divided by its weight, (a, b, a^2 + b^2, 1) / w^2,
    r^2 / w^2 = q1 a' + q2 b' + D^2 / w^2 + g'          (three FMAs),
whose reciprocal square root is w / r.
Pair rows (the 7 x 7 Gauss-Legendre rectangle rule): p = F d, da0 = p1 - a0, the row's
C = D^2 + (a0^2 + b^2) - 2 (p1 a0 + p2 b) and the two nodes a0 -+ s of a pair
r^2 = C + s^2 -+ 2 da0 s.

For a field point at distance ratio D/L >= 2 the expansion cancels at most a factor
(D + L)^2 / (D - L)^2 <= 9.  The checks: in FP64 the relative error of w/r stays within a
few ulp (the method's own accuracy floor is about 10 ulp, Sec. 4); in FP32 it stays below
the mixed path's 1e-6 budget down to DR 2 and near the FP32 unit roundoff at DR >= 3.
"""
import numpy as np
import pytest

L = np.longdouble


def _need_long_double():
    if np.finfo(np.longdouble).nmant < 60:
        pytest.skip("long double is not wider than double on this platform")


def _fma(a, b, c, t):
    """fma in precision t (exact product of the operands, one rounding)."""
    return (a.astype(L) * b.astype(L) + c.astype(L)).astype(t)


def _frames(n, rng):
    # as the library builds them: f1 along an edge, f3 the normal from a cross product,
    # f2 = f3 x f1 (orthonormal to rounding)
    f1 = rng.normal(size=(n, 3))
    f1 /= np.linalg.norm(f1, axis=1)[:, None]
    f3 = np.cross(f1, rng.normal(size=(n, 3)))
    f3 /= np.linalg.norm(f3, axis=1)[:, None]
    f2 = np.cross(f3, f1)
    return f1, f2, f3


def _setup(n, dr_lo, dr_hi, seed):
    rng = np.random.default_rng(seed)
    f1, f2, f3 = _frames(n, rng)
    size = np.exp(rng.uniform(np.log(1e-3), np.log(10.0), n))  # element size L
    c = rng.uniform(-100.0, 100.0, (n, 3))                          # centroid far from the origin too
    a = rng.uniform(-1.0, 1.0, n) * size * 0.7                      # node in the element plane, |n| <= L
    b = rng.uniform(-1.0, 1.0, n) * size * 0.7
    w = np.exp(rng.uniform(np.log(0.005), np.log(0.3), n))          # positive weight
    dr = np.exp(rng.uniform(np.log(dr_lo), np.log(dr_hi), n))
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    P = c + u * (dr * size)[:, None]
    return f1, f2, f3, c, a, b, w, P


def expanded_errors(t, n=200_000, dr_lo=2.0, dr_hi=100.0, seed=5):
    """Relative error of w/r from the kernels' expanded form in precision t."""
    _need_long_double()
    f1, f2, f3, c, a, b, w, P = _setup(n, dr_lo, dr_hi, seed)
    d = P - c  # FP64, as in the kernels
    D2 = _fma(d[:, 0], d[:, 0], _fma(d[:, 1], d[:, 1], d[:, 2] * d[:, 2], np.float64), np.float64)
    dt = d.astype(t)
    g1, g2 = (-2.0 * f1).astype(t), (-2.0 * f2).astype(t)
    q1 = _fma(dt[:, 0], g1[:, 0], _fma(dt[:, 1], g1[:, 1], (dt[:, 2] * g1[:, 2]).astype(t), t), t)
    q2 = _fma(dt[:, 0], g2[:, 0], _fma(dt[:, 1], g2[:, 1], (dt[:, 2] * g2[:, 2]).astype(t), t), t)
    iw2 = 1.0 / (w * w)
    g = _fma(a, a, b * b, np.float64)
    ap, bp, gp, iw = (a * iw2).astype(t), (b * iw2).astype(t), (g * iw2).astype(t), iw2.astype(t)
    x = _fma(q1, ap, _fma(q2, bp, _fma(D2.astype(t), iw, gp, t), t), t)
    got = 1 / np.sqrt(x.astype(L))
    # reference relative to the centroid (P - c of two doubles is exact in long double)
    n_ = a.astype(L)[:, None] * f1.astype(L) + b.astype(L)[:, None] * f2.astype(L)
    r = np.sqrt(np.sum((P.astype(L) - c.astype(L) - n_) ** 2, axis=1))
    exact = w.astype(L) / r
    return np.abs((got - exact) / exact).astype(np.float64)


def pair_row_errors(t, n=200_000, dr_lo=2.0, dr_hi=100.0, seed=6):
    """Relative error of 1/r for both nodes a0 -+ s of a pair row in precision t."""
    _need_long_double()
    f1, f2, f3, c, a, b, w, P = _setup(n, dr_lo, dr_hi, seed)
    a0 = a * 0.01                                              # parallelogram shift of the row
    s = np.abs(a)                                              # half distance of the pair
    d64 = P - c
    D2 = _fma(d64[:, 0], d64[:, 0], _fma(d64[:, 1], d64[:, 1], d64[:, 2] * d64[:, 2], np.float64), np.float64)
    d = d64.astype(t)
    p1, p2 = [_fma(d[:, 0], f[:, 0].astype(t), _fma(d[:, 1], f[:, 1].astype(t), (d[:, 2] * f[:, 2].astype(t)).astype(t), t), t)
              for f in (f1, f2)]
    q1, q2 = (-2 * p1).astype(t), (-2 * p2).astype(t)
    at0, bt = a0.astype(t), b.astype(t)
    g0 = _fma(a0, a0, b * b, np.float64).astype(t)  # staged in FP64, rounded to t
    C = _fma(q1, at0, _fma(q2, bt, (D2.astype(t) + g0).astype(t), t), t)
    da0 = (p1 - at0).astype(t)
    st = s.astype(t)
    u = (C + (st * st).astype(t)).astype(t)
    errs = []
    for sign in (-1.0, 1.0):  # node a0 + s: r^2 = u - 2 da0 s; node a0 - s: u + 2 da0 s
        x = _fma((sign * 2.0 * da0).astype(t), st, u, t)
        got = 1 / np.sqrt(x.astype(L))
        n_ = (a0.astype(L) - sign * s.astype(L))[:, None] * f1.astype(L) + b.astype(L)[:, None] * f2.astype(L)
        exact = 1 / np.sqrt(np.sum((P.astype(L) - c.astype(L) - n_) ** 2, axis=1))
        errs.append(np.abs((got - exact) / exact).astype(np.float64))
    return np.concatenate(errs)


@pytest.mark.parametrize("form", [expanded_errors, pair_row_errors])
def test_fp64_forms_round_like_the_differences(form):
    """At distance ratio >= 3 (the default switch) within 2 ulp, down to 2 within 3 ulp; the
    difference form (p - n)^2 of a correctly rounded point rounds to about 1 ulp."""
    ulp = np.finfo(np.float64).eps
    e3 = form(np.float64, dr_lo=3.0, seed=9) / ulp
    e2 = form(np.float64) / ulp
    print(f"FP64 {form.__name__}: DR>=3 max {e3.max():.2f} ulp, DR>=2 max {e2.max():.2f}, median {np.median(e2):.2f}")
    assert e3.max() < 2.0 and e2.max() < 3.0 and np.median(e2) < 0.5


@pytest.mark.parametrize("form", [expanded_errors, pair_row_errors])
def test_fp32_forms_within_the_mixed_budget(form):
    e2 = form(np.float32)                     # distance ratios 2 .. 100
    e3 = form(np.float32, dr_lo=3.0, seed=9)  # 3 .. 100
    eps = np.finfo(np.float32).eps
    print(f"FP32 {form.__name__}: DR>=2 max {e2.max():.2e}, DR>=3 max {e3.max():.2e} ({e3.max() / eps:.1f} eps)")
    assert e2.max() < 1e-6
    assert e3.max() < 8 * eps
