"""Pins of the error normalisers and of the distance-ratio switch that every GPU parity
gate depends on.

The gates divide an error by a sum of per-element magnitudes computed by the oracle
(the potential's sum of |phi_j|, the field's sum of |E_j|, the collocation rows' sums per
right-hand side, the gradient's per-element and per-term scales).  A scale slip there (a
doubled constant, an L1 instead of a Euclidean norm, the wrong right-hand side) would
make a gate vacuous, so each is checked here against values obtained independently:
single-element calls, sign flips, closed forms and the point-charge limit.

The distance ratio DR = D / L with L the average side length (Sec. 2) decides where the
rule is applied directly and where the element is subdivided.  L is computed here with
numpy from the vertices ((a + b + c) / 3 for a triangle, the mean of the four sides,
(a + b) / 2, for a rectangle) and points are placed a relative 1e-9 inside and outside
D = 3 L: the oracle must call the first near and the second far.  Too small an L would
fail the inside points, too large an L (the perimeter, a + b, the longest side) the
outside ones.
"""
import numpy as np
import pytest

import ref_integrals as RI

K_SI = 1.0 / (4.0 * np.pi * 8.8541878188e-12)


def rand_tri(rng, scale=1.0):
    A = rng.normal(size=3) * scale
    B = A + rng.normal(size=3) * scale
    C = A + rng.normal(size=3) * scale
    return np.concatenate([A, B, C])


def rand_rect(rng, aspect=3.0):
    e1 = rng.normal(size=3)
    e2 = rng.normal(size=3)
    e2 -= (e2 @ e1) / (e1 @ e1) * e1
    e1 *= aspect / np.linalg.norm(e1)
    e2 *= 1.0 / np.linalg.norm(e2)
    return np.concatenate([rng.normal(size=3), e1, e2])


def numpy_L(kind, g):
    if kind == 0:
        A, B, C = g[0:3], g[3:6], g[6:9]
        return (np.linalg.norm(B - A) + np.linalg.norm(C - B) + np.linalg.norm(A - C)) / 3.0
    return 0.5 * (np.linalg.norm(g[3:6]) + np.linalg.norm(g[6:9]))


def numpy_centroid(kind, g):
    if kind == 0:
        return (g[0:3] + g[3:6] + g[6:9]) / 3.0
    return g[0:3] + 0.5 * g[3:6] + 0.5 * g[6:9]


def split(kind, g):
    g = np.asarray(g, float)[None, :]
    return (g, None) if kind == 0 else (None, g)


def far_points(cen, L, rng, n=8, dr=(4.0, 40.0)):
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    r = np.exp(rng.uniform(np.log(dr[0]), np.log(dr[1]), n)) * L
    return cen + d * r[:, None]


# ----------------------------------------------------------- distance ratio, L ------
@pytest.mark.parametrize("kind", [0, 1])
def test_distance_ratio_switch_uses_average_side(orc, kind):
    rng = np.random.default_rng(31 + kind)
    for _ in range(20):
        g = rand_tri(rng) if kind == 0 else rand_rect(rng, aspect=rng.uniform(1.0, 6.0))
        L = numpy_L(kind, g)
        cen = numpy_centroid(kind, g)
        c_orc, _, L_orc = orc.element_geometry(kind, g)
        assert np.allclose(c_orc, cen, rtol=0, atol=1e-15 * np.abs(g).max() * 4)
        assert abs(L_orc - L) <= 4e-16 * L
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        for f, near in ((1.0 - 1e-9, 1), (1.0 + 1e-9, 0)):
            P = cen + 3.0 * L * f * d
            _, st = orc.element(kind, g, P, orc.params(), mode=1)
            assert st["near_pairs"] == near, (kind, f, L)
            # the threshold scales with near_dr: at near_dr 5 the same point is near
            _, st5 = orc.element(kind, g, P, orc.params(near_dr=5.0), mode=1)
            assert st5["near_pairs"] == 1


# ------------------------------------------------------ potential / field sums ------
@pytest.mark.parametrize("kind", [0, 1])
def test_single_element_normalisers_equal_magnitudes(orc, kind):
    """One element of positive density: abs_phi = |phi| and abs_E = |E| (Euclidean)."""
    rng = np.random.default_rng(5 + kind)
    g = rand_tri(rng) if kind == 0 else rand_rect(rng)
    cen, L = numpy_centroid(kind, g), numpy_L(kind, g)
    pts = np.concatenate([far_points(cen, L, rng), far_points(cen, L, rng, dr=(0.05, 2.5))])
    tri, rect = split(kind, g)
    ref = orc.evaluate(tri, rect, np.array([0.7]), pts, orc.params(), with_abs=True)
    assert np.allclose(ref["abs_phi"], np.abs(ref["phi"]), rtol=1e-15, atol=0)
    assert np.allclose(ref["abs_E"], np.linalg.norm(ref["E"], axis=1), rtol=1e-15, atol=0)
    # negative density: the magnitudes, not the signed values
    neg = orc.evaluate(tri, rect, np.array([-0.7]), pts, orc.params(), with_abs=True)
    assert np.array_equal(neg["abs_phi"], ref["abs_phi"]) and np.array_equal(neg["abs_E"], ref["abs_E"])
    assert np.all(neg["phi"] < 0) == np.all(ref["phi"] > 0)


def test_two_elements_normalisers_add_magnitudes(orc):
    """sigma = (+1, -1): the sums cancel, the normalisers add the two single-element
    magnitudes obtained from separate calls."""
    rng = np.random.default_rng(9)
    t = rand_tri(rng)
    r = rand_rect(rng)
    r[0:3] += 0.3
    pts = rng.normal(size=(40, 3)) * 4.0
    both = orc.evaluate(t[None, :], r[None, :], np.array([1.0, -1.0]), pts, orc.params(), with_abs=True)
    one = orc.evaluate(t[None, :], None, np.array([1.0]), pts, orc.params(), with_abs=True)
    two = orc.evaluate(None, r[None, :], np.array([1.0]), pts, orc.params(), with_abs=True)
    assert np.allclose(both["abs_phi"], np.abs(one["phi"]) + np.abs(two["phi"]), rtol=1e-14, atol=0)
    assert np.allclose(both["abs_E"], np.linalg.norm(one["E"], axis=1) + np.linalg.norm(two["E"], axis=1),
                       rtol=1e-14, atol=0)
    assert np.allclose(both["phi"], one["phi"] - two["phi"], rtol=0, atol=1e-14 * both["abs_phi"].max())


def test_normaliser_constant_is_coulomb(orc):
    """A far point sees the element as its total charge: abs_phi -> K |Q| / D and
    abs_E -> K |Q| / D^2 with K = 1 / (4 pi eps0) (SI, Sec. 2)."""
    rng = np.random.default_rng(2)
    g = rand_rect(rng)
    area = np.linalg.norm(g[3:6]) * np.linalg.norm(g[6:9])
    cen = numpy_centroid(1, g)
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    D = 1e4 * numpy_L(1, g)
    ref = orc.evaluate(None, g[None, :], np.array([-2.0]), (cen + D * d)[None, :], orc.params(), with_abs=True)
    Q = 2.0 * area
    assert abs(ref["abs_phi"][0] / (K_SI * Q / D) - 1.0) < 1e-7
    assert abs(ref["abs_E"][0] / (K_SI * Q / D ** 2) - 1.0) < 1e-7


# ------------------------------------------------------------------ collocation -----
def test_collocation_normaliser_per_right_hand_side(orc):
    """abs[r][k] = K sum_j |sigma_rj| |phi_j(c_k)| for every right-hand side r, with
    phi_j from single-element evaluations at the centroids (including the element's own
    on-element integral)."""
    rng = np.random.default_rng(21)
    tris = np.stack([rand_tri(rng, 0.5) + np.tile(rng.normal(size=3) * 2, 3) for _ in range(4)])
    rects = np.stack([rand_rect(rng, 2.0) for _ in range(3)])
    rects[:, 0:3] += rng.normal(size=(3, 3)) * 2
    ne = 7
    sig = rng.normal(size=(3, ne))
    sig[1] *= 1e-3
    sig[2] = np.abs(sig[2])
    col = orc.collocation(tris, rects, sig)
    cen = np.concatenate([[numpy_centroid(0, g) for g in tris], [numpy_centroid(1, g) for g in rects]])
    phi = np.zeros((ne, ne))  # phi[j][k]: unit-density potential of element j at centroid k
    for j in range(ne):
        t, r = (tris[j:j + 1], None) if j < 4 else (None, rects[j - 4:j - 3])
        phi[j] = orc.evaluate(t, r, np.array([1.0]), cen, orc.params())["phi"]
    expect = np.abs(sig)[:, :, None] * np.abs(phi)[None, :, :]  # [r][j][k]
    assert col["abs"].shape == (3, ne)
    assert np.allclose(col["abs"], expect.sum(axis=1), rtol=1e-13, atol=0)
    assert np.allclose(col["out"], np.einsum("rj,jk->rk", sig, phi), rtol=0, atol=1e-13 * col["abs"].max())
    # the all-positive right-hand side has no cancellation: its normaliser is its value
    assert np.allclose(col["abs"][2], np.abs(col["out"][2]), rtol=1e-12)


# --------------------------------------------------------------------- gradient -----
def test_gradient_normaliser_is_frobenius_norm_of_closed_form(orc):
    """One rectangle, sigma = 1: abs_G = K |G|_F with G the closed-form Hessian of the
    uniformly charged rectangle (all nine entries: the off-diagonal ones count twice)."""
    rng = np.random.default_rng(4)
    g = rand_rect(rng, 2.0)
    cen, L = numpy_centroid(1, g), numpy_L(1, g)
    pts = far_points(cen, L, rng, n=6, dr=(6.0, 60.0))
    ref = orc.gradient(None, g[None, :], np.array([1.0]), pts, orc.params())
    for k, P in enumerate(pts):
        H = K_SI * RI.rect_gradient_closed_form(g, P)
        assert abs(ref["abs_G"][k] / np.linalg.norm(H) - 1.0) < 1e-9
        # and the per-term scale tends to it: sqrt(6) |q| / r^3 per term, r -> D
    # point-charge limit of the per-term scale: K |Q| sqrt(6) / D^3
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    D = 1e4 * L
    far = orc.gradient(None, g[None, :], np.array([-3.0]), (cen + D * d)[None, :], orc.params())
    Q = 3.0 * np.linalg.norm(g[3:6]) * np.linalg.norm(g[6:9])
    assert abs(far["abs_T"][0] / (K_SI * Q * np.sqrt(6.0) / D ** 3) - 1.0) < 1e-7
    assert abs(far["abs_G"][0] / (K_SI * Q * np.sqrt(6.0) / D ** 3) - 1.0) < 1e-7


def test_gradient_normalisers_add_over_elements(orc):
    """sigma = (+1, -1) on two elements: abs_G and abs_T are the sums of the single-element
    values from separate calls."""
    rng = np.random.default_rng(12)
    t = rand_tri(rng)
    r = rand_rect(rng)
    r[0:3] += 0.5
    pts = rng.normal(size=(30, 3)) * 5.0
    both = orc.gradient(t[None, :], r[None, :], np.array([1.0, -1.0]), pts, orc.params())
    one = orc.gradient(t[None, :], None, np.array([1.0]), pts, orc.params())
    two = orc.gradient(None, r[None, :], np.array([1.0]), pts, orc.params())
    fro = lambda G: np.linalg.norm(orc.gradient_matrix(G), axis=(1, 2))  # noqa: E731
    assert np.allclose(one["abs_G"], fro(one["G"]), rtol=1e-14, atol=0)
    assert np.allclose(both["abs_G"], fro(one["G"]) + fro(two["G"]), rtol=1e-14, atol=0)
    assert np.allclose(both["abs_T"], one["abs_T"] + two["abs_T"], rtol=1e-14, atol=0)
