"""Pins of the oracle's field gradient dE_i/dx_j (the conclusions: higher derivatives of
the potential follow from the same point charges of Eq. 4.1).

References independent of the oracle:
* rectangles: the closed-form Hessian of the uniformly charged rectangle (corner sums of
  textbook antiderivatives), itself checked against nested Gauss-Legendre quadrature of
  the gradient kernel;
* triangles: nested Gauss-Legendre at distance ratios >= 2 and, closer in, Richardson
  central differences of the semi-analytic field;
* meshes: trace-free (Laplace), finite differences of the oracle's own (pinned) field,
  and the point-charge limit far away.
"""
import numpy as np
import pytest

import oracle
import ref_integrals as RI
from paper_1606_03743_amd import workloads as W


def _rect():
    e1 = np.array([1.3, 0.2, 0.0])
    e2 = np.array([-0.2, 1.3, 0.5])
    e2 = 0.6 * (e2 - (e2 @ e1) / (e1 @ e1) * e1)
    g = np.concatenate([[0.2, -0.1, 0.3], e1, e2])
    L = 0.5 * (np.linalg.norm(e1) + np.linalg.norm(e2))
    return g, g[0:3] + 0.5 * e1 + 0.5 * e2, L


def _tri():
    g = np.array([0.1, 0.2, -0.3, 1.2, 0.1, 0.2, 0.3, 0.9, -0.1])
    A, B, C = g[0:3], g[3:6], g[6:9]
    L = (np.linalg.norm(B - A) + np.linalg.norm(C - B) + np.linalg.norm(A - C)) / 3
    return g, (A + B + C) / 3, L


def _points(cen, L, drs, seed):
    rng = np.random.default_rng(seed)
    out = []
    for dr in drs:
        d = rng.normal(size=3)
        out.append((dr, cen + dr * L * d / np.linalg.norm(d)))
    return out


def _rel(a, b):
    return np.abs(a - b).max() / np.linalg.norm(b)


def test_rect_closed_form_is_the_quadrature():
    """The reference Hessian itself against direct quadrature of the kernel.  The corner
    sums cancel to a result ~DR^-3 smaller than their terms: tolerance eps * DR^3."""
    g, cen, L = _rect()
    for dr, P in _points(cen, L, [2.0, 4.0, 10.0, 40.0], 3):
        tol = max(1e-14, 4e-16 * dr ** 3)
        assert _rel(RI.rect_gradient_closed_form(g, P), RI.gl2_gradient(1, g, P, 64)) < tol, dr


@pytest.mark.parametrize("seed", [1, 2])
def test_rect_gradient_matches_closed_form(orc, seed):
    g, cen, L = _rect()
    for dr, P in _points(cen, L, [30, 10, 4, 3.01, 2.9, 2, 1, 0.5, 0.2, 0.05], seed):
        o, _ = orc.element(1, g, P, grad=True)
        G = orc.gradient_matrix(o[4:10])
        assert _rel(G, RI.rect_gradient_closed_form(g, P)) < 1e-10, dr


def test_triangle_gradient_matches_quadrature_and_fan(orc):
    g, cen, L = _tri()

    def fd(P, h):
        G = np.zeros((3, 3))
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            d1 = (RI.fan(0, g, P + e, 48, 32)[1:] - RI.fan(0, g, P - e, 48, 32)[1:]) / (2 * h)
            d2 = (RI.fan(0, g, P + 2 * e, 48, 32)[1:] - RI.fan(0, g, P - 2 * e, 48, 32)[1:]) / (4 * h)
            G[:, j] = (4 * d1 - d2) / 3
        return G

    for dr, P in _points(cen, L, [10, 3.5, 2.5, 1.0, 0.5, 0.2], 2):
        o, st = orc.element(0, g, P, grad=True)
        G = orc.gradient_matrix(o[4:10])
        if dr >= 2:
            assert _rel(G, RI.gl2_gradient(0, g, P, 64)) < 1e-13, dr
        assert _rel(G, fd(P, 1e-3 * L)) < 1e-8, dr
        if dr < 3:
            assert st["leaves"] > 0


def test_gradient_and_field_share_the_dispatch(orc):
    """Field part of a gradient call equals the plain field call bit for bit."""
    g, cen, L = _tri()
    for dr, P in _points(cen, L, [5.0, 1.0, 0.1], 4):
        a, sa = orc.element(0, g, P)
        b, sb = orc.element(0, g, P, grad=True)
        assert np.array_equal(a, b[:4]) and sa == sb


@pytest.fixture(scope="module")
def mesh():
    tri, rect = W.cylinder(1.0, -1.0, 1.0, 12, 3, 36)
    sig = np.random.default_rng(3).normal(size=tri.shape[0] + rect.shape[0])
    return tri, rect, sig


def test_mesh_gradient_trace_free_and_derivative_of_field(orc, mesh):
    tri, rect, sig = mesh
    rng = np.random.default_rng(8)
    far = np.ascontiguousarray(rng.uniform(-3.0, 3.0, size=(6, 3)) + np.array([0, 0, 4.0]))
    near, _ = W.near_points(tri, rect, 6, rng)
    pts = np.concatenate([far, near])
    res = orc.gradient(tri, rect, sig, pts)
    G, aG = res["G"], res["abs_G"]
    assert np.all(np.isfinite(G)) and np.all(aG > 0)
    # Laplace: the gradient of a source-free field is trace-free
    assert np.all(np.abs(G[:, 0] + G[:, 1] + G[:, 2]) <= 1e-13 * aG)
    # per-term scale: at least the per-element one (triangle inequality), equal to it for
    # a point far from every element (each element is then one cluster of like terms)
    aT = res["abs_T"]
    assert np.all(aT >= aG * (1 - 1e-13))
    assert np.all(aT[:6] <= 1.05 * aG[:6]) and np.any(aT[6:] > 1.5 * aG[6:])
    # dE/dx by Richardson central differences of the oracle's field
    M = orc.gradient_matrix(G)
    for p in range(pts.shape[0]):
        h = 1e-4  # small against every element size and distance
        cols = []
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            st = np.stack([pts[p] + e, pts[p] - e, pts[p] + 2 * e, pts[p] - 2 * e])
            E = orc.evaluate(tri, rect, sig, st)["E"]
            d1 = (E[0] - E[1]) / (2 * h)
            d2 = (E[2] - E[3]) / (4 * h)
            cols.append((4 * d1 - d2) / 3)
        fd = np.stack(cols, axis=1)
        assert np.abs(M[p] - fd).max() <= 1e-6 * aG[p], p


def test_far_gradient_is_point_charge(orc):
    """Far from a charged sphere the gradient is that of its total charge at the centre
    (the icosahedral mesh has no dipole, and its quadrupole vanishes by symmetry)."""
    tri = W.icosphere(2, 1.0)
    sig = np.full(tri.shape[0], 1e-9)
    area = 0.5 * np.linalg.norm(np.cross(tri[:, 3:6] - tri[:, 0:3], tri[:, 6:9] - tri[:, 0:3]), axis=1)
    Q = float(np.sum(sig * area))
    K = orc.coulomb_constant()
    rng = np.random.default_rng(11)
    d = rng.normal(size=(5, 3))
    d *= (40.0 / np.linalg.norm(d, axis=1))[:, None]
    G = orc.gradient_matrix(orc.gradient(tri, None, sig, d)["G"])
    for p in range(5):
        r = np.linalg.norm(d[p])
        ref = K * Q * (r * r * np.eye(3) - 3.0 * np.outer(d[p], d[p])) / r ** 5
        assert _rel(G[p], ref) < 1e-6


def test_on_element_gradient_is_nan(orc):
    g, cen, L = _tri()
    o, st = orc.element(0, g, cen, grad=True)
    assert np.all(np.isfinite(o[:4])) and np.all(np.isnan(o[4:10])) and st["on_surface"] == 1
    tri = g.reshape(1, 9)
    res = orc.gradient(tri, None, np.ones(1), np.stack([cen, cen + np.array([0, 0, 1.0])]))
    assert np.all(np.isnan(res["G"][0])) and np.all(np.isfinite(res["G"][1]))


def test_dr_rule_gradient_accuracy(orc, mesh):
    """The distance-ratio rule levels (chosen for the field) keep the gradient accurate."""
    tri, rect, sig = mesh
    rng = np.random.default_rng(4)
    d = rng.normal(size=(60, 3))
    pts = d * (np.geomspace(2.5, 120.0, 60) / np.linalg.norm(d, axis=1))[:, None]
    a = orc.gradient(tri, rect, sig, pts)
    b = orc.gradient(tri, rect, sig, pts, prm=orc.params(dr_rules=True))
    err = np.abs(a["G"] - b["G"]).max(axis=1) / a["abs_G"]
    assert 0 < err.max() < 1e-12
