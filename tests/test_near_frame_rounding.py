"""Node geometry of the FP64 near-field walk (host model of the kernel's arithmetic, FP64,
against long double).

The near kernel works in each element's frame (origin at the centroid c computed on the
host, f1, f2 in the plane, f3 the normal): the field point becomes p = F (P - c), a
triangle vertex V the triple F (V - c), a rectangle its corner F (P0 - c) and its sides
F e1, F e2.  A child of the subdivision (lattice level k, cell (i, j), size h = 2^-k) has
its Gaussian points at the barycentric or natural combinations of these triples, and the
offsets d = p - node give 1/|d| and d/|d|^3 (Sec. 4, Eq. 4.1).

Two inputs make the third frame coordinate of the vertices matter although the element is
flat: the frame of a sliver triangle is known only to eps times its aspect ratio, and the
rounded centroid of a small element far from the origin lies beside the element's plane by
a rounding of the coordinates.  Keeping those rounding-level heights makes the nodes the
exact combinations of the vertices; the checks compare the frame form with the
three-dimensional form relative to the first vertex (which needs no frame) on the inputs
where dropping the heights fails: points beside a sliver in its plane, and points 1e-9 L
above small elements at the depth cap (24 levels).  The normaliser is the sum of the terms'
magnitudes, sum w/r^2.
"""
import numpy as np
import pytest

import oracle

LD = np.longdouble


def _need_long_double():
    if np.finfo(np.longdouble).nmant < 60:
        pytest.skip("long double is not wider than double on this platform")


def _frame_tri(A, B, C):
    # as the library builds it: f1 along B - A, f3 the normal from a cross product, f2 = f3 x f1
    N = np.cross(B - A, C - A)
    N /= np.linalg.norm(N)
    F1 = (B - A) / np.linalg.norm(B - A)
    return np.array([F1, np.cross(N, F1), N]), (A + B + C) / 3.0


def _frame_rect(P0, e1, e2):
    N = np.cross(e1, e2)
    N /= np.linalg.norm(N)
    F1 = e2 / np.linalg.norm(e2)
    return np.array([F1, np.cross(N, F1), N]), P0 + 0.5 * e1 + 0.5 * e2


def _field(d, w):
    r = np.sqrt(np.sum(d * d, axis=-1))
    return np.sum((w / r**3)[:, None] * d, axis=0), np.sum(w / r**2)


def _tri_child_cases(rng, n, beside):
    lam, wts = oracle.tri_rule(33)
    for _ in range(n):
        c = rng.uniform(-2.0, 2.0, 3)
        size = 10.0 ** rng.uniform(-4.0, 0.0)
        ar = 10.0 ** rng.uniform(0.0, 2.0)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        v = np.cross(u, rng.normal(size=3))
        v /= np.linalg.norm(v)
        A, B, C = c, c + size * u, c + 0.5 * size * u + (size / ar) * v
        if beside:  # in the plane beyond vertex B; the child at B at level 5
            P = B + 0.01 * (B - A)
            k, i, j = 5, 31, 0
        else:  # 1e-9 .. 1e-8 L above the element; the child under the point at level 24
            L = (np.linalg.norm(B - A) + np.linalg.norm(C - B) + np.linalg.norm(A - C)) / 3.0
            s, t = rng.random(2)
            if s + t > 1.0:
                s, t = 1.0 - s, 1.0 - t
            N = np.cross(B - A, C - A)
            P = A + s * (B - A) + t * (C - A) + L * 10.0 ** rng.uniform(-9.0, -8.0) * N / np.linalg.norm(N)
            k = 24
            i, j = int(s * 2**k), int(t * 2**k)
            if i + j >= 2**k:
                i, j = 2**k - 1 - j, j
        h = 2.0**-k
        yield (A, B, C), P, (i, j, h), lam, wts


def _tri_forms(A, B, C, P, cell, lam, wts):
    i, j, h = cell
    lb, lc = lam[:, 1], lam[:, 2]
    # reference: long double, relative to A
    eB, eC = B.astype(LD) - A.astype(LD), C.astype(LD) - A.astype(LD)
    q = (i * h) * eB + (j * h) * eC + lb[:, None] * (h * eB) + lc[:, None] * (h * eC)
    E_ref, S = _field((P.astype(LD) - A.astype(LD)) - q, wts.astype(LD))
    # three dimensions relative to A (FP64)
    eB64, eC64 = B - A, C - A
    V0 = (i * h) * eB64 + (j * h) * eC64
    E_3d, _ = _field((P - A) - (V0 + lb[:, None] * (h * eB64) + lc[:, None] * (h * eC64)), wts)
    # the element's frame, with and without the vertices' third coordinate (FP64)
    F, c = _frame_tri(A, B, C)
    out = {}
    for keep in (True, False):
        loc = np.array([F @ (V - c) for V in (A, B, C)])
        if not keep:
            loc[:, 2] = 0.0
        p = F @ (P - c)
        u, v = loc[1] - loc[0], loc[2] - loc[0]
        x0 = (i * h) * u + ((j * h) * v + loc[0])
        d = (p - x0) - lb[:, None] * (h * u) - lc[:, None] * (h * v)
        E_l, _ = _field(d, wts)
        out[keep] = F.T @ E_l
    err = lambda E: float(np.sum(np.abs(E - E_ref.astype(float))) / float(S))
    return err(E_3d), err(out[True]), err(out[False])


@pytest.mark.parametrize("beside", [True, False])
def test_triangle_vertex_heights_keep_the_nodes_exact(beside):
    _need_long_double()
    rng = np.random.default_rng(3 if beside else 5)
    e3d, ekeep, edrop = [], [], []
    for (A, B, C), P, cell, lam, wts in _tri_child_cases(rng, 120, beside):
        a, b, c = _tri_forms(A, B, C, P, cell, lam, wts)
        e3d.append(a); ekeep.append(b); edrop.append(c)
    e3d, ekeep, edrop = max(e3d), max(ekeep), max(edrop)
    # with the heights: the rounding of the three-dimensional form
    assert ekeep <= 4.0 * e3d + 1e-15
    # without them the frame's error shows (documents why they are kept)
    assert edrop > 30.0 * ekeep


def test_rectangle_corner_keeps_the_plane():
    """Points 1e-9 .. 1e-8 L above small rectangles far from the origin, at the depth cap:
    the rounded centroid lies beside the plane by ~1e-16 of the coordinates, i.e. by up to
    1e-4 of such a point's height; with the corner P0 - c in three frame coordinates the
    frame form matches the three-dimensional form."""
    _need_long_double()
    xy, wts = oracle.rect_rule(7)
    x, y = xy[:, 0], xy[:, 1]
    rng = np.random.default_rng(7)
    worst = {"3d": 0.0, "corner": 0.0, "centred": 0.0}
    for _ in range(120):
        c = rng.uniform(-2.0, 2.0, 3)
        size = 10.0 ** rng.uniform(-4.0, 0.0)
        ar = 10.0 ** rng.uniform(0.0, 2.0)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        v = np.cross(u, rng.normal(size=3))
        v /= np.linalg.norm(v)
        P0, e1, e2 = c, size * u, (size / ar) * v
        Lr = 0.5 * (np.linalg.norm(e1) + np.linalg.norm(e2))
        s, t = rng.random(2)
        N = np.cross(e1, e2)
        P = P0 + s * e1 + t * e2 + Lr * 10.0 ** rng.uniform(-9.0, -8.0) * N / np.linalg.norm(N)
        h = 2.0**-24
        i, j = int(s / h), int(t / h)
        E1, E2 = e1.astype(LD), e2.astype(LD)
        q = ((i + 0.5) * h) * E1 + ((j + 0.5) * h) * E2
        q = q + (x[:, None] * (0.5 * h)) * E1 + (y[:, None] * (0.5 * h)) * E2
        E_ref, S = _field((P.astype(LD) - P0.astype(LD)) - q, wts.astype(LD))
        cen = ((i + 0.5) * h) * e1 + ((j + 0.5) * h) * e2
        E_3d, _ = _field((P - P0) - (cen + (x[:, None] * (0.5 * h)) * e1 + (y[:, None] * (0.5 * h)) * e2), wts)
        F, cc = _frame_rect(P0, e1, e2)
        gm, bt, al = F[0] @ e1 / 2.0, F[1] @ e1 / 2.0, np.linalg.norm(e2) / 2.0
        p = F @ (P - cc)
        res = {}
        for name, corner, hz in (("corner", F @ (P0 - cc), (F[2] @ e1, F[2] @ e2)),
                                 ("centred", np.array([-(gm + al), -bt, 0.0]), (0.0, 0.0))):
            cx = ((i + 0.5) * h) * (2 * gm) + (((j + 0.5) * h) * (2 * al) + corner[0])
            cy = ((i + 0.5) * h) * (2 * bt) + corner[1]
            cz = ((i + 0.5) * h) * hz[0] + (((j + 0.5) * h) * hz[1] + corner[2])
            da = (p[0] - cx) - x * (h * gm) - y * (h * al)
            db = (p[1] - cy) - x * (h * bt)
            d = np.stack([da, db, np.full_like(da, p[2] - cz)], axis=1)
            E_l, _ = _field(d, wts)
            res[name] = F.T @ E_l
        for name, E in (("3d", E_3d), ("corner", res["corner"]), ("centred", res["centred"])):
            worst[name] = max(worst[name], float(np.sum(np.abs(E - E_ref.astype(float))) / float(S)))
    assert worst["corner"] <= 4.0 * worst["3d"] + 1e-15
    assert worst["centred"] > 100.0 * worst["corner"]
