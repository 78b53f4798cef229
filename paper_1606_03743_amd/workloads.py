"""Seeded synthetic inputs: electrode meshes, charge densities and field points.

This module only builds inputs.  It holds none of the cubature, Coulomb-sum,
classification or subdivision arithmetic, and both the GPU tests and the oracle
tests draw their inputs from it.

The paper measures on KATRIN main-spectrometer meshes of 1.5 million triangles or
rectangles with solved charge densities (Sec. 5, Sec. 6).  Those meshes are not
available, so the workloads here stand in for them with the same element kinds,
a spread of aspect ratios, random densities, and field points of which most are
far from every element while some lie close to one.

Geometry formats (FP64, row-major):
  tri  [n][9] = A, B, C
  rect [n][9] = P0 (corner), e1 (x side vector), e2 (y side vector), e1 . e2 = 0
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 20161606


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
def icosphere(subdivisions: int = 3, radius: float = 1.0) -> np.ndarray:
    """Icosahedron refined by midpoint subdivision, vertices projected to the sphere.

    20 * 4**subdivisions flat triangles, outward orientation.
    """
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    verts = [tuple(x) for x in v]
    for _ in range(subdivisions):
        cache = {}
        vlist = verts

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                m = (np.array(vlist[i]) + np.array(vlist[j])) / 2.0
                m /= np.linalg.norm(m)
                cache[key] = len(vlist)
                vlist.append(tuple(m))
            return cache[key]

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        f = np.array(nf, dtype=np.int64)
        verts = vlist
    V = np.array(verts) * radius
    tri = np.concatenate([V[f[:, 0]], V[f[:, 1]], V[f[:, 2]]], axis=1)
    return np.ascontiguousarray(tri)


def _ring_counts(n_boundary: int, n_tri: int) -> np.ndarray:
    """Vertex counts v_1..v_n of concentric rings for a disk with n_tri triangles.

    A fan to ring 1 gives v_1 triangles and the strip between rings i-1 and i gives
    v_{i-1} + v_i, so the total is 2 * sum(v) - v_n.  Rings are spaced so that the
    triangles are close to equilateral; the outer ring has n_boundary vertices.
    """
    if (n_tri - n_boundary) % 2:
        raise ValueError("n_tri - n_boundary must be even")
    target = (n_tri - n_boundary) // 2  # sum of v_1..v_{n-1}
    c = math.pi * math.sqrt(3.0)       # v_i ~ c i gives equilateral-like cells
    n = max(2, int(round(math.sqrt(2.0 * target / c) + 0.5)))
    i = np.arange(1, n)
    # rings next to the rim taper by at most 1.2x per ring towards n_boundary
    cap = np.floor(n_boundary * 1.2 ** np.minimum(n - i, 40)).astype(np.int64)

    def counts(cc):
        return np.maximum(3, np.minimum(np.round(cc * i), cap)).astype(np.int64)

    lo, hi = 0.0, 4.0 * target
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if counts(mid).sum() <= target:
            lo = mid
        else:
            hi = mid
    v = counts(lo)
    diff = target - int(v.sum())
    free = np.nonzero(v < cap)[0]
    if diff < 0 or diff > free.size:
        raise RuntimeError("ring construction failed")
    for k in free[np.linspace(0, free.size - 1, num=diff, dtype=np.int64)] if diff else []:
        v[k] += 1
    v = np.concatenate([v, [n_boundary]])
    if 2 * int(v.sum()) - n_boundary != n_tri or v.min() < 3:
        raise RuntimeError("ring construction failed")
    return v


def disk_triangles(radius: float, z: float, n_boundary: int, n_tri: int, up: bool) -> np.ndarray:
    """Deterministic ring triangulation of the regular n_boundary-gon of the given radius.

    The outer ring's vertices sit at angles 2 pi k / n_boundary, matching a mantle
    polygon with the same corner count.  Normal +z if up, else -z.
    """
    v = _ring_counts(n_boundary, n_tri)
    n = len(v)
    rings = []
    for i, cnt in enumerate(v, start=1):
        r = radius * i / n
        off = 0.0 if i == n else 0.5 * (i % 2)
        ang = 2.0 * math.pi * (np.arange(cnt) + off) / cnt
        if i == n:
            x, y = radius * np.cos(ang), radius * np.sin(ang)
        else:
            x, y = r * np.cos(ang), r * np.sin(ang)
        rings.append((ang, np.stack([x, y, np.full(cnt, z)], axis=1)))
    tris = []
    center = np.array([0.0, 0.0, z])
    a1, p1 = rings[0]
    for k in range(len(a1)):
        tris.append((center, p1[k], p1[(k + 1) % len(a1)]))
    for i in range(1, n):
        aa, pa = rings[i - 1]
        ab, pb = rings[i]
        na, nb = len(aa), len(ab)
        # unwrap angles so both walks start at their first vertex
        ua = np.concatenate([aa, [aa[0] + 2 * math.pi]])
        ub = np.concatenate([ab, [ab[0] + 2 * math.pi]])
        ia = ib = 0
        while ia < na or ib < nb:
            adv_a = ib >= nb or (ia < na and ua[ia + 1] <= ub[ib + 1])
            if adv_a:
                tris.append((pa[ia % na], pb[ib % nb], pa[(ia + 1) % na]))
                ia += 1
            else:
                tris.append((pa[ia % na], pb[ib % nb], pb[(ib + 1) % nb]))
                ib += 1
    T = np.array([np.concatenate(t) for t in tris])
    # orient
    A, B, C = T[:, 0:3], T[:, 3:6], T[:, 6:9]
    nz = np.cross(B - A, C - A)[:, 2]
    flip = (nz < 0) if up else (nz > 0)
    T[flip] = np.concatenate([A[flip], C[flip], B[flip]], axis=1)
    if T.shape[0] != n_tri:
        raise RuntimeError("triangle count mismatch")
    return np.ascontiguousarray(T)


def graded_heights(length: float, n_z: int, width: float) -> np.ndarray:
    """Ring heights h_k = width * (1 + 3 t_k^p), t_k = |2(k+1/2)/n_z - 1|, sum = length.

    Aspect ratios h/width stay within [1, 4]; p is found by bisection.
    """
    t = np.abs(2.0 * (np.arange(n_z) + 0.5) / n_z - 1.0)
    mean_ar = length / (n_z * width)
    if not (1.0 < mean_ar < 4.0):
        raise ValueError("mean aspect ratio outside (1, 4)")
    lo, hi = 1e-6, 1e6
    for _ in range(200):
        p = math.sqrt(lo * hi)
        m = np.mean(1.0 + 3.0 * t ** p)
        if m > mean_ar:
            lo = p
        else:
            hi = p
    h = width * (1.0 + 3.0 * t ** p)
    return h * (length / h.sum())


def cylinder_mantle(radius: float, z0: float, z1: float, n_theta: int, n_z: int) -> np.ndarray:
    """Flat rectangles on the n_theta-gon prism; e1 along the chord, e2 along z."""
    w = 2.0 * radius * math.sin(math.pi / n_theta)
    h = graded_heights(z1 - z0, n_z, w)
    zb = z0 + np.concatenate([[0.0], np.cumsum(h)])
    zb[-1] = z1
    th = 2.0 * math.pi * np.arange(n_theta + 1) / n_theta
    cx, cy = radius * np.cos(th), radius * np.sin(th)
    J, K = np.meshgrid(np.arange(n_theta), np.arange(n_z), indexing="xy")
    J, K = J.ravel(), K.ravel()
    P0 = np.stack([cx[J], cy[J], zb[K]], axis=1)
    e1 = np.stack([cx[J + 1] - cx[J], cy[J + 1] - cy[J], np.zeros_like(J, dtype=np.float64)], axis=1)
    e2 = np.stack([np.zeros(J.size), np.zeros(J.size), zb[K + 1] - zb[K]], axis=1)
    return np.ascontiguousarray(np.concatenate([P0, e1, e2], axis=1))


def cylinder(radius, z0, z1, n_theta, n_z, cap_tris):
    """Closed cylinder: graded rectangle mantle + two ring-triangulated caps."""
    rect = cylinder_mantle(radius, z0, z1, n_theta, n_z)
    top = disk_triangles(radius, z1, n_theta, cap_tris, up=True)
    bot = disk_triangles(radius, z0, n_theta, cap_tris, up=False)
    return np.concatenate([bot, top], axis=0), rect


# --------------------------------------------------------------------------
# element facts used only to place points (no cubature arithmetic)
# --------------------------------------------------------------------------
def _tri_parts(tri):
    A, B, C = tri[:, 0:3], tri[:, 3:6], tri[:, 6:9]
    cen = (A + B + C) / 3.0
    n = np.cross(B - A, C - A)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    L = (np.linalg.norm(B - C, axis=1) + np.linalg.norm(C - A, axis=1) + np.linalg.norm(A - B, axis=1)) / 3.0
    return cen, n, L


def _rect_parts(rect):
    P0, e1, e2 = rect[:, 0:3], rect[:, 3:6], rect[:, 6:9]
    cen = P0 + 0.5 * e1 + 0.5 * e2
    n = np.cross(e1, e2)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    L = 0.5 * (np.linalg.norm(e1, axis=1) + np.linalg.norm(e2, axis=1))
    return cen, n, L


def aspect_ratios(tri, rect):
    """Triangle: longest side / its height; rectangle: long side / short side (Sec. 2)."""
    out = {}
    if tri is not None and len(tri):
        A, B, C = tri[:, 0:3], tri[:, 3:6], tri[:, 6:9]
        s = np.stack([np.linalg.norm(B - C, axis=1), np.linalg.norm(C - A, axis=1),
                      np.linalg.norm(A - B, axis=1)], axis=1)
        area = 0.5 * np.linalg.norm(np.cross(B - A, C - A), axis=1)
        lmax = s.max(axis=1)
        out["tri"] = lmax / (2.0 * area / lmax)
    if rect is not None and len(rect):
        a = np.linalg.norm(rect[:, 3:6], axis=1)
        b = np.linalg.norm(rect[:, 6:9], axis=1)
        out["rect"] = np.maximum(a, b) / np.minimum(a, b)
    return out


def points_on_elements(tri, rect, idx, rng):
    """Uniform random points on elements idx (global index: triangles first)."""
    nt = 0 if tri is None else tri.shape[0]
    P = np.empty((idx.size, 3))
    nrm = np.empty((idx.size, 3))
    L = np.empty(idx.size)
    it = idx < nt
    if it.any():
        T = tri[idx[it]]
        u, v = rng.random(it.sum()), rng.random(it.sum())
        su = np.sqrt(u)
        la, lb = 1.0 - su, su * (1.0 - v)
        lc = 1.0 - la - lb
        P[it] = la[:, None] * T[:, 0:3] + lb[:, None] * T[:, 3:6] + lc[:, None] * T[:, 6:9]
        _, n, l = _tri_parts(T)
        nrm[it], L[it] = n, l
    ir = ~it
    if ir.any():
        R = rect[idx[ir] - nt]
        x, y = rng.random(ir.sum()), rng.random(ir.sum())
        P[ir] = R[:, 0:3] + x[:, None] * R[:, 3:6] + y[:, None] * R[:, 6:9]
        _, n, l = _rect_parts(R)
        nrm[ir], L[ir] = n, l
    return P, nrm, L


def far_points_box(tri, rect, n, lo, hi, rng, margin=3.0):
    """n points uniform in the box [lo, hi], kept only if every element centroid is at
    least margin * (largest L of that element kind) away: a sufficient condition for
    every pair to be at distance ratio >= margin."""
    from scipy.spatial import cKDTree

    trees = []
    for parts, arr in ((_tri_parts, tri), (_rect_parts, rect)):
        if arr is not None and len(arr):
            cen, _, L = parts(arr)
            trees.append((cKDTree(cen), margin * L.max()))
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    out = []
    have = 0
    rounds = 0
    while have < n:
        rounds += 1
        if rounds > 200 or (rounds > 20 and have == 0):
            raise ValueError("the box leaves (almost) no room for far points: refine the mesh")
        m = int((n - have) * 1.3) + 64
        cand = lo + (hi - lo) * rng.random((m, 3))
        ok = np.ones(m, dtype=bool)
        for tree, rad in trees:
            d, _ = tree.query(cand, k=1, distance_upper_bound=rad)
            ok &= ~(d < rad)
        cand = cand[ok]
        out.append(cand)
        have += cand.shape[0]
    return np.ascontiguousarray(np.concatenate(out)[:n])


def near_points(tri, rect, n, rng, hmin_ratio=1e-3, hmax_ratio=2.0):
    """n points above random elements: uniform point on the element, offset along
    +-normal by h = L * 10^U(log10 hmin_ratio, log10 hmax_ratio)."""
    ne = (0 if tri is None else tri.shape[0]) + (0 if rect is None else rect.shape[0])
    idx = rng.integers(0, ne, size=n)
    P, nrm, L = points_on_elements(tri, rect, idx, rng)
    h = L * 10.0 ** rng.uniform(math.log10(hmin_ratio), math.log10(hmax_ratio), size=n)
    sgn = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    return np.ascontiguousarray(P + (sgn * h)[:, None] * nrm), idx


def shell_points(n, rmin, rmax, rng):
    """Uniform in volume in the spherical shell rmin <= r <= rmax, isotropic."""
    r = (rmin ** 3 + rng.random(n) * (rmax ** 3 - rmin ** 3)) ** (1.0 / 3.0)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.ascontiguousarray(d * r[:, None])


# --------------------------------------------------------------------------
# particle tracks (serving queries)
# --------------------------------------------------------------------------
def track_points(n, rng, r_wall=0.95, z_wall=4.9, step=1e-3):
    """n points spaced `step` apart along a straight track that reflects specularly
    off the cylinder r = r_wall and the planes z = +-z_wall."""
    r0 = r_wall * math.sqrt(rng.random())
    ph = 2.0 * math.pi * rng.random()
    p = np.array([r0 * math.cos(ph), r0 * math.sin(ph), rng.uniform(-z_wall, z_wall)])
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    out = np.empty((n, 3))
    k = 0
    s0 = 0.0  # arc length from p to the next sample
    while k < n:
        # distance along d to the next wall
        t_hit = math.inf
        a = d[0] ** 2 + d[1] ** 2
        if a > 1e-300:
            b = p[0] * d[0] + p[1] * d[1]
            c = p[0] ** 2 + p[1] ** 2 - r_wall ** 2
            disc = b * b - a * c
            if disc > 0:
                t = (-b + math.sqrt(disc)) / a
                if t > 1e-12:
                    t_hit = t
        if d[2] > 0:
            t_hit = min(t_hit, (z_wall - p[2]) / d[2])
        elif d[2] < 0:
            t_hit = min(t_hit, (-z_wall - p[2]) / d[2])
        t_hit = max(t_hit, 0.0)
        m = 0 if s0 > t_hit else int((t_hit - s0) // step) + 1
        m = min(m, n - k)
        if m:
            s = s0 + step * np.arange(m)
            out[k:k + m] = p + s[:, None] * d
            k += m
        # advance to the wall and reflect
        p = p + t_hit * d
        s0 = s0 + step * m - t_hit
        rr = math.hypot(p[0], p[1])
        if abs(abs(p[2]) - z_wall) < 1e-9 * z_wall:
            d[2] = -d[2]
        elif rr > 0:
            nr = np.array([p[0] / rr, p[1] / rr, 0.0])
            d = d - 2.0 * np.dot(d, nr) * nr
    return out


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    tri: np.ndarray
    rect: np.ndarray
    sigma: np.ndarray            # [n_rhs, n_E]
    points: np.ndarray | None    # [n, 3]
    tri_rule: int
    rect_gl_n: int
    info: dict = field(default_factory=dict)

    @property
    def n_elements(self):
        return self.tri.shape[0] + self.rect.shape[0]


def _rngs(seed, k):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(k)]


def icosphere_workload(n_points=4096) -> Workload:
    """Icosphere R=1 (1,280 triangles), densities U[-1,1], points uniform in volume in
    the shell 2 <= r <= 10, 7-point triangle rule."""
    r_sig, r_pts = _rngs(SEED_BASE + 0, 2)
    tri = icosphere(3, 1.0)
    sigma = r_sig.uniform(-1.0, 1.0, size=(1, tri.shape[0]))
    pts = shell_points(n_points, 2.0, 10.0, r_pts)
    return Workload("icosphere-1280tri-4096pts-tri7", tri, np.zeros((0, 9)), sigma, pts, 7, 7,
                    {"seed": SEED_BASE + 0})


def cylinder_workload(n_theta=250, n_z=200, cap_tris=50_000, n_points=1_000_000, near_frac=0.3,
                      seed=SEED_BASE + 1, tri_rule=33, rect_gl_n=7, name=None) -> Workload:
    """Cylinder R=1, z in [-5, 5]: graded rectangle mantle (aspect ratios 1-4) and
    ring-triangulated caps; densities N(0,1); points: (1-near_frac) uniform in the box
    1.2x the electrode with every element at distance ratio >= 3, near_frac placed
    above random elements at h = L * 10^U(-3, log10 2) (distance ratio < 3)."""
    r_sig, r_far, r_near, r_mix = _rngs(seed, 4)
    tri, rect = cylinder(1.0, -5.0, 5.0, n_theta, n_z, cap_tris)
    sigma = r_sig.standard_normal((1, tri.shape[0] + rect.shape[0]))
    n_near = int(round(near_frac * n_points))
    n_far = n_points - n_near
    far = far_points_box(tri, rect, n_far, (-1.2, -1.2, -6.0), (1.2, 1.2, 6.0), r_far)
    near, near_el = near_points(tri, rect, n_near, r_near)
    pts = np.concatenate([far, near], axis=0)
    perm = r_mix.permutation(n_points)
    is_near = np.concatenate([np.zeros(n_far, bool), np.ones(n_near, bool)])[perm]
    pts = np.ascontiguousarray(pts[perm])
    name = name or f"cylinder-{tri.shape[0]}tri-{rect.shape[0]}rect-{n_points}pts-tri{tri_rule}-gl{rect_gl_n}"
    return Workload(name, tri, rect, sigma, pts, tri_rule, rect_gl_n,
                    {"seed": seed, "is_near": is_near})


def cylinder_150k(n_points=1_000_000) -> Workload:
    """100,000 cap triangles + 50,000 mantle rectangles, 1,000,000 points, 30 % near."""
    return cylinder_workload(250, 200, 50_000, n_points, 0.3, SEED_BASE + 1)


def nested_cylinders_workload(inner=(200, 200, 20_000), outer=(300, 200, 30_000), n_rhs=8,
                              seed=SEED_BASE + 3) -> Workload:
    """Nested coaxial cylinders: inner R=1, z in [-5,5]; outer R=2, z in [-6,6];
    densities N(0,1) for n_rhs right-hand sides; collocation points are the centroids.
    Default sizes: 40k+60k rectangles and 40k+60k triangles = 200,000 elements."""
    (r_sig,) = _rngs(seed, 1)
    t1, q1 = cylinder(1.0, -5.0, 5.0, inner[0], inner[1], inner[2])
    t2, q2 = cylinder(2.0, -6.0, 6.0, outer[0], outer[1], outer[2])
    tri = np.ascontiguousarray(np.concatenate([t1, t2]))
    rect = np.ascontiguousarray(np.concatenate([q1, q2]))
    sigma = r_sig.standard_normal((n_rhs, tri.shape[0] + rect.shape[0]))
    return Workload(f"nested-cylinders-{tri.shape[0]}tri-{rect.shape[0]}rect-{n_rhs}rhs-tri33-gl7",
                    tri, rect, sigma, None, 33, 7, {"seed": seed})


def serving_geometry(n_theta=600, n_z=500, cap_tris=350_000, seed=SEED_BASE + 4) -> Workload:
    """Cylinder as above with 1,000,000 elements (700k cap triangles, 300k mantle
    rectangles), densities N(0,1), no points (queries come from `serving_queries`)."""
    (r_sig,) = _rngs(seed, 1)
    tri, rect = cylinder(1.0, -5.0, 5.0, n_theta, n_z, cap_tris)
    sigma = r_sig.standard_normal((1, tri.shape[0] + rect.shape[0]))
    return Workload(f"serving-cylinder-{tri.shape[0]}tri-{rect.shape[0]}rect-tri33-gl7",
                    tri, rect, sigma, None, 33, 7, {"seed": seed})


def serving_query_sizes(n_queries, seed=SEED_BASE + 4, max_log2=16):
    """Query sizes n = round(2^U(0, max_log2)) in [1, 2^max_log2]."""
    rng = np.random.default_rng([seed, 1])
    return np.clip(np.rint(2.0 ** rng.uniform(0.0, max_log2, size=n_queries)), 1, 2 ** max_log2).astype(np.int64)


def serving_query(i, n, seed=SEED_BASE + 4):
    """Points of query i: a particle track of n steps inside the electrode volume."""
    return track_points(int(n), np.random.default_rng([seed, 2, int(i)]))


def poisson_arrivals(n_queries, rate, seed=SEED_BASE + 4):
    """Arrival times (s) of an open-loop Poisson process with the given rate (1/s)."""
    rng = np.random.default_rng([seed, 3])
    return np.cumsum(rng.exponential(1.0 / rate, size=n_queries))
