"""Seeded synthetic inputs: sizes, structure and determinism of the generators."""
import numpy as np
import pytest

from paper_1606_03743_amd import workloads as W


def test_icosphere_workload():
    w = W.icosphere_workload()
    assert w.tri.shape == (1280, 9) and w.rect.shape == (0, 9)
    r = np.linalg.norm(w.points, axis=1)
    assert w.points.shape == (4096, 3) and r.min() >= 2.0 and r.max() <= 10.0
    assert np.all(np.abs(w.sigma) <= 1.0)
    V = w.tri.reshape(-1, 3)
    assert np.allclose(np.linalg.norm(V, axis=1), 1.0)
    # closed, outward: total signed volume = (1/6) sum A . (B x C) > 0
    vol = np.sum(np.einsum("ij,ij->i", w.tri[:, 0:3], np.cross(w.tri[:, 3:6], w.tri[:, 6:9]))) / 6
    assert 4.0 < vol < 4.19


def test_cylinder_mesh_structure():
    tri, rect = W.cylinder(1.0, -5.0, 5.0, 250, 200, 50_000)
    assert tri.shape == (100_000, 9) and rect.shape == (50_000, 9)
    ar = W.aspect_ratios(tri, rect)
    assert ar["rect"].min() >= 1.0 - 1e-9 and ar["rect"].max() <= 4.0 + 1e-9
    assert ar["tri"].max() <= 4.0
    # rectangles are exact rectangles, mantle height 10
    assert np.max(np.abs(np.einsum("ij,ij->i", rect[:, 3:6], rect[:, 6:9]))) == 0.0
    assert abs(rect[:, 8].reshape(200, 250)[:, 0].sum() - 10.0) < 1e-12
    # caps tile the 250-gon exactly
    A, B, C = tri[:, 0:3], tri[:, 3:6], tri[:, 6:9]
    area = 0.5 * np.linalg.norm(np.cross(B - A, C - A), axis=1)
    poly = 250 / 2 * np.sin(2 * np.pi / 250)
    assert abs(area[:50_000].sum() - poly) < 1e-12 and abs(area[50_000:].sum() - poly) < 1e-12


@pytest.mark.parametrize("nb,nt", [(8, 40), (12, 36), (200, 20_000), (300, 30_000), (600, 350_000)])
def test_ring_counts(nb, nt):
    v = W._ring_counts(nb, nt)
    assert 2 * v.sum() - v[-1] == nt and v[-1] == nb and v.min() >= 3


def test_cylinder_points_small():
    w = W.cylinder_workload(40, 20, 400, n_points=2000, near_frac=0.3, seed=7)
    isn = w.info["is_near"]
    assert w.points.shape == (2000, 3) and isn.sum() == 600
    # far points: every centroid farther than 3 x the largest L of its kind
    from scipy.spatial import cKDTree

    for parts, arr in ((W._tri_parts, w.tri), (W._rect_parts, w.rect)):
        cen, _, L = parts(arr)
        d, _ = cKDTree(cen).query(w.points[~isn])
        assert d.min() >= 3.0 * L.max()
    # near points: distance ratio < 3 to at least one element
    cen = np.concatenate([W._tri_parts(w.tri)[0], W._rect_parts(w.rect)[0]])
    L = np.concatenate([W._tri_parts(w.tri)[2], W._rect_parts(w.rect)[2]])
    P = w.points[isn]
    dr = np.linalg.norm(P[:, None, :] - cen[None, :, :], axis=2) / L[None, :]
    assert np.all(dr.min(axis=1) < 3.0)


def test_determinism():
    a = W.cylinder_workload(40, 20, 400, n_points=500, seed=3)
    b = W.cylinder_workload(40, 20, 400, n_points=500, seed=3)
    assert np.array_equal(a.points, b.points) and np.array_equal(a.sigma, b.sigma)
    assert np.array_equal(W.serving_query(5, 300), W.serving_query(5, 300))


def test_serving_queries():
    n = W.serving_query_sizes(20_000)
    assert n.min() >= 1 and n.max() <= 65536
    assert 4000 < n.mean() < 8000  # log-uniform on [1, 2^16]: mean (2^16 - 1) / (16 ln 2) ~ 5909
    q = W.serving_query(3, 20_000)
    assert np.hypot(q[:, 0], q[:, 1]).max() <= 0.95 + 1e-9 and np.abs(q[:, 2]).max() <= 4.9 + 1e-9
    step = np.linalg.norm(np.diff(q, axis=0), axis=1)
    assert step.max() <= 1e-3 + 1e-12 and np.median(step) > 0.999e-3
    t = W.poisson_arrivals(1000, 50.0)
    assert np.all(np.diff(t) > 0) and 15 < t[-1] < 25


def test_far_points_guard():
    """A mesh too coarse for the box raises instead of sampling forever."""
    with pytest.raises(ValueError):
        W.cylinder_workload(24, 18, 96, n_points=100, seed=1)
