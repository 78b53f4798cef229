"""Allocation-free evaluation (bemc_eval_noalloc) through the C ABI: the same potential and
field as bemc_eval on the same points, on consecutive calls whose second input is smaller
(the static workspace keeps the first call's contents), in both precisions, and both
against the oracle (Sec. 4, Eq. 4.1 with the subdivision below distance ratio 3).
Tolerances as in the parity tests: FP64 1e-12, mixed 1e-6, errors normalised by the
oracle's sums of per-element magnitudes."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1606_03743_amd import bemc, workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-6}
MAX_POINTS = 1 << 16  # the workspace's point limit (bemc.h)


def torch_mod():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


@pytest.fixture(scope="module")
def cyl():
    w = W.cylinder_workload(40, 30, 1200, n_points=5000, near_frac=0.3, seed=303)
    return w


def make_ctx(w):
    ctx = bemc.Context(0)
    ctx.set_rules(w.tri_rule, w.rect_gl_n)
    ctx.upload_geometry(w.tri, w.rect)
    ctx.upload_densities(w.sigma)
    return ctx


def nerr(phi, E, ref):
    ep = np.abs(phi - ref["phi"]) / ref["abs_phi"]
    ee = np.sum(np.abs(E - ref["E"]), axis=1) / ref["abs_E"]
    return ep.max(), ee.max()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_eval_on_consecutive_calls(cyl, precision):
    torch = torch_mod()
    w = cyl
    ctx = make_ctx(w)
    lib = bemc.load_library()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    prec = bemc.FP64 if precision == "fp64" else bemc.MIXED
    # a full call, then a smaller one over other points
    for sl in (slice(0, 5000), slice(3100, 4833)):
        P = w.points[sl]
        n = P.shape[0]
        print(f"noalloc {precision}: {n} points", flush=True)
        pts = torch.tensor(np.ascontiguousarray(P.T), dtype=torch.float64, device="cuda:0")
        phi_a = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
        E_a = torch.full((3, n), float("nan"), dtype=torch.float64, device="cuda:0")
        rc = lib.bemc_eval_noalloc(ctx.h, ctypes.c_void_p(pts.data_ptr()), n, prec, 0,
                                   ctypes.c_void_p(phi_a.data_ptr()), ctypes.c_void_p(E_a.data_ptr()), stream)
        assert rc == bemc.OK, lib.bemc_last_error()
        st_a = ctx.stats()
        phi_b, E_b, _ = ctx.eval(pts, precision=precision)
        st_b = ctx.stats()
        torch.cuda.synchronize()
        ref = oracle.evaluate(w.tri, w.rect, w.sigma[0], P, oracle.params(33, 7), with_abs=True)
        assert st_a["near_pairs"] == st_b["near_pairs"] == ref["stats"]["near_pairs"] > 0
        assert st_a["leaves"] == st_b["leaves"]
        a = (phi_a.cpu().numpy(), E_a.cpu().numpy().T.copy())
        b = (phi_b.cpu().numpy(), E_b.cpu().numpy().T.copy())
        assert np.isfinite(a[0]).all() and np.isfinite(a[1]).all()
        d_p = np.abs(a[0] - b[0]) / ref["abs_phi"]
        d_e = np.sum(np.abs(a[1] - b[1]), axis=1) / ref["abs_E"]
        assert d_p.max() <= TOL[precision] and d_e.max() <= TOL[precision]
        ep, ee = nerr(a[0], a[1], ref)
        print(f"  vs eval {d_p.max():.2e} {d_e.max():.2e}; vs oracle {ep:.2e} {ee:.2e}", flush=True)
        assert ep <= TOL[precision] and ee <= TOL[precision]
    ctx.close()


def test_noalloc_potential_only_and_limits(cyl):
    torch = torch_mod()
    w = cyl
    ctx = make_ctx(w)
    P = w.points[:777]
    pts = torch.tensor(np.ascontiguousarray(P.T), dtype=torch.float64, device="cuda:0")
    phi = torch.empty(777, dtype=torch.float64, device="cuda:0")
    ctx.eval_noalloc(pts, phi)  # no field requested
    ref_phi, _, _ = ctx.eval(pts)
    torch.cuda.synchronize()
    assert torch.equal(phi, ref_phi)  # same split, same order: identical
    # more points than the workspace holds: refused on the host, nothing enqueued
    big = torch.zeros((3, MAX_POINTS + 1), dtype=torch.float64, device="cuda:0")
    out = torch.empty(MAX_POINTS + 1, dtype=torch.float64, device="cuda:0")
    with pytest.raises(bemc.BemcError) as ei:
        ctx.eval_noalloc(big, out)
    assert ei.value.code == bemc.E_LIMIT
    ctx.close()


def test_noalloc_near_pair_overflow_is_reported():
    """65,536 points just above the elements of a fine mesh have more near pairs than the
    workspace's list: the call still returns at once, stats() reports BEMC_E_LIMIT, and the
    next call on fewer points is exact again."""
    torch = torch_mod()
    w = W.cylinder_workload(40, 30, 1200, n_points=10, seed=78)
    rng = np.random.default_rng(9)
    idx = rng.integers(0, w.n_elements, MAX_POINTS)
    P, nrm, L = W.points_on_elements(w.tri, w.rect, idx, rng)
    q = np.ascontiguousarray(P + nrm * (1e-3 * L)[:, None])
    ctx = make_ctx(w)
    pts = torch.tensor(np.ascontiguousarray(q.T), dtype=torch.float64, device="cuda:0")
    phi = torch.empty(MAX_POINTS, dtype=torch.float64, device="cuda:0")
    E = torch.empty((3, MAX_POINTS), dtype=torch.float64, device="cuda:0")
    assert ctx.eval_noalloc(pts, phi, E) == bemc.OK
    with pytest.raises(bemc.BemcError) as ei:
        ctx.stats()
    assert ei.value.code == bemc.E_LIMIT and "near pairs" in str(ei.value)
    sub = pts[:, :2000].contiguous()
    phi2 = torch.empty(2000, dtype=torch.float64, device="cuda:0")
    E2 = torch.empty((3, 2000), dtype=torch.float64, device="cuda:0")
    ctx.eval_noalloc(sub, phi2, E2)
    st = ctx.stats()
    torch.cuda.synchronize()
    ref = oracle.evaluate(w.tri, w.rect, w.sigma[0], q[:2000], oracle.params(33, 7), with_abs=True)
    assert st["near_pairs"] == ref["stats"]["near_pairs"]
    ep, ee = nerr(phi2.cpu().numpy(), E2.cpu().numpy().T.copy(), ref)
    assert ep <= 1e-12 and ee <= 1e-12
    ctx.close()
