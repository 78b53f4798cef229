"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle, element by
element, on seeded inputs.

Error measure (per field point): the potential error divided by the sum of the absolute
per-element potentials, and the L1 field error divided by the sum of the per-element field
magnitudes (both sums from the oracle).  Random-sign densities make the plain relative
error ill-conditioned where contributions cancel; this normalisation bounds the
accumulated rounding of an N-term sum independently of that cancellation.
Tolerances: FP64 path 1e-12, mixed path 1e-6.
"""
import numpy as np
import pytest

import oracle
from paper_1606_03743_amd import bemc, workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-6}


def torch_mod():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def nerr(phi, E, ref):
    ep = np.abs(phi - ref["phi"]) / ref["abs_phi"]
    ee = np.sum(np.abs(E - ref["E"]), axis=1) / ref["abs_E"]
    return ep, ee


def run_gpu(ctx, pts_np, precision):
    torch = torch_mod()
    pts = torch.tensor(np.ascontiguousarray(pts_np.T), dtype=torch.float64, device="cuda:0")
    phi, E, rc = ctx.eval(pts, precision=precision)
    torch.cuda.synchronize()
    return phi.cpu().numpy(), E.cpu().numpy().T.copy(), rc


def make_ctx(w, tri_rule=None, rect_gl_n=None):
    ctx = bemc.Context(0)
    ctx.set_rules(tri_rule or w.tri_rule, rect_gl_n or w.rect_gl_n)
    ctx.upload_geometry(w.tri, w.rect)
    ctx.upload_densities(w.sigma)
    return ctx


@pytest.fixture(scope="module")
def sphere():
    w = W.icosphere_workload()
    ref = oracle.evaluate(w.tri, w.rect, w.sigma[0], w.points, oracle.params(tri_rule=7), with_abs=True)
    return w, ref


@pytest.fixture(scope="module")
def cyl():
    w = W.cylinder_workload(40, 30, 1200, n_points=3000, near_frac=0.3, seed=101)
    ref = oracle.evaluate(w.tri, w.rect, w.sigma[0], w.points, oracle.params(33, 7), with_abs=True)
    return w, ref


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_icosphere_full(sphere, precision):
    """1,280-triangle icosphere, 4,096 points in 2 <= r <= 10, 7-point rule: every pair far."""
    w, ref = sphere
    ctx = make_ctx(w)
    phi, E, rc = run_gpu(ctx, w.points, precision)
    st = ctx.stats()
    ctx.close()
    assert rc == 0 and st["near_pairs"] == 0 and ref["stats"]["near_pairs"] == 0
    assert st["pairs"] == 4096 * 1280 and st["node_interactions"] == 4096 * 1280 * 7
    ep, ee = nerr(phi, E, ref)
    print(f"icosphere {precision}: phi {ep.max():.2e} E {ee.max():.2e}")
    assert ep.max() <= TOL[precision] and ee.max() <= TOL[precision]
    if precision == "mixed":  # but not FP64-exact: the FP32 path really ran
        assert ep.max() > 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cylinder_with_near_field(cyl, precision):
    """Triangles (33-point rule) + rectangles (7 x 7 Gauss), 30 % of points near an element."""
    w, ref = cyl
    ctx = make_ctx(w)
    phi, E, rc = run_gpu(ctx, w.points, precision)
    st = ctx.stats()
    ctx.close()
    assert rc == 0
    assert st["near_pairs"] == ref["stats"]["near_pairs"] > 0
    assert st["leaves"] > 0 and st["cap_hits"] == 0
    ep, ee = nerr(phi, E, ref)
    print(f"cylinder {precision}: phi {ep.max():.2e} E {ee.max():.2e}, near pairs {st['near_pairs']}, "
          f"leaves gpu {st['leaves']} oracle {ref['stats']['leaves']}")
    assert ep.max() <= TOL[precision] and ee.max() <= TOL[precision]
    assert abs(st["leaves"] - ref["stats"]["leaves"]) <= 0.001 * ref["stats"]["leaves"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_uniform_density_plain_relative_error(cyl, precision):
    """sigma = 1 everywhere: no cancellation between elements, so the paper's plain relative
    error of the potential (Sec. 2) is well conditioned and gated directly; the field is
    gated by its norm against the sum of per-element field magnitudes as above."""
    w, _ = cyl
    ones = np.ones(w.n_elements)
    ref = oracle.evaluate(w.tri, w.rect, ones, w.points, oracle.params(33, 7), with_abs=True)
    ctx = bemc.Context(0)
    ctx.upload_geometry(w.tri, w.rect)
    ctx.upload_densities(ones)
    phi, E, _ = run_gpu(ctx, w.points, precision)
    ctx.close()
    rel = np.abs(phi - ref["phi"]) / np.abs(ref["phi"])
    print(f"sigma=1 {precision}: plain relative phi max {rel.max():.2e} median {np.median(rel):.2e}")
    assert rel.max() <= TOL[precision]
    assert np.allclose(ref["phi"], ref["abs_phi"])  # all contributions positive
    _, ee = nerr(phi, E, ref)
    assert ee.max() <= TOL[precision]


@pytest.mark.parametrize("n", [1, 2, 255, 511, 513, 1025])
def test_ragged_point_counts(cyl, n):
    w, ref = cyl
    ctx = make_ctx(w)
    idx = np.arange(n) * 7 % w.points.shape[0]
    phi, E, _ = run_gpu(ctx, w.points[idx], "fp64")
    ctx.close()
    sub = {k: ref[k][idx] for k in ("phi", "E", "abs_phi", "abs_E")}
    ep, ee = nerr(phi, E, sub)
    assert ep.max() <= 1e-12 and ee.max() <= 1e-12


def test_near_list_overflow_regrows(cyl):
    w, ref = cyl
    ctx = make_ctx(w)
    ctx.set_near_capacity(8, grow=True)
    phi, E, _ = run_gpu(ctx, w.points, "fp64")
    st = ctx.stats()
    ctx.close()
    assert st["near_capacity"] >= st["near_pairs"] > 8
    ep, ee = nerr(phi, E, ref)
    assert ep.max() <= 1e-12 and ee.max() <= 1e-12


def test_fixed_near_list_overflow_is_reported(cyl):
    """A fixed near-pair list never makes the host wait; an evaluation that overflows it is
    reported by stats() and, once it has finished, by the next call; a growing list then
    gives the oracle's result."""
    torch = torch_mod()
    w, ref = cyl
    ctx = make_ctx(w)
    ctx.set_near_capacity(8)
    pts = torch.tensor(np.ascontiguousarray(w.points.T), dtype=torch.float64, device="cuda:0")
    _, _, rc = ctx.eval(pts)
    assert rc == 0
    with pytest.raises(bemc.BemcError) as ei:
        ctx.stats()
    assert ei.value.code == bemc.E_LIMIT and "near pairs" in str(ei.value)
    ctx.eval(pts)
    torch.cuda.synchronize()
    with pytest.raises(bemc.BemcError) as ei:
        ctx.eval(pts)
    assert ei.value.code == bemc.E_LIMIT
    ctx.set_near_capacity(8, grow=True)
    phi, E, rc = run_gpu(ctx, w.points, "fp64")
    st = ctx.stats()
    ctx.close()
    assert rc == 0 and st["near_capacity"] >= st["near_pairs"] == ref["stats"]["near_pairs"]
    ep, ee = nerr(phi, E, ref)
    assert ep.max() <= 1e-12 and ee.max() <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("near_dr,after_upload", [(2.0, False), (10.0, False), (10.0, True)])
def test_other_near_thresholds(precision, near_dr, after_upload):
    """The distance-ratio switch at 2 (the smallest accepted: far sums expanded about the
    centroid down to DR 2) and at 10, against the oracle with the same threshold; also set
    after the geometry is resident (the thresholds and the near walk's element records are
    then rewritten on the device)."""
    w = W.cylinder_workload(40, 30, 1200, n_points=1500, near_frac=0.3, seed=23)
    ref = oracle.evaluate(w.tri, w.rect, w.sigma[0], w.points, oracle.params(33, 7, near_dr=near_dr), with_abs=True)
    ctx = bemc.Context(0)
    ctx.set_rules(33, 7, 3.0 if after_upload else near_dr)
    ctx.upload_geometry(w.tri, w.rect)
    ctx.upload_densities(w.sigma)
    if after_upload:
        run_gpu(ctx, w.points, precision)  # at 3 first
        ctx.set_rules(33, 7, near_dr)
    phi, E, rc = run_gpu(ctx, w.points, precision)
    st = ctx.stats()
    with pytest.raises(bemc.BemcError):
        ctx.set_rules(33, 7, 1.9)
    ctx.close()
    assert rc == 0 and st["near_pairs"] == ref["stats"]["near_pairs"] > 0
    ep, ee = nerr(phi, E, ref)
    print(f"near_dr {near_dr} {precision}: phi {ep.max():.2e} E {ee.max():.2e}, near pairs {st['near_pairs']}")
    assert ep.max() <= TOL[precision] and ee.max() <= TOL[precision]


@pytest.mark.parametrize("max_depth", [0, 1, 3])
def test_small_depth_caps(max_depth):
    """Depth caps 0 (the rule on the whole element for every near pair), 1 and 3: both near
    walks (a lane per pair, and a wavefront per pair for the points closest to an element)
    stop there and apply the rule to the capped nodes, as the oracle does; leaves and capped
    leaves match exactly."""
    w = W.cylinder_workload(40, 30, 1200, n_points=1500, near_frac=0.3, seed=29)
    ref = oracle.evaluate(w.tri, w.rect, w.sigma[0], w.points, oracle.params(33, 7, max_depth=max_depth),
                          with_abs=True)
    ctx = bemc.Context(0)
    ctx.set_rules(33, 7, 3.0, max_depth)
    ctx.upload_geometry(w.tri, w.rect)
    ctx.upload_densities(w.sigma)
    for prec in ("fp64", "mixed"):
        phi, E, rc = run_gpu(ctx, w.points, prec)
        st = ctx.stats()
        assert rc == 0 and st["near_pairs"] == ref["stats"]["near_pairs"] > 0
        assert st["max_depth"] == ref["stats"]["max_depth"] == max_depth
        for k in ("leaves", "cap_hits"):
            assert st[k] == ref["stats"][k], (k, st[k], ref["stats"][k])
        ep, ee = nerr(phi, E, ref)
        print(f"depth cap {max_depth} {prec}: phi {ep.max():.2e} E {ee.max():.2e}, cap hits {st['cap_hits']}")
        assert ep.max() <= TOL[prec] and ee.max() <= TOL[prec]
    ctx.close()


@pytest.mark.parametrize("tri_rule,gl", [(4, 2), (7, 3), (12, 5), (19, 7), (33, 8)])
def test_other_rules(tri_rule, gl):
    """Generic (run-time node count) kernels and every triangle table."""
    w = W.cylinder_workload(40, 30, 1200, n_points=700, near_frac=0.3, seed=5, tri_rule=tri_rule, rect_gl_n=gl)
    ref = oracle.evaluate(w.tri, w.rect, w.sigma[0], w.points, oracle.params(tri_rule, gl), with_abs=True)
    ctx = make_ctx(w)
    for prec in ("fp64", "mixed"):
        phi, E, _ = run_gpu(ctx, w.points, prec)
        ep, ee = nerr(phi, E, ref)
        assert ep.max() <= TOL[prec] and ee.max() <= TOL[prec], (prec, ep.max(), ee.max())
    ctx.close()


def test_points_on_elements():
    """Field points lying on an element: principal value, warning status."""
    w = W.cylinder_workload(40, 30, 1200, n_points=200, near_frac=0.5, seed=9)
    rng = np.random.default_rng(3)
    idx = rng.integers(0, w.n_elements, 40)
    on, _, _ = W.points_on_elements(w.tri, w.rect, idx, rng)
    pts = np.concatenate([w.points, on])
    ref = oracle.evaluate(w.tri, w.rect, w.sigma[0], pts, oracle.params(), with_abs=True)
    ctx = make_ctx(w)
    phi, E, rc = run_gpu(ctx, pts, "fp64")
    st = ctx.stats()
    ctx.close()
    assert rc == 0 and st["status"] == bemc.W_ON_SURFACE
    assert st["on_surface"] == ref["stats"]["on_surface"] >= 40
    ep, ee = nerr(phi, E, ref)
    assert ep.max() <= 1e-12 and ee.max() <= 1e-12


def test_single_kind_geometries():
    rng = np.random.default_rng(1)
    tri = W.icosphere(2, 1.0)
    rect = W.cylinder_mantle(1.0, -1.0, 1.0, 12, 3)
    pts = np.concatenate([W.shell_points(300, 1.5, 4.0, rng), rng.uniform(-0.9, 0.9, (200, 3)) * [0.5, 0.5, 1]])
    for t, r in ((tri, None), (None, rect)):
        ne = (0 if t is None else t.shape[0]) + (0 if r is None else r.shape[0])
        sig = rng.standard_normal(ne)
        ref = oracle.evaluate(t, r, sig, pts, oracle.params(), with_abs=True)
        ctx = bemc.Context(0)
        ctx.upload_geometry(t, r)
        ctx.upload_densities(sig)
        phi, E, _ = run_gpu(ctx, pts, "fp64")
        ctx.close()
        ep, ee = nerr(phi, E, ref)
        assert ep.max() <= 1e-12 and ee.max() <= 1e-12


def test_empty_and_errors():
    torch = torch_mod()
    w = W.cylinder_workload(40, 30, 1200, n_points=10, seed=9)
    ctx = bemc.Context(0)
    with pytest.raises(bemc.BemcError) as ei:
        ctx.eval(torch.zeros((3, 4), dtype=torch.float64, device="cuda:0"))
    assert ei.value.code == bemc.E_NO_GEOMETRY
    bad = w.tri.copy()
    bad[3, 3:6] = bad[3, 0:3]  # zero-area triangle
    with pytest.raises(bemc.BemcError) as ei:
        ctx.upload_geometry(bad, w.rect)
    assert ei.value.code == bemc.E_DEGENERATE_ELEMENT
    skew = w.rect.copy()
    skew[0, 6] += 0.01
    with pytest.raises(bemc.BemcError) as ei:
        ctx.upload_geometry(w.tri, skew)
    assert ei.value.code == bemc.E_NOT_RECTANGLE
    tiny = w.rect.copy()
    tiny[0, 3:9] *= 1e-170  # sides of 1e-172: the area underflows
    with pytest.raises(bemc.BemcError) as ei:
        ctx.upload_geometry(w.tri, tiny)
    assert ei.value.code == bemc.E_DEGENERATE_ELEMENT
    nan = w.tri.copy()
    nan[0, 0] = np.nan
    with pytest.raises(bemc.BemcError) as ei:
        ctx.upload_geometry(nan, w.rect)
    assert ei.value.code == bemc.E_NONFINITE
    ctx.upload_geometry(w.tri, w.rect)
    ctx.upload_densities(w.sigma)
    phi, E, rc = ctx.eval(torch.zeros((3, 0), dtype=torch.float64, device="cuda:0"))
    assert rc == 0 and phi.numel() == 0
    with pytest.raises(bemc.BemcError) as ei:
        ctx.eval(torch.zeros((3, 4), dtype=torch.float64, device="cuda:0"), rhs=1)
    assert ei.value.code == bemc.E_INVALID_ARG
    with pytest.raises(bemc.BemcError):
        ctx.set_rules(tri_rule=5)
    # index range: n >= 2^31 is rejected before any pointer is read or kernel launched
    small = torch.zeros((3, 4), dtype=torch.float64, device="cuda:0")
    out = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    rc = ctx.lib.bemc_eval(ctx.h, small.data_ptr(), 1 << 31, 0, 0, out.data_ptr(), None, None)
    assert rc == bemc.E_LIMIT
    rc = ctx.lib.bemc_eval_gradient(ctx.h, small.data_ptr(), 1 << 31, 0, 0, out.data_ptr(), None)
    assert rc == bemc.E_LIMIT
    ctx.close()


def test_far_field_is_deterministic(sphere):
    w, _ = sphere
    ctx = make_ctx(w)
    a = run_gpu(ctx, w.points, "fp64")
    b = run_gpu(ctx, w.points, "fp64")
    ctx.close()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_results_are_reproducible_bit_for_bit(cyl, precision):
    """With near pairs: the near-field sums are formed per point in element order, so two
    runs, and a run whose near-pair list overflowed and was regrown, agree bit for bit --
    for the field, the gradient and the collocation product."""
    torch = torch_mod()
    w, _ = cyl
    ctx = make_ctx(w)
    a = run_gpu(ctx, w.points, precision)
    b = run_gpu(ctx, w.points, precision)
    ctx.set_near_capacity(8, grow=True)  # forces a larger list and a repeated list pass
    c = run_gpu(ctx, w.points, precision)
    assert ctx.stats()["near_pairs"] > 8
    for x, y in ((a, b), (a, c)):
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
    pts = torch.tensor(np.ascontiguousarray(w.points.T), dtype=torch.float64, device="cuda:0")
    g1 = ctx.eval_gradient(pts, precision)[0].cpu().numpy()
    g2 = ctx.eval_gradient(pts, precision)[0].cpu().numpy()
    assert np.array_equal(g1, g2)
    sig = torch.tensor(np.stack([w.sigma[0], -w.sigma[0] ** 2]), device="cuda:0")
    o1 = ctx.collocation(sig, precision).cpu().numpy()
    o2 = ctx.collocation(sig, precision).cpu().numpy()
    assert np.array_equal(o1, o2)
    ctx.close()


# --------------------------------------------------------------- collocation -----
@pytest.fixture(scope="module")
def nested():
    t1, q1 = W.cylinder(1.0, -1.0, 1.0, 16, 4, 64)
    t2, q2 = W.cylinder(2.0, -1.5, 1.5, 24, 4, 144)
    tri, rect = np.concatenate([t1, t2]), np.concatenate([q1, q2])
    # eight right-hand sides per launch, as on the 200,000-element collocation workload
    sig = np.random.default_rng(8).standard_normal((8, tri.shape[0] + rect.shape[0]))
    sig[3] = np.abs(sig[3])  # one density of one sign: no cancellation in its rows
    sig[5] *= 1e-3           # right-hand sides of very different magnitudes
    ref = oracle.collocation(tri, rect, sig)
    return tri, rect, sig, ref


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_collocation_matvec(nested, precision):
    torch = torch_mod()
    tri, rect, sig, ref = nested
    ctx = bemc.Context(0)
    ctx.upload_geometry(tri, rect)
    s = torch.tensor(sig, dtype=torch.float64, device="cuda:0")
    out = ctx.collocation(s, precision=precision)
    torch.cuda.synchronize()
    st = ctx.stats()
    ctx.close()
    out = out.cpu().numpy()
    ne = sig.shape[1]
    assert st["on_surface"] == ne  # every row has its self term
    # normalised by each right-hand side's own row sum of |sigma_j phi_j| (oracle)
    err = np.abs(out - ref["out"]) / ref["abs"]
    print(f"collocation {precision}: max per right-hand side " + " ".join(f"{e:.1e}" for e in err.max(axis=1)))
    assert out.shape == (8, ne)
    assert err.max() <= TOL[precision]


def test_collocation_reuses_its_near_stage(nested):
    """Consecutive products on one context reuse the first one's near-pair list and near
    records (unit-density potentials): products with other densities match the oracle and a
    fresh context bit for bit, also after a field evaluation in between (which ends the
    reuse) and after a change of the near threshold (which forms the near stage anew)."""
    torch = torch_mod()
    tri, rect, sig, ref = nested
    ne = sig.shape[1]
    s8 = torch.tensor(sig, dtype=torch.float64, device="cuda:0")
    s2 = torch.tensor(sig[[4, 1]] * 3.0, dtype=torch.float64, device="cuda:0")

    def fresh(s, near_dr=3.0):
        c = bemc.Context(0)
        c.set_rules(33, 7, near_dr)
        c.upload_geometry(tri, rect)
        o = c.collocation(s, precision="fp64").cpu().numpy()
        st = c.stats()
        c.close()
        return o, st

    want8, st8 = fresh(s8)
    want2, _ = fresh(s2)
    ctx = bemc.Context(0)
    ctx.upload_geometry(tri, rect)
    ctx.upload_densities(sig[0])
    first = ctx.collocation(s8, precision="fp64").cpu().numpy()
    again = ctx.collocation(s2, precision="fp64").cpu().numpy()  # reuses the near stage
    st = ctx.stats()
    assert np.array_equal(first, want8) and np.array_equal(again, want2)
    for k in ("near_pairs", "leaves", "on_surface"):
        assert st[k] == st8[k], k
    ref2 = oracle.collocation(tri, rect, sig[[4, 1]] * 3.0)
    assert (np.abs(again - ref2["out"]) / ref2["abs"]).max() <= 1e-12
    # a field evaluation overwrites the buffers; the next product forms its near stage again
    pts = torch.tensor(np.ascontiguousarray(W.shell_points(300, 0.5, 3.0, np.random.default_rng(4)).T),
                       device="cuda:0")
    ctx.eval(pts, "fp64")
    after_eval = ctx.collocation(s2, precision="fp64").cpu().numpy()
    mixed = ctx.collocation(s8, precision="mixed").cpu().numpy()  # reuses it, mixed far field
    assert np.array_equal(after_eval, want2)
    assert (np.abs(mixed - ref["out"]) / ref["abs"]).max() <= 1e-6
    # another near threshold: the near stage is formed anew, with more near pairs
    ctx.set_rules(33, 7, 4.0)
    wider = ctx.collocation(s8, precision="fp64").cpu().numpy()
    st4 = ctx.stats()
    ctx.close()
    want4, st4_fresh = fresh(s8, 4.0)
    assert np.array_equal(wider, want4) and st4["near_pairs"] == st4_fresh["near_pairs"] > st8["near_pairs"]
    assert wider.shape == (8, ne)


# ------------------------------------------------------------ full-size sampled ----
def test_full_size_cylinder_sampled():
    """The benchmark workload at full size (150,000 elements, 1,000,000 points) in the
    launch configuration the benchmark uses; the oracle checks a sample of points."""
    torch = torch_mod()
    w = W.cylinder_150k()
    ctx = make_ctx(w)
    pts = torch.tensor(np.ascontiguousarray(w.points.T), dtype=torch.float64, device="cuda:0")
    res = {}
    for prec in ("fp64", "mixed"):
        phi, E, rc = ctx.eval(pts, precision=prec)
        torch.cuda.synchronize()
        res[prec] = (phi.cpu().numpy(), E.cpu().numpy().T.copy(), ctx.stats())
    ctx.close()
    rng = np.random.default_rng(42)
    isn = w.info["is_near"]
    idx = np.concatenate([rng.choice(np.nonzero(~isn)[0], 96, replace=False),
                          rng.choice(np.nonzero(isn)[0], 96, replace=False)])
    ref = oracle.evaluate(w.tri, w.rect, w.sigma[0], w.points[idx], oracle.params(33, 7), with_abs=True)
    for prec in ("fp64", "mixed"):
        phi, E, st = res[prec]
        sub_ref = ref
        ep, ee = nerr(phi[idx], E[idx], sub_ref)
        print(f"full-size {prec}: phi {ep.max():.2e} E {ee.max():.2e}; near pairs {st['near_pairs']}, "
              f"far {st['far_ms']:.1f} ms near {st['near_ms']:.1f} ms")
        assert ep.max() <= TOL[prec] and ee.max() <= TOL[prec]
        assert np.all(np.isfinite(phi)) and np.all(np.isfinite(E))


# ------------------------------------------------ rule choice by distance ratio ------
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_dr_rules_parity(cyl, precision):
    """Far pairs take 7/12/19/33 (triangles) and B2/B3/B4/7x7 (rectangles) by distance
    ratio; the points are Morton-ordered inside the library and returned in input order."""
    w, ref_fixed = cyl
    ref = oracle.evaluate(w.tri, w.rect, w.sigma[0], w.points, oracle.params(33, 7, dr_rules=True), with_abs=True)
    ctx = make_ctx(w)
    ctx.set_dr_rules(True)
    phi, E, rc = run_gpu(ctx, w.points, precision)
    st = ctx.stats()
    ctx.close()
    assert rc == 0 and st["near_pairs"] == ref["stats"]["near_pairs"]
    fixed_terms = w.points.shape[0] * (w.tri.shape[0] * 33 + w.rect.shape[0] * 49)
    assert 0 < st["node_interactions"] < fixed_terms
    ep, ee = nerr(phi, E, ref)
    print(f"dr rules {precision}: phi {ep.max():.2e} E {ee.max():.2e}; terms {st['node_interactions']:.3e} "
          f"vs {fixed_terms:.3e} fixed")
    assert ep.max() <= TOL[precision] and ee.max() <= TOL[precision]
    ep, ee = nerr(phi, E, ref_fixed)  # the coarser rules stay at the fixed rules' accuracy
    assert ep.max() <= TOL[precision] and ee.max() <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_dr_rules_custom_limits_and_rules(precision):
    """Other limits and other finest rules (19-point triangles, Table B4 rectangles): the
    run-time node-count kernel, checked against the oracle with the same settings.  Rules
    coarser than the third level are rejected while the rule choice is on."""
    w = W.cylinder_workload(40, 30, 1200, n_points=1500, near_frac=0.3, seed=23)
    tri_dr, rect_dr = (60.0, 20.0, 8.0), (90.0, 30.0, 10.0)
    prm = oracle.params(19, rect_gl_n=0, rect_table_n=17, dr_rules=True, tri_dr=tri_dr, rect_dr=rect_dr)
    ref = oracle.evaluate(w.tri, w.rect, w.sigma[0], w.points, prm, with_abs=True)
    ctx = bemc.Context(0)
    ctx.set_rules(19, -17)
    ctx.set_dr_rules(True, tri_dr, rect_dr)
    with pytest.raises(bemc.BemcError):
        ctx.set_rules(12, -17)
    with pytest.raises(bemc.BemcError):
        ctx.set_rules(19, -12)
    ctx.upload_geometry(w.tri, w.rect)
    ctx.upload_densities(w.sigma)
    phi, E, _ = run_gpu(ctx, w.points, precision)
    st = ctx.stats()
    ctx.close()
    assert st["near_pairs"] == ref["stats"]["near_pairs"] and st["leaves"] == ref["stats"]["leaves"]
    ep, ee = nerr(phi, E, ref)
    print(f"dr custom {precision}: phi {ep.max():.2e} E {ee.max():.2e}")
    assert ep.max() <= TOL[precision] and ee.max() <= TOL[precision]


def band_points(centre, L, dr, n, rng):
    """n points at distance dr * L from `centre`, isotropic directions."""
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return centre + dr * L * v


@pytest.mark.parametrize("kind", ["tri", "rect"])
def test_dr_rules_single_level_bands(kind):
    """One element; each evaluation holds only points just above or just below one of the
    level limits (distance ratio limit * (1 +- 1e-6)), so every wavefront needs exactly one
    level: the executed terms are n x that level's node count, the per-pair count equals
    them, and the result equals the oracle's per-pair choice to 1e-14 (plain relative
    error: one positive element, no cancellation)."""
    torch = torch_mod()
    rng = np.random.default_rng(2024)
    if kind == "tri":
        tri = np.array([[0.1, -0.2, 0.05, 1.3, 0.1, -0.1, 0.4, 1.1, 0.3]])
        rect = np.zeros((0, 9))
        a, b, c = (np.linalg.norm(tri[0, 3:6] - tri[0, 0:3]), np.linalg.norm(tri[0, 6:9] - tri[0, 3:6]),
                   np.linalg.norm(tri[0, 0:3] - tri[0, 6:9]))
        L = (a + b + c) / 3.0
        centre = (tri[0, 0:3] + tri[0, 3:6] + tri[0, 6:9]) / 3.0
        limits, nodes = (100.0, 25.0, 10.0, 3.0), (7, 12, 19, 33)
    else:
        tri = np.zeros((0, 9))
        e1, e2 = np.array([0.8, 0.3, 0.0]), np.array([-0.3 * 0.5, 0.8 * 0.5, 0.7])
        e2 -= e1 * (e1 @ e2) / (e1 @ e1)
        rect = np.concatenate([[0.2, 0.1, -0.3], e1, e2])[None, :]
        L = 0.5 * (np.linalg.norm(e1) + np.linalg.norm(e2))
        centre = rect[0, 0:3] + 0.5 * e1 + 0.5 * e2
        limits, nodes = (150.0, 40.0, 15.0, 3.0), (7, 12, 17, 49)
    sigma = np.array([[0.7]])
    ctx = bemc.Context(0)
    ctx.set_rules(33, 7)
    ctx.set_dr_rules(True)
    ctx.upload_geometry(tri, rect)
    ctx.upload_densities(sigma)
    n = 320
    prm = oracle.params(33, 7, dr_rules=True)
    for lvl, lim in enumerate(limits):
        # just above the limit: this level; just below: the next finer one (none below DR 3)
        cases = [(lim * (1 + 1e-6), nodes[lvl])]
        if lvl < 3:
            cases.append((lim * (1 - 1e-6), nodes[lvl + 1]))
        for dr, want in cases:
            P = band_points(centre, L, dr, n, rng)
            for precision in ("fp64", "mixed"):
                phi, E, _ = run_gpu(ctx, P, precision)
                st = ctx.stats()
                assert st["near_pairs"] == 0
                assert st["node_interactions"] == n * want, (kind, dr, st["node_interactions"], n * want)
                assert st["node_interactions_pair_rule"] == n * want
                if precision == "fp64":
                    ref = oracle.evaluate(tri, rect, sigma[0], P, prm, with_abs=True)
                    rp = np.abs(phi - ref["phi"]) / np.abs(ref["phi"])
                    re = np.linalg.norm(E - ref["E"], axis=1) / np.linalg.norm(ref["E"], axis=1)
                    print(f"band {kind} DR {dr:.6g}: {want} nodes, phi {rp.max():.1e} E {re.max():.1e}")
                    assert rp.max() <= 1e-14 and re.max() <= 1e-14
    ctx.close()


@pytest.mark.parametrize("table", [4, 7, 12, 17, 33])
def test_rectangle_table_rules(table):
    w = W.cylinder_workload(40, 30, 1200, n_points=600, near_frac=0.3, seed=17)
    ref = oracle.evaluate(w.tri, w.rect, w.sigma[0], w.points, oracle.params(33, rect_gl_n=0, rect_table_n=table),
                          with_abs=True)
    ctx = bemc.Context(0)
    ctx.set_rules(33, -table)
    ctx.upload_geometry(w.tri, w.rect)
    ctx.upload_densities(w.sigma)
    for precision in ("fp64", "mixed"):
        phi, E, _ = run_gpu(ctx, w.points, precision)
        ep, ee = nerr(phi, E, ref)
        assert ep.max() <= TOL[precision] and ee.max() <= TOL[precision]
    ctx.close()


def test_dr_rules_full_size_sampled():
    torch = torch_mod()
    w = W.cylinder_150k()
    ctx = make_ctx(w)
    ctx.set_dr_rules(True)
    pts = torch.tensor(np.ascontiguousarray(w.points.T), dtype=torch.float64, device="cuda:0")
    res = {}
    for prec in ("fp64", "mixed"):
        phi, E, _ = ctx.eval(pts, precision=prec)
        torch.cuda.synchronize()
        res[prec] = (phi.cpu().numpy(), E.cpu().numpy().T.copy(), ctx.stats())
    ctx.close()
    rng = np.random.default_rng(43)
    idx = rng.choice(w.points.shape[0], 128, replace=False)
    ref = oracle.evaluate(w.tri, w.rect, w.sigma[0], w.points[idx], oracle.params(33, 7), with_abs=True)
    for prec in ("fp64", "mixed"):
        phi, E, st = res[prec]
        ep, ee = nerr(phi[idx], E[idx], ref)
        print(f"dr full-size {prec}: phi {ep.max():.2e} E {ee.max():.2e}; terms {st['node_interactions']:.3e}, "
              f"far {st['far_ms']:.1f} ms")
        assert ep.max() <= TOL[prec] and ee.max() <= TOL[prec]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_translation_far_from_the_origin(cyl, precision):
    """The same geometry and points moved by (1e3, -2e3, 5e2), i.e. coordinates 1e5 times the
    element size: offsets are formed relative to element centroids (far field) and first
    vertices (near field), so parity with the oracle on the same moved inputs holds at the
    usual tolerance.  (Against the unmoved run the inputs themselves differ: rounding the
    coordinates at 2e3 moves a point by ~2e-13, which is 1e-8 of its height above an element
    at 1e-3 L.)"""
    w, _ = cyl
    shift = np.array([1e3, -2e3, 5e2])
    tri = w.tri + np.tile(shift, 3)
    rect = w.rect.copy()
    rect[:, 0:3] += shift
    pts = w.points + shift
    ref = oracle.evaluate(tri, rect, w.sigma[0], pts, oracle.params(33, 7), with_abs=True)
    ctx = bemc.Context(0)
    ctx.upload_geometry(tri, rect)
    ctx.upload_densities(w.sigma)
    phi, E, _ = run_gpu(ctx, pts, precision)
    ctx.close()
    ep, ee = nerr(phi, E, ref)
    print(f"translated {precision}: phi {ep.max():.2e} E {ee.max():.2e}")
    assert ep.max() <= TOL[precision] and ee.max() <= TOL[precision]


def test_million_elements_sampled():
    """1,000,000 elements (the serving geometry) and 200,000 points on particle tracks
    inside it, plus points near its elements: FP64 and mixed, a sample checked against the
    oracle (element indices, chunking and the near-list regrouping at a million elements)."""
    torch = torch_mod()
    g = W.serving_geometry()
    rng = np.random.default_rng(61)
    tracks = np.concatenate([W.serving_query(i, 20_000) for i in range(9)])
    near, _ = W.near_points(g.tri, g.rect, 20_000, rng)
    pts = np.concatenate([tracks, near])
    ctx = bemc.Context(0)
    ctx.upload_geometry(g.tri, g.rect)
    ctx.upload_densities(g.sigma)
    tp = torch.tensor(np.ascontiguousarray(pts.T), dtype=torch.float64, device="cuda:0")
    res = {}
    for prec in ("fp64", "mixed"):
        phi, E, _ = ctx.eval(tp, prec)
        torch.cuda.synchronize()
        res[prec] = (phi.cpu().numpy(), E.cpu().numpy().T.copy(), ctx.stats())
    ctx.close()
    idx = np.concatenate([rng.choice(tracks.shape[0], 24, replace=False),
                          tracks.shape[0] + rng.choice(near.shape[0], 24, replace=False)])
    ref = oracle.evaluate(g.tri, g.rect, g.sigma[0], pts[idx], oracle.params(33, 7), with_abs=True)
    for prec in ("fp64", "mixed"):
        phi, E, st = res[prec]
        assert st["pairs"] == pts.shape[0] * 1_000_000 and st["near_pairs"] > 0
        ep, ee = nerr(phi[idx], E[idx], ref)
        print(f"1M elements {prec}: phi {ep.max():.2e} E {ee.max():.2e}; near pairs {st['near_pairs']}, "
              f"far {st['far_ms']:.0f} ms")
        assert ep.max() <= TOL[prec] and ee.max() <= TOL[prec]
        assert np.all(np.isfinite(phi)) and np.all(np.isfinite(E))


def rotated_skewed(w, seed=71, skew=5e-11):
    """The workload under a random rotation, with every other rectangle made a parallelogram:
    e2 gains a component of relative size `skew` along e1 (inside the upload's orthogonality
    tolerance of 1e-10, so the element is accepted and evaluated as the parallelogram it is)."""
    rng = np.random.default_rng(seed)
    R, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    tri = (w.tri.reshape(-1, 3, 3) @ R.T).reshape(-1, 9)
    rect = (w.rect.reshape(-1, 3, 3) @ R.T).reshape(-1, 9)
    e1, e2 = rect[:, 3:6], rect[:, 6:9]
    f = skew * np.linalg.norm(e2, axis=1) / np.linalg.norm(e1, axis=1)
    f[1::2] = 0.0
    rect[:, 6:9] = e2 + f[:, None] * e1
    return tri, rect, w.points @ R.T


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("dr", [False, True])
def test_rotated_geometry_and_parallelograms(cyl, precision, dr):
    """Elements in general orientation (every element frame has nonzero components on all
    axes) and rectangles skewed at 5e-11: parity with the oracle on the same inputs, fixed
    rules and rules by distance ratio (the 7 x 7 rows and the Table B levels)."""
    w, _ = cyl
    tri, rect, pts = rotated_skewed(w)
    ref = oracle.evaluate(tri, rect, w.sigma[0], pts, oracle.params(33, 7, dr_rules=dr), with_abs=True)
    ctx = bemc.Context(0)
    ctx.upload_geometry(tri, rect)
    ctx.upload_densities(w.sigma)
    ctx.set_dr_rules(dr)
    phi, E, _ = run_gpu(ctx, pts, precision)
    st = ctx.stats()
    ctx.close()
    assert st["near_pairs"] == ref["stats"]["near_pairs"]
    ep, ee = nerr(phi, E, ref)
    print(f"rotated, skewed, dr={dr} {precision}: phi {ep.max():.2e} E {ee.max():.2e}")
    assert ep.max() <= TOL[precision] and ee.max() <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_rotated_gradient_and_collocation(cyl, precision):
    """Field gradient and collocation product on the rotated, skewed geometry: the tensor's
    rotation from the element frames and the potential-only sums."""
    torch = torch_mod()
    w, _ = cyl
    tri, rect, pts = rotated_skewed(w, seed=72)
    pts = pts[::3]
    ref = oracle.gradient(tri, rect, w.sigma[0], pts, oracle.params(33, 7))
    ctx = bemc.Context(0)
    ctx.upload_geometry(tri, rect)
    ctx.upload_densities(w.sigma)
    tp = torch.tensor(np.ascontiguousarray(pts.T), dtype=torch.float64, device="cuda:0")
    G, rc = ctx.eval_gradient(tp, precision=precision)
    torch.cuda.synchronize()
    G = G.cpu().numpy().T
    eg = np.abs(G - ref["G"]).max(axis=1) / ref["abs_T"]
    print(f"rotated gradient {precision}: {eg.max():.2e}")
    assert rc == 0 and eg.max() <= TOL[precision]
    sig = np.random.default_rng(9).standard_normal(tri.shape[0] + rect.shape[0])
    refc = oracle.collocation(tri, rect, sig)
    out = ctx.collocation(torch.tensor(sig[None, :], dtype=torch.float64, device="cuda:0"), precision=precision)
    torch.cuda.synchronize()
    ctx.close()
    ec = np.abs(out.cpu().numpy()[0] - refc["out"][0]) / refc["abs"][0]
    print(f"rotated collocation {precision}: {ec.max():.2e}")
    assert ec.max() <= TOL[precision]


@pytest.mark.parametrize("scale", [1e-7, 1e4])
def test_scaled_geometry(cyl, scale):
    """The cylinder workload scaled to nanometre elements (1e-7) and to 250 m elements (1e4):
    field and gradient in both precisions against the oracle on the same inputs (no overflow
    or underflow in the FP32 sums; the gradient's FP32 products use unit vectors)."""
    torch = torch_mod()
    w, _ = cyl
    tri, rect, pts = w.tri * scale, w.rect.copy(), w.points[::2] * scale
    rect[:, 0:3] *= scale
    rect[:, 3:9] *= scale
    ref = oracle.evaluate(tri, rect, w.sigma[0], pts, oracle.params(33, 7), with_abs=True)
    refg = oracle.gradient(tri, rect, w.sigma[0], pts, oracle.params(33, 7))
    ctx = bemc.Context(0)
    ctx.upload_geometry(tri, rect)
    ctx.upload_densities(w.sigma)
    tp = torch.tensor(np.ascontiguousarray(pts.T), dtype=torch.float64, device="cuda:0")
    for precision in ("fp64", "mixed"):
        phi, E, _ = ctx.eval(tp, precision=precision)
        G, _ = ctx.eval_gradient(tp, precision=precision)
        torch.cuda.synchronize()
        ep, ee = nerr(phi.cpu().numpy(), E.cpu().numpy().T.copy(), ref)
        eg = np.abs(G.cpu().numpy().T - refg["G"]).max(axis=1) / refg["abs_T"]
        print(f"scale {scale:g} {precision}: phi {ep.max():.2e} E {ee.max():.2e} grad {eg.max():.2e}")
        assert ep.max() <= TOL[precision] and ee.max() <= TOL[precision] and eg.max() <= TOL[precision]
    ctx.close()
