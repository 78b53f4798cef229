"""GPU parity on seeded random element soups: triangles of any shape and orientation,
rectangles in random orientation with aspect ratios up to 10, sizes over 1.5 decades, every
rule family (triangle rules 4-33, Gauss-Legendre n x n, Tables B), far points and points
from 1e-3 L to 2 L above random elements; fixed rules and rules by distance ratio, FP64 and
mixed.  The oracle runs on the same inputs with the same settings.  Same error measure and
tolerances as the other parity tests (FP64 1e-12, mixed 1e-6).
"""
import numpy as np
import pytest

import oracle
from paper_1606_03743_amd import bemc, workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-6}
TRI_RULES = (4, 7, 12, 19, 33)
RECT_RULES = (1, 2, 3, 4, 5, 6, 7, 8, -4, -7, -12, -17, -33)  # n x n Gauss-Legendre, or Table B (negative)


def soup(seed, n_tri=300, n_rect=200, n_far=1500, n_near=500):
    rng = np.random.default_rng(seed)
    c = rng.uniform(-2.0, 2.0, (n_tri, 3))
    s = 10.0 ** rng.uniform(-2.0, -0.5, n_tri)
    tri = (c[:, None, :] + rng.standard_normal((n_tri, 3, 3)) * s[:, None, None]).reshape(-1, 9)
    u = rng.standard_normal((n_rect, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    v = np.cross(u, rng.standard_normal((n_rect, 3)))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    la = 10.0 ** rng.uniform(-2.0, -0.5, n_rect)
    lb = la * 10.0 ** rng.uniform(-1.0, 1.0, n_rect)
    p0 = rng.uniform(-2.0, 2.0, (n_rect, 3))
    rect = np.concatenate([p0, u * la[:, None], v * lb[:, None]], axis=1)
    sigma = rng.standard_normal(n_tri + n_rect)
    far = rng.uniform(-3.0, 3.0, (n_far, 3))
    near, _ = W.near_points(tri, rect, n_near, rng)
    pts = np.concatenate([far, near])
    return tri, rect, sigma, pts, rng


def rules_for(rng, dr):
    if dr:  # the finest level must be at least the 19-point rule / Table B4
        return int(rng.choice((19, 33))), int(rng.choice((5, 6, 7, 8, -17, -33)))
    return int(rng.choice(TRI_RULES)), int(rng.choice(RECT_RULES))


def oracle_params(tri_rule, rect_rule, dr):
    if rect_rule > 0:
        return oracle.params(tri_rule, rect_gl_n=rect_rule, dr_rules=dr)
    return oracle.params(tri_rule, rect_gl_n=0, rect_table_n=-rect_rule, dr_rules=dr)


@pytest.mark.parametrize("dr", [False, True])
@pytest.mark.parametrize("seed", range(6))
def test_random_soup(seed, dr):
    import torch

    assert torch.cuda.is_available()
    tri, rect, sigma, pts, rng = soup(1000 + seed)
    tri_rule, rect_rule = rules_for(rng, dr)
    ref = oracle.evaluate(tri, rect, sigma, pts, oracle_params(tri_rule, rect_rule, dr), with_abs=True)
    ctx = bemc.Context(0)
    ctx.set_rules(tri_rule, rect_rule)
    ctx.upload_geometry(tri, rect)
    ctx.upload_densities(sigma)
    ctx.set_dr_rules(dr)
    tp = torch.tensor(np.ascontiguousarray(pts.T), dtype=torch.float64, device="cuda:0")
    for precision in ("fp64", "mixed"):
        phi, E, _ = ctx.eval(tp, precision=precision)
        torch.cuda.synchronize()
        st = ctx.stats()
        phi = phi.cpu().numpy()
        E = E.cpu().numpy().T
        ep = np.abs(phi - ref["phi"]) / ref["abs_phi"]
        ee = np.sum(np.abs(E - ref["E"]), axis=1) / ref["abs_E"]
        print(f"soup {seed} rules {tri_rule}/{rect_rule} dr={dr} {precision}: phi {ep.max():.2e} "
              f"E {ee.max():.2e}; near pairs {st['near_pairs']}")
        assert st["near_pairs"] == ref["stats"]["near_pairs"]
        assert ep.max() <= TOL[precision] and ee.max() <= TOL[precision]
    ctx.close()


@pytest.mark.parametrize("seed", range(3))
def test_random_soup_gradient_and_collocation(seed):
    """The field gradient (per-term scale abs_T) and the collocation product (self terms on
    every row) on the same kind of soups."""
    import torch

    assert torch.cuda.is_available()
    tri, rect, sigma, pts, rng = soup(2000 + seed, n_far=600, n_near=300)
    tri_rule, rect_rule = rules_for(rng, False)
    prm = oracle_params(tri_rule, rect_rule, False)
    refg = oracle.gradient(tri, rect, sigma, pts, prm)
    refc = oracle.collocation(tri, rect, sigma, prm=prm)
    ctx = bemc.Context(0)
    ctx.set_rules(tri_rule, rect_rule)
    ctx.upload_geometry(tri, rect)
    ctx.upload_densities(sigma)
    tp = torch.tensor(np.ascontiguousarray(pts.T), dtype=torch.float64, device="cuda:0")
    s = torch.tensor(sigma[None, :], dtype=torch.float64, device="cuda:0")
    for precision in ("fp64", "mixed"):
        G, rc = ctx.eval_gradient(tp, precision=precision)
        out = ctx.collocation(s, precision=precision)
        torch.cuda.synchronize()
        eg = np.abs(G.cpu().numpy().T - refg["G"]).max(axis=1) / refg["abs_T"]
        ec = np.abs(out.cpu().numpy()[0] - refc["out"][0]) / refc["abs"][0]
        print(f"soup {seed} rules {tri_rule}/{rect_rule} {precision}: gradient {eg.max():.2e} "
              f"collocation {ec.max():.2e}")
        assert rc == 0 and eg.max() <= TOL[precision] and ec.max() <= TOL[precision]
    ctx.close()
