"""Serving at the scale of the serving benchmark: the 1,000,000-element cylinder resident in
HBM, queries of 1, 4,096 and 65,536 points along particle tracks inside the electrode and
one query next to the electrode surface (near field), FP64 and mixed, one rule per kind and
the rule choice by distance ratio.  Each query alone equals the same query in a mix of
concurrent queries, and 32 sampled points of every query agree with the oracle (Sec. 4,
Eq. 4.1 with the subdivision below distance ratio 3).  A second test forces the growth of a
batch slot's near-pair list."""
import numpy as np
import pytest

import oracle
from paper_1606_03743_amd import bemc, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    import torch

    assert torch.cuda.is_available()
    g = W.serving_geometry()
    sizes = [1, 4096, 65536]
    queries = [np.ascontiguousarray(W.serving_query(1000 + i, s)) for i, s in enumerate(sizes)]
    near, _ = W.near_points(g.tri, g.rect, 3000, np.random.default_rng(12))
    queries.append(np.ascontiguousarray(near))
    return g, queries


def serve(g, queries, precision, dr, alone, **cfg):
    ctx = bemc.Context(0)
    ctx.set_dr_rules(dr)
    ctx.upload_geometry(g.tri, g.rect)
    ctx.upload_densities(g.sigma)
    ctx.server_start(precision=precision, **cfg)
    phis = [np.full(len(q), np.nan) for q in queries]
    Es = [np.full((len(q), 3), np.nan) for q in queries]
    if alone:
        infos = [ctx.server_wait(ctx.server_submit(q, p, e), 100.0) for q, p, e in zip(queries, phis, Es)]
    else:
        # the longest query first: while its batch runs, the others wait and are packed together
        order = sorted(range(len(queries)), key=lambda i: -len(queries[i]))
        ts = {i: ctx.server_submit(queries[i], phis[i], Es[i]) for i in order}
        infos = [ctx.server_wait(ts[i], 100.0) for i in range(len(queries))]
    ctx.server_stop()
    ctx.close()
    assert all(i["done"] == 1 and i["status"] == 0 for i in infos)
    return phis, Es, infos


@pytest.mark.parametrize("precision,tol,dr", [("fp64", 1e-12, False), ("mixed", 1e-6, False),
                                              ("fp64", 1e-12, True), ("mixed", 1e-6, True)])
def test_serving_full_geometry(big, precision, tol, dr):
    g, queries = big
    cfg = dict(mem_budget_bytes=16 << 30, max_batch_points=1 << 16)
    print(f"serving 1M elements: {precision} dr={dr} alone", flush=True)
    pa, Ea, _ = serve(g, queries, precision, dr, alone=True, n_streams=2, small_query_points=4096, **cfg)
    print(f"serving 1M elements: {precision} dr={dr} mix", flush=True)
    # one stream: the queries after the 65,536-point one queue behind it and share a batch
    pm, Em, im = serve(g, queries, precision, dr, alone=False, n_streams=1, small_query_points=0, **cfg)
    longest = int(np.argmax([len(q) for q in queries]))
    assert len({i["batch_id"] for k, i in enumerate(im) if k != longest}) == 1
    assert im[longest]["batch_id"] not in {i["batch_id"] for k, i in enumerate(im) if k != longest}
    rng = np.random.default_rng(31)
    sel = [rng.choice(len(q), min(32, len(q)), replace=False) for q in queries]
    P = np.concatenate([q[s] for q, s in zip(queries, sel)])
    ref = oracle.evaluate(g.tri, g.rect, g.sigma[0], P, oracle.params(33, 7, dr_rules=dr), with_abs=True)
    assert ref["stats"]["near_pairs"] > 0
    off = 0
    for q, s, a, b, ea, eb in zip(queries, sel, pa, pm, Ea, Em):
        sl = slice(off, off + len(s))
        off += len(s)
        assert np.isfinite(a).all() and np.isfinite(b).all()
        d_p = np.abs(a[s] - b[s]) / ref["abs_phi"][sl]
        d_e = np.sum(np.abs(ea[s] - eb[s]), axis=1) / ref["abs_E"][sl]
        assert d_p.max() <= tol and d_e.max() <= tol
        for phi, E in ((a, ea), (b, eb)):
            ep = np.abs(phi[s] - ref["phi"][sl]) / ref["abs_phi"][sl]
            ee = np.sum(np.abs(E[s] - ref["E"][sl]), axis=1) / ref["abs_E"][sl]
            print(f"  query of {len(q)} points: phi {ep.max():.2e} E {ee.max():.2e}")
            assert ep.max() <= tol and ee.max() <= tol


def test_serving_near_list_growth():
    """A batch of 4,096 points just above a fine mesh has more near pairs than a slot's
    initial list (16 per point of the batch size): the list grows and the batch completes
    with the oracle's result."""
    w = W.cylinder_workload(40, 30, 1200, n_points=10, seed=78)
    rng = np.random.default_rng(8)
    idx = rng.integers(0, w.n_elements, 4096)
    P, nrm, L = W.points_on_elements(w.tri, w.rect, idx, rng)
    q = np.ascontiguousarray(P + nrm * (1e-3 * L)[:, None])
    ref = oracle.evaluate(w.tri, w.rect, w.sigma[0], q, oracle.params(33, 7), with_abs=True)
    assert ref["stats"]["near_pairs"] > 16 * 4096
    for precision, tol in (("fp64", 1e-12), ("mixed", 1e-6)):
        (phi,), (E,), (info,) = serve(w, [q], precision, False, alone=True, mem_budget_bytes=1 << 30,
                                      max_batch_points=4096, n_streams=2)
        ep = np.abs(phi - ref["phi"]) / ref["abs_phi"]
        ee = np.sum(np.abs(E - ref["E"]), axis=1) / ref["abs_E"]
        assert ep.max() <= tol and ee.max() <= tol
