"""HIP-graph replays of the fit's device phase and of predictions
(KRR_OPT_GRAPHS) against direct launches: every replay must give the same
bits as the direct call on the same inputs.  The inputs are rewritten in
place between replays (same pointers, new values), so a replay that reused
stale results would fail; eager work of the program and synchronisations
run between the replays.  Mixed precision (the first refinement steps run
inside the graph, the rest outside), FP64, a change of partition shapes
(a new capture), and routed / averaged predictions; the fit graphs with
the multi-launch and with the persistent factorisation."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1805_00569_amd import datagen, krr
from _parity import ew

pytestmark = pytest.mark.gpu


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.fixture(scope="module")
def ctxs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g = krr.Context(0)
    g.set_option(krr.OPT_GRAPHS, 1)
    e = krr.Context(0)
    yield g, e
    g.close()
    e.close()


def _alphas(models, p):
    return [[m.alpha(j).cpu().numpy() for j in range(p)] for m in models]


@pytest.fixture(params=[0, 1], ids=["launches", "persistent"])
def persistent(request, ctxs):
    """The graph context's factorisation: one launch per stage, or the
    persistent launch (whose task plans the graphs must find resident)."""
    ctxs[0].set_option(krr.OPT_PERSISTENT, request.param)
    yield request.param
    ctxs[0].set_option(krr.OPT_PERSISTENT, 0)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_fit_replays_equal_direct_fits(ctxs, dev, prec, persistent):
    gctx, ectx = ctxs
    st = torch.cuda.Stream()
    w = datagen.small(515, 5000, 12, k=300, p=6, comps=6, dtype=np.float32 if prec == "mixed" else np.float64)
    params = [krr.Params(sigma=2.0, lam=1e-2, prec=prec, refine_tol=1e-8, max_refine=20),
              krr.Params(sigma=datagen.median_heuristic_sigma(w.X), lam=1e-1, prec=prec, refine_tol=1e-8,
                         max_refine=20)]
    print(f"graphs: fit {prec} persistent={persistent}", flush=True)
    with torch.cuda.stream(st):
        X, y = _t(w.X, dev), _t(w.y.astype(w.X.dtype), dev)
        C, a, _ = ectx.partition(X, 6, "kmeans", lloyd_iters=8, seed=5)
        c0 = gctx.graph_counts()
        g = np.random.default_rng(7)
        for rep in range(5):
            # new label values in the same buffer
            y.copy_(_t((w.y * (1.0 + 0.1 * rep) + 0.01 * g.standard_normal(w.n)).astype(w.X.dtype), dev))
            mg, ig, sg = gctx.fit(X, y, a, C, 6, params)
            me, ie, se = ectx.fit(X, y, a, C, 6, params)
            assert sg == se == 0
            ag, ae = _alphas(mg, 6), _alphas(me, 6)
            for q in range(2):
                for j in range(6):
                    assert np.array_equal(ag[q][j], ae[q][j]), (rep, q, j)
            keys = ("status", "refine_iters", "fallback", "rel_residual", "err_est", "kappa_bound")
            assert [[r[k] for k in keys] for r in ig] == [[r[k] for k in keys] for r in ie]
            yh_g = gctx.predict(mg[0], _t(w.Xt, dev)).cpu().numpy()
            yh_e = ectx.predict(me[0], _t(w.Xt, dev)).cpu().numpy()
            assert np.array_equal(yh_g, yh_e)
            torch.cuda.synchronize()
            for m in mg + me:
                m.free()
        c1 = gctx.graph_counts()
    print(f"  captures {c1[0] - c0[0]}, replays {c1[1] - c0[1]}", flush=True)
    assert c1[0] - c0[0] >= 1 and c1[1] - c0[1] >= 2
    # the last replay against the oracle
    yo = y.cpu().numpy().astype(np.float64)
    om = O.fit(w.X, yo, a.cpu().numpy(), C.cpu().numpy(), 6, params[0].sigma, params[0].lam)
    tol = 1e-10 if prec == "fp64" else 1e-6
    for j in range(6):
        assert ew(ag[0][j], om.alphas[j]) < tol


def test_fit_graph_follows_a_change_of_shapes(ctxs, dev, persistent):
    gctx, ectx = ctxs
    st = torch.cuda.Stream()
    w = datagen.small(516, 4000, 8, k=100, p=5, comps=5, dtype=np.float32)
    params = [krr.Params(sigma=2.0, lam=1e-2, prec="mixed", refine_tol=1e-8, max_refine=20)]
    print(f"graphs: shape change persistent={persistent}", flush=True)
    c0 = gctx.graph_counts()
    with torch.cuda.stream(st):
        X, y = _t(w.X, dev), _t(w.y.astype(np.float32), dev)
        a = torch.empty(w.n, dtype=torch.int32, device=dev)
        for rep, seed in enumerate((1, 1, 1, 2, 2, 2, 1)):
            C, a2, _ = ectx.partition(X, 5, "kmeans", lloyd_iters=3 + seed, seed=seed)
            a.copy_(a2)   # the same assignment buffer, different partitions
            mg, _, sg = gctx.fit(X, y, a, C, 5, params)
            me, _, se = ectx.fit(X, y, a, C, 5, params)
            assert sg == se == 0
            for j in range(5):
                assert np.array_equal(mg[0].alpha(j).cpu().numpy(), me[0].alpha(j).cpu().numpy()), (rep, j)
            for m in mg + me:
                m.free()
            torch.cuda.synchronize()
    c1 = gctx.graph_counts()
    print(f"  captures {c1[0] - c0[0]}, replays {c1[1] - c0[1]}", flush=True)
    assert c1[0] - c0[0] >= 2 and c1[1] - c0[1] >= 2   # a graph per shape, replayed


@pytest.mark.parametrize("route", ["nearest", "average"])
def test_predict_replays_equal_direct_predictions(ctxs, dev, route):
    gctx, ectx = ctxs
    st = torch.cuda.Stream()
    w = datagen.small(517, 3000, 10, k=700, p=4, comps=4, dtype=np.float64)
    params = [krr.Params(sigma=1.5, lam=1e-2, prec="fp64")]
    print(f"graphs: predict {route}", flush=True)
    with torch.cuda.stream(st):
        X, y = _t(w.X, dev), _t(w.y, dev)
        C, a, _ = ectx.partition(X, 4, "kmeans", lloyd_iters=5, seed=9)
        m, _, s0 = gctx.fit(X, y, a, C, 4, params)
        me, _, s1 = ectx.fit(X, y, a, C, 4, params)
        assert s0 == s1 == 0
        Xt = _t(w.Xt, dev)
        out = torch.empty(w.Xt.shape[0], dtype=torch.float64, device=dev)
        c0 = gctx.graph_counts()
        g = np.random.default_rng(3)
        for rep in range(5):
            Xt.copy_(_t(w.Xt + 0.05 * g.standard_normal(w.Xt.shape), dev))   # new queries, same buffer
            yg = gctx.predict(m[0], Xt, route=route, out=out)   # the same output buffer every call
            ye = ectx.predict(me[0], Xt, route=route)   # direct launches
            assert torch.equal(yg, ye), rep
            yo, _ = O.predict(O.fit(w.X, w.y, a.cpu().numpy(), C.cpu().numpy(), 4, 1.5, 1e-2), Xt.cpu().numpy(),
                              route)
            assert np.max(np.abs(yg.cpu().numpy() - yo)) <= 1e-10 * max(np.max(np.abs(yo)), 1e-3)
            torch.cuda.synchronize()
        c1 = gctx.graph_counts()
        m[0].free()
        me[0].free()
    print(f"  captures {c1[0] - c0[0]}, replays {c1[1] - c0[1]}", flush=True)
    # the first calls run directly (one may grow the workspace, which changes the key)
    assert c1[0] - c0[0] == 1 and c1[1] - c0[1] >= 2
