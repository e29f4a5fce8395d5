"""The persistent factorisation (one launch for every stage of every system,
device task queues, KRR_OPT_PERSISTENT = 1) against the multi-launch
sequence (KRR_OPT_PERSISTENT = 0, the default): the same tile bodies run in
the same order inside each system, so alpha, the refinement record and the
predictions must be identical bit for bit -- for balanced and ragged batches,
in mixed precision (BF16 packed path and its FP32-update fallback), FP32 and
FP64, and for fewer systems than XCDs (one shared queue).  Both are also
checked against the FP64 oracle.  The give-up path is forced from the host
with a zero wait limit: the launch must end and the fit report KRR_EDEVICE
(or, if no task had to wait, succeed with the same results); the context
stays usable."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1805_00569_amd import datagen, krr
from _parity import ew

pytestmark = pytest.mark.gpu


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _fit(ctx, X, y, a, C, p, params, persistent):
    ctx.set_option(krr.OPT_PERSISTENT, 1 if persistent else 0)
    try:
        models, info, st = ctx.fit(X, y, a, C, p, params)
    finally:
        ctx.set_option(krr.OPT_PERSISTENT, 0)
    alphas = [[m.alpha(j).cpu().numpy() for j in range(p)] for m in models]
    return models, info, st, alphas


CASES = [
    # name, n, d, p, method, prec, sigma, lam, panel
    ("balanced_mixed", 4096, 20, 8, "kbalance", "mixed", 3.0, 1e-2, 16),
    ("ragged_mixed", 9000, 12, 11, "kmeans", "mixed", 2.0, 1e-2, 4),
    ("ragged_mixed_fallback", 5000, 10, 9, "kmeans", None, 0.0, 1e-1, 6),
    ("ragged_fp32", 7000, 16, 10, "kmeans", "fp32", 2.0, 1e-2, 5),
    ("ragged_fp64", 5000, 8, 9, "kmeans", "fp64", 1.5, 1e-2, 3),
    ("few_systems_mixed", 6000, 16, 3, "kmeans", "mixed", 2.0, 1e-2, 16),
    ("one_system_fp64", 3000, 6, 1, "kmeans", "fp64", 1.0, 1e-3, 8),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_persistent_equals_launch_sequence(ctx, dev, case):
    name, n, d, p, method, prec, sigma, lam, panel = case
    w = datagen.small(300 + n, n, d, k=200, p=p, comps=p, dtype=np.float32 if prec != "fp64" else np.float64)
    if prec is None:   # median-heuristic sigma in mixed precision: systems take the FP32-update fallback
        prec, sigma = "mixed", datagen.median_heuristic_sigma(w.X)
    print(f"persistent vs launches: {name} n={n} d={d} p={p} {prec} sigma={sigma:.3f} panel={panel}", flush=True)
    X, y = _t(w.X, dev), _t(w.y.astype(w.X.dtype), dev)
    C, a, sz = ctx.partition(X, p, method, lloyd_iters=8, seed=n)
    params = [krr.Params(sigma=sigma, lam=lam, prec=prec, refine_tol=1e-8, max_refine=30),
              krr.Params(sigma=sigma * 1.5, lam=lam, prec=prec, refine_tol=1e-8, max_refine=30)]
    ctx.set_option(krr.OPT_PANEL_TILES, panel)
    try:
        m1, i1, s1, a1 = _fit(ctx, X, y, a, C, p, params, True)
        m0, i0, s0, a0 = _fit(ctx, X, y, a, C, p, params, False)
    finally:
        ctx.set_option(krr.OPT_PANEL_TILES, 0)
    assert s1 == s0 == 0
    for q in range(2):
        for j in range(p):
            assert np.array_equal(a1[q][j], a0[q][j]), (q, j)
    keys = ("status", "refine_iters", "fallback", "rel_residual", "kappa_est", "err_est", "kappa_bound")
    assert [[r[k] for k in keys] for r in i1] == [[r[k] for k in keys] for r in i0]
    if prec == "mixed":
        print(f"  fallbacks {sum(r['fallback'] for r in i1)}, steps max {max(r['refine_iters'] for r in i1)}",
              flush=True)
    yh1 = ctx.predict(m1[0], _t(w.Xt, dev)).cpu().numpy()
    yh0 = ctx.predict(m0[0], _t(w.Xt, dev)).cpu().numpy()
    assert np.array_equal(yh1, yh0)
    # and against the oracle
    a_np, C_np = a.cpu().numpy(), C.cpu().numpy()
    yo = w.y.astype(w.X.dtype).astype(np.float64)
    om = O.fit(w.X, yo, a_np, C_np, p, params[0].sigma, params[0].lam)
    tol = {"fp64": 1e-10, "mixed": 1e-6, "fp32": 1e-2}[prec]
    for j in range(p):
        assert ew(a1[0][j], om.alphas[j]) < tol, j
    for m in m1 + m0:
        m.free()


def test_persistent_gives_up_when_forced(ctx, dev):
    w = datagen.small(41, 6000, 10, k=10, p=6, comps=6, dtype=np.float32)
    X, y = _t(w.X, dev), _t(w.y.astype(np.float32), dev)
    C, a, _ = ctx.partition(X, 6, "kmeans", lloyd_iters=5, seed=4)
    params = [krr.Params(sigma=2.0, lam=1e-2, prec="mixed", refine_tol=1e-6, max_refine=10)]
    print("persistent: forced give-up (wait limit 0 ms)", flush=True)
    ref, _, st = ctx.fit(X, y, a, C, 6, params)
    assert st == 0
    ctx.set_option(krr.OPT_PERSIST_WAIT_MS, 0)
    try:
        try:
            models, info, st = ctx.fit(X, y, a, C, 6, params)
            gave_up = False
        except krr.KrrError as e:
            assert e.status == krr.KRR_EDEVICE and "gave up" in str(e)
            gave_up = True
    finally:
        ctx.set_option(krr.OPT_PERSIST_WAIT_MS, 30000)
    if not gave_up:
        for j in range(6):
            assert np.array_equal(models[0].alpha(j).cpu().numpy(), ref[0].alpha(j).cpu().numpy())
        models[0].free()
    print(f"  gave up: {gave_up}", flush=True)
    again, _, st = ctx.fit(X, y, a, C, 6, params)   # the context still works
    assert st == 0
    for j in range(6):
        assert np.array_equal(again[0].alpha(j).cpu().numpy(), ref[0].alpha(j).cpu().numpy())
    again[0].free()
    ref[0].free()


@pytest.mark.parametrize("prec", ["mixed", "fp32", "fp64"])
def test_factor_streams_give_identical_results(ctx, dev, prec):
    """KRR_OPT_FACTOR_STREAMS: the launch sequence split into groups of
    systems factored at the same time on 1, 2, 3 or 4 streams gives the same
    alpha bit for bit (ragged K-means batch of 24 systems, 16 and 8 of them
    needed for two groups of eight), and the context keeps working."""
    w = datagen.small(900, 20000, 12, k=200, p=24, comps=24, dtype=np.float64 if prec == "fp64" else np.float32)
    X, y = _t(w.X, dev), _t(w.y.astype(w.X.dtype), dev)
    C, a, sz = ctx.partition(X, 24, "kmeans", lloyd_iters=6, seed=3)
    print(f"factor streams {prec}: sizes {sorted(sz.cpu().numpy().tolist())[:3]}..{int(sz.max())}", flush=True)
    params = [krr.Params(sigma=2.0, lam=1e-2, prec=prec, refine_tol=1e-8, max_refine=30)]
    ref = None
    try:
        for fs in (1, 2, 3, 4):
            ctx.set_option(krr.OPT_FACTOR_STREAMS, fs)
            models, info, st = ctx.fit(X, y, a, C, 24, params)
            assert st == 0
            al = [models[0].alpha(j).cpu().numpy() for j in range(24)]
            rows = [(r["status"], r["refine_iters"], r["fallback"]) for r in info]
            for m in models:
                m.free()
            if ref is None:
                ref = (al, rows)
            else:
                assert rows == ref[1], fs
                for j in range(24):
                    assert np.array_equal(al[j], ref[0][j]), (fs, j)
    finally:
        ctx.set_option(krr.OPT_FACTOR_STREAMS, 2)
    with pytest.raises(krr.KrrError):
        ctx.set_option(krr.OPT_FACTOR_STREAMS, 5)
