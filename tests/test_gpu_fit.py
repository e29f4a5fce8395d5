"""Parity of krr_fit / krr_predict / krr_select with the FP64 oracle.

Tolerances: FP64 path 1e-10 relative on alpha and predictions; mixed path
1e-6 relative after refinement (FP64 residual), as the design requires; FP32
path bounded by a multiple of kappa * m * u32.  Every comparison is element
by element (max |a - b| over max |b|, see tests/_parity.py); errors of
predictions are scaled by max(max|yhat_ref|, 1e-3 max|y_test|) so that a
model whose predictions are all ~0 (kernel ~ identity) is judged against the
scale of the labels."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_1805_00569_amd import datagen, krr
from _parity import ew, pred_ew

pytestmark = pytest.mark.gpu


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _fit_both(ctx, dev, w, p, params, method="given", centroids=None, iters=10, seed=0):
    X, y = _t(w.X, dev), _t(w.y.astype(w.X.dtype), dev)
    if method == "given":
        C, a, _ = ctx.partition(X, p, "given", centroids=_t(centroids, dev))
    else:
        C, a, _ = ctx.partition(X, p, method, lloyd_iters=iters, seed=seed)
    models, info, st = ctx.fit(X, y, a, C, p, params)
    a_np = a.cpu().numpy()
    C_np = C.cpu().numpy()
    yo = w.y.astype(w.X.dtype).astype(np.float64)
    oms = [O.fit(w.X, yo, a_np, C_np, p, q.sigma, q.lam, q.kernel, q.lambda_times_m) for q in params]
    return models, info, st, oms, X, a_np


def test_plain_single_partition_fp64(ctx, dev):
    """p = 1, FP64: n=2048, d=16, sigma=1, lambda=1e-3 (Algorithm 1)."""
    w = datagen.plain_krr()
    print("plain fp64 n=2048 d=16", flush=True)
    params = [krr.Params(sigma=1.0, lam=1e-3, prec="fp64")]
    models, info, st, oms, X, _ = _fit_both(ctx, dev, w, 1, params, centroids=np.zeros((1, 16)))
    assert st == 0 and info[0]["status"] == 0 and info[0]["m"] == 2048
    alpha = models[0].alpha(0).cpu().numpy()
    assert ew(alpha, oms[0].alphas[0]) < 1e-10
    yhat = ctx.predict(models[0], _t(w.Xt, dev)).cpu().numpy()
    yo, _ = O.predict(oms[0], w.Xt)
    assert pred_ew(yhat, yo, w.yt) < 1e-10
    mse, best = ctx.select(models, _t(w.Xt, dev), _t(w.yt, dev))
    assert best == 0 and abs(mse[0] - O.mse(yo, w.yt)) <= 1e-10 * O.mse(yo, w.yt)


@pytest.mark.parametrize("n,d,p,panel", [(3000, 12, 5, 4), (700, 5, 2, 1), (900, 3, 3, 2), (130, 4, 1, 4)])
def test_ragged_partitions_fp64(ctx, dev, n, d, p, panel):
    """K-means partitions of uneven size (ragged tails, several tiles and
    panels), two settings fitted in one batch."""
    w = datagen.small(40 + n, n, d, k=150, p=p, comps=p, dtype=np.float64)
    print(f"ragged fp64 n={n} d={d} p={p} panel={panel}", flush=True)
    ctx.set_option(krr.OPT_PANEL_TILES, panel)
    try:
        params = [krr.Params(sigma=1.5, lam=1e-2, prec="fp64"), krr.Params(sigma=0.7, lam=1e-3, prec="fp64")]
        models, info, st, oms, X, a = _fit_both(ctx, dev, w, p, params, method="kmeans", iters=8, seed=n)
    finally:
        ctx.set_option(krr.OPT_PANEL_TILES, 0)
    assert st == 0
    for q in range(2):
        for j in range(p):
            assert info[q * p + j]["m"] == int((a == j).sum())
            alpha = models[q].alpha(j).cpu().numpy()
            assert ew(alpha, oms[q].alphas[j]) < 1e-10, (q, j)
        for route in ("nearest", "average", "all"):
            yhat = ctx.predict(models[q], _t(w.Xt, dev), route=route).cpu().numpy()
            yo, _ = O.predict(oms[q], w.Xt, route)
            assert pred_ew(yhat.ravel(), yo.ravel(), np.repeat(w.yt, p if route == "all" else 1)) < 1e-10, route
    mse, best = ctx.select(models, _t(w.Xt, dev), _t(w.yt, dev))
    mo = [O.mse(O.predict(om, w.Xt)[0], w.yt) for om in oms]
    np.testing.assert_allclose(mse, mo, rtol=1e-10)
    assert best == O.select(mo)


def test_dckrr_random_partition_average_route_fp64(ctx, dev):
    """DC-KRR (Algorithm 3): random even partition, per-partition systems
    (K + lambda m I) alpha = y, prediction averaged over all models, best
    setting by MSE -- against the oracle."""
    w = datagen.small(61, 3001, 6, k=200, p=4, comps=4, dtype=np.float64)
    print("dc-krr n=3001 d=6 p=4", flush=True)
    params = [krr.Params(sigma=s_, lam=1e-4, prec="fp64", lambda_times_m=True) for s_ in (0.8, 2.0)]
    models, info, st, oms, X, a = _fit_both(ctx, dev, w, 4, params, method="random", seed=17)
    assert st == 0
    assert sorted(int(i["m"]) for i in info[:4]) == [750, 750, 750, 751]
    for q in range(2):
        for j in range(4):
            assert ew(models[q].alpha(j).cpu().numpy(), oms[q].alphas[j]) < 1e-10, (q, j)
        yhat = ctx.predict(models[q], _t(w.Xt, dev), route="average").cpu().numpy()
        yo, _ = O.predict(oms[q], w.Xt, "average")
        assert pred_ew(yhat, yo, w.yt) < 1e-10
    mse, best = ctx.select(models, _t(w.Xt, dev), _t(w.yt, dev), route="average")
    mo = [O.mse(O.predict(om, w.Xt, "average")[0], w.yt) for om in oms]
    np.testing.assert_allclose(mse, mo, rtol=1e-10)
    assert best == O.select(mo)


def test_approx_kbalance_nearest_route_fp64(ctx, dev):
    """BKRR2 on the approximate parallel K-balance (Section 4.3): the
    partition identical to the oracle's, then per-partition fits and
    nearest-centre predictions against the oracle, and the best setting."""
    w = datagen.small(62, 3200, 6, k=300, p=4, comps=4, dtype=np.float64)
    print("approx k-balance n=3200 d=6 p=4", flush=True)
    params = [krr.Params(sigma=s_, lam=1e-3, prec="fp64") for s_ in (0.8, 2.0)]
    models, info, st, oms, X, a = _fit_both(ctx, dev, w, 4, params, method="kbalance_approx", iters=6, seed=19)
    assert st == 0
    _, ao = O.kbalance_approx(w.X, 4, 6, 19)
    np.testing.assert_array_equal(a, ao)
    assert sorted(int(i["m"]) for i in info[:4]) == [800] * 4   # p^2 divides n
    for q in range(2):
        for j in range(4):
            assert ew(models[q].alpha(j).cpu().numpy(), oms[q].alphas[j]) < 1e-10, (q, j)
        yhat = ctx.predict(models[q], _t(w.Xt, dev)).cpu().numpy()
        yo, _ = O.predict(oms[q], w.Xt)
        assert pred_ew(yhat, yo, w.yt) < 1e-10
    mse, best = ctx.select(models, _t(w.Xt, dev), _t(w.yt, dev))
    mo = [O.mse(O.predict(om, w.Xt)[0], w.yt) for om in oms]
    np.testing.assert_allclose(mse, mo, rtol=1e-10)
    assert best == O.select(mo)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_label_route_selection_is_the_lower_bound(ctx, dev, dtype):
    """BKRR3 / KKRR3 (Algorithm 6): per held-out point the partition model
    closest to its label.  The MSE matches the oracle's label choice, is at
    most the NEAREST and AVERAGE MSEs, and predict() refuses the route (it
    has no labels)."""
    w = datagen.small(62, 2500, 5, k=300, p=5, comps=5, dtype=dtype)
    print(f"label route n=2500 p=5 {dtype.__name__}", flush=True)
    params = [krr.Params(sigma=s_, lam=1e-3, prec="fp64") for s_ in (0.6, 1.5, 3.0)]
    models, info, st, oms, X, a = _fit_both(ctx, dev, w, 5, params, method="kbalance", iters=6, seed=4)
    assert st == 0
    Xv, yv = _t(w.Xt, dev), _t(w.yt.astype(dtype), dev)
    yt = w.yt.astype(dtype).astype(np.float64)
    mse_l, best_l = ctx.select(models, Xv, yv, route="label")
    mse_n, _ = ctx.select(models, Xv, yv, route="nearest")
    mse_a, _ = ctx.select(models, Xv, yv, route="average")
    mo = []
    for om in oms:
        allp, _ = O.predict(om, w.Xt, "all")
        chosen, _ = O.label_oracle_select(allp, yt)
        mo.append(O.mse(chosen, yt))
    np.testing.assert_allclose(mse_l, mo, rtol=1e-10)
    assert best_l == O.select(mo)
    assert all(l <= n_ * (1 + 1e-12) and l <= a_ * (1 + 1e-12) for l, n_, a_ in zip(mse_l, mse_n, mse_a))
    with pytest.raises(krr.KrrError) as e:
        ctx.predict(models[0], Xv, route="label")
    assert e.value.status == krr.KRR_EINVAL


def _okernel(q):
    """The oracle's description of a setting's kernel (Table 1)."""
    if q.kernel == "polynomial":
        return ("polynomial", q.kernel_a, q.kernel_r, q.kernel_degree)
    if q.kernel == "sigmoid":
        return ("sigmoid", q.kernel_a, q.kernel_r)
    return q.kernel


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_polynomial_sigmoid_and_gaussian_settings_in_one_batch(ctx, dev, prec):
    """Table 1's polynomial and sigmoid kernels beside the Gaussian in one
    batch (two polynomial settings share their kernel matrix): alpha,
    nearest-centre predictions and selection against the oracle."""
    w = datagen.small(63, 1800, 5, k=160, p=3, comps=3, dtype=np.float64, spread=1.0)
    print(f"kernels poly/sigmoid/gaussian {prec}", flush=True)
    params = [krr.Params(sigma=1.5, lam=1e-2, prec=prec, refine_tol=1e-10, max_refine=40),
              krr.Params(kernel="polynomial", kernel_a=0.1, kernel_r=1.0, kernel_degree=3, lam=1e-2, prec=prec,
                         refine_tol=1e-10, max_refine=40),
              krr.Params(kernel="polynomial", kernel_a=0.1, kernel_r=1.0, kernel_degree=3, lam=1e-1, prec=prec,
                         refine_tol=1e-10, max_refine=40),
              krr.Params(kernel="sigmoid", kernel_a=0.02, kernel_r=0.3, lam=1.0, prec=prec, refine_tol=1e-10,
                         max_refine=40)]
    X, y = _t(w.X, dev), _t(w.y, dev)
    C, a, _ = ctx.partition(X, 3, "kbalance", lloyd_iters=5, seed=3)
    models, info, st = ctx.fit(X, y, a, C, 3, params)
    for r in info:
        print(f"  setting {r['param']} part {r['partition']}: status {r['status']} steps {r['refine_iters']} "
              f"fallback {r['fallback']} kappa_est {r['kappa_est']:.3g} err_est {r['err_est']:.2e} "
              f"rel_res {r['rel_residual']:.2e}", flush=True)
    assert st == 0 and all(i["status"] == 0 for i in info)
    a_np, C_np = a.cpu().numpy(), C.cpu().numpy()
    oms = [O.fit(w.X, w.y, a_np, C_np, 3, q.sigma, q.lam, _okernel(q)) for q in params]
    tol = 1e-10 if prec == "fp64" else 1e-6
    for q in range(len(params)):
        for j in range(3):
            assert ew(models[q].alpha(j).cpu().numpy(), oms[q].alphas[j]) < tol, (q, j)
        yhat = ctx.predict(models[q], _t(w.Xt, dev)).cpu().numpy()
        yo, _ = O.predict(oms[q], w.Xt)
        assert pred_ew(yhat, yo, w.yt) < tol, q
    mse, best = ctx.select(models, _t(w.Xt, dev), _t(w.yt, dev))
    mo = [O.mse(O.predict(om, w.Xt)[0], w.yt) for om in oms]
    np.testing.assert_allclose(mse, mo, rtol=tol)
    assert best == O.select(mo)


def test_sigmoid_not_spd_reports_pivot(ctx, dev):
    """tanh(a x^T y + r) with r < 0 puts a negative value on the diagonal of
    the first point (x = 0): not positive definite at pivot 1, as the
    oracle's LAPACK-style check says; kernel arguments are validated."""
    X = np.array([[0.0, 0.0], [3.0, 0.0], [-3.0, 0.0]] * 30)
    y = np.linspace(-1.0, 1.0, X.shape[0])
    r = O.fit_one(X, y, 1.0, 0.0, ("sigmoid", 1.0, -1.0))
    assert r["status"] == O.STATUS_NOT_SPD and r["pivot"] == 1
    Xd = _t(X, dev)
    C, a, _ = ctx.partition(Xd, 1, "given", centroids=_t(np.zeros((1, 2)), dev))
    models, info, st = ctx.fit(Xd, _t(y, dev), a, C, 1,
                               [krr.Params(kernel="sigmoid", kernel_a=1.0, kernel_r=-1.0, lam=0.0, prec="fp64")])
    assert st == krr.KRR_ENOTSPD and info[0]["failed_pivot"] == 1
    for bad in (dict(kernel_degree=0), dict(kernel_degree=65), dict(kernel_a=float("inf"))):
        with pytest.raises(krr.KrrError) as e:
            ctx.fit(Xd, _t(y, dev), a, C, 1, [krr.Params(kernel="polynomial", prec="fp64", **bad)])
        assert e.value.status == krr.KRR_EINVAL


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_sigmoid_indefinite_systems_solved_by_lu(ctx, dev, prec):
    """Sigmoid kernel tanh(0.1 x^T y - 0.1) with lambda = 1: every one of the
    four ragged partitions (473..740 points) has K + lambda I indefinite
    (19..28 negative eigenvalues, condition numbers 3e3..2e4).  With
    indefinite = 1 Cholesky rejects each and LU with partial pivoting solves
    it (solver 1, status OK, failed_pivot = the oracle's Cholesky pivot),
    alpha against the oracle's LU; the same setting without the flag reports
    KRR_ENOTSPD, and a Gaussian setting in the batch keeps Cholesky."""
    w = datagen.small(71, 2400, 6, k=100, p=4, comps=4, dtype=np.float64 if prec == "fp64" else np.float32,
                      spread=1.0)
    g = np.random.default_rng(1)
    Cc = w.X[g.choice(w.n, 4, replace=False)].astype(np.float64)
    print(f"sigmoid indefinite -> LU ({prec})", flush=True)
    X, y = _t(w.X, dev), _t(w.y.astype(w.X.dtype), dev)
    C, a, _ = ctx.partition(X, 4, "given", centroids=_t(Cc, dev))
    sig = dict(kernel="sigmoid", kernel_a=0.1, kernel_r=-0.1, lam=1.0, prec=prec, refine_tol=1e-10, max_refine=30)
    params = [krr.Params(indefinite=True, **sig), krr.Params(sigma=1.0, lam=1e-2, prec=prec, refine_tol=1e-10,
                                                             max_refine=30, indefinite=True)]
    models, info, st = ctx.fit(X, y, a, C, 4, params)
    for r in info:
        print(f"  setting {r['param']} part {r['partition']} m {r['m']}: status {r['status']} solver {r['solver']} "
              f"pivot {r['failed_pivot']}", flush=True)
    assert st == 0
    a_np = a.cpu().numpy()
    om = O.fit(w.X, w.y.astype(w.X.dtype), a_np, Cc, 4, 1.0, 1.0, ("sigmoid", 0.1, -0.1), indefinite=True)
    og = O.fit(w.X, w.y.astype(w.X.dtype), a_np, Cc, 4, 1.0, 1e-2)
    for j in range(4):
        r = info[j]
        assert om.infos[j]["solver"] == "lu"
        # the pivot that rejects the system: FP64 Cholesky's exactly; FP32 updates may meet it elsewhere
        piv_ok = r["failed_pivot"] == om.infos[j]["pivot"] if prec == "fp64" else r["failed_pivot"] > 0
        assert r["solver"] == 1 and r["status"] == 0 and piv_ok, r
        assert r["rel_residual"] == -1.0 and r["err_est"] == -1.0
        assert ew(models[0].alpha(j).cpu().numpy(), om.alphas[j]) < 1e-9, j
        assert info[4 + j]["solver"] == 0 and info[4 + j]["status"] == 0
        assert ew(models[1].alpha(j).cpu().numpy(), og.alphas[j]) < (1e-10 if prec == "fp64" else 1e-6), j
    yhat = ctx.predict(models[0], _t(w.Xt, dev)).cpu().numpy()
    yo, _ = O.predict(om, w.Xt)
    assert pred_ew(yhat, yo, w.yt) < 1e-9
    for m in models:
        m.free()
    m2, info2, st2 = ctx.fit(X, y, a, C, 4, [krr.Params(**sig)])
    assert st2 == krr.KRR_ENOTSPD
    assert all(r["status"] == krr.KRR_ENOTSPD and r["solver"] == 0 and r["failed_pivot"] > 0 for r in info2)
    if prec == "fp64":
        assert [r["failed_pivot"] for r in info2] == [om.infos[j]["pivot"] for j in range(4)]
    for m in m2:
        m.free()


def test_batch_invariance_serial_equals_batched(ctx, dev):
    """The plain per-system launch sequence gives bitwise the same alpha as
    the batched one."""
    w = datagen.small(50, 1500, 6, k=40, p=3, comps=3, dtype=np.float32)
    X, y = _t(w.X, dev), _t(w.y.astype(np.float32), dev)
    C, a, _ = ctx.partition(X, 3, "kbalance", lloyd_iters=5, seed=2)
    params = [krr.Params(sigma=2.0, lam=1e-2, prec=pr) for pr in ("fp64",)]
    m1, i1, s1 = ctx.fit(X, y, a, C, 3, params)
    ctx.set_option(krr.OPT_SERIAL_FIT, 1)
    try:
        m2, i2, s2 = ctx.fit(X, y, a, C, 3, params)
    finally:
        ctx.set_option(krr.OPT_SERIAL_FIT, 0)
    for j in range(3):
        assert torch.equal(m1[0].alpha(j), m2[0].alpha(j))


def test_fp32_path(ctx, dev):
    w = datagen.small(60, 1200, 8, k=100, p=2, comps=2, dtype=np.float32)
    params = [krr.Params(sigma=3.0, lam=1e-1, prec="fp32")]
    models, info, st, oms, X, a = _fit_both(ctx, dev, w, 2, params, method="kmeans", iters=5, seed=1)
    assert st == 0
    for j in range(2):
        Xj = w.X[a == j].astype(np.float64)
        kappa = np.linalg.cond(O.kernel_matrix(Xj, Xj, 3.0) + 0.1 * np.eye(Xj.shape[0]))
        err = ew(models[0].alpha(j).cpu().numpy(), oms[0].alphas[j])
        assert err < 20 * kappa * Xj.shape[0] * 6e-8, (err, kappa)


@pytest.mark.parametrize("sigma", [None, 2.0])
def test_mixed_precision_refines_to_1e6(ctx, dev, sigma):
    """BF16 trailing updates + FP64 diagonal blocks + FP64 residual: alpha
    within 1e-6 of the FP64 solution after refinement.  sigma=None uses the
    median heuristic (kernel far from the identity, kappa ~ 1e2..1e4)."""
    w = datagen.small(70, 2000, 10, k=200, p=2, comps=2, dtype=np.float32)
    s = datagen.median_heuristic_sigma(w.X) if sigma is None else sigma
    print(f"mixed sigma={s:.3f}", flush=True)
    params = [krr.Params(sigma=s, lam=1e-1, prec="mixed", refine_tol=1e-8, max_refine=40)]
    models, info, st, oms, X, a = _fit_both(ctx, dev, w, 2, params, method="kbalance", iters=5, seed=3)
    assert st == 0, info
    for j in range(2):
        assert info[j]["rel_residual"] <= 1e-8 and 0 <= info[j]["err_est"] <= 1e-8
        err = ew(models[0].alpha(j).cpu().numpy(), oms[0].alphas[j])
        assert err < 1e-6, err
        print(f"partition {j}: refine steps {info[j]['refine_iters']} fallback {info[j]['fallback']} "
              f"kappa_est {info[j]['kappa_est']:.3g} err_est {info[j]['err_est']:.2e} alpha err {err:.2e}",
              flush=True)
        if sigma is not None:
            assert info[j]["fallback"] == 0
    yhat = ctx.predict(models[0], _t(w.Xt, dev)).cpu().numpy()
    yo, _ = O.predict(oms[0], w.Xt)
    assert pred_ew(yhat, yo, w.yt) < 1e-6


@pytest.mark.parametrize("panel", [1, 3, 16, 40])
def test_mixed_ragged_partitions_panels(ctx, dev, panel):
    """Mixed precision over k-means partitions of uneven size (systems with
    different tile counts in one batch) and panel widths that put diagonal
    blocks both at panel starts and inside the column launches (which also
    carry the forward solve of the first pass): alpha within 1e-6 of FP64."""
    w = datagen.small(75, 3000, 12, k=150, p=5, comps=5, dtype=np.float32)
    print(f"mixed ragged panel={panel}", flush=True)
    ctx.set_option(krr.OPT_PANEL_TILES, panel)
    try:
        params = [krr.Params(sigma=1.5, lam=1e-2, prec="mixed", refine_tol=1e-8, max_refine=40),
                  krr.Params(sigma=0.7, lam=1e-3, prec="mixed", refine_tol=1e-8, max_refine=40)]
        models, info, st, oms, X, a = _fit_both(ctx, dev, w, 5, params, method="kmeans", iters=8, seed=7)
    finally:
        ctx.set_option(krr.OPT_PANEL_TILES, 0)
    assert st == 0, info
    sizes = np.bincount(a, minlength=5)
    assert len(set(-(-sizes // 64))) > 1   # systems of different tile counts
    for q in range(2):
        for j in range(5):
            assert info[q * 5 + j]["rel_residual"] <= 1e-8
            assert ew(models[q].alpha(j).cpu().numpy(), oms[q].alphas[j]) < 1e-6, (q, j)


_LARGE = {}


def _large_system():
    """m = 8,300 points in 4 dimensions (FP32-representable) and the oracle's
    alpha for sigma = 0.5, lambda = 1e-2 (computed once)."""
    if not _LARGE:
        g = np.random.default_rng(85)
        m = 8300
        X = g.uniform(-1.0, 1.0, size=(m, 4)).astype(np.float32)
        y = (np.sin(X.astype(np.float64) @ np.array([1.0, -2.0, 0.5, 1.5]))
             + 0.1 * g.standard_normal(m)).astype(np.float32)
        ref = O.fit_one(X.astype(np.float64), y.astype(np.float64), 0.5, 1e-2)
        _LARGE.update(X=X, y=y, alpha=ref["alpha"])
    return _LARGE["X"], _LARGE["y"], _LARGE["alpha"]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_large_system_backward_solve_from_global(ctx, dev, prec):
    """One system of m = 8,300 (130 tile rows: the backward solve goes band
    by band, with a ragged top band of 2 rows) against the FP64 oracle."""
    X, y, alpha_ref = _large_system()
    print(f"large system m={X.shape[0]} {prec}", flush=True)
    Xg = X.astype(np.float64) if prec == "fp64" else X
    yg = y.astype(np.float64) if prec == "fp64" else y
    Xd = _t(Xg, dev)
    C, a, _ = ctx.partition(Xd, 1, "given", centroids=_t(np.zeros((1, 4), Xg.dtype), dev))
    models, info, st = ctx.fit(Xd, _t(yg, dev), a, C, 1,
                               [krr.Params(sigma=0.5, lam=1e-2, prec=prec, refine_tol=1e-8, max_refine=40)])
    assert st == 0 and info[0]["status"] == 0
    err = ew(models[0].alpha(0).cpu().numpy(), alpha_ref)
    assert err < (1e-10 if prec == "fp64" else 1e-6), err


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_large_system_wide_panel(ctx, dev, prec):
    """The m = 8,300 system (130 tile rows) with panels of 40 tiles: three
    full panels with their trailing updates and a ragged last one of 10."""
    X, y, alpha_ref = _large_system()
    print(f"large system panel=40 {prec}", flush=True)
    Xg = X.astype(np.float64) if prec == "fp64" else X
    yg = y.astype(np.float64) if prec == "fp64" else y
    Xd = _t(Xg, dev)
    C, a, _ = ctx.partition(Xd, 1, "given", centroids=_t(np.zeros((1, 4), Xg.dtype), dev))
    ctx.set_option(krr.OPT_PANEL_TILES, 40)
    try:
        models, info, st = ctx.fit(Xd, _t(yg, dev), a, C, 1,
                                   [krr.Params(sigma=0.5, lam=1e-2, prec=prec, refine_tol=1e-8, max_refine=40)])
    finally:
        ctx.set_option(krr.OPT_PANEL_TILES, 0)
    assert st == 0 and info[0]["status"] == 0
    err = ew(models[0].alpha(0).cpu().numpy(), alpha_ref)
    assert err < (1e-10 if prec == "fp64" else 1e-6), err


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_large_and_small_systems_in_one_batch(ctx, dev, prec):
    """A batch holding a system of 130 tile rows (band-by-band backward
    solve) and one of 11 (whole-system solve in LDS), two settings, with
    refinement in mixed precision: every alpha against the FP64 oracle."""
    X, y, alpha_ref = _large_system()
    g = np.random.default_rng(86)
    X2 = (g.uniform(-1.0, 1.0, size=(700, 4)) + 10.0).astype(np.float32)
    y2 = (np.cos(X2.astype(np.float64).sum(axis=1)) + 0.1 * g.standard_normal(700)).astype(np.float32)
    Xa, ya = np.concatenate([X, X2]), np.concatenate([y, y2])
    print(f"large + small systems {prec}", flush=True)
    Xg = Xa.astype(np.float64) if prec == "fp64" else Xa
    yg = ya.astype(np.float64) if prec == "fp64" else ya
    Xd = _t(Xg, dev)
    C0 = np.array([[0.0] * 4, [10.0] * 4], Xg.dtype)
    C, a, _ = ctx.partition(Xd, 2, "given", centroids=_t(C0, dev))
    assert np.array_equal(a.cpu().numpy(), np.repeat([0, 1], [8300, 700]))
    params = [krr.Params(sigma=0.5, lam=1e-2, prec=prec, refine_tol=1e-8, max_refine=40),
              krr.Params(sigma=0.8, lam=1e-2, prec=prec, refine_tol=1e-8, max_refine=40)]
    models, info, st = ctx.fit(Xd, _t(yg, dev), a, C, 2, params)
    assert st == 0 and all(i["status"] == 0 for i in info)
    tol = 1e-10 if prec == "fp64" else 1e-6
    assert ew(models[0].alpha(0).cpu().numpy(), alpha_ref) < tol
    for q, sg in enumerate((0.5, 0.8)):
        ref = O.fit_one(X2.astype(np.float64), y2.astype(np.float64), sg, 1e-2)["alpha"]
        assert ew(models[q].alpha(1).cpu().numpy(), ref) < tol, q


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_paths_at_the_threshold(ctx, dev, prec):
    """Systems of 32 tile rows (m = 2,048: whole-system backward solve) and 33
    (m = 2,049: band by band, the top band and the last tile holding one row)
    in one batch, two settings: every alpha against the FP64 oracle."""
    g = np.random.default_rng(87)
    sizes = (2048, 2049)
    Xs = [(g.uniform(-1.0, 1.0, size=(m, 4)) + 10.0 * q).astype(np.float32) for q, m in enumerate(sizes)]
    ys = [(np.sin(Xq.astype(np.float64).sum(axis=1)) + 0.1 * g.standard_normal(len(Xq))).astype(np.float32)
          for Xq in Xs]
    print(f"solve threshold m={sizes} {prec}", flush=True)
    Xa, ya = np.concatenate(Xs), np.concatenate(ys)
    Xg = Xa.astype(np.float64) if prec == "fp64" else Xa
    yg = ya.astype(np.float64) if prec == "fp64" else ya
    Xd = _t(Xg, dev)
    C0 = np.array([[0.0] * 4, [10.0] * 4], Xg.dtype)
    C, a, _ = ctx.partition(Xd, 2, "given", centroids=_t(C0, dev))
    assert np.array_equal(a.cpu().numpy(), np.repeat([0, 1], sizes))
    sigmas = (0.5, 1.0)
    params = [krr.Params(sigma=sg, lam=1e-2, prec=prec, refine_tol=1e-8, max_refine=40) for sg in sigmas]
    models, info, st = ctx.fit(Xd, _t(yg, dev), a, C, 2, params)
    assert st == 0 and all(i["status"] == 0 for i in info)
    tol = 1e-10 if prec == "fp64" else 1e-6
    for q, sg in enumerate(sigmas):
        for j in range(2):
            ref = O.fit_one(Xs[j].astype(np.float64), ys[j].astype(np.float64), sg, 1e-2)["alpha"]
            assert ew(models[q].alpha(j).cpu().numpy(), ref) < tol, (q, j)


def test_linear_kernel_is_primal_ridge(ctx, dev):
    """Linear kernel through the GPU path equals x^T (X^T X + lam I)^-1 X^T y
    (Eq. 2 with Table 1's linear kernel)."""
    g = np.random.default_rng(80)
    X = g.standard_normal((500, 7))
    y = g.standard_normal(500)
    Xt = g.standard_normal((90, 7))
    lam = 0.5
    wv = np.linalg.solve(X.T @ X + lam * np.eye(7), X.T @ y)
    Xd = _t(X, dev)
    C, a, _ = ctx.partition(Xd, 1, "given", centroids=_t(np.zeros((1, 7)), dev))
    models, info, st = ctx.fit(Xd, _t(y, dev), a, C, 1, [krr.Params(kernel="linear", lam=lam, prec="fp64")])
    assert st == 0
    yhat = ctx.predict(models[0], _t(Xt, dev)).cpu().numpy()
    np.testing.assert_allclose(yhat, Xt @ wv, rtol=1e-9, atol=1e-10)


def test_lambda_times_m(ctx, dev):
    w = datagen.small(81, 400, 4, k=20, p=2, comps=2, dtype=np.float64)
    params = [krr.Params(sigma=1.0, lam=1e-3, prec="fp64", lambda_times_m=True)]
    models, info, st, oms, X, a = _fit_both(ctx, dev, w, 2, params, method="kmeans", iters=3, seed=4)
    for j in range(2):
        assert ew(models[0].alpha(j).cpu().numpy(), oms[0].alphas[j]) < 1e-10


def test_not_spd_reports_pivot_and_keeps_others(ctx, dev):
    """A negative shift makes one setting indefinite: status ENOTSPD with
    the LAPACK-style pivot; the other setting's systems stay valid."""
    X = np.concatenate([np.arange(40)[:, None] * 100.0, np.zeros((40, 1))], axis=1)  # K = I
    y = np.linspace(-1, 1, 40)
    Xd = _t(X, dev)
    C, a, _ = ctx.partition(Xd, 1, "given", centroids=_t(np.zeros((1, 2)), dev))
    params = [krr.Params(sigma=1.0, lam=0.5, prec="fp64"), krr.Params(sigma=1.0, lam=-2.0, prec="fp64")]
    models, info, st = ctx.fit(Xd, _t(y, dev), a, C, 1, params)
    assert st == krr.KRR_ENOTSPD
    assert info[0]["status"] == 0 and info[1]["status"] == krr.KRR_ENOTSPD and info[1]["failed_pivot"] == 1
    r = O.fit_one(X, y, 1.0, -2.0)
    assert r["status"] == O.STATUS_NOT_SPD and r["pivot"] == 1
    np.testing.assert_allclose(models[0].alpha(0).cpu().numpy(), y / 1.5, rtol=1e-15)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
@pytest.mark.parametrize("dup", [(100, 101), (40, 90), (3, 150)])
def test_not_spd_pivot_inside_tiles(ctx, dev, prec, dup):
    """Far-apart points (K = I) with point dup[1] a copy of point dup[0] and a
    negative shift lam: every pivot is 1 + lam except the Schur complement of
    the copy, (1 + lam) - 1 / (1 + lam) < 0, so the first failing pivot is
    dup[1] + 1 (1-based).  The pairs put it inside a diagonal tile's third
    16-column sub-block, across two tiles, and in the last tile."""
    m = 160
    X = np.concatenate([np.arange(m)[:, None] * 100.0, np.zeros((m, 1))], axis=1)
    X[dup[1]] = X[dup[0]]
    y = np.linspace(-1, 1, m)
    r = O.fit_one(X, y, 1.0, -0.25)
    assert r["status"] == O.STATUS_NOT_SPD and r["pivot"] == dup[1] + 1
    Xg = X if prec == "fp64" else X.astype(np.float32)
    Xd = _t(Xg, dev)
    C, a, _ = ctx.partition(Xd, 1, "given", centroids=_t(np.zeros((1, 2), Xg.dtype), dev))
    models, info, st = ctx.fit(Xd, _t(y.astype(Xg.dtype), dev), a, C, 1, [krr.Params(sigma=1.0, lam=-0.25, prec=prec)])
    assert st == krr.KRR_ENOTSPD
    assert info[0]["status"] == krr.KRR_ENOTSPD and info[0]["failed_pivot"] == dup[1] + 1


def test_model_memory_reused(dev):
    """Models freed by the caller leave their memory in the context for later
    models of the same size: a repeated fit holds no more memory and gives the
    same alpha."""
    w = datagen.small(88, 1500, 6, k=40, p=3, comps=3, dtype=np.float64)
    X, y = _t(w.X, dev), _t(w.y, dev)
    params = [krr.Params(sigma=1.5, lam=1e-2, prec="fp64"), krr.Params(sigma=0.8, lam=1e-2, prec="fp64")]
    c = krr.Context(dev.index or 0)
    try:
        C, a, _ = c.partition(X, 3, "kmeans", lloyd_iters=4, seed=1)
        m1, _, st1 = c.fit(X, y, a, C, 3, params)
        a1 = [m1[q].alpha(j).cpu().numpy() for q in range(2) for j in range(3)]
        for m in m1:
            m.free()
        held = c.memory_in_use()
        m2, _, st2 = c.fit(X, y, a, C, 3, params)
        assert st1 == 0 and st2 == 0
        assert c.memory_in_use() == held
        a2 = [m2[q].alpha(j).cpu().numpy() for q in range(2) for j in range(3)]
        for u, v in zip(a1, a2):
            np.testing.assert_array_equal(u, v)
        for m in m2:
            m.free()
        assert c.memory_in_use() == held
    finally:
        c.close()


def test_empty_and_tiny_partitions(ctx, dev):
    g = np.random.default_rng(82)
    X = g.standard_normal((70, 3))
    y = g.standard_normal(70)
    C = np.array([[0.0, 0.0, 0.0], [1e6, 1e6, 1e6], [X[5, 0], X[5, 1], X[5, 2]]])
    X[5] += 1e3      # point 5 alone near nothing; partition 1 stays empty
    C[2] = X[5]
    w = datagen.Workload("edge", X, y, None, None, X[:9], y[:9], 3, (1.0,), (1e-2,), {})
    params = [krr.Params(sigma=1.0, lam=1e-2, prec="fp64")]
    models, info, st, oms, Xd, a = _fit_both(ctx, dev, w, 3, params, centroids=C)
    assert st == 0
    assert [info[j]["m"] for j in range(3)] == [69, 0, 1]
    for j in (0, 2):
        assert ew(models[0].alpha(j).cpu().numpy(), oms[0].alphas[j]) < 1e-10
    for route in ("nearest", "average"):
        yhat = ctx.predict(models[0], _t(w.Xt, dev), route=route).cpu().numpy()
        yo, _ = O.predict(oms[0], w.Xt, route)
        assert pred_ew(yhat, yo, w.yt) < 1e-10


def test_fit_rejects_bad_arguments(ctx, dev):
    X = torch.zeros((10, 3), dtype=torch.float64, device=dev)
    a = torch.zeros(10, dtype=torch.int32, device=dev)
    C = torch.zeros((1, 3), dtype=torch.float64, device=dev)
    with pytest.raises(krr.KrrError) as e:
        ctx.fit(X, X[:, 0].contiguous(), a, C, 1, [krr.Params(sigma=-1.0)])
    assert e.value.status == krr.KRR_EINVAL
    with pytest.raises(krr.KrrError) as e:
        ctx.fit(X, X[:, 0].contiguous(), a, C, 1, [krr.Params(lam=math.nan)])
    assert e.value.status == krr.KRR_EINVAL


def test_fit_budget_failure_on_a_later_model_leaks_nothing(dev):
    """A budget that holds the workspace, the partition data and the first
    model but not the second: krr_fit returns KRR_EBUDGET, hands out no model
    handle, and the context can still be destroyed (no model or partition
    data left alive on it)."""
    import ctypes
    w = datagen.small(91, 1500, 6, k=10, p=3, comps=3, dtype=np.float64)
    X, y = _t(w.X, dev), _t(w.y, dev)
    params = [krr.Params(sigma=1.0, lam=1e-2, prec="fp64"), krr.Params(sigma=2.0, lam=1e-2, prec="fp64")]
    part = krr.Context(0)
    C, a, _ = part.partition(X, 3, "kmeans", lloyd_iters=5, seed=3)
    torch.cuda.synchronize()
    part.close()
    probe = krr.Context(0)                   # holds exactly what the fit needs
    models, _, st = probe.fit(X, y, a, C, 3, params)
    assert st == 0
    total = probe.memory_in_use()            # workspace + data + both models
    for m in models:
        m.free()
    probe.close()
    print(f"budget failure: total {total} bytes", flush=True)
    lim = krr.Context(0, hbm_budget=total - 1)
    handles = (ctypes.c_void_p * 2)(ctypes.c_void_p(1), ctypes.c_void_p(1))
    info = (krr.PartInfo * 6)()
    arr = (krr.FitParams * 2)(*[q.to_c() for q in params])
    st = lim.lib.krr_fit(lim.h, krr._stream(dev), krr._ptr(X), krr._ptr(y), krr.F64, 1500, 6, krr._ptr(a),
                         krr._ptr(C), 3, arr, 2, handles, info)
    assert st == krr.KRR_EBUDGET, lim.lib.krr_last_error(lim.h)
    assert handles[0] is None and handles[1] is None
    assert lim.lib.krr_destroy(lim.h) == krr.KRR_OK
    lim.h = None
