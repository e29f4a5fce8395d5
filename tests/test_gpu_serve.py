"""Serving runtime (continuous batching) on the GPU.

A resident BKRR2 model (K-balance partitions, nearest-centre route,
Algorithm 5) answers predict requests; fit requests are independent
problems (Eq. 6).  Checks: every result is the same alone and in a mix of
concurrent requests (1e-12 relative, element by element; only the
summation split of a prediction may differ), predictions and fits agree with the direct library
calls and with the FP64 oracle (the resident model in mixed precision,
refined: predictions element by element within 1e-6; fit requests in FP32
at the FP32 path's bound), the admission budget is respected, and bad
requests are rejected before queueing."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1805_00569_amd import datagen, krr
from _parity import ew, pred_ew

pytestmark = pytest.mark.gpu

SIGMA, LAM = 2.0, 1e-2


@pytest.fixture(scope="module")
def resident(ctx, dev):
    pools = datagen.serving_pools(seed=7, n=8192, d=16, comps=8, n_queries=2048, fit_ds=(4, 16), fit_rows=900,
                                  fit_comps=4)
    w = pools.resident
    X = torch.from_numpy(w.X).to(dev)
    y = torch.from_numpy(w.y.astype(np.float32)).to(dev)
    C, a, _ = ctx.partition(X, 8, "kbalance", lloyd_iters=10, seed=3)
    models, info, st = ctx.fit(X, y, a, C, 8, [krr.Params(sigma=SIGMA, lam=LAM, prec="mixed", refine_tol=1e-10,
                                                          max_refine=30)])
    assert st == 0
    yield pools, models[0], X, a.cpu().numpy(), C.cpu().numpy()
    models[0].free()


def _fit_params():
    return krr.Params(sigma=SIGMA, lam=LAM, prec="fp32")


def test_serve_alone_equals_mix(ctx, dev, resident):
    pools, model, X, a_np, C_np = resident
    print("serve: alone vs mix", flush=True)
    srv = krr.Server(ctx, model, predict_workers=2, fit_workers=2, max_batch_fits=8, max_batch_points=4096)
    try:
        q_alone = datagen.take_rows(pools.queries, 100, 300)
        f_X = datagen.take_rows(pools.fit_X[4], 50, 333)
        f_y = datagen.take_rows(pools.fit_y[4][:, None], 50, 333)[:, 0]
        y_alone, info = srv.wait(srv.submit_predict(q_alone))
        assert info["status"] == 0 and info["batch_requests"] == 1
        al_alone, info = srv.wait(srv.submit_fit(f_X, f_y, _fit_params()))
        assert info["status"] == 0

        # direct library calls give the same numbers
        y_direct = ctx.predict(model, torch.from_numpy(q_alone).to(dev)).cpu().numpy()
        assert ew(y_alone, y_direct) < 1e-12

        # a burst of mixed requests with the two probes in the middle
        g = np.random.default_rng(11)
        tickets, probes = [], {}
        for i in range(60):
            if i == 25:
                probes["p"] = srv.submit_predict(q_alone)
            if i == 31:
                probes["f"] = srv.submit_fit(f_X, f_y, _fit_params())
            if g.random() < 0.25:
                fd = int(g.choice([4, 16]))
                m = int(g.integers(64, 800))
                off = int(g.integers(0, 900))
                fy = datagen.take_rows(pools.fit_y[fd][:, None], off, m)[:, 0]
                tickets.append(("fit", srv.submit_fit(datagen.take_rows(pools.fit_X[fd], off, m), fy, _fit_params()),
                                fd, off, m))
            else:
                k = int(g.integers(1, 700))
                off = int(g.integers(0, 2048))
                tickets.append(("predict", srv.submit_predict(datagen.take_rows(pools.queries, off, k)), k, off))
        y_mix, info_p = srv.wait(probes["p"])
        al_mix, info_f = srv.wait(probes["f"])
        assert info_p["status"] == 0 and info_f["status"] == 0
        assert ew(y_mix, y_alone) < 1e-12
        assert ew(al_mix, al_alone) < 1e-12
        batched = 0
        for t in tickets:
            out, inf = srv.wait(t[1])
            assert inf["status"] == 0
            batched = max(batched, inf["batch_requests"])
            if t[0] == "predict":
                ref = ctx.predict(model, torch.from_numpy(datagen.take_rows(pools.queries, t[3], t[2])).to(dev))
                assert ew(out, ref.cpu().numpy()) < 1e-12
        assert batched > 1, "no request was batched with another"
        s = srv.stats()
        assert s["predict_requests"] + s["fit_requests"] == 2 + 2 + len(tickets)
        assert s["failed"] == 0 and s["predict_p99_ms"] >= s["predict_p50_ms"] > 0
    finally:
        srv.close()

    # the fit result against the FP64 oracle (FP32 path: kappa-scaled bound)
    Xf = f_X.astype(np.float64)
    om = O.fit(Xf, f_y.astype(np.float64), np.zeros(333, np.int32), np.zeros((1, 4)), 1, SIGMA, LAM,
               "gaussian", False)
    kappa = np.linalg.cond(O.kernel_matrix(Xf, Xf, SIGMA) + LAM * np.eye(333))
    err = ew(al_alone, om.alphas[0])
    assert err < 20 * kappa * 333 * 6e-8, (err, kappa)


def test_serve_predictions_match_oracle(ctx, dev, resident):
    pools, model, X, a_np, C_np = resident
    print("serve: predictions vs oracle", flush=True)
    w = pools.resident
    om = O.fit(w.X.astype(np.float64), w.y.astype(np.float32).astype(np.float64), a_np, C_np, 8, SIGMA, LAM,
               "gaussian", False)
    srv = krr.Server(ctx, model, predict_workers=1, fit_workers=0)
    try:
        q = datagen.take_rows(pools.queries, 0, 257)
        yhat, info = srv.wait(srv.submit_predict(q))
        yo, _ = O.predict(om, q.astype(np.float64))
        # element by element, relative to max(|y_ref|_inf, 1e-3 |y|_inf)
        assert pred_ew(yhat, yo, w.y) < 1e-6
        with pytest.raises(krr.KrrError) as e:
            srv.submit_fit(q, q[:, 0], _fit_params())
        assert e.value.status == krr.KRR_ESTATE
    finally:
        srv.close()


def test_serve_admission_budget(ctx, dev, resident):
    pools, model, *_ = resident
    print("serve: admission budget", flush=True)
    # 24 MiB: two predict workers hold at most 2 x 2.9 MB (batches of 2,048
    # points, d = 16); each fit worker gets ~9.7 MB, i.e. three fit requests
    # of m <= 740 at a time
    budget = 24 << 20
    srv = krr.Server(ctx, model, predict_workers=2, fit_workers=2, max_batch_fits=4, max_batch_points=2048,
                     hbm_budget=budget)
    try:
        ts = []
        for i in range(12):
            m = 300 + 40 * i
            ts.append(srv.submit_fit(datagen.take_rows(pools.fit_X[16], 7 * i, m),
                                     datagen.take_rows(pools.fit_y[16][:, None], 7 * i, m)[:, 0], _fit_params()))
            ts.append(srv.submit_predict(datagen.take_rows(pools.queries, 13 * i, 1000)))
        for t in ts:
            _, inf = srv.wait(t)
            assert inf["status"] == 0
        s = srv.stats()
        assert 0 < s["max_inflight_bytes"] <= budget
        # device memory actually held by the workers' contexts together
        assert 0 < s["max_device_bytes"] <= budget
        with pytest.raises(krr.KrrError) as e:
            srv.submit_fit(datagen.take_rows(pools.fit_X[16], 0, 2000),   # alone above a fit worker's share
                           datagen.take_rows(pools.fit_y[16][:, None], 0, 2000)[:, 0], _fit_params())
        assert e.value.status == krr.KRR_EBUDGET
        with pytest.raises(krr.KrrError) as e:
            srv.submit_predict(np.zeros((0, 16), np.float32))
        assert e.value.status == krr.KRR_EINVAL
        with pytest.raises(krr.KrrError) as e:
            srv.submit_predict(np.zeros((4096, 16), np.float32))   # above max_batch_points
        assert e.value.status == krr.KRR_EINVAL
    finally:
        srv.close()
    with pytest.raises(krr.KrrError) as e:   # a budget the predict workers alone would fill
        krr.Server(ctx, model, predict_workers=2, fit_workers=1, max_batch_points=2048, hbm_budget=4 << 20)
    assert e.value.status == krr.KRR_EINVAL
