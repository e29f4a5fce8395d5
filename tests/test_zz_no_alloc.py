"""krr_predict_noalloc: the prediction entry point that allocates no device
memory (its temporaries live in a fixed per-GPU scratch array).  Checked
through the C ABI against krr_predict on the same model and inputs -- the
same kernels with the same launch shapes, so the values must agree bit for
bit -- and against the FP64 oracle at the FP64 tolerance (1e-10), on two
calls in a row, the second with fewer points, for every route."""
import gc

import numpy as np
import pytest
import torch

import oracle as O
from paper_1805_00569_amd import datagen, krr
from _parity import pred_ew

pytestmark = pytest.mark.gpu


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.fixture(scope="module")
def fitted():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    ctx = krr.Context(0)
    n, d, p = 3000, 12, 5
    w = datagen.small(77, n, d, k=900, p=p, comps=p, dtype=np.float64)
    X, y = _t(w.X, dev), _t(w.y, dev)
    C, a, _ = ctx.partition(X, p, "kmeans", lloyd_iters=8, seed=5)
    models, info, st = ctx.fit(X, y, a, C, p, [krr.Params(sigma=1.5, lam=1e-2, prec="fp64")])
    assert st == 0
    om = O.fit(w.X, w.y, a.cpu().numpy(), C.cpu().numpy(), p, 1.5, 1e-2)
    yield ctx, dev, w, models[0], om, p
    models[0].free()
    ctx.close()


@pytest.mark.parametrize("route", ["nearest", "all", "average"])
def test_noalloc_equals_predict_on_two_calls(fitted, route):
    ctx, dev, w, model, om, p = fitted
    print(f"noalloc predict route={route}", flush=True)
    for k in (900, 131):   # second call smaller: stale scratch contents from the first must not matter
        Xt = _t(w.Xt[:k], dev)
        shape = (k, p) if route == "all" else (k,)
        out = torch.full(shape, float("nan"), dtype=torch.float64, device=dev)
        rout = torch.full((k,), -7, dtype=torch.int32, device=dev)
        # no collection inside the measured call: freeing an unreachable tensor
        # left by earlier tests would move torch's count without any allocation
        gc.collect()
        gc.disable()
        try:
            torch.cuda.synchronize()
            mem0, alloc0 = ctx.memory_in_use(), torch.cuda.memory_allocated(dev)
            ctx.predict_noalloc(model, Xt, out, route=route, route_out=rout)
            torch.cuda.synchronize()
            mem1, alloc1 = ctx.memory_in_use(), torch.cuda.memory_allocated(dev)
        finally:
            gc.enable()
        assert mem1 == mem0 and alloc1 == alloc0
        ref, rref = ctx.predict(model, Xt, route=route, want_route=True)
        got = out.cpu().numpy()
        assert np.array_equal(got, ref.cpu().numpy()), (route, k)
        assert np.array_equal(rout.cpu().numpy(), rref.cpu().numpy()), (route, k)
        yo, _ = O.predict(om, w.Xt[:k], route)
        ro, _ = O.assign(w.Xt[:k], om.centroids)
        assert np.array_equal(rout.cpu().numpy(), ro)
        assert pred_ew(got.ravel(), yo.ravel(), np.repeat(w.yt[:k], p if route == "all" else 1)) < 1e-10


def test_noalloc_rejects_oversized_call_before_any_work(fitted):
    ctx, dev, w, model, om, p = fitted
    k = 300_000   # ALL needs k * p * 8 bytes of partial sums: far above the fixed scratch
    print(f"noalloc oversize k={k} p={p}", flush=True)
    Xt = torch.zeros((k, w.X.shape[1]), dtype=torch.float64, device=dev)
    out = torch.full((k, p), float("nan"), dtype=torch.float64, device=dev)
    with pytest.raises(krr.KrrError) as e:
        ctx.predict_noalloc(model, Xt, out, route="all")
    assert e.value.status == krr.KRR_EINVAL and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.isnan(out).all()
    # the next call still works
    k2 = 64
    out2 = torch.empty(k2, dtype=torch.float64, device=dev)
    ctx.predict_noalloc(model, _t(w.Xt[:k2], dev), out2)
    ref = ctx.predict(model, _t(w.Xt[:k2], dev))
    assert torch.equal(out2, ref)
