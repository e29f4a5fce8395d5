"""CSR input (Sections 5.5 and 6): the device expansion to the dense matrix
is identical, bit for bit, to the oracle's; a malformed structure is an
error; a fit on the expanded sparse input matches the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1805_00569_amd import krr

pytestmark = pytest.mark.gpu


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _random_csr(g, n, d, density, dtype, repeats=True):
    counts = g.binomial(d, density, n)
    counts[:: 7] = 0                                    # empty rows
    indptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    nnz = int(indptr[-1])
    indices = np.empty(nnz, np.int32)
    for i in range(n):
        row = g.choice(d, counts[i], replace=False)
        if repeats and counts[i] > 2:
            row[-1] = row[0]                             # a repeated column, summed in storage order
        indices[indptr[i]:indptr[i + 1]] = row           # unsorted
    values = g.standard_normal(nnz).astype(dtype)
    return indptr, indices, values


@pytest.mark.parametrize("n,d,density,dtype", [(5000, 90, 0.3, np.float32), (5000, 90, 0.3, np.float64),
                                               (257, 600, 0.02, np.float32), (1, 3, 1.0, np.float64)])
def test_csr_expansion_bitexact(ctx, dev, n, d, density, dtype):
    print(f"csr n={n} d={d} density={density} {dtype.__name__}", flush=True)
    g = np.random.default_rng(n + d)
    indptr, indices, values = _random_csr(g, n, d, density, dtype)
    X = ctx.csr_to_dense(_t(indptr, dev), _t(indices, dev), _t(values, dev), d).cpu().numpy()
    Xo = O.csr_to_dense(indptr, indices, values, n, d)
    assert X.dtype == Xo.dtype
    np.testing.assert_array_equal(X, Xo)


def test_csr_no_entries(ctx, dev):
    """nnz = 0: the all-zero matrix (no index or value buffers)."""
    print("csr nnz=0", flush=True)
    X = ctx.csr_to_dense(_t(np.zeros(6, np.int64), dev), torch.empty(0, dtype=torch.int32, device=dev),
                         torch.empty(0, dtype=torch.float32, device=dev), 9)
    assert X.shape == (5, 9) and not X.any()


@pytest.mark.parametrize("indptr,indices", [([0, 2, 1], [0, 1]), ([1, 1, 2], [0, 1]), ([0, 1, 2], [0, 4]),
                                            ([0, 1, 1], [0, 1]), ([0, 1, 2], [-1, 0])])
def test_csr_malformed_is_an_error(ctx, dev, indptr, indices):
    """Structures the oracle rejects: decreasing or offset row pointers, a
    last pointer short of nnz, a column outside [0, d).  The kernel checks
    every pointer and index before use, so nothing is read or written out of
    bounds; the call returns KRR_EINVAL."""
    print(f"csr malformed {indptr} {indices}", flush=True)
    with pytest.raises(ValueError):
        O.csr_to_dense(indptr, indices, np.ones(len(indices)), 2, 4)
    with pytest.raises(krr.KrrError) as e:
        ctx.csr_to_dense(_t(np.array(indptr, np.int64), dev), _t(np.array(indices, np.int32), dev),
                         _t(np.ones(len(indices)), dev), 4)
    assert e.value.status == krr.KRR_EINVAL


def test_fit_on_sparse_input_matches_oracle(ctx, dev):
    """Sparse FP64 input (15% of 40 features nonzero) through CSR, p = 3
    K-means partitions, one setting: alpha and predictions against the FP64
    oracle on the same dense matrix."""
    g = np.random.default_rng(61)
    n, d = 1500, 40
    indptr, indices, values = _random_csr(g, n, d, 0.15, np.float64, repeats=False)
    Xo = O.csr_to_dense(indptr, indices, values, n, d)
    y = np.sin(Xo[:, :5].sum(axis=1)) + 0.05 * g.standard_normal(n)
    tp, ti, tv = _random_csr(g, 200, d, 0.15, np.float64, repeats=False)
    print("csr fit n=1500 d=40 p=3", flush=True)
    X = ctx.csr_to_dense(_t(indptr, dev), _t(indices, dev), _t(values, dev), d)
    Xt = ctx.csr_to_dense(_t(tp, dev), _t(ti, dev), _t(tv, dev), d)
    C, a, _ = ctx.partition(X, 3, "kmeans", lloyd_iters=5, seed=4)
    params = [krr.Params(sigma=2.0, lam=1e-2, prec="fp64")]
    models, info, st = ctx.fit(X, _t(y, dev), a, C, 3, params)
    assert st == 0
    om = O.fit(Xo, y, a.cpu().numpy(), C.cpu().numpy(), 3, 2.0, 1e-2, "gaussian", False)
    for j in range(3):
        ref = om.alphas[j]
        got = models[0].alpha(j).cpu().numpy()
        assert np.linalg.norm(got - ref) <= 1e-10 * max(np.linalg.norm(ref), 1e-300), j
    yhat = ctx.predict(models[0], Xt).cpu().numpy()
    yref, _ = O.predict(om, O.csr_to_dense(tp, ti, tv, 200, d))
    assert np.linalg.norm(yhat - yref) <= 1e-10 * max(np.linalg.norm(yref), 1e-300)
