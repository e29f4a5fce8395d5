"""Parity of the partition kernels with the oracle: assignment indices, the
Lloyd centres (the exactly rounded member sums divided by the count on both
sides) and the K-balance memberships must be identical bit for bit on the same seeded
inputs.  The k-means++ picks are compared too; the GPU forms the cumulative
D^2 weights in a different (blocked) order, so each test also checks that
every pick of the oracle is further from a rounding tie than the bound of
the two orders (``kpp_ambiguous`` in tests/_parity.py): there the picks must
agree, and equal picks make every later step bit-exact."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1805_00569_amd import datagen
from _parity import kpp_ambiguous

pytestmark = pytest.mark.gpu


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("n,d,p,dtype", [(131072, 90, 32, np.float32), (2048, 16, 1, np.float64),
                                         (1000, 7, 5, np.float64), (257, 90, 64, np.float32),
                                         (300, 600, 9, np.float64), (5, 3, 5, np.float32)])
def test_assign_given_bitexact(ctx, dev, n, d, p, dtype):
    print(f"assign n={n} d={d} p={p} {dtype.__name__}", flush=True)
    g = np.random.default_rng(n + d + p)
    X = (g.standard_normal((n, d)) * g.uniform(0.5, 2, d)).astype(dtype)
    C = g.standard_normal((p, d))
    if p >= 3:
        C[p - 1] = C[1]                      # planted duplicate centre
        C[0] = X[min(3, n - 1)].astype(np.float64)   # a point sitting on a centre
    Cg, a, sz = ctx.partition(_t(X, dev), p, "given", centroids=_t(C, dev))
    ao, _ = O.assign(X, C)
    np.testing.assert_array_equal(a.cpu().numpy(), ao)
    np.testing.assert_array_equal(sz.cpu().numpy(), np.bincount(ao, minlength=p))
    np.testing.assert_array_equal(Cg.cpu().numpy(), C)


def test_kmeans_seeding_and_lloyd_bitexact(ctx, dev):
    w = datagen.gaussian_mixture(seed=31, n=8192, d=90, comps=16, lo=128, hi=2000)
    for iters in (0, 1, 7):
        print(f"kmeans iters={iters}", flush=True)
        C, a, sz = ctx.partition(_t(w.X, dev), 16, "kmeans", lloyd_iters=iters, seed=123)
        tr = []
        C0, idx = O.kmeanspp(w.X, 16, 123, tr)
        assert kpp_ambiguous(tr, w.X.shape[0]) == 0
        Co, ao, _, _ = O.lloyd(w.X, C0, iters)
        np.testing.assert_array_equal(C.cpu().numpy(), Co)
        np.testing.assert_array_equal(a.cpu().numpy(), ao)
        np.testing.assert_array_equal(sz.cpu().numpy(), np.bincount(ao, minlength=16))


@pytest.mark.parametrize("n,d,p,dtype", [(20000, 90, 3, np.float32), (9000, 130, 2, np.float64),
                                         (3001, 7, 5, np.float64), (2000, 400, 3, np.float32)])
def test_lloyd_means_long_sums(ctx, dev, n, d, p, dtype):
    """Clusters of hundreds to thousands of members (many row splits of the
    mean step; in FP64 several limb normalisations per thread) and more than
    64 features (several feature slices): the Lloyd centres equal the
    oracle's exactly rounded means bit for bit.  The 400-feature rows are too
    wide for the staged assignment and take its unstaged kernel."""
    print(f"lloyd means n={n} d={d} p={p} {dtype.__name__}", flush=True)
    g = np.random.default_rng(n + d)
    X = (g.standard_normal((n, d)) * g.uniform(0.5, 2, d) + 3.0 * g.standard_normal((1, d))).astype(dtype)
    C, a, sz = ctx.partition(_t(X, dev), p, "kmeans", lloyd_iters=4, seed=n)
    tr = []
    C0, _ = O.kmeanspp(X, p, n, tr)
    assert kpp_ambiguous(tr, n) == 0
    Co, ao, _, _ = O.lloyd(X, C0, 4)
    np.testing.assert_array_equal(a.cpu().numpy(), ao)
    np.testing.assert_array_equal(C.cpu().numpy(), Co)
    assert sz.cpu().numpy().max() > 256   # clusters of hundreds of members


def test_kbalance_bitexact(ctx, dev):
    w = datagen.balanced(seed=32, n=8192, k_test=16, p=16)
    print("kbalance n=8192 p=16", flush=True)
    C, a, sz = ctx.partition(_t(w.X, dev), 16, "kbalance", lloyd_iters=5, seed=7)
    tr = []
    Co, ao = O.kbalance(w.X, 16, 5, 7, tr)
    assert kpp_ambiguous(tr, w.X.shape[0]) == 0
    np.testing.assert_array_equal(a.cpu().numpy(), ao)
    np.testing.assert_array_equal(C.cpu().numpy(), Co)
    assert sz.cpu().numpy().tolist() == [512] * 16


def test_kbalance_ragged_capacity(ctx, dev):
    w = datagen.small(33, 1003, 5, comps=3, dtype=np.float64)
    C, a, sz = ctx.partition(_t(w.X, dev), 7, "kbalance", lloyd_iters=4, seed=3)
    Co, ao = O.kbalance(w.X, 7, 4, 3)
    np.testing.assert_array_equal(a.cpu().numpy(), ao)
    np.testing.assert_array_equal(C.cpu().numpy(), Co)
    assert sz.cpu().numpy().max() <= 144


@pytest.mark.parametrize("p", [1, 2, 13, 16, 17])
def test_kbalance_many_blocks_with_ties(ctx, dev, p):
    """K-balance (Algorithm 4) over ~80 blocks of 256 points, several centres
    filling inside one group of 16 blocks, on integer-grid points where equal
    distances are common (the lowest centre index wins); p <= 16 and p > 16
    take different event kernels."""
    g = np.random.default_rng(40 + p)
    n = 20011
    X = g.integers(0, 4, size=(n, 3)).astype(np.float64)
    X[: n // 3] += 10.0 * g.integers(0, 3, size=(n // 3, 1))   # uneven clusters: centres fill at different times
    print(f"kbalance n={n} p={p} (ties)", flush=True)
    C, a, sz = ctx.partition(_t(X, dev), p, "kbalance", lloyd_iters=3, seed=5)
    Co, ao = O.kbalance(X, p, 3, 5)
    np.testing.assert_array_equal(a.cpu().numpy(), ao)
    np.testing.assert_array_equal(C.cpu().numpy(), Co)
    assert sz.cpu().numpy().max() <= -(-n // p)


@pytest.mark.parametrize("case", ["balanced", "ties", "ragged", "one_point_segments"])
def test_kbalance_approx_bitexact(ctx, dev, case):
    """Approximate parallel K-balance (Section 4.3): p even segments of the
    samples, each with its own greedy pass at capacity ceil(n_q / p), then
    the member-mean centres, bit for bit.  Cases: p^2 | n (every partition
    exactly n / p), integer-grid ties, a ragged split, and p = n (one sample
    per segment)."""
    if case == "balanced":
        w = datagen.balanced(seed=34, n=8192, k_test=16, p=16)
        X, p, iters = w.X, 16, 5
    elif case == "ties":
        g = np.random.default_rng(41)
        X = g.integers(0, 4, size=(20011, 3)).astype(np.float64)
        X[: 20011 // 3] += 10.0 * g.integers(0, 3, size=(20011 // 3, 1))
        p, iters = 13, 3
    elif case == "ragged":
        X, p, iters = datagen.small(35, 1003, 5, comps=3, dtype=np.float64).X, 7, 4
    else:
        X = np.random.default_rng(42).standard_normal((300, 4)).astype(np.float32)
        p, iters = 300, 2
    n = X.shape[0]
    print(f"kbalance_approx {case} n={n} p={p}", flush=True)
    C, a, sz = ctx.partition(_t(X, dev), p, "kbalance_approx", lloyd_iters=iters, seed=11)
    Co, ao = O.kbalance_approx(X, p, iters, 11)
    np.testing.assert_array_equal(a.cpu().numpy(), ao)
    np.testing.assert_array_equal(C.cpu().numpy(), Co)
    sizes = sz.cpu().numpy()
    np.testing.assert_array_equal(sizes, np.bincount(ao, minlength=p))
    if n % (p * p) == 0:
        assert sizes.tolist() == [n // p] * p
    assert sizes.max() <= p * -(-(-(-n // p)) // p)


@pytest.mark.parametrize("n,d,p,seed,dtype", [(20011, 90, 16, 5, np.float32), (4096, 8, 7, 1, np.float64),
                                              (65536, 4, 64, 9, np.float32), (5, 3, 5, 2, np.float64),
                                              (37, 2, 1, 3, np.float32)])
def test_random_partition_bitexact(ctx, dev, n, d, p, seed, dtype):
    """DC-KRR divide step (Algorithm 3): the shuffled even split and its
    member-mean centres, bit for bit; sizes differ by at most one (n = 65536
    needs no cycle-walking, 20011 does)."""
    print(f"random partition n={n} d={d} p={p} seed={seed}", flush=True)
    g = np.random.default_rng(n + p)
    X = (g.standard_normal((n, d)) * g.uniform(0.5, 2, d)).astype(dtype)
    C, a, sz = ctx.partition(_t(X, dev), p, "random", seed=seed)
    Co, ao = O.random_partition(X, p, seed)
    np.testing.assert_array_equal(a.cpu().numpy(), ao)
    np.testing.assert_array_equal(sz.cpu().numpy(), np.bincount(ao, minlength=p))
    np.testing.assert_array_equal(C.cpu().numpy(), Co)
    assert sz.max().item() - sz.min().item() <= 1


def test_kmeans_converges_early(ctx, dev):
    # well separated clusters: Lloyd reaches a fixed point before the cap
    w = datagen.small(34, 2000, 4, comps=4, spread=50.0)
    C, a, _ = ctx.partition(_t(w.X, dev), 4, "kmeans", lloyd_iters=50, seed=1)
    tr = []
    C0, _ = O.kmeanspp(w.X, 4, 1, tr)
    assert kpp_ambiguous(tr, w.X.shape[0]) == 0
    Co, ao, passes, deltas = O.lloyd(w.X, C0, 50)
    assert passes < 50
    np.testing.assert_array_equal(C.cpu().numpy(), Co)
    np.testing.assert_array_equal(a.cpu().numpy(), ao)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_kmeans_with_empty_clusters(ctx, dev, dtype):
    """Three distinct rows, each repeated, and p = 5: after three k-means++
    picks every D^2 weight is zero, so the last picks duplicate earlier
    centres (total 0: the point at floor(u n)), ties send every point to the
    lowest-index duplicate, and the other duplicates stay empty and keep their
    centres through the Lloyd passes; all of it bit for bit."""
    print(f"kmeans empty clusters {dtype.__name__}", flush=True)
    rows = np.array([[0.0, 1.0, 2.0], [5.0, -1.0, 0.5], [-3.0, 4.0, 1.5]])
    X = np.repeat(rows, [120, 90, 90], axis=0).astype(dtype)
    X = X[np.random.default_rng(8).permutation(X.shape[0])]
    C, a, sz = ctx.partition(_t(X, dev), 5, "kmeans", lloyd_iters=6, seed=4)
    C0, _ = O.kmeanspp(X, 5, 4)
    Co, ao, _, _ = O.lloyd(X, C0, 6)
    np.testing.assert_array_equal(a.cpu().numpy(), ao)
    np.testing.assert_array_equal(C.cpu().numpy(), Co)
    szo = np.bincount(ao, minlength=5)
    np.testing.assert_array_equal(sz.cpu().numpy(), szo)
    assert (szo == 0).sum() == 2


def test_partition_rejects_bad_arguments(ctx, dev):
    from paper_1805_00569_amd import krr
    X = torch.zeros((10, 3), dtype=torch.float32, device=dev)
    with pytest.raises(krr.KrrError) as e:
        ctx.partition(X, 11, "kmeans")
    assert e.value.status == krr.KRR_EINVAL


@pytest.mark.parametrize("n,d,p,dtype", [(6000, 20, 3, np.float32), (6000, 20, 3, np.float64),
                                         (140000, 5, 1, np.float32)])
def test_means_exact_over_the_whole_range(ctx, dev, n, d, p, dtype):
    """Member means of the random even split (no distances, so any finite
    values may be used): magnitudes over most of the format's exponent range,
    subnormals, large values that cancel, exact zeros and a column of tiny
    values; the centres equal the oracle's exactly rounded means bit for bit.
    Rows 0..9 hold planted extremes.  The single partition of 140,000 rows
    gives each thread of the mean step more than 128 terms (limbs normalised
    inside the loop, not only at its end)."""
    print(f"means whole range n={n} d={d} p={p} {dtype.__name__}", flush=True)
    g = np.random.default_rng(77)
    lo, hi = (-140, 100) if dtype == np.float32 else (-1060, 1000)
    e = g.integers(lo, hi, (n, d)).astype(float)
    X = (g.standard_normal((n, d)) * np.exp2(e)).astype(dtype)
    big = np.finfo(dtype).max / 8
    X[0:4, 0] = [big, -big, big, -big]               # cancel exactly
    X[4:8, 1] = np.finfo(dtype).smallest_subnormal   # subnormal terms
    X[8:10, :] = 0.0
    X[:, 2] = np.finfo(dtype).smallest_subnormal * g.integers(-5, 6, n)   # a column of tiny values
    C, a, sz = ctx.partition(_t(X, dev), p, "random", seed=5)
    Co, ao = O.random_partition(X, p, 5)
    np.testing.assert_array_equal(a.cpu().numpy(), ao)
    Cg = C.cpu().numpy()
    np.testing.assert_array_equal(Cg, Co)
    assert np.array_equal(np.signbit(Cg), np.signbit(Co))   # same sign of zero too
