"""Seeded synthetic workloads shaped like the paper's experiments.

This module only draws input arrays.  It holds none of the method's
arithmetic (no distances, no kernels, no solves), so both the CPU oracle and
the GPU path can be fed from it without sharing any computation.

Every array comes from ``numpy.random.default_rng(SeedSequence([seed, stream]))``
with a fixed stream number per role, so a test can regenerate any single
array without drawing the others:

    stream 0  training inputs          stream 3  label function parameters
    stream 1  validation inputs        stream 4  label noise
    stream 2  test inputs              stream 5  mixture / feature-scale parameters

The paper's datasets (MSD, d=90; cadata, d=8; Table 2 of Section 5.1) are not
available, so the shapes below stand in for them: d=90 and a few thousand
points per partition, as in the weak-scaling runs of Section 5.3.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

S_XTRAIN, S_XVAL, S_XTEST, S_LABEL, S_NOISE, S_MIX = 0, 1, 2, 3, 4, 5


def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(stream)]))


@dataclasses.dataclass
class Workload:
    name: str
    X: np.ndarray            # n x d, row-major
    y: np.ndarray            # n
    Xv: np.ndarray | None    # validation inputs (model selection)
    yv: np.ndarray | None
    Xt: np.ndarray           # test inputs
    yt: np.ndarray
    p: int                   # number of partitions
    sigmas: tuple
    lambdas: tuple
    meta: dict

    @property
    def n(self):
        return self.X.shape[0]

    @property
    def d(self):
        return self.X.shape[1]


# ---------------------------------------------------------------------------
# label functions (drawn parameters only; evaluated here because the labels
# are part of the input, not of the method)
# ---------------------------------------------------------------------------

def _sin3_labels(X, seed, stream_noise, noise=0.1):
    # y = sin(x0 + x1 + x2) + noise * N(0, 1)
    base = np.sin(X[:, 0].astype(np.float64) + X[:, 1] + X[:, 2])
    return base + noise * rng(seed, stream_noise).standard_normal(X.shape[0])


@dataclasses.dataclass
class TanhNet:
    W1: np.ndarray
    b1: np.ndarray
    w2: np.ndarray

    @staticmethod
    def draw(seed, d, hidden=64):
        g = rng(seed, S_LABEL)
        W1 = g.standard_normal((hidden, d)) / math.sqrt(d)
        b1 = g.standard_normal(hidden)
        w2 = g.standard_normal(hidden) / math.sqrt(hidden)
        return TanhNet(W1, b1, w2)

    def __call__(self, X):
        return np.tanh(X.astype(np.float64) @ self.W1.T + self.b1) @ self.w2


def _noise(seed, stream_offset, k, scale):
    return scale * rng(seed, S_NOISE * 1000 + stream_offset).standard_normal(k)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def plain_krr(seed=1, n=2048, k=512, d=16):
    """Single partition (p=1), FP64: x ~ N(0, I), y = sin(x0+x1+x2) + 0.1 N(0,1)."""
    X = rng(seed, S_XTRAIN).standard_normal((n, d))
    Xt = rng(seed, S_XTEST).standard_normal((k, d))
    y = _sin3_labels(X, seed, S_NOISE)
    yt = np.sin(Xt[:, 0] + Xt[:, 1] + Xt[:, 2]) + 0.1 * rng(seed, S_NOISE + 100).standard_normal(k)
    return Workload("plain_krr_fp64_n2048_d16", X, y, None, None, Xt, yt, 1,
                    (1.0,), (1e-3,), {"dtype": "f64"})


def balanced(seed=2, n=65536, k_test=8192, d=90, p=16, val_frac=0.1,
             sigmas=(0.5, 1.0, 2.0), lambdas=(1e-4, 1e-2), dtype=np.float32):
    """Balanced-partition workload: x = s * z, z ~ N(0, I), s_k ~ U[0.5, 2];
    y = random two-layer tanh network + 0.05 N(0, 1); hold-out set of
    ceil(val_frac * n) points for model selection."""
    s = rng(seed, S_MIX).uniform(0.5, 2.0, d)
    k_val = int(math.ceil(val_frac * n))
    X = (rng(seed, S_XTRAIN).standard_normal((n, d)) * s).astype(dtype)
    Xv = (rng(seed, S_XVAL).standard_normal((k_val, d)) * s).astype(dtype)
    Xt = (rng(seed, S_XTEST).standard_normal((k_test, d)) * s).astype(dtype)
    f = TanhNet.draw(seed, d)
    y = f(X) + _noise(seed, 0, n, 0.05)
    yv = f(Xv) + _noise(seed, 1, k_val, 0.05)
    yt = f(Xt) + _noise(seed, 2, k_test, 0.05)
    return Workload(f"balanced_n{n}_d{d}_p{p}", X, y, Xv, yv, Xt, yt, p,
                    tuple(sigmas), tuple(lambdas), {"feature_scale": s, "dtype": "f32"})


def zipf_clipped_counts(n, comps, alpha=1.1, lo=512, hi=14000):
    """Component counts proportional to r^-alpha (r = 1..comps), water-filled
    into [lo, hi] so that they sum to n."""
    w = np.arange(1, comps + 1, dtype=np.float64) ** (-alpha)
    w /= w.sum()

    def total(scale):
        return np.clip(n * w * scale, lo, hi).sum()

    a, b = 1e-6, 1e6
    for _ in range(200):
        mid = math.sqrt(a * b)
        if total(mid) < n:
            a = mid
        else:
            b = mid
    c = np.clip(n * w * b, lo, hi)
    base = np.floor(c).astype(np.int64)
    rem = int(n - base.sum())
    order = np.argsort(-(c - base), kind="stable")
    i = 0
    while rem > 0:
        j = order[i % comps]
        if base[j] < hi:
            base[j] += 1
            rem -= 1
        i += 1
    while rem < 0:
        j = order[::-1][i % comps]
        if base[j] > lo:
            base[j] -= 1
            rem += 1
        i += 1
    return base


def gaussian_mixture(seed=3, n=131072, d=90, comps=32, mean_scale=3.0, alpha=1.1,
                     lo=512, hi=14000, k_test=8192, dtype=np.float32, raw=False):
    """Mixture of `comps` unit-covariance Gaussians with means ~ N(0, mean_scale^2 I)
    and Zipf(alpha) weights; component sizes water-filled into [lo, hi]
    (raw=True keeps the unclipped proportional counts).  Points are shuffled so
    that the input order carries no component information."""
    g = rng(seed, S_MIX)
    mu = g.standard_normal((comps, d)) * mean_scale
    if raw:
        w = np.arange(1, comps + 1, dtype=np.float64) ** (-alpha)
        counts = np.floor(n * w / w.sum()).astype(np.int64)
        counts[0] += n - counts.sum()
    else:
        counts = zipf_clipped_counts(n, comps, alpha, lo, hi)
    comp = np.repeat(np.arange(comps), counts)
    perm = g.permutation(n)
    comp = comp[perm]
    X = (mu[comp] + rng(seed, S_XTRAIN).standard_normal((n, d))).astype(dtype)
    ct = rng(seed, S_XTEST + 10).choice(comps, size=k_test, p=counts / counts.sum())
    Xt = (mu[ct] + rng(seed, S_XTEST).standard_normal((k_test, d))).astype(dtype)
    f = TanhNet.draw(seed, d)
    y = f(X) + _noise(seed, 0, n, 0.05)
    yt = f(Xt) + _noise(seed, 2, k_test, 0.05)
    return Workload(f"gmm_n{n}_d{d}_k{comps}", X, y, None, None, Xt, yt, comps,
                    (2.0,), (1e-2,), {"counts": counts, "means": mu, "dtype": "f32"})


def median_heuristic_sigma(X, sample=2048, seed=0):
    """sigma = sqrt(median pairwise squared distance / 2) on a seeded subsample
    (a stress setting that makes K far from the identity)."""
    g = rng(seed, 99)
    idx = g.choice(X.shape[0], size=min(sample, X.shape[0]), replace=False)
    Z = X[idx].astype(np.float64)
    sq = (Z * Z).sum(1)
    D = sq[:, None] + sq[None, :] - 2.0 * Z @ Z.T
    iu = np.triu_indices(Z.shape[0], 1)
    return float(math.sqrt(max(np.median(D[iu]), 1e-300) / 2.0))


def small(seed, n, d, k=64, p=4, dtype=np.float64, comps=None, spread=3.0):
    """Small seeded problem for parity tests: a `comps`-component mixture (or
    N(0, I) when comps is None) with sin labels."""
    g = rng(seed, S_MIX)
    if comps:
        mu = g.standard_normal((comps, d)) * spread
        c = g.integers(0, comps, n)
        ct = g.integers(0, comps, k)
        X = mu[c] + rng(seed, S_XTRAIN).standard_normal((n, d))
        Xt = mu[ct] + rng(seed, S_XTEST).standard_normal((k, d))
    else:
        X = rng(seed, S_XTRAIN).standard_normal((n, d))
        Xt = rng(seed, S_XTEST).standard_normal((k, d))
    X = X.astype(dtype)
    Xt = Xt.astype(dtype)
    y = np.sin(X[:, 0].astype(np.float64) + X[:, min(1, d - 1)]) + 0.1 * rng(seed, S_NOISE).standard_normal(n)
    yt = np.sin(Xt[:, 0].astype(np.float64) + Xt[:, min(1, d - 1)])
    return Workload(f"small_s{seed}_n{n}_d{d}", X, y, None, None, Xt, yt, p,
                    (1.0,), (1e-2,), {})


# ---------------------------------------------------------------------------
# serving workload: a request stream over a resident partitioned model
# ---------------------------------------------------------------------------
S_TRACE = 40   # arrival trace streams are S_TRACE + a per-rate offset


@dataclasses.dataclass
class ServingPools:
    """Payload pools the requests of a trace slice from.

    resident: the training set of the resident model (a `comps`-component
    mixture, like the ragged-partition workload); queries: points from the
    same distribution; fit_X[d], fit_y[d]: mixture points and labels of
    dimension d for fit requests."""
    resident: Workload
    queries: np.ndarray
    fit_X: dict
    fit_y: dict


def serving_pools(seed=5, n=262144, d=90, comps=64, n_queries=16384, fit_ds=(8, 32, 90), fit_rows=8192,
                  fit_comps=32):
    res = gaussian_mixture(seed=seed, n=n, d=d, comps=comps, lo=max(64, n // comps // 8),
                           hi=max(n // comps * 4, 1), k_test=n_queries)
    fit_X, fit_y = {}, {}
    for fd in fit_ds:
        w = gaussian_mixture(seed=seed * 1000 + fd, n=fit_rows, d=fd, comps=fit_comps,
                             lo=max(1, fit_rows // fit_comps // 8), hi=fit_rows, k_test=1)
        fit_X[fd] = w.X
        fit_y[fd] = w.y.astype(np.float32)
    return ServingPools(res, res.Xt, fit_X, fit_y)


@dataclasses.dataclass
class TraceRequest:
    t: float        # arrival time, seconds from the start of the trace
    kind: str       # "predict" or "fit"
    rows: int       # query points (predict) or training points (fit)
    d: int
    offset: int     # first row in the pool (wrapping)


def serving_trace(seed=5, rate=100.0, seconds=2.0, fit_frac=0.1, fit_rows=(256, 8192), fit_ds=(8, 32, 90),
                  query_rows=(1, 1024), d_model=90, pool_queries=16384, pool_fit=8192):
    """Poisson arrivals at `rate` per second for `seconds`; each request is a
    fit with probability fit_frac (m uniform in fit_rows, d uniform over
    fit_ds) and otherwise a prediction of a uniform number of query points in
    query_rows.  Sizes and pool offsets only; payloads come from the pools."""
    g = rng(seed, S_TRACE + int(round(rate)))
    out, t = [], 0.0
    while True:
        t += g.exponential(1.0 / rate)
        if t >= seconds:
            break
        if g.random() < fit_frac:
            m = int(g.integers(fit_rows[0], fit_rows[1] + 1))
            fd = int(fit_ds[g.integers(0, len(fit_ds))])
            out.append(TraceRequest(t, "fit", m, fd, int(g.integers(0, pool_fit))))
        else:
            k = int(g.integers(query_rows[0], query_rows[1] + 1))
            out.append(TraceRequest(t, "predict", k, d_model, int(g.integers(0, pool_queries))))
    return out


def take_rows(pool, offset, rows):
    """rows consecutive rows of pool starting at offset, wrapping around."""
    idx = (offset + np.arange(rows)) % pool.shape[0]
    return np.ascontiguousarray(pool[idx])
