"""Element-wise parity measures and oracle helpers shared by the GPU tests.

Every floating-point comparison is element by element: the largest
difference over the vector, divided by the largest magnitude of the
reference, so that one wrong entry cannot hide in a norm over thousands of
correct ones.  Predictions of a model whose outputs are all close to zero
(a kernel close to the identity) are judged against the scale of the labels
instead: the denominator is max(max|yhat_ref|, 1e-3 max|y|).
"""
from __future__ import annotations

import concurrent.futures
import math
import multiprocessing

import numpy as np

import oracle as O

# k-means++ decisions: unit roundoff of FP64
U64 = 2.0 ** -53


def ew(a, b) -> float:
    """max_i |a_i - b_i| / max_i |b_i| (0 for two empty vectors)."""
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    assert a.shape == b.shape, (a.shape, b.shape)
    if b.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def pred_ew(yhat, yref, ytrue) -> float:
    """Element-wise prediction error, scaled by max(max|yref|, 1e-3 max|ytrue|)."""
    yhat = np.asarray(yhat, np.float64).ravel()
    yref = np.asarray(yref, np.float64).ravel()
    den = max(float(np.max(np.abs(yref))) if yref.size else 0.0,
              1e-3 * float(np.max(np.abs(np.asarray(ytrue, np.float64)))), 1e-300)
    return float(np.max(np.abs(yhat - yref)) / den) if yref.size else 0.0


def kpp_ambiguous(trace, n: int) -> int:
    """Number of k-means++ decisions whose threshold lies within the rounding
    gap of another summation order of the cumulative weights.

    The oracle forms the cumulative D^2 weight S as the sequential running
    sum; the GPU sums the same nonnegative weights in blocks of 256 (in-block
    running sums, block totals summed in order, one add of the block offset).
    Both are within gamma_k * E of the exact prefix E, with k = n for the
    running sum and k = 256 + ceil(n / 256) + 1 for the blocked one
    (gamma_k = k u / (1 - k u), Higham, Accuracy and Stability, Section 4.2),
    and the thresholds u_t * total differ by at most the same amount plus
    one rounding.  A decision whose margins S_i - thr and thr - S_{i-1} both
    exceed twice that bound is taken the same way by both orders."""
    kb = 256 + math.ceil(n / 256) + 1

    def gam(k):
        return k * U64 / (1.0 - k * U64)

    amb = 0
    for rec in trace:
        if rec["thr"] is None:
            continue
        bound = 2.0 * (gam(n) + gam(kb) + 2 * U64) * rec["total"]
        if not (rec["at"] - rec["thr"] > bound and rec["thr"] - rec["below"] > bound):
            amb += 1
    return amb


def _fit_worker(args):
    Xj, yj, sigma, lam, kernel, ltm = args
    try:
        import threadpoolctl
        with threadpoolctl.threadpool_limits(1):
            return O.fit_one(Xj, yj, sigma, lam, kernel, ltm)["alpha"]
    except ImportError:
        return O.fit_one(Xj, yj, sigma, lam, kernel, ltm)["alpha"]


def oracle_alphas(jobs, workers: int = 8):
    """alpha of O.fit_one for every (Xj, yj, sigma, lambda, kernel,
    lambda_times_m) job, in worker processes started fresh (spawn: nothing of
    the GPU process is inherited), one BLAS thread each."""
    if len(jobs) <= 1:
        return [_fit_worker(j) for j in jobs]
    ctx = multiprocessing.get_context("spawn")
    with concurrent.futures.ProcessPoolExecutor(max_workers=min(workers, len(jobs)), mp_context=ctx) as ex:
        return list(ex.map(_fit_worker, jobs))
