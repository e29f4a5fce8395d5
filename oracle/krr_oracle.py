"""Reference (oracle) implementation of partitioned kernel ridge regression.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain FP64 CPU statement
of what the GPU library computes.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library never calls it
and shares no code with it.

It follows You, Demmel, Hsieh, Vuduc, "Accurate, Fast and Scalable Kernel
Ridge Regression on Parallel and Distributed Systems" (ICS'18):

* Section 2.3, Eqs. (6)-(7) and Algorithm 1: kernel matrix, the solve of
  (K + lambda I) alpha = y, prediction, MSE (Eq. 3).
* Table 1: Gaussian, linear, polynomial and sigmoid kernels.
* Section 2.4, Algorithm 2: K-means (assignment, change count, mean update).
* Section 3.2, Algorithm 3 (DC-KRR): random even partition, averaged models.
* Section 4.3, Algorithm 4: K-balance (capacity-constrained greedy pass in
  sample order, then centre recompute); Algorithm 5 (BKRR2): per-partition
  fits, nearest-centre routing of test points, MSE reduce, best parameters.
* Section 4.1 (KKRR): average of all partition models; Section 4.2 (KKRR2):
  nearest-centre model only.

Readings taken where the paper is silent (each is listed in the design notes):

* lambda is the absolute diagonal shift (K + lambda I); ``lambda_times_m``
  reproduces the per-partition lambda*m of Algorithms 3, 5, 6.
* Squared distances are accumulated in FP64, sequentially over the feature
  index, each subtract / multiply / add rounded on its own (no fused
  multiply-add).  Comparisons use the squared value; ties go to the lowest
  centre index (the strict "<" over ascending j of Algorithm 4).
* K-means initialisation ("randomly" in Algorithm 2) is k-means++ (D^2
  sampling) driven by SplitMix64 uniforms; the cumulative D^2 weight is the
  plain sequential running sum in point order, see ``kmeanspp``.
* Lloyd stops after ``iters`` passes or when no assignment changed; an empty
  cluster keeps its previous centre; the returned partition is the assignment
  to the final centres.
* The mean of a cluster (Algorithm 2) is its members' exactly rounded FP64
  sum (the exact sum of the values rounded once, to nearest, ties to even;
  ``math.fsum``) divided by the count in FP64; it depends on no order of the
  members.
* K-balance capacity is ceil(n/p); the recompute of centres (optional in the
  paper) is done.
* The approximate parallel K-balance (Section 4.3, after Algorithm 4) splits
  the samples in input order into p even segments, rows
  [floor(q n / p), floor((q + 1) n / p)), as a row scatter would; each
  segment runs the greedy pass with capacity ceil(n_q / p) (the paper's
  n / p^2 when p^2 divides n), then the centres are recomputed as member
  means over all segments.
* CSR input (Sections 5.5 and 6) is expanded to the dense n x d matrix;
  repeated columns of a row are added in storage order in the values' dtype.
* DC-KRR's shuffle (Algorithm 3) is a keyed Feistel permutation with
  cycle-walking, and the even split gives partition j the shuffled rows
  [floor(j n / p), floor((j + 1) n / p)); see ``shuffle_positions``.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15

STATUS_OK, STATUS_NOT_SPD = 0, -4


# ---------------------------------------------------------------------------
# SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
# generators", OOPSLA 2014) -- written from its published definition.
# ---------------------------------------------------------------------------

def splitmix64_outputs(seed: int, count: int) -> list[int]:
    state = seed & MASK64
    out = []
    for _ in range(count):
        state = (state + GOLDEN_GAMMA) & MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        out.append(z ^ (z >> 31))
    return out


def uniforms(seed: int, count: int) -> np.ndarray:
    """u_t = (top 53 bits of the t-th SplitMix64 output) * 2^-53, in [0, 1)."""
    return np.array([(z >> 11) * (2.0 ** -53) for z in splitmix64_outputs(seed, count)],
                    dtype=np.float64)


# ---------------------------------------------------------------------------
# distances and assignment (Algorithm 2 step "argmin_j ||x_i - CT_j||")
# ---------------------------------------------------------------------------

def dist2(A: np.ndarray, B: np.ndarray, chunk: int = 8192) -> np.ndarray:
    """Squared Euclidean distances between rows of A (na x d) and B (nb x d),
    FP64, summed sequentially over the feature index with separate roundings."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    na, d = A.shape
    out = np.empty((na, B.shape[0]), dtype=np.float64)
    for r0 in range(0, na, chunk):
        a = A[r0:r0 + chunk]
        acc = np.zeros((a.shape[0], B.shape[0]), dtype=np.float64)
        for k in range(d):
            diff = a[:, k, None] - B[None, :, k]
            sq = diff * diff
            acc = acc + sq
        out[r0:r0 + chunk] = acc
    return out


def assign(X: np.ndarray, C: np.ndarray):
    """Nearest centre per point: (index int32, squared distance).  np.argmin
    returns the first minimum, i.e. the lowest centre index on ties."""
    D = dist2(X, C)
    idx = np.argmin(D, axis=1).astype(np.int32)
    return idx, D[np.arange(D.shape[0]), idx]


# ---------------------------------------------------------------------------
# K-means (Algorithm 2) with k-means++ initialisation
# ---------------------------------------------------------------------------

def running_sum(w: np.ndarray) -> np.ndarray:
    """Inclusive prefix sums S_i = (...((w_0 + w_1) + w_2) ... + w_i), FP64,
    one rounding per addition, strictly in index order.  (NumPy's
    add.accumulate is this left-to-right recurrence; np.sum is pairwise and
    is not used for it.)"""
    return np.add.accumulate(np.asarray(w, dtype=np.float64))


def kmeanspp(X: np.ndarray, k: int, seed: int, trace: list | None = None) -> tuple[np.ndarray, np.ndarray]:
    """k-means++ seeding.  First centre: point floor(u_0 n).  Centre t: the
    smallest i whose cumulative D^2 weight S_i exceeds u_t * S_{n-1}, where
    D^2 is the squared distance to the nearest centre chosen so far and S is
    the sequential running sum in point order.  Returns (centres k x d FP64,
    chosen indices).  `trace` (optional list) receives, for t >= 1, a dict
    with the threshold, the total and the running sums just below and at the
    pick (for checking how far a decision is from a rounding tie)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    u = uniforms(seed, k)
    chosen = [min(int(math.floor(u[0] * n)), n - 1)]
    D2 = dist2(X, X[chosen[0]][None, :])[:, 0]
    for t in range(1, k):
        S = running_sum(D2)
        total = S[-1]
        if not total > 0.0:
            i = min(int(math.floor(u[t] * n)), n - 1)
            thr = None
        else:
            thr = u[t] * total
            i = int(np.argmax(S > thr))      # first index with S_i > thr
        if trace is not None:
            trace.append({"t": t, "pick": i, "thr": thr, "total": float(total),
                          "below": float(S[i - 1]) if i > 0 else 0.0, "at": float(S[i])})
        chosen.append(i)
        D2 = np.minimum(D2, dist2(X, X[i][None, :])[:, 0])
    return X[chosen].copy(), np.array(chosen, dtype=np.int64)


def member_means(X: np.ndarray, a: np.ndarray, C_prev: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Algorithm 2 mean step: CT_j = (sum of members) / count_j; an empty
    cluster keeps C_prev[j].  Algorithm 2 leaves the rounding of the sum open;
    here it is the exact sum of the member values rounded once to FP64
    (math.fsum: nearest, ties to even), which no order of the members
    changes, then one FP64 division by the count."""
    X = np.asarray(X, dtype=np.float64)
    k = C_prev.shape[0]
    C = C_prev.copy()
    counts = np.bincount(a, minlength=k).astype(np.int64)
    for j in range(k):
        if counts[j] == 0:
            continue
        members = X[a == j]
        total = np.array([math.fsum(members[:, f]) for f in range(members.shape[1])])
        C[j] = total / float(counts[j])
    return C, counts


def lloyd(X: np.ndarray, C0: np.ndarray, iters: int):
    """Lloyd iterations of Algorithm 2.  Returns (final centres, assignment to
    the final centres, number of passes run, list of change counts)."""
    C = np.asarray(C0, dtype=np.float64).copy()
    prev = None
    deltas = []
    for _ in range(iters):
        a, _ = assign(X, C)
        delta = int(a.shape[0]) if prev is None else int(np.count_nonzero(a != prev))
        deltas.append(delta)
        prev = a
        C, _ = member_means(X, a, C)
        if delta == 0:
            break
    a, _ = assign(X, C)
    return C, a, len(deltas), deltas


def kmeans(X, k, iters, seed, trace: list | None = None):
    """k-means++ seeding, then Lloyd (Algorithm 2); `trace` as in kmeanspp."""
    C0, _ = kmeanspp(X, k, seed, trace)
    C, a, _, _ = lloyd(X, C0, iters)
    return C, a


def kbalance_greedy(X: np.ndarray, C: np.ndarray, cap: int) -> np.ndarray:
    """Algorithm 4 greedy pass: samples in input order; each goes to its
    nearest centre among those holding fewer than `cap` samples (strict "<"
    over ascending centre index, so the lowest index wins ties)."""
    D = dist2(X, C)
    p = C.shape[0]
    CS = [0] * p
    MB = np.empty(X.shape[0], dtype=np.int32)
    for i in range(X.shape[0]):
        row = D[i]
        best, bestd = -1, math.inf
        for j in range(p):
            if CS[j] < cap and row[j] < bestd:
                best, bestd = j, row[j]
        if best < 0:        # every centre full: unreachable when cap*p >= n
            best = 0
        CS[best] += 1
        MB[i] = best
    return MB


def kbalance(X, p, iters, seed, trace: list | None = None):
    """K-balance (Algorithm 4): K-means centres, greedy capacity-ceil(n/p)
    pass, then centres recomputed as member means."""
    C, _ = kmeans(X, p, iters, seed, trace)
    n = X.shape[0]
    cap = -(-n // p)
    MB = kbalance_greedy(X, C, cap)
    C2, _ = member_means(X, MB, C)
    return C2, MB


def kbalance_approx(X, p, iters, seed):
    """Approximate parallel K-balance (Section 4.3): the same K-means centres,
    the samples split in input order into p even segments (one per node),
    each segment's own greedy pass with capacity ceil(n_q / p) (n / p^2 per
    node and centre), then centres recomputed as member means."""
    C, _ = kmeans(X, p, iters, seed)
    n = X.shape[0]
    MB = np.empty(n, dtype=np.int32)
    for q in range(p):
        lo, hi = q * n // p, (q + 1) * n // p
        if hi > lo:
            MB[lo:hi] = kbalance_greedy(X[lo:hi], C, -(-(hi - lo) // p))
    C2, _ = member_means(X, MB, C)
    return C2, MB


# ---------------------------------------------------------------------------
# Sparse input (Section 5.5 and Section 6: the n x d input matrix held in CSR)
# ---------------------------------------------------------------------------

def csr_to_dense(indptr, indices, values, n: int, d: int) -> np.ndarray:
    """The dense n x d matrix of a CSR (compressed sparse row) input: row i
    holds values[k] at column indices[k] for indptr[i] <= k < indptr[i + 1].
    Columns repeated within a row are added in storage order, starting from
    zero, in the values' dtype.  A malformed structure (indptr[0] != 0,
    indptr decreasing, indptr[n] != nnz, a column outside [0, d)) raises
    ValueError."""
    indptr = np.asarray(indptr, dtype=np.int64)
    indices = np.asarray(indices, dtype=np.int64)
    values = np.asarray(values)
    nnz = values.shape[0]
    if indptr.shape != (n + 1,) or indices.shape != (nnz,):
        raise ValueError("CSR arrays of the wrong length")
    if indptr[0] != 0 or indptr[n] != nnz or np.any(indptr[1:] < indptr[:-1]):
        raise ValueError("malformed CSR row pointers")
    if nnz and (indices.min() < 0 or indices.max() >= d):
        raise ValueError("CSR column index out of range")
    X = np.zeros((n, d), dtype=values.dtype)
    for i in range(n):
        for k in range(int(indptr[i]), int(indptr[i + 1])):
            j = int(indices[k])
            X[i, j] = X[i, j] + values[k]
    return X


# ---------------------------------------------------------------------------
# DC-KRR divide step (Section 3.2, Algorithm 3): shuffle the rows of [X, y],
# then hand them out evenly by rows
# ---------------------------------------------------------------------------

SHUFFLE_ROUNDS = 8


def _mix64(z: int) -> int:
    """Output function of SplitMix64 (Steele, Lea, Flood 2014): two
    xor-shift-multiply rounds and a final xor-shift of a 64-bit value."""
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def shuffle_positions(n: int, seed: int) -> np.ndarray:
    """pos[i] = the row that point i takes in the shuffled matrix of Algorithm 3.

    The paper does not say how to shuffle.  Here the shuffle is a keyed
    pseudo-random permutation, computed for every point on its own: a
    balanced Feistel network of SHUFFLE_ROUNDS rounds on b-bit values (b the
    smallest even number >= 2 with 2^b >= n; halves of h = b/2 bits; round r
    maps (L, R) to (R, L xor F_r(R)) with F_r(R) = the low h bits of the
    SplitMix64 output function of (K_r + R) mod 2^64, K_r = the r-th
    SplitMix64 output of the seed), restricted to [0, n) by cycle-walking
    (Black & Rogaway, "Ciphers with arbitrary finite domains", CT-RSA 2002):
    an image outside [0, n) is mapped again until it falls inside."""
    keys = splitmix64_outputs(seed, SHUFFLE_ROUNDS)
    b = 2
    while (1 << b) < n:
        b += 2
    h = b // 2
    mask = (1 << h) - 1

    def feistel(v: int) -> int:
        left, right = v >> h, v & mask
        for key in keys:
            left, right = right, left ^ (_mix64((key + right) & MASK64) & mask)
        return (left << h) | right

    pos = np.empty(n, dtype=np.int64)
    for i in range(n):
        v = feistel(i)
        while v >= n:
            v = feistel(v)
        pos[i] = v
    return pos


def random_partition(X: np.ndarray, p: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Algorithm 3's even split of the shuffled rows: shuffled row pos goes to
    partition j with floor(j n / p) <= pos < floor((j + 1) n / p), i.e.
    j = ceil((pos + 1) p / n) - 1 (sizes differ by at most one).  The centres
    (for nearest-centre routing; Algorithm 3 itself averages all models) are
    the member means, summed as in Algorithm 2's mean step."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    pos = shuffle_positions(n, seed)
    a = (((pos + 1) * p + n - 1) // n - 1).astype(np.int32)
    C, _ = member_means(X, a, np.zeros((p, X.shape[1])))
    return C, a


def partition(X, p, method, iters=20, seed=0, centroids=None):
    """Returns (centroids p x d FP64, assignment int32[n], sizes int64[p])."""
    if method == "random":
        C, a = random_partition(X, p, seed)
    elif method == "given":
        C = np.asarray(centroids, dtype=np.float64)
        a, _ = assign(X, C)
    elif method == "kmeans":
        C, a = kmeans(X, p, iters, seed)
    elif method == "kbalance":
        C, a = kbalance(X, p, iters, seed)
    elif method == "kbalance_approx":
        C, a = kbalance_approx(X, p, iters, seed)
    else:
        raise ValueError(method)
    return C, a, np.bincount(a, minlength=p).astype(np.int64)


def gather(a: np.ndarray, p: int):
    """Stable grouping of points by partition: (permutation, offsets[p+1])."""
    perm = np.argsort(a, kind="stable")
    sizes = np.bincount(a, minlength=p)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return perm, offsets


# ---------------------------------------------------------------------------
# kernel ridge regression (Section 2.3)
# ---------------------------------------------------------------------------

def kernel_matrix(A, B, sigma, kernel="gaussian"):
    """Table 1: Gaussian exp(-||a-b||^2 / (2 sigma^2)) by direct difference;
    linear a^T b; polynomial (a x^T y + r)^d given as ("polynomial", a, r, d)
    with an integer d >= 1; sigmoid tanh(a x^T y + r) given as
    ("sigmoid", a, r).  The sigmoid kernel is not positive semi-definite in
    general, so K + lambda I may not be either (the solve then reports the
    failing pivot)."""
    name = kernel if isinstance(kernel, str) else kernel[0]
    if name == "gaussian":
        return np.exp(-dist2(A, B) / (2.0 * sigma * sigma))
    G = np.asarray(A, np.float64) @ np.asarray(B, np.float64).T
    if name == "linear":
        return G
    if name == "polynomial":
        _, a, r, deg = kernel
        return (a * G + r) ** int(deg)
    if name == "sigmoid":
        _, a, r = kernel
        return np.tanh(a * G + r)
    raise ValueError(kernel)


def solve_lu(A, b):
    """Solution of the (possibly indefinite) system A x = b by LU with
    partial pivoting (LAPACK dgetrf / dgetrs through SciPy).  Returns
    (x, singular): singular when a zero pivot makes A numerically singular."""
    lu, piv = scipy.linalg.lu_factor(np.asarray(A, np.float64), check_finite=False)
    if np.any(np.diag(lu) == 0.0):
        return np.full(A.shape[0], np.nan), True
    return scipy.linalg.lu_solve((lu, piv), np.asarray(b, np.float64), check_finite=False), False


def fit_one(Xj, yj, sigma, lam, kernel="gaussian", lambda_times_m=False, indefinite=False):
    """Solve (K + lambda_eff I) alpha = y by Cholesky (Eq. 6, Algorithm 1).
    With `indefinite`, a system whose Cholesky factorisation meets a
    non-positive pivot (the sigmoid kernel of Table 1 is not positive
    semi-definite in general) is solved by LU with partial pivoting instead
    (solve_lu) and reported with solver "lu".
    Returns dict(alpha, status, pivot, backward_error, lambda_eff, solver)."""
    m = Xj.shape[0]
    lam_eff = lam * m if lambda_times_m else lam
    if m == 0:   # an empty partition (K-means may leave a cluster empty) has no system
        return {"alpha": np.zeros(0), "status": STATUS_OK, "pivot": 0, "backward_error": 0.0,
                "lambda_eff": lam_eff}
    A = kernel_matrix(Xj, Xj, sigma, kernel)
    A[np.diag_indices(m)] += lam_eff
    yj = np.asarray(yj, dtype=np.float64)
    try:
        c = scipy.linalg.cho_factor(A, lower=True, check_finite=False)
    except np.linalg.LinAlgError as e:
        # LAPACK dpotrf reports the order of the first non-positive leading minor
        piv = _first_bad_pivot(A)
        if indefinite:
            alpha, singular = solve_lu(A, yj)
            if not singular:
                r = A @ alpha - yj
                be = np.linalg.norm(r) / (np.linalg.norm(A, 2 if m <= 512 else "fro") * np.linalg.norm(alpha)
                                          + np.linalg.norm(yj))
                return {"alpha": alpha, "status": STATUS_OK, "pivot": piv, "backward_error": float(be),
                        "lambda_eff": lam_eff, "solver": "lu"}
        return {"alpha": np.full(m, np.nan), "status": STATUS_NOT_SPD, "pivot": piv,
                "backward_error": math.inf, "lambda_eff": lam_eff, "err": str(e), "solver": "none"}
    alpha = scipy.linalg.cho_solve(c, yj, check_finite=False)
    r = A @ alpha - yj
    be = np.linalg.norm(r) / (np.linalg.norm(A, 2 if m <= 512 else "fro") * np.linalg.norm(alpha)
                              + np.linalg.norm(yj))
    return {"alpha": alpha, "status": STATUS_OK, "pivot": 0, "backward_error": float(be),
            "lambda_eff": lam_eff, "solver": "cholesky"}


def _first_bad_pivot(A):
    """1-based order of the first leading principal minor that is not
    positive definite (the LAPACK dpotrf `info` convention)."""
    m = A.shape[0]
    L = np.zeros_like(A)
    for j in range(m):
        s = A[j, j] - L[j, :j] @ L[j, :j]
        if not s > 0.0:
            return j + 1
        L[j, j] = math.sqrt(s)
        L[j + 1:, j] = (A[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return 0


class Model:
    """One (sigma, lambda) setting fitted on every partition."""

    def __init__(self, Xparts, alphas, centroids, sigma, lam, kernel, infos):
        self.Xparts = Xparts
        self.alphas = alphas
        self.centroids = centroids
        self.sigma = sigma
        self.lam = lam
        self.kernel = kernel
        self.infos = infos


def fit(X, y, a, centroids, p, sigma, lam, kernel="gaussian", lambda_times_m=False, indefinite=False):
    """Per-partition fits (Algorithm 5 training phase)."""
    perm, off = gather(a, p)
    Xparts, alphas, infos = [], [], []
    for j in range(p):
        idx = perm[off[j]:off[j + 1]]
        Xj = np.asarray(X, np.float64)[idx]
        r = fit_one(Xj, np.asarray(y, np.float64)[idx], sigma, lam, kernel, lambda_times_m, indefinite)
        Xparts.append(Xj)
        alphas.append(r["alpha"])
        infos.append(r)
    return Model(Xparts, alphas, np.asarray(centroids, np.float64), sigma, lam, kernel, infos)


def predict_one(Xj, alpha, Xt, sigma, kernel="gaussian"):
    """Eq. (7): y~(x^) = sum_i alpha_i K(x_i, x^)."""
    if Xj.shape[0] == 0:
        return np.zeros(np.asarray(Xt).shape[0])
    return kernel_matrix(Xt, Xj, sigma, kernel) @ alpha


def predict(model: Model, Xt, route="nearest"):
    """nearest: the model of the closest centre (KKRR2 / BKRR2);
    average: mean over all partition models (KKRR / BKRR);
    all: k x p matrix of every model's prediction (BKRR3 / KKRR3)."""
    Xt = np.asarray(Xt, np.float64)
    p = len(model.alphas)
    if route == "nearest":
        r, _ = assign(Xt, model.centroids)
        yhat = np.zeros(Xt.shape[0])
        for j in range(p):
            sel = np.nonzero(r == j)[0]
            if sel.size:
                yhat[sel] = predict_one(model.Xparts[j], model.alphas[j], Xt[sel], model.sigma, model.kernel)
        return yhat, r
    allp = np.stack([predict_one(model.Xparts[j], model.alphas[j], Xt, model.sigma, model.kernel)
                     for j in range(p)], axis=1)
    if route == "average":
        return allp.mean(axis=1), None
    if route == "all":
        return allp, None
    raise ValueError(route)


def mse(yhat, ytrue):
    """Eq. (3)."""
    e = np.asarray(yhat, np.float64) - np.asarray(ytrue, np.float64)
    return float(np.mean(e * e))


def select(mses):
    """Best model: lowest MSE, strict '<' so the first in order wins ties
    (Algorithm 5, final comparison)."""
    best, bestv = -1, math.inf
    for i, v in enumerate(mses):
        if v < bestv:
            best, bestv = i, v
    return best


def label_oracle_select(allp, ytrue):
    """BKRR3 / KKRR3 (Algorithm 6): per test point the model whose prediction
    is closest to the true label (first index on ties)."""
    e = (allp - np.asarray(ytrue, np.float64)[:, None]) ** 2
    idx = np.argmin(e, axis=1)
    return allp[np.arange(allp.shape[0]), idx], idx


# ---------------------------------------------------------------------------
# work accounting
# ---------------------------------------------------------------------------

def fit_flops(m, d):
    """Algorithmic flops of one fit: m^3/3 (Cholesky) + m^2 d (lower-triangle
    Gram) + m^2/2 (exp, counted as one) + 2 m^2 (two triangular solves)."""
    m = float(m)
    return m ** 3 / 3.0 + m * m * d + m * m / 2.0 + 2.0 * m * m


def predict_flops(m, d):
    return 2.0 * m * d + 3.0 * m


def partitioned_speedup(n, p, n_partitioned=None):
    """Per-processor flop ratio of one global n x n Cholesky spread over p
    processors (n^3/p) against one local (n'/p)^3 factorisation per
    processor, n' = n_partitioned (default n): p^2 when n' = n (Section 5.2)."""
    n2 = n if n_partitioned is None else n_partitioned
    return (n ** 3 / p) / ((n2 / p) ** 3)
