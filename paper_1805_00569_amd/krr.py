"""Python binding of the C ABI in include/krr.h (argument marshalling only).

Every step of the computation runs in the HIP library ``libkrr.so``; this
module converts torch tensors to device pointers, takes the current HIP
stream, and turns negative status codes into ``KrrError``.  If the library is
not built, importing it raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkrr.so")

KRR_OK, KRR_EINVAL, KRR_ENOMEM, KRR_EBUDGET, KRR_ENOTSPD, KRR_ENOCONV, KRR_EDEVICE, KRR_ESTATE = \
    0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EBUDGET", -4: "ENOTSPD", -5: "ENOCONV",
                -6: "EDEVICE", -7: "ESTATE"}
F32, F64 = 0, 1
PART = {"kmeans": 0, "kbalance": 1, "given": 2, "random": 3, "kbalance_approx": 4}
PREC = {"fp64": 0, "fp32": 1, "mixed": 2}
ROUTE = {"nearest": 0, "average": 1, "all": 2, "label": 3}
KERNEL = {"gaussian": 0, "linear": 1, "polynomial": 2, "sigmoid": 3}
OPT_PANEL_TILES, OPT_SERIAL_FIT, OPT_SYNC_CHECK, OPT_TIMING, OPT_PERSISTENT, OPT_PERSIST_WAIT_MS, OPT_GRAPHS = \
    0, 1, 2, 3, 4, 5, 6
OPT_AUTOTUNE = 7
OPT_FACTOR_STREAMS = 8
OPT_COLUMN_PAIRS = 9


class KrrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class FitParams(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("lambda_", ctypes.c_double), ("kernel", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("refine_tol", ctypes.c_double), ("max_refine", ctypes.c_int32),
                ("lambda_times_m", ctypes.c_int32), ("kernel_a", ctypes.c_double), ("kernel_r", ctypes.c_double),
                ("kernel_degree", ctypes.c_int32), ("indefinite", ctypes.c_int32)]


class PartInfo(ctypes.Structure):
    _fields_ = [("partition", ctypes.c_int32), ("param", ctypes.c_int32), ("m", ctypes.c_int32),
                ("status", ctypes.c_int32), ("failed_pivot", ctypes.c_int32), ("refine_iters", ctypes.c_int32),
                ("fallback", ctypes.c_int32), ("solver", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("kappa_est", ctypes.c_double), ("err_est", ctypes.c_double), ("kappa_bound", ctypes.c_double)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("predict_workers", ctypes.c_int32), ("fit_workers", ctypes.c_int32),
                ("max_batch_fits", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("max_batch_points", ctypes.c_int64), ("hbm_budget_bytes", ctypes.c_size_t)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("kind", ctypes.c_int32), ("batch_requests", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("queue_ms", ctypes.c_double), ("run_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double)]


class ServeStats(ctypes.Structure):
    _fields_ = [("predict_requests", ctypes.c_int64), ("fit_requests", ctypes.c_int64),
                ("points", ctypes.c_int64), ("fit_rows", ctypes.c_int64),
                ("predict_batches", ctypes.c_int64), ("fit_batches", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("max_inflight_bytes", ctypes.c_int64),
                ("max_device_bytes", ctypes.c_int64),
                ("predict_p50_ms", ctypes.c_double), ("predict_p99_ms", ctypes.c_double),
                ("fit_p50_ms", ctypes.c_double), ("fit_p99_ms", ctypes.c_double),
                ("span_ms", ctypes.c_double)]


_P = ctypes.c_void_p
_SIGS = {
    "krr_create": ([ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(_P)], ctypes.c_int),
    "krr_destroy": ([_P], ctypes.c_int),
    "krr_last_error": ([_P], ctypes.c_char_p),
    "krr_set_option": ([_P, ctypes.c_int32, ctypes.c_int64], ctypes.c_int),
    "krr_memory_in_use": ([_P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "krr_autotune": ([_P, _P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "krr_graph_counts": ([_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "krr_timing_report": ([_P, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "krr_csr_to_dense": ([_P, _P, _P, _P, _P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, _P],
                         ctypes.c_int),
    "krr_partition": ([_P, _P, _P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                       ctypes.c_int32, ctypes.c_uint64, _P, _P, _P], ctypes.c_int),
    "krr_fit": ([_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _P, _P, ctypes.c_int32,
                 ctypes.POINTER(FitParams), ctypes.c_int32, ctypes.POINTER(_P), ctypes.POINTER(PartInfo)],
                ctypes.c_int),
    "krr_predict": ([_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _P, _P], ctypes.c_int),
    "krr_predict_noalloc": ([_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _P, _P], ctypes.c_int),
    "krr_select": ([_P, _P, ctypes.POINTER(_P), ctypes.c_int32, _P, _P, ctypes.c_int32, ctypes.c_int64,
                    ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "krr_model_alpha": ([_P, _P, _P, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "krr_model_free": ([_P], ctypes.c_int),
    "krr_server_create": ([_P, _P, ctypes.POINTER(ServerConfig), ctypes.POINTER(_P)], ctypes.c_int),
    "krr_server_destroy": ([_P], ctypes.c_int),
    "krr_server_last_error": ([_P], ctypes.c_char_p),
    "krr_server_submit_predict": ([_P, _P, ctypes.c_int64, _P, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "krr_server_submit_fit": ([_P, _P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(FitParams), _P,
                               ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "krr_server_wait": ([_P, ctypes.c_int64, ctypes.POINTER(RequestInfo)], ctypes.c_int),
    "krr_server_stats": ([_P, ctypes.c_int32, ctypes.POINTER(ServeStats)], ctypes.c_int),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libkrr.so and declare the exported signatures.  Raises if the
    library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: run `python -c 'import __graft_entry__ as g; g.build()'` first")
    lib = ctypes.CDLL(path)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _dtype_code(t):
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


@dataclasses.dataclass
class Params:
    sigma: float = 1.0
    lam: float = 1e-3
    kernel: str = "gaussian"
    prec: str = "fp64"
    refine_tol: float = 1e-6
    max_refine: int = 30
    lambda_times_m: bool = False
    kernel_a: float = 1.0      # polynomial / sigmoid: (a x^T y + r)^d, tanh(a x^T y + r)
    kernel_r: float = 1.0
    kernel_degree: int = 2
    indefinite: bool = False   # solve systems Cholesky rejects by LU with partial pivoting

    def to_c(self):
        return FitParams(float(self.sigma), float(self.lam), KERNEL[self.kernel], PREC[self.prec],
                         float(self.refine_tol), int(self.max_refine), int(bool(self.lambda_times_m)),
                         float(self.kernel_a), float(self.kernel_r), int(self.kernel_degree),
                         int(bool(self.indefinite)))


class Model:
    def __init__(self, ctx, handle, params):
        self.ctx = ctx
        self.handle = handle
        self.params = params

    def alpha(self, j):
        """alpha of partition j, FP64 device tensor (points in increasing
        original index order)."""
        m = ctypes.c_int64(0)
        out = torch.empty(max(int(self._m[j]), 1), dtype=torch.float64, device=self.ctx.device)
        self.ctx._check(self.ctx.lib.krr_model_alpha(self.ctx.h, _stream(self.ctx.device), self.handle, j,
                                                    _ptr(out), ctypes.byref(m)))
        return out[: m.value]

    def free(self):
        if self.handle:
            self.ctx.lib.krr_model_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Context:
    """One library context bound to a GPU."""

    def __init__(self, device=0, hbm_budget=0):
        self.lib = load_library()
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        h = ctypes.c_void_p()
        st = self.lib.krr_create(self.device.index or 0, int(hbm_budget), ctypes.byref(h))
        if st != KRR_OK:
            raise KrrError(st, "krr_create failed")
        self.h = h

    def _check(self, st):
        if st != KRR_OK:
            raise KrrError(st, self.lib.krr_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.krr_destroy(self.h)
            self.h = None

    def set_option(self, option, value):
        self._check(self.lib.krr_set_option(self.h, int(option), int(value)))

    def memory_in_use(self):
        v = ctypes.c_size_t(0)
        self._check(self.lib.krr_memory_in_use(self.h, ctypes.byref(v)))
        return v.value

    def autotune(self, prec, m, d, n_sys=8):
        """Time trial fits and record the fastest panel width for (prec, size
        class of m) on this context.  Returns (width, median fit ms)."""
        w, ms = ctypes.c_int32(0), ctypes.c_double(0.0)
        self._check(self.lib.krr_autotune(self.h, _stream(self.device), PREC[prec], int(m), int(d), int(n_sys),
                                          ctypes.byref(w), ctypes.byref(ms)))
        return w.value, ms.value

    def graph_counts(self):
        """(graphs captured, graph replays) on this context."""
        c, r = ctypes.c_int64(0), ctypes.c_int64(0)
        self._check(self.lib.krr_graph_counts(self.h, ctypes.byref(c), ctypes.byref(r)))
        return c.value, r.value

    def timing_report(self):
        """Per-kernel-class event timing since the last report (see
        krr_timing_report): {class: {"count", "ms", "flops"}}."""
        import json
        need = ctypes.c_size_t(0)
        self._check(self.lib.krr_timing_report(self.h, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(max(need.value, 2) + 4096)
        self._check(self.lib.krr_timing_report(self.h, buf, len(buf), ctypes.byref(need)))
        return json.loads(buf.value.decode() or "{}")

    def csr_to_dense(self, indptr, indices, values, d):
        """Dense n x d matrix (dtype of `values`) from CSR device tensors:
        indptr int64[n + 1], indices int32[nnz], values float32/float64[nnz]."""
        if indptr.dtype != torch.int64 or indices.dtype != torch.int32:
            raise TypeError("indptr must be int64 and indices int32")
        n, nnz = indptr.numel() - 1, values.numel()
        if indices.numel() != nnz:
            raise ValueError("indices and values differ in length")
        X = torch.empty((n, d), dtype=values.dtype, device=self.device)
        self._check(self.lib.krr_csr_to_dense(self.h, _stream(self.device), _ptr(indptr),
                                              _ptr(indices) if nnz else None, _ptr(values) if nnz else None,
                                              _dtype_code(values), n, d, nnz, _ptr(X)))
        return X

    def partition(self, X, p, method="kmeans", lloyd_iters=20, seed=0, centroids=None):
        """Returns (centroids p x d FP64, assign int32[n], sizes int64[p])."""
        n, d = X.shape
        C = (centroids.to(torch.float64).contiguous().clone() if centroids is not None
             else torch.empty((p, d), dtype=torch.float64, device=self.device))
        a = torch.empty(n, dtype=torch.int32, device=self.device)
        sz = torch.empty(p, dtype=torch.int64, device=self.device)
        self._check(self.lib.krr_partition(self.h, _stream(self.device), _ptr(X), _dtype_code(X), n, d, p,
                                           PART[method], lloyd_iters, ctypes.c_uint64(seed & (2 ** 64 - 1)),
                                           _ptr(C), _ptr(a), _ptr(sz)))
        return C, a, sz

    def fit(self, X, y, assign, centroids, p, params, raise_on_fail=False):
        """Fit every (setting, partition) system in one batch.  Returns
        (list of Model, list of info dicts, status)."""
        n, d = X.shape
        if y.dtype != X.dtype:
            raise TypeError("y must have the dtype of X")
        arr = (FitParams * len(params))(*[q.to_c() for q in params])
        handles = (ctypes.c_void_p * len(params))()
        info = (PartInfo * (len(params) * p))()
        st = self.lib.krr_fit(self.h, _stream(self.device), _ptr(X), _ptr(y), _dtype_code(X), n, d, _ptr(assign),
                              _ptr(centroids), p, arr, len(params), handles, info)
        if st not in (KRR_OK, KRR_ENOTSPD, KRR_ENOCONV) or (raise_on_fail and st != KRR_OK):
            self._check(st)
        models = [Model(self, handles[q], params[q]) for q in range(len(params))]
        infos = [{f: getattr(r, f) for f, _ in PartInfo._fields_} for r in info]
        sizes = {r["partition"]: r["m"] for r in infos}
        for mdl in models:
            mdl._m = sizes
        return models, infos, st

    def predict(self, model, Xt, route="nearest", want_route=False, out=None):
        """Predictions FP64 (k, or k x p for "all"), into `out` when given."""
        k = Xt.shape[0]
        p = len(model._m)
        if out is None:
            out = torch.empty((k, p) if route == "all" else (k,), dtype=torch.float64, device=self.device)
        r = torch.empty(k, dtype=torch.int32, device=self.device) if want_route else None
        self._check(self.lib.krr_predict(self.h, _stream(self.device), model.handle, _ptr(Xt), _dtype_code(Xt), k,
                                         ROUTE[route], _ptr(out), _ptr(r)))
        return (out, r) if want_route else out

    def predict_noalloc(self, model, Xt, yhat, route="nearest", route_out=None):
        """krr_predict_noalloc into caller-allocated outputs: yhat FP64 (k, or
        k x p for "all"), route_out int32[k] or None."""
        self._check(self.lib.krr_predict_noalloc(self.h, _stream(self.device), model.handle, _ptr(Xt),
                                                 _dtype_code(Xt), Xt.shape[0], ROUTE[route], _ptr(yhat),
                                                 _ptr(route_out)))
        return yhat

    def select(self, models, Xv, yv, route="nearest"):
        k = Xv.shape[0]
        hs = (ctypes.c_void_p * len(models))(*[m.handle for m in models])
        mse = (ctypes.c_double * len(models))()
        best = ctypes.c_int32(-1)
        self._check(self.lib.krr_select(self.h, _stream(self.device), hs, len(models), _ptr(Xv), _ptr(yv),
                                        _dtype_code(Xv), k, ROUTE[route], mse, ctypes.byref(best)))
        return list(mse), best.value

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request server around a resident model (see the
    serving section of include/krr.h).  Requests carry host numpy arrays;
    the arrays are kept referenced here until the request is waited for."""

    def __init__(self, ctx, model, predict_workers=2, fit_workers=1, max_batch_fits=16,
                 max_batch_points=16384, hbm_budget=0):
        self.ctx = ctx
        self.lib = ctx.lib
        self.model = model
        cfg = ServerConfig(int(predict_workers), int(fit_workers), int(max_batch_fits), 0,
                           int(max_batch_points), int(hbm_budget))
        h = ctypes.c_void_p()
        st = self.lib.krr_server_create(ctx.h, model.handle, ctypes.byref(cfg), ctypes.byref(h))
        if st != KRR_OK:
            raise KrrError(st, "krr_server_create failed: " + ctx.lib.krr_last_error(ctx.h).decode())
        self.h = h
        self._keep = {}

    def _check(self, st):
        if st != KRR_OK:
            raise KrrError(st, self.lib.krr_server_last_error(self.h).decode())

    def submit_predict(self, Xq):
        """Xq: host float32 k x d.  Returns a ticket."""
        import numpy as np
        Xq = np.ascontiguousarray(Xq, dtype=np.float32)
        out = np.empty(Xq.shape[0], dtype=np.float64)
        t = ctypes.c_int64(0)
        self._check(self.lib.krr_server_submit_predict(self.h, Xq.ctypes.data, Xq.shape[0], out.ctypes.data,
                                                        ctypes.byref(t)))
        self._keep[t.value] = (Xq, out)
        return t.value

    def submit_fit(self, X, y, params):
        """X: host float32 m x d, y: host float32 m, params: Params.  Returns a ticket."""
        import numpy as np
        X = np.ascontiguousarray(X, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        out = np.empty(X.shape[0], dtype=np.float64)
        cp = params.to_c()
        t = ctypes.c_int64(0)
        self._check(self.lib.krr_server_submit_fit(self.h, X.ctypes.data, y.ctypes.data, X.shape[0], X.shape[1],
                                                    ctypes.byref(cp), out.ctypes.data, ctypes.byref(t)))
        self._keep[t.value] = (X, y, out)
        return t.value

    def wait(self, ticket):
        """Block until the request is done.  Returns (result array, info dict);
        a failed request raises KrrError."""
        info = RequestInfo()
        st = self.lib.krr_server_wait(self.h, int(ticket), ctypes.byref(info))
        keep = self._keep.pop(int(ticket), None)
        if st != KRR_OK:
            raise KrrError(st, self.lib.krr_server_last_error(self.h).decode())
        return keep[-1], {f: getattr(info, f) for f, _ in RequestInfo._fields_}

    def stats(self, reset=False):
        s = ServeStats()
        self._check(self.lib.krr_server_stats(self.h, int(bool(reset)), ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in ServeStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.lib.krr_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def exported_symbols(header=None):
    """Function names declared in include/krr.h."""
    import re
    header = header or os.path.join(os.path.dirname(_HERE), "include", "krr.h")
    src = open(header).read()
    return sorted(set(re.findall(r"^\s*(?:krr_status|const char\*)\s+(krr_\w+)\s*\(", src, re.M)))
