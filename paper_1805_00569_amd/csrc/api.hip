// C ABI entry points (declared in include/krr.h): argument validation, the
// context's workspace pool and budget accounting, and error translation.  No
// C++ exception crosses the ABI.
#include "common.hpp"

#include <cstring>

namespace krr {

// Released model blocks are kept for reuse by later models of the same
// rounded size, so fits repeated with the same shapes allocate nothing; the
// cache holds at most MODEL_CACHE_BLOCKS blocks, is emptied before an
// allocation would exceed the budget, and is freed with the context.  Its
// bytes count as held by the context.
constexpr size_t MODEL_CACHE_BLOCKS = 64;

void drain(krr_ctx ctx) {
  if (ctx->capturing) fail(KRR_ESTATE, "synchronisation inside a graph capture");
  if (ctx->in_call) KRR_HIP(hipStreamSynchronize(ctx->cur_stream));
  for (auto& m : ctx->marks) KRR_HIP(hipEventSynchronize(m.second));
}

StreamScope::StreamScope(krr_ctx c, hipStream_t s) : ctx(c) {
  ctx->cur_stream = s;
  ctx->in_call = true;
}

StreamScope::~StreamScope() {
  ctx->in_call = false;
  hipEvent_t ev = nullptr;
  for (auto& m : ctx->marks)
    if (m.first == ctx->cur_stream) ev = m.second;
  if (ev == nullptr) {
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipStreamSynchronize(ctx->cur_stream);   // no event: nothing of this call may stay queued
      return;
    }
    ctx->marks.emplace_back(ctx->cur_stream, ev);
  }
  if (hipEventRecord(ev, ctx->cur_stream) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(ctx->cur_stream);
  }
}

static void drop_model_cache(krr_ctx ctx) {
  if (ctx->model_cache.empty()) return;
  drain(ctx);
  for (auto& kv : ctx->model_cache) (void)hipFree(kv.second);
  ctx->model_cache.clear();
  ctx->cache_bytes = 0;
}

static void charge(krr_ctx ctx, size_t add) {
  if (ctx->budget == 0) return;
  if (ctx->ws_bytes + ctx->model_bytes + ctx->cache_bytes + add > ctx->budget) drop_model_cache(ctx);
  if (ctx->ws_bytes + ctx->model_bytes + add > ctx->budget)
    fail(KRR_EBUDGET, "HBM budget exceeded: holding " + std::to_string(ctx->ws_bytes + ctx->model_bytes) +
                          " bytes, need " + std::to_string(add) + " more, budget " + std::to_string(ctx->budget));
}

void* ws_get(krr_ctx ctx, const std::string& name, size_t bytes) {
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  DevBuf& b = ctx->ws[name];
  if (b.bytes >= bytes) return b.ptr;
  if (ctx->capturing) fail(KRR_ESTATE, "workspace '" + name + "' would grow inside a graph capture");
  ctx->ws_epoch += 1;
  const size_t old = b.bytes;
  charge(ctx, bytes - old);
  for (int i = 0; i < krr_ctx_s::PersistCache::kSlots; ++i)   // a cached plan is gone with its buffer
    if (name == "persist_plan" + std::to_string(i)) ctx->persist.slot[i] = krr_ctx_s::PersistPlan{};
  if (b.ptr != nullptr) {
    drain(ctx);  // the old buffer may still be in use by this context's queued work
    KRR_HIP(hipFree(b.ptr));
    b.ptr = nullptr;
    b.bytes = 0;
    ctx->ws_bytes -= old;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    fail(KRR_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed (" + name + ")");
  }
  b.ptr = p;
  b.bytes = bytes;
  ctx->ws_bytes += bytes;
  return p;
}

void* model_alloc(krr_ctx ctx, size_t bytes) {
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  const auto it = ctx->model_cache.find(bytes);
  if (it != ctx->model_cache.end()) {
    void* p = it->second;
    ctx->model_cache.erase(it);
    ctx->cache_bytes -= bytes;
    ctx->model_bytes += bytes;
    return p;
  }
  charge(ctx, bytes);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    fail(KRR_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed (model)");
  }
  ctx->model_bytes += bytes;
  return p;
}

// The caller guarantees that no queued work still uses the block.
void model_release(krr_ctx ctx, void* p, size_t bytes) {
  if (p == nullptr) return;
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  ctx->model_bytes -= std::min(ctx->model_bytes, bytes);
  if (ctx->model_cache.size() < MODEL_CACHE_BLOCKS) {
    ctx->model_cache.emplace(bytes, p);
    ctx->cache_bytes += bytes;
  } else {
    (void)hipFree(p);
  }
}

void graph_drop_all(krr_ctx ctx) {
  if (ctx->graph_cache.empty() && ctx->graph_seen.empty()) return;
  drain(ctx);
  for (auto& kv : ctx->graph_cache)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  ctx->graph_cache.clear();
  ctx->graph_seen.clear();
}

void ws_release_all(krr_ctx ctx) {
  drain(ctx);
  for (auto& kv : ctx->ws)
    if (kv.second.ptr != nullptr) {
      KRR_HIP(hipFree(kv.second.ptr));
      ctx->ws_bytes -= kv.second.bytes;
    }
  ctx->ws.clear();
  ctx->ws_epoch += 1;
  for (auto& pl : ctx->persist.slot) pl = krr_ctx_s::PersistPlan{};   // the plans lived in the workspace
}

void* pinned_named(krr_ctx ctx, const std::string& name, size_t bytes) {
  auto& b = ctx->pinned_bufs[name];
  if (b.second >= bytes) return b.first;
  if (b.first != nullptr) {
    drain(ctx);
    (void)hipHostFree(b.first);
    b.first = nullptr;
    b.second = 0;
  }
  bytes = std::max(bytes, size_t(1) << 16);
  KRR_HIP(hipHostMalloc(&b.first, bytes, hipHostMallocDefault));
  b.second = bytes;
  return b.first;
}

void* pinned_get(krr_ctx ctx, size_t bytes) {
  if (ctx->pinned_bytes >= bytes) return ctx->pinned;
  if (ctx->pinned != nullptr) {
    drain(ctx);
    (void)hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
  }
  bytes = std::max(bytes, size_t(1) << 16);
  KRR_HIP(hipHostMalloc(&ctx->pinned, bytes, hipHostMallocDefault));
  ctx->pinned_bytes = bytes;
  return ctx->pinned;
}

void check_launch(krr_ctx ctx, hipStream_t s, const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) fail(KRR_EDEVICE, std::string("launch of ") + what + ": " + hipGetErrorString(e));
  if (ctx->sync_check && !ctx->capturing) {
    const hipError_t e2 = hipStreamSynchronize(s);
    if (e2 != hipSuccess) fail(KRR_EDEVICE, std::string("after ") + what + ": " + hipGetErrorString(e2));
  }
}

static hipEvent_t ev_get(krr_ctx ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

KernelTimer::KernelTimer(krr_ctx c, hipStream_t st, const char* name, double f, int major, double by)
    : ctx(c), s(st), cls(name), flops(f), bytes(by) {
  if (ctx->timing == 0 || (ctx->timing == 1 && !major) || ctx->noalloc || ctx->capturing) return;
  a = ev_get(ctx);
  b = ev_get(ctx);
  if (a == nullptr || b == nullptr || hipEventRecord(a, s) != hipSuccess) {
    a = b = nullptr;
  }
}

KernelTimer::~KernelTimer() {
  if (a == nullptr) return;
  if (hipEventRecord(b, s) == hipSuccess) ctx->pending.push_back({cls, a, b, flops, bytes});
}

// Adds the pending launches to the per-class totals: summed durations, and
// the time covered by the union of a class's launch intervals (all positions
// relative to the first pending launch's start event); the classes named
// "chol_*" are also united into the class "chol" (the factorisation).
static void collect_timing(krr_ctx ctx) {
  KRR_HIP(hipDeviceSynchronize());
  std::map<std::string, std::vector<std::pair<float, float>>> iv;
  const hipEvent_t ref = ctx->pending.empty() ? nullptr : ctx->pending.front().a;
  for (auto& p : ctx->pending) {
    float ms = 0.f, t0 = 0.f, t1 = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      krr_timing_agg& g = ctx->timing_agg[p.cls];
      g.count += 1;
      g.ms += ms;
      g.flops += p.flops;
      g.bytes += p.bytes;
      if (hipEventElapsedTime(&t0, ref, p.a) == hipSuccess && hipEventElapsedTime(&t1, ref, p.b) == hipSuccess) {
        iv[p.cls].emplace_back(t0, t1);
        if (std::strncmp(p.cls, "chol_", 5) == 0) iv["chol"].emplace_back(t0, t1);
      }
    }
  }
  for (auto& kv : iv) {
    auto& v = kv.second;
    std::sort(v.begin(), v.end());
    double busy = 0.0, lo = v.front().first, hi = v.front().second;
    for (const auto& x : v) {
      if (x.first > hi) {
        busy += hi - lo;
        lo = x.first;
        hi = x.second;
      } else {
        hi = std::max(hi, (double)x.second);
      }
    }
    busy += hi - lo;
    ctx->timing_agg[kv.first].busy_ms += busy;
  }
  for (auto& p : ctx->pending) {
    ctx->ev_pool.push_back(p.a);
    ctx->ev_pool.push_back(p.b);
  }
  ctx->pending.clear();
}

struct DeviceGuard {
  int old = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&old) != hipSuccess) old = -1;
    KRR_HIP(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    if (old >= 0) (void)hipSetDevice(old);
  }
};

template <typename F>
static krr_status guarded(krr_ctx ctx, F&& f) {
  if (ctx == nullptr) return KRR_EINVAL;
  try {
    DeviceGuard g(ctx->device);
    f();
    ctx->last_error.clear();
    return KRR_OK;
  } catch (const Error& e) {
    ctx->last_error = e.msg;
    return e.status;
  } catch (const std::exception& e) {
    ctx->last_error = e.what();
    return KRR_EDEVICE;
  } catch (...) {
    ctx->last_error = "unknown error";
    return KRR_EDEVICE;
  }
}

krr_status run_guarded(krr_ctx ctx, const std::function<void()>& f) { return guarded(ctx, f); }

}  // namespace krr

krr_part_data::~krr_part_data() {
  if (ctx != nullptr) {
    krr::model_release(ctx, base, bytes);
    ctx->n_datas -= 1;
  }
}

using namespace krr;

extern "C" {

krr_status krr_create(int device, size_t hbm_budget_bytes, krr_ctx* out) {
  if (out == nullptr) return KRR_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return KRR_EINVAL;
  try {   // library set-up on this device: the no-allocation scratch address
    DeviceGuard g(device);
    noalloc_scratch_init(device);
  } catch (const Error& e) {
    return e.status;
  }
  krr_ctx c = new (std::nothrow) krr_ctx_s();
  if (c == nullptr) return KRR_ENOMEM;
  c->device = device;
  c->budget = hbm_budget_bytes;
  tune_load(c);
  {
    DeviceGuard g(device);
    bool ok = true;
    for (auto& st : c->side) ok = ok && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    for (auto& ev : c->side_ev) ok = ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      for (auto ev : c->side_ev)
        if (ev) (void)hipEventDestroy(ev);
      for (auto st : c->side)
        if (st) (void)hipStreamDestroy(st);
      delete c;
      return KRR_EDEVICE;
    }
  }
  *out = c;
  return KRR_OK;
}

krr_status krr_destroy(krr_ctx ctx) {
  if (ctx == nullptr) return KRR_EINVAL;
  if (ctx->n_models > 0 || ctx->n_datas > 0) {
    ctx->last_error = "models still alive on this context";
    return KRR_ESTATE;
  }
  (void)hipSetDevice(ctx->device);
  try {
    drain(ctx);
  } catch (const Error&) {
    (void)hipDeviceSynchronize();
  }
  for (auto& kv : ctx->graph_cache)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  for (auto& m : ctx->marks) (void)hipEventDestroy(m.second);
  ctx->marks.clear();
  for (auto& kv : ctx->ws)
    if (kv.second.ptr) (void)hipFree(kv.second.ptr);
  drop_model_cache(ctx);
  for (auto& p : ctx->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  for (auto& kv : ctx->pinned_bufs)
    if (kv.second.first) (void)hipHostFree(kv.second.first);
  for (auto ev : ctx->side_ev)
    if (ev) (void)hipEventDestroy(ev);
  for (auto st : ctx->side)
    if (st) (void)hipStreamDestroy(st);
  delete ctx;
  return KRR_OK;
}

const char* krr_last_error(krr_ctx ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

krr_status krr_set_option(krr_ctx ctx, int32_t option, int64_t value) {
  return guarded(ctx, [&] {
    switch (option) {
      case KRR_OPT_PANEL_TILES:
        KRR_REQUIRE(value >= 0 && value <= 64, "panel width must be 1..64 tiles (0: the precision's default)");
        ctx->panel_tiles = (int)value;
        break;
      case KRR_OPT_SERIAL_FIT:
        ctx->serial_fit = value ? 1 : 0;
        break;
      case KRR_OPT_SYNC_CHECK:
        ctx->sync_check = value ? 1 : 0;
        break;
      case KRR_OPT_PERSISTENT:
        ctx->persistent = value ? 1 : 0;
        break;
      case KRR_OPT_FACTOR_STREAMS:
        KRR_REQUIRE(value >= 1 && value <= krr_ctx_s::kMaxFactorStreams, "factor streams must be 1..4");
        ctx->factor_streams = (int)value;
        break;
      case KRR_OPT_AUTOTUNE:
        ctx->autotune = value ? 1 : 0;
        break;
      case KRR_OPT_COLUMN_PAIRS:
        ctx->column_pairs = value ? 1 : 0;
        break;
      case KRR_OPT_GRAPHS:
        graph_drop_all(ctx);
        ctx->graphs = value ? 1 : 0;
        break;
      case KRR_OPT_PERSIST_WAIT_MS:
        KRR_REQUIRE(value >= 0, "the wait limit must be >= 0 ms");
        ctx->persist_wait_ms = value;
        break;
      case KRR_OPT_TIMING:
        KRR_REQUIRE(value >= 0 && value <= 2, "timing must be 0, 1 or 2");
        collect_timing(ctx);
        ctx->timing_agg.clear();
        ctx->timing = (int)value;
        break;
      default:
        fail(KRR_EINVAL, "unknown option");
    }
  });
}

krr_status krr_timing_report(krr_ctx ctx, char* buf, size_t cap, size_t* needed) {
  return guarded(ctx, [&] {
    collect_timing(ctx);
    std::string js = "{";
    bool first = true;
    char tmp[256];
    for (auto& kv : ctx->timing_agg) {
      std::snprintf(tmp, sizeof(tmp),
                    "%s\"%s\": {\"count\": %lld, \"ms\": %.6f, \"busy_ms\": %.6f, \"flops\": %.6e, \"bytes\": %.6e}",
                    first ? "" : ", ", kv.first.c_str(), (long long)kv.second.count, kv.second.ms, kv.second.busy_ms,
                    kv.second.flops, kv.second.bytes);
      js += tmp;
      first = false;
    }
    js += "}";
    if (needed != nullptr) *needed = js.size() + 1;
    if (buf != nullptr && cap > 0) {
      const size_t nb = std::min(cap - 1, js.size());
      std::memcpy(buf, js.data(), nb);
      buf[nb] = 0;
      ctx->timing_agg.clear();
    }
  });
}

krr_status krr_graph_counts(krr_ctx ctx, int64_t* captured, int64_t* replayed) {
  if (ctx == nullptr || captured == nullptr || replayed == nullptr) return KRR_EINVAL;
  *captured = ctx->graph_captures;
  *replayed = ctx->graph_replays;
  return KRR_OK;
}

krr_status krr_memory_in_use(krr_ctx ctx, size_t* bytes) {
  if (ctx == nullptr || bytes == nullptr) return KRR_EINVAL;
  *bytes = ctx->ws_bytes + ctx->model_bytes + ctx->cache_bytes;
  return KRR_OK;
}

krr_status krr_csr_to_dense(krr_ctx ctx, hipStream_t stream, const int64_t* indptr, const int32_t* indices,
                            const void* values, int32_t dtype, int64_t n, int32_t d, int64_t nnz, void* X) {
  return guarded(ctx, [&] {
    KRR_REQUIRE(indptr && X, "null pointer argument");
    KRR_REQUIRE(nnz == 0 || (indices && values), "null pointer argument");
    KRR_REQUIRE(dtype == KRR_F32 || dtype == KRR_F64, "dtype must be KRR_F32 or KRR_F64");
    KRR_REQUIRE(n >= 1 && d >= 1 && nnz >= 0, "n and d must be >= 1, nnz >= 0");
    KRR_REQUIRE(n < (int64_t(1) << 31) - 1, "n must fit in int32");
    StreamScope ss(ctx, stream);
    run_csr_to_dense(ctx, stream, indptr, indices, values, dtype, n, d, nnz, X);
  });
}

krr_status krr_partition(krr_ctx ctx, hipStream_t stream, const void* X, int32_t dtype, int64_t n, int32_t d,
                         int32_t p, int32_t method, int32_t lloyd_iters, uint64_t seed, double* centroids,
                         int32_t* assign, int64_t* sizes) {
  return guarded(ctx, [&] {
    KRR_REQUIRE(X && centroids && assign && sizes, "null pointer argument");
    KRR_REQUIRE(dtype == KRR_F32 || dtype == KRR_F64, "dtype must be KRR_F32 or KRR_F64");
    KRR_REQUIRE(n >= 1 && d >= 1, "n and d must be >= 1");
    KRR_REQUIRE(n < (int64_t(1) << 31) - 1, "n must fit in int32");
    KRR_REQUIRE(p >= 1 && p <= n && p <= 1024, "p must be in [1, min(n, 1024)]");
    KRR_REQUIRE(method == KRR_PART_KMEANS || method == KRR_PART_KBALANCE || method == KRR_PART_GIVEN ||
                    method == KRR_PART_RANDOM || method == KRR_PART_KBALANCE_APPROX,
                "unknown partition method");
    KRR_REQUIRE(lloyd_iters >= 0 && lloyd_iters <= 100000, "lloyd_iters out of range");
    StreamScope ss(ctx, stream);
    run_partition(ctx, stream, X, dtype, n, d, p, method, lloyd_iters, seed, centroids, assign, sizes);
  });
}

krr_status krr_fit(krr_ctx ctx, hipStream_t stream, const void* X, const void* y, int32_t dtype, int64_t n,
                   int32_t d, const int32_t* assign, const double* centroids, int32_t p,
                   const krr_fit_params* params, int32_t n_params, krr_model* models_out,
                   krr_part_info* info_out) {
  krr_status st = KRR_OK;
  krr_status g = guarded(ctx, [&] {
    KRR_REQUIRE(X && y && assign && centroids && params && models_out && info_out, "null pointer argument");
    KRR_REQUIRE(dtype == KRR_F32 || dtype == KRR_F64, "dtype must be KRR_F32 or KRR_F64");
    KRR_REQUIRE(n >= 1 && d >= 1 && n < (int64_t(1) << 31) - 1, "bad n or d");
    KRR_REQUIRE(p >= 1 && p <= n && p <= 1024, "p must be in [1, min(n, 1024)]");
    KRR_REQUIRE(n_params >= 1 && n_params <= 4096, "n_params must be in [1, 4096]");
    KRR_REQUIRE((int64_t)n_params * p <= 65535, "n_params * p must be <= 65535 (systems per batch)");
    for (int q = 0; q < n_params; ++q) {
      const krr_fit_params& P = params[q];
      KRR_REQUIRE(P.kernel == KRR_KERNEL_GAUSSIAN || P.kernel == KRR_KERNEL_LINEAR ||
                      P.kernel == KRR_KERNEL_POLYNOMIAL || P.kernel == KRR_KERNEL_SIGMOID,
                  "unknown kernel");
      KRR_REQUIRE(P.kernel != KRR_KERNEL_GAUSSIAN || P.sigma > 0.0, "sigma must be > 0");
      KRR_REQUIRE((P.kernel != KRR_KERNEL_POLYNOMIAL && P.kernel != KRR_KERNEL_SIGMOID) ||
                      (std::isfinite(P.kernel_a) && std::isfinite(P.kernel_r)),
                  "kernel_a and kernel_r must be finite");
      KRR_REQUIRE(P.kernel != KRR_KERNEL_POLYNOMIAL || (P.kernel_degree >= 1 && P.kernel_degree <= 64),
                  "kernel_degree must be in [1, 64]");
      KRR_REQUIRE(std::isfinite(P.lambda), "lambda must be finite");
      KRR_REQUIRE(P.prec == KRR_PREC_FP64 || P.prec == KRR_PREC_FP32 || P.prec == KRR_PREC_MIXED,
                  "unknown precision");
      KRR_REQUIRE(P.prec == params[0].prec, "all settings of one call must share the precision");
      KRR_REQUIRE(P.max_refine >= 0 && P.max_refine <= 1000, "max_refine out of range");
      KRR_REQUIRE(P.indefinite == 0 || P.indefinite == 1, "indefinite must be 0 or 1");
    }
    for (int q = 0; q < n_params; ++q) models_out[q] = nullptr;
    StreamScope ss(ctx, stream);
    run_fit(ctx, stream, X, y, dtype, n, d, assign, centroids, p, params, n_params, models_out, info_out);
    for (int q = 0; q < n_params * p; ++q) {
      if (info_out[q].status == KRR_ENOTSPD) st = KRR_ENOTSPD;
      else if (info_out[q].status == KRR_ENOCONV && st == KRR_OK) st = KRR_ENOCONV;
    }
  });
  if (g != KRR_OK) return g;
  if (st != KRR_OK) ctx->last_error = "one or more systems failed; see info_out";
  return st;
}

krr_status krr_predict(krr_ctx ctx, hipStream_t stream, krr_model model, const void* Xt, int32_t dtype, int64_t k,
                       int32_t route, double* yhat, int32_t* route_out) {
  return guarded(ctx, [&] {
    KRR_REQUIRE(model && Xt && yhat, "null pointer argument");
    KRR_REQUIRE(model->ctx == ctx, "model belongs to another context");
    KRR_REQUIRE(dtype == KRR_F32 || dtype == KRR_F64, "dtype must be KRR_F32 or KRR_F64");
    KRR_REQUIRE(k >= 1 && k < (int64_t(1) << 31) - 1, "k must be >= 1");
    KRR_REQUIRE(route == KRR_ROUTE_NEAREST || route == KRR_ROUTE_AVERAGE || route == KRR_ROUTE_ALL,
                "unknown route");
    StreamScope ss(ctx, stream);
    run_predict(ctx, stream, model, Xt, dtype, k, route, yhat, route_out);
  });
}

krr_status krr_predict_noalloc(krr_ctx ctx, hipStream_t stream, krr_model model, const void* Xt, int32_t dtype,
                               int64_t k, int32_t route, double* yhat, int32_t* route_out) {
  return guarded(ctx, [&] {
    KRR_REQUIRE(model && Xt && yhat, "null pointer argument");
    KRR_REQUIRE(model->ctx == ctx, "model belongs to another context");
    KRR_REQUIRE(dtype == KRR_F32 || dtype == KRR_F64, "dtype must be KRR_F32 or KRR_F64");
    KRR_REQUIRE(k >= 1 && k < (int64_t(1) << 31) - 1, "k must be >= 1");
    KRR_REQUIRE(route == KRR_ROUTE_NEAREST || route == KRR_ROUTE_AVERAGE || route == KRR_ROUTE_ALL,
                "unknown route");
    run_predict_noalloc(ctx, stream, model, Xt, dtype, k, route, yhat, route_out);
  });
}

krr_status krr_select(krr_ctx ctx, hipStream_t stream, const krr_model* models, int32_t n_models, const void* Xv,
                      const void* yv, int32_t dtype, int64_t k, int32_t route, double* mse_out,
                      int32_t* best_out) {
  return guarded(ctx, [&] {
    KRR_REQUIRE(models && Xv && yv && mse_out && best_out, "null pointer argument");
    KRR_REQUIRE(n_models >= 1, "n_models must be >= 1");
    for (int i = 0; i < n_models; ++i) KRR_REQUIRE(models[i] && models[i]->ctx == ctx, "bad model handle");
    KRR_REQUIRE(dtype == KRR_F32 || dtype == KRR_F64, "dtype must be KRR_F32 or KRR_F64");
    KRR_REQUIRE(k >= 1 && k < (int64_t(1) << 31) - 1, "k must be >= 1");
    KRR_REQUIRE(route == KRR_ROUTE_NEAREST || route == KRR_ROUTE_AVERAGE || route == KRR_ROUTE_LABEL,
                "route must be NEAREST, AVERAGE or LABEL");
    StreamScope ss(ctx, stream);
    run_select(ctx, stream, models, n_models, Xv, yv, dtype, k, route, mse_out, best_out);
  });
}

krr_status krr_model_alpha(krr_ctx ctx, hipStream_t stream, krr_model model, int32_t j, double* alpha,
                           int64_t* m) {
  return guarded(ctx, [&] {
    KRR_REQUIRE(model && alpha && m, "null pointer argument");
    KRR_REQUIRE(model->ctx == ctx, "model belongs to another context");
    KRR_REQUIRE(j >= 0 && j < model->data->p, "partition index out of range");
    const int64_t mj = model->data->offsets[j + 1] - model->data->offsets[j];
    *m = mj;
    StreamScope ss(ctx, stream);
    if (mj > 0)
      KRR_HIP(hipMemcpyAsync(alpha, model->alpha + model->voff[j], (size_t)mj * 8, hipMemcpyDeviceToDevice,
                             stream));
  });
}

krr_status krr_model_free(krr_model model) {
  if (model == nullptr) return KRR_OK;
  krr_ctx ctx = model->ctx;
  (void)hipSetDevice(ctx->device);
  // only this context's queued work can still read the model (every entry
  // point checks that a model belongs to the calling context): wait for that,
  // not for the whole device
  try {
    drain(ctx);
  } catch (const Error&) {
    (void)hipDeviceSynchronize();
  }
  model_release(ctx, model->alpha, model->bytes);
  model->data.reset();
  ctx->n_models -= 1;
  delete model;
  return KRR_OK;
}

}  // extern "C"
