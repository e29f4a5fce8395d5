// Serving runtime: continuous batching of predict and fit requests around a
// resident partitioned model.  Predict requests are routed to the model of
// the nearest partition centre and evaluated with Eq. 7 (KKRR2 / BKRR2,
// Section 4.2, Algorithm 5); fit requests are independent problems
// (K + lambda I) alpha = y (Eq. 6, Algorithm 1) that are solved together as
// one ragged batch, one partition per request.
//
// Threads: every worker owns a context (workspace pool, pinned staging) and a
// stream, so batches of different workers overlap on the device; the request
// queues, the admission budget and the statistics are shared under one
// mutex.  No worker ever synchronises the device: each waits on its own
// stream only.
//
// Device memory: the HBM budget is split between the workers' contexts, so
// the memory they hold together never exceeds it.  Each predict worker gets
// twice the estimate of a full predict batch; the fit workers share the rest
// equally.  A fit request larger than one fit worker's share is rejected at
// submission, a fit batch is only formed within one share, and a fit worker
// whose retained workspace plus its next batch would exceed its share frees
// its workspace first (its stream is idle between batches).
#include "common.hpp"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

namespace krr {
namespace {

using Clock = std::chrono::steady_clock;

double now_ms() {
  return std::chrono::duration<double, std::milli>(Clock::now().time_since_epoch()).count();
}

enum { KIND_PREDICT = 0, KIND_FIT = 1 };

struct Request {
  int64_t ticket = 0;
  int kind = KIND_PREDICT;
  const float* X = nullptr;   // predict: k x d queries; fit: m x d points
  const float* y = nullptr;   // fit labels
  double* out = nullptr;      // predict: yhat; fit: alpha
  int64_t rows = 0;
  int32_t d = 0;
  krr_fit_params params{};
  size_t need = 0;            // admission estimate, bytes
  double t_submit = 0, t_start = 0, t_done = 0;
  int32_t status = KRR_OK;
  int32_t batch_requests = 0;
  bool done = false;
};

struct Worker {
  int kind = KIND_PREDICT;
  krr_ctx ctx = nullptr;
  size_t share = 0;       // device memory the worker's context may hold (0 = no cap)
  size_t held = 0;        // device memory its context held after its last batch
  hipStream_t stream = nullptr;
  std::thread thread;
  void* host = nullptr;   // pinned staging owned by the worker (the context's own
  size_t host_bytes = 0;  // pinned buffer is used inside the fit and predict paths)
};

// Device memory a fit of m points in d dimensions holds while it runs: the
// packed lower-triangle factor storage, the inverse diagonal blocks, the FP64
// copy and BF16 operand packs of the mixed path, vectors and staged inputs.
size_t fit_need(int64_t m, int d, int prec, int panel_tiles) {
  const int64_t T = ceil_div(m, NB);
  const size_t tiles = (size_t)(T * (T + 1) / 2);
  const size_t aes = prec == KRR_PREC_FP64 ? 8 : 4;
  size_t b = tiles * NB * NB * aes + (size_t)T * NB * NB * aes;
  if (prec == KRR_PREC_MIXED) {
    b += tiles * NB * NB * 8;                                   // FP64 copy for the residual
    b += (size_t)T * 4 * 2 * panel_tiles * 512 * 2;             // BF16 operand packs
    b += (size_t)T * T * NB * 8;                                // residual partials
  }
  b += (size_t)T * NB * 8 * 6 + (size_t)m * d * 4 * 3 + (size_t)m * 24;
  return b + (size_t(1) << 20);
}

size_t predict_need(int64_t k, int d) { return (size_t)k * ((size_t)d * 4 * 2 + 64) + (size_t(1) << 20); }

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  int64_t idx = (int64_t)std::ceil(q * (double)v.size()) - 1;
  idx = std::max<int64_t>(0, std::min<int64_t>(idx, (int64_t)v.size() - 1));
  return v[idx];
}

bool same_setting(const krr_fit_params& a, const krr_fit_params& b) {
  return a.sigma == b.sigma && a.lambda == b.lambda && a.kernel == b.kernel && a.prec == b.prec &&
         a.refine_tol == b.refine_tol && a.max_refine == b.max_refine && a.lambda_times_m == b.lambda_times_m &&
         a.kernel_a == b.kernel_a && a.kernel_r == b.kernel_r && a.kernel_degree == b.kernel_degree;
}

}  // namespace
}  // namespace krr

struct krr_server_s {
  krr_model model = nullptr;
  int device = 0;
  int32_t d_model = 0;
  krr_server_config cfg{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<krr::Request*> queue[2];
  std::unordered_map<int64_t, krr::Request*> requests;
  int64_t next_ticket = 1;
  size_t inflight = 0;
  size_t fit_share = 0;       // per fit worker (0 = no cap)
  size_t max_held = 0;        // peak device memory held by all worker contexts together
  bool stopping = false;
  std::vector<krr::Worker*> workers;
  std::string last_error;
  // statistics since creation or the last reset
  int64_t n_done[2] = {0, 0};
  int64_t points = 0, fit_rows = 0, batches[2] = {0, 0}, failed = 0;
  size_t max_inflight = 0;
  std::vector<double> latency[2];
  double t_first = -1.0, t_last = -1.0;
};

namespace krr {
namespace {

void grow_host(Worker* W, size_t bytes) {
  if (W->host_bytes >= bytes) return;
  if (W->host != nullptr) (void)hipHostFree(W->host);   // the worker's stream is idle here
  W->host = nullptr;
  W->host_bytes = 0;
  bytes = std::max(bytes, size_t(1) << 20);
  KRR_HIP(hipHostMalloc(&W->host, bytes, hipHostMallocDefault));
  W->host_bytes = bytes;
}

// Oldest requests of the worker's kind that fit the caps and the budget.
// Called with the server lock held; the head is admissible.
std::vector<Request*> take_batch(krr_server S, int kind, size_t& need) {
  std::vector<Request*> b;
  std::deque<Request*>& q = S->queue[kind];
  const size_t budget = S->cfg.hbm_budget_bytes;
  auto fits_budget = [&](size_t add) {
    return budget == 0 ||
           (S->inflight + need + add <= budget && (kind == KIND_PREDICT || need + add <= S->fit_share));
  };
  if (kind == KIND_PREDICT) {
    int64_t pts = 0;
    while (!q.empty()) {
      Request* r = q.front();
      if (!b.empty() && (pts + r->rows > S->cfg.max_batch_points || !fits_budget(r->need))) break;
      b.push_back(r);
      pts += r->rows;
      need += r->need;
      q.pop_front();
    }
  } else {
    Request* head = q.front();
    int64_t rows = 0;
    for (auto it = q.begin(); it != q.end() && (int)b.size() < S->cfg.max_batch_fits;) {
      Request* r = *it;
      const bool match = r->d == head->d && same_setting(r->params, head->params);
      if (match && (b.empty() || (fits_budget(r->need) && rows + r->rows < (int64_t(1) << 30)))) {
        b.push_back(r);
        rows += r->rows;
        need += r->need;
        it = q.erase(it);
      } else if (match) {
        break;   // keep the arrival order among requests of one setting
      } else {
        ++it;
      }
    }
  }
  return b;
}

bool admissible(krr_server S, int kind) {
  const std::deque<Request*>& q = S->queue[kind];
  if (q.empty()) return false;
  const size_t budget = S->cfg.hbm_budget_bytes;
  return budget == 0 || S->inflight + q.front()->need <= budget;
}

void set_error(krr_server S, const std::string& msg) {
  std::lock_guard<std::mutex> lk(S->mu);
  S->last_error = msg;
}

// One routed prediction for the concatenated queries of the batch.
int32_t run_predict_batch(krr_server S, Worker* W, const std::vector<Request*>& batch) {
  const int d = S->d_model;
  int64_t k = 0;
  for (Request* r : batch) k += r->rows;
  const size_t xb = ((size_t)k * d * 4 + 255) & ~size_t(255);
  grow_host(W, xb + (size_t)k * 8);
  char* h = (char*)W->host;
  int64_t o = 0;
  for (Request* r : batch) {
    std::memcpy(h + (size_t)o * d * 4, r->X, (size_t)r->rows * d * 4);
    o += r->rows;
  }
  StreamScope ss(W->ctx, W->stream);
  char* dv = (char*)ws_get(W->ctx, "serve_predict", xb + (size_t)k * 8);
  double* dy = (double*)(dv + xb);
  KRR_HIP(hipMemcpyAsync(dv, h, (size_t)k * d * 4, hipMemcpyHostToDevice, W->stream));
  run_predict(W->ctx, W->stream, S->model, dv, KRR_F32, k, KRR_ROUTE_NEAREST, dy, nullptr);
  double* hy = (double*)(h + xb);
  KRR_HIP(hipMemcpyAsync(hy, dy, (size_t)k * 8, hipMemcpyDeviceToHost, W->stream));
  KRR_HIP(hipStreamSynchronize(W->stream));
  o = 0;
  for (Request* r : batch) {
    std::memcpy(r->out, hy + o, (size_t)r->rows * 8);
    o += r->rows;
  }
  return KRR_OK;
}

// One ragged batch: request i is partition i of a fit with given assignment.
int32_t run_fit_batch(krr_server S, Worker* W, const std::vector<Request*>& batch) {
  (void)S;
  const int d = batch[0]->d;
  const int p = (int)batch.size();
  int64_t n = 0;
  for (Request* r : batch) n += r->rows;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t xb = al((size_t)n * d * 4), yb = al((size_t)n * 4), ab = al((size_t)n * 4),
               cb = al((size_t)p * d * 8);
  grow_host(W, xb + yb + ab + (size_t)n * 8);
  char* h = (char*)W->host;
  float* hx = (float*)h;
  float* hyv = (float*)(h + xb);
  int32_t* ha = (int32_t*)(h + xb + yb);
  int64_t o = 0;
  for (int i = 0; i < p; ++i) {
    Request* r = batch[i];
    std::memcpy(hx + (size_t)o * d, r->X, (size_t)r->rows * d * 4);
    std::memcpy(hyv + o, r->y, (size_t)r->rows * 4);
    for (int64_t t = 0; t < r->rows; ++t) ha[o + t] = i;
    o += r->rows;
  }
  StreamScope ss(W->ctx, W->stream);
  size_t need = 0;
  for (Request* r : batch) need += r->need;
  if (W->share != 0 && W->held + need > W->share) {
    ws_release_all(W->ctx);   // retained buffers of earlier batches would not leave room
    W->held = 0;
  }
  char* dv = (char*)ws_get(W->ctx, "serve_fit", xb + yb + ab + cb);
  KRR_HIP(hipMemcpyAsync(dv, h, xb + yb + ab, hipMemcpyHostToDevice, W->stream));
  double* dc = (double*)(dv + xb + yb + ab);
  KRR_HIP(hipMemsetAsync(dc, 0, (size_t)p * d * 8, W->stream));   // centres are not used for routing
  std::vector<krr_part_info> info(p);
  FitDirect fd;
  run_fit(W->ctx, W->stream, dv, dv + xb, KRR_F32, n, d, (const int32_t*)(dv + xb + yb), dc, p, &batch[0]->params,
          1, nullptr, info.data(), &fd);
  double* ho = (double*)(h + xb + yb + ab);   // inputs were consumed by the fit's synchronisation
  o = 0;
  for (int i = 0; i < p; ++i) {
    KRR_REQUIRE(fd.m[i] == batch[i]->rows, "partition size does not match the request");
    if (fd.m[i] > 0)
      KRR_HIP(hipMemcpyAsync(ho + o, fd.alpha + fd.v_off[i], (size_t)fd.m[i] * 8, hipMemcpyDeviceToHost, W->stream));
    o += fd.m[i];
  }
  KRR_HIP(hipStreamSynchronize(W->stream));
  o = 0;
  for (int i = 0; i < p; ++i) {
    std::memcpy(batch[i]->out, ho + o, (size_t)batch[i]->rows * 8);
    batch[i]->status = info[i].status;
    o += batch[i]->rows;
  }
  return KRR_OK;
}

void worker_loop(krr_server S, Worker* W) {
  (void)hipSetDevice(S->device);
  for (;;) {
    std::vector<Request*> batch;
    size_t need = 0;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return admissible(S, W->kind) || (S->stopping && S->queue[W->kind].empty()); });
      if (S->queue[W->kind].empty()) return;   // stopping, nothing left
      batch = take_batch(S, W->kind, need);
      S->inflight += need;
      S->max_inflight = std::max(S->max_inflight, S->inflight);
      const double t = now_ms();
      for (Request* r : batch) {
        r->t_start = t;
        r->batch_requests = (int32_t)batch.size();
        r->status = KRR_OK;
      }
    }
    int32_t st = KRR_OK;
    std::string msg;
    try {
      st = W->kind == KIND_PREDICT ? run_predict_batch(S, W, batch) : run_fit_batch(S, W, batch);
    } catch (const Error& e) {
      st = e.status;
      msg = e.msg;
    } catch (const std::exception& e) {
      st = KRR_EDEVICE;
      msg = e.what();
    }
    size_t held = 0;
    (void)krr_memory_in_use(W->ctx, &held);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      const double t = now_ms();
      S->inflight -= need;
      W->held = held;
      size_t tot = 0;
      for (Worker* V : S->workers) tot += V->held;
      S->max_held = std::max(S->max_held, tot);
      if (st != KRR_OK) S->last_error = msg;
      S->batches[W->kind] += 1;
      for (Request* r : batch) {
        if (st != KRR_OK) r->status = st;
        r->t_done = t;
        r->done = true;
        S->n_done[r->kind] += 1;
        if (r->kind == KIND_PREDICT) S->points += r->rows;
        else S->fit_rows += r->rows;
        if (r->status != KRR_OK) S->failed += 1;
        S->latency[r->kind].push_back(t - r->t_submit);
        S->t_last = std::max(S->t_last, t);
      }
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
}

krr_status submit(krr_server S, Request* r) {
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->stopping) {
    delete r;
    S->last_error = "server is stopping";
    return KRR_ESTATE;
  }
  r->ticket = S->next_ticket++;
  r->t_submit = now_ms();
  if (S->t_first < 0) S->t_first = r->t_submit;
  S->requests[r->ticket] = r;
  S->queue[r->kind].push_back(r);
  lk.unlock();
  S->cv_work.notify_all();
  return KRR_OK;
}

}  // namespace
}  // namespace krr

using namespace krr;

extern "C" {

krr_status krr_server_create(krr_ctx owner, krr_model model, const krr_server_config* cfg, krr_server* out) {
  if (out == nullptr) return KRR_EINVAL;
  *out = nullptr;
  if (owner == nullptr || model == nullptr || cfg == nullptr) return KRR_EINVAL;
  if (model->ctx != owner || !model->data) return KRR_EINVAL;
  if (cfg->predict_workers < 1 || cfg->predict_workers > 16 || cfg->fit_workers < 0 || cfg->fit_workers > 16 ||
      cfg->max_batch_fits < 1 || cfg->max_batch_fits > 1024 || cfg->max_batch_points < 1 || cfg->reserved != 0)
    return KRR_EINVAL;
  if (model->data->dtype != KRR_F32) {
    owner->last_error = "the resident model must be fitted on FP32 inputs (queries arrive as FP32)";
    return KRR_EINVAL;
  }
  krr_server S = new (std::nothrow) krr_server_s();
  if (S == nullptr) return KRR_ENOMEM;
  S->model = model;
  S->device = owner->device;
  S->d_model = model->data->d;
  S->cfg = *cfg;
  const int nw = cfg->predict_workers + cfg->fit_workers;
  // split of the budget between the workers' contexts
  size_t pshare = 0;
  if (cfg->hbm_budget_bytes != 0) {
    pshare = 2 * predict_need(cfg->max_batch_points, S->d_model);
    const size_t preserve = pshare * (size_t)cfg->predict_workers;
    if (preserve >= cfg->hbm_budget_bytes ||
        (cfg->fit_workers > 0 && (cfg->hbm_budget_bytes - preserve) / (size_t)cfg->fit_workers < (size_t(1) << 20))) {
      owner->last_error = "HBM budget of " + std::to_string(cfg->hbm_budget_bytes) +
                          " bytes leaves no room: the predict workers need " + std::to_string(preserve) +
                          " bytes for batches of max_batch_points, and every fit worker at least 1 MiB";
      delete S;
      return KRR_EINVAL;
    }
    S->fit_share = cfg->fit_workers > 0 ? (cfg->hbm_budget_bytes - preserve) / (size_t)cfg->fit_workers : 0;
  }
  krr_status st = KRR_OK;
  for (int i = 0; i < nw && st == KRR_OK; ++i) {
    Worker* W = new Worker();
    W->kind = i < cfg->predict_workers ? KIND_PREDICT : KIND_FIT;
    W->share = W->kind == KIND_PREDICT ? pshare : S->fit_share;
    st = krr_create(S->device, W->share, &W->ctx);
    if (st == KRR_OK) {
      (void)hipSetDevice(S->device);
      if (hipStreamCreateWithFlags(&W->stream, hipStreamNonBlocking) != hipSuccess) st = KRR_EDEVICE;
    }
    S->workers.push_back(W);
  }
  if (st != KRR_OK) {
    for (Worker* W : S->workers) {
      if (W->stream) (void)hipStreamDestroy(W->stream);
      if (W->ctx) (void)krr_destroy(W->ctx);
      delete W;
    }
    delete S;
    return st;
  }
  for (Worker* W : S->workers) W->thread = std::thread(worker_loop, S, W);
  *out = S;
  return KRR_OK;
}

krr_status krr_server_destroy(krr_server S) {
  if (S == nullptr) return KRR_EINVAL;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
  }
  S->cv_work.notify_all();
  for (Worker* W : S->workers)
    if (W->thread.joinable()) W->thread.join();
  for (Worker* W : S->workers) {
    if (W->stream) (void)hipStreamDestroy(W->stream);
    if (W->host) (void)hipHostFree(W->host);
    if (W->ctx) (void)krr_destroy(W->ctx);
    delete W;
  }
  for (auto& kv : S->requests) delete kv.second;
  delete S;
  return KRR_OK;
}

const char* krr_server_last_error(krr_server S) { return S ? S->last_error.c_str() : "null server"; }

krr_status krr_server_submit_predict(krr_server S, const float* Xq, int64_t k, double* yhat, int64_t* ticket) {
  if (S == nullptr) return KRR_EINVAL;
  if (Xq == nullptr || yhat == nullptr || ticket == nullptr || k < 1 || k > S->cfg.max_batch_points) {
    set_error(S, "predict: null pointer, or k outside [1, max_batch_points]");
    return KRR_EINVAL;
  }
  Request* r = new (std::nothrow) Request();
  if (r == nullptr) return KRR_ENOMEM;
  r->kind = KIND_PREDICT;
  r->X = Xq;
  r->out = yhat;
  r->rows = k;
  r->d = S->d_model;
  r->need = predict_need(k, S->d_model);
  if (S->cfg.hbm_budget_bytes != 0 && r->need > S->cfg.hbm_budget_bytes) {
    delete r;
    set_error(S, "predict request alone exceeds the HBM budget");
    return KRR_EBUDGET;
  }
  const krr_status st = submit(S, r);
  if (st == KRR_OK) *ticket = r->ticket;
  return st;
}

krr_status krr_server_submit_fit(krr_server S, const float* X, const float* y, int64_t m, int32_t d,
                                 const krr_fit_params* params, double* alpha, int64_t* ticket) {
  if (S == nullptr) return KRR_EINVAL;
  if (X == nullptr || y == nullptr || params == nullptr || alpha == nullptr || ticket == nullptr || m < 1 ||
      m >= (int64_t(1) << 30) || d < 1) {
    set_error(S, "fit: null pointer or bad size");
    return KRR_EINVAL;
  }
  const krr_fit_params& P = *params;
  const bool ar = P.kernel == KRR_KERNEL_POLYNOMIAL || P.kernel == KRR_KERNEL_SIGMOID;
  if ((P.kernel != KRR_KERNEL_GAUSSIAN && P.kernel != KRR_KERNEL_LINEAR && !ar) ||
      (P.kernel == KRR_KERNEL_GAUSSIAN && !(P.sigma > 0.0)) || !std::isfinite(P.lambda) ||
      (ar && !(std::isfinite(P.kernel_a) && std::isfinite(P.kernel_r))) ||
      (P.kernel == KRR_KERNEL_POLYNOMIAL && (P.kernel_degree < 1 || P.kernel_degree > 64)) ||
      (P.prec != KRR_PREC_FP64 && P.prec != KRR_PREC_FP32 && P.prec != KRR_PREC_MIXED) || P.max_refine < 0 ||
      P.max_refine > 1000 || (P.indefinite != 0 && P.indefinite != 1)) {
    set_error(S, "fit: bad settings");
    return KRR_EINVAL;
  }
  if (S->cfg.fit_workers == 0) {
    set_error(S, "fit: the server has no fit workers");
    return KRR_ESTATE;
  }
  Request* r = new (std::nothrow) Request();
  if (r == nullptr) return KRR_ENOMEM;
  r->kind = KIND_FIT;
  r->X = X;
  r->y = y;
  r->out = alpha;
  r->rows = m;
  r->d = d;
  r->params = P;
  r->need = fit_need(m, d, P.prec, default_panel_tiles(P.prec));
  if (S->cfg.hbm_budget_bytes != 0 && r->need > S->fit_share) {
    delete r;
    set_error(S, "fit request alone (" + std::to_string(fit_need(m, d, P.prec, default_panel_tiles(P.prec))) +
                     " bytes) exceeds a fit worker's share of the HBM budget (" + std::to_string(S->fit_share) +
                     " bytes)");
    return KRR_EBUDGET;
  }
  const krr_status st = submit(S, r);
  if (st == KRR_OK) *ticket = r->ticket;
  return st;
}

krr_status krr_server_wait(krr_server S, int64_t ticket, krr_request_info* info) {
  if (S == nullptr) return KRR_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->requests.find(ticket);
  if (it == S->requests.end()) {
    S->last_error = "unknown ticket";
    return KRR_EINVAL;
  }
  Request* r = it->second;
  S->cv_done.wait(lk, [&] { return r->done; });
  if (info != nullptr) {
    info->status = r->status;
    info->kind = r->kind;
    info->batch_requests = r->batch_requests;
    info->reserved = 0;
    info->queue_ms = r->t_start - r->t_submit;
    info->run_ms = r->t_done - r->t_start;
    info->total_ms = r->t_done - r->t_submit;
  }
  const krr_status st = (krr_status)r->status;
  S->requests.erase(it);
  delete r;
  return st;
}

krr_status krr_server_stats(krr_server S, int32_t reset, krr_serve_stats* out) {
  if (S == nullptr || out == nullptr) return KRR_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  out->predict_requests = S->n_done[KIND_PREDICT];
  out->fit_requests = S->n_done[KIND_FIT];
  out->points = S->points;
  out->fit_rows = S->fit_rows;
  out->predict_batches = S->batches[KIND_PREDICT];
  out->fit_batches = S->batches[KIND_FIT];
  out->failed = S->failed;
  out->max_inflight_bytes = (int64_t)S->max_inflight;
  out->max_device_bytes = (int64_t)S->max_held;
  out->predict_p50_ms = percentile(S->latency[KIND_PREDICT], 0.50);
  out->predict_p99_ms = percentile(S->latency[KIND_PREDICT], 0.99);
  out->fit_p50_ms = percentile(S->latency[KIND_FIT], 0.50);
  out->fit_p99_ms = percentile(S->latency[KIND_FIT], 0.99);
  out->span_ms = (S->t_first >= 0 && S->t_last >= 0) ? S->t_last - S->t_first : 0.0;
  if (reset) {
    S->n_done[0] = S->n_done[1] = 0;
    S->points = S->fit_rows = 0;
    S->batches[0] = S->batches[1] = 0;
    S->failed = 0;
    S->max_inflight = S->inflight;
    S->max_held = 0;
    for (Worker* V : S->workers) S->max_held += V->held;
    S->latency[0].clear();
    S->latency[1].clear();
    S->t_first = S->t_last = -1.0;
  }
  return KRR_OK;
}

}  // extern "C"
