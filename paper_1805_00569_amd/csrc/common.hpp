// Shared host/device definitions of the KRR library (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/krr.h"

namespace krr {

// Square tile edge of every blocked matrix in the library.  A system of size m
// holds T = ceil(m / NB) tile rows; its lower triangle is stored as T(T+1)/2
// contiguous NB x NB tiles, tile (i, j) (i >= j) at index i(i+1)/2 + j, each
// tile column-major (element (r, c) at c * NB + r).
constexpr int NB = 64;

struct Error {
  krr_status status;
  std::string msg;
};

[[noreturn]] inline void fail(krr_status s, const std::string& m) { throw Error{s, m}; }

#define KRR_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      ::krr::fail(KRR_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

#define KRR_REQUIRE(cond, msg)                       \
  do {                                                \
    if (!(cond)) ::krr::fail(KRR_EINVAL, (msg));      \
  } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t tri(int64_t t) { return t * (t + 1) / 2; }

// A grow-only device allocation.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// Table 1's polynomial and sigmoid kernels from the inner product g = x^T y:
// (a g + r)^d by binary powering and tanh(a g + r); each operation rounded on
// its own.
__device__ __forceinline__ double poly_kernel(double g, double a, double r, int deg) {
  double b = a * g + r, v = 1.0;
  for (int e = deg; e > 0; e >>= 1) {
    if (e & 1) v *= b;
    b *= b;
  }
  return v;
}

// Default Cholesky panel width (64-wide tiles) of a precision: measured
// fastest for the batched fits of systems of a few thousand points (mixed
// precision: 24; the FP32 and FP64 matrix-core paths: 16).
constexpr int default_panel_tiles(int prec) { return prec == KRR_PREC_MIXED ? 24 : 16; }

// Per-system descriptor of one batched solve (K_s + lambda_s I) alpha_s = y_s.
struct SysDesc {
  int32_t m;        // number of points in the partition
  int32_t T;        // tile rows, ceil(m / NB)
  int32_t part;     // partition index
  int32_t param;    // setting index
  int64_t a_off;    // element offset of the system's packed lower tiles
  int64_t w_off;    // element offset of its T inverse diagonal tiles
  int64_t v_off;    // offset of its padded vectors (T * NB entries)
  int64_t x_off;    // first row of the partition in the grouped inputs
  double neg_inv_2s2;  // -1 / (2 sigma^2)
  double lambda;       // diagonal shift actually used
  int32_t kernel;      // krr_kernel
  int32_t level;       // precision level that factors this system in the current pass
  double ka, kr;       // polynomial / sigmoid: a and r of Table 1
  int32_t kdeg;        // polynomial degree
  int32_t wp;          // Cholesky panel width of this system (64-wide tiles)
  int64_t pk_off;      // element offset of its BF16 panel-pack slot (mixed precision)
  int64_t k_off;       // mixed precision: element offset of the FP64 kernel tiles (without the
                       // shift) shared by the settings of this partition with the same kernel and sigma
  int32_t g_sys;       // the system of this partition in the first setting that shares its kernel tiles
  int32_t pad_;
};

// Device-side status of one system.
struct SysStatus {
  int32_t status;        // KRR_OK or KRR_ENOTSPD
  int32_t failed_pivot;  // 1-based, 0 = none
  int32_t refine_iters;
  int32_t converged;     // refinement reached the tolerance
  int32_t stalled;       // refinement stopped reducing the residual
  int32_t corr;          // corrections applied with the factor in use
  double rel_residual;
  double prev_rel;
  double ynorm;
  double kappa_l;        // (max_i L_ii / min_i L_ii)^2 of the factor in use: a lower bound of kappa_2(A)
  double kappa_u;        // an upper bound of kappa_2 of the FP64 system (Gershgorin; -1: not formed)
  double dnorm;          // ||delta||_inf of the last correction (-1: none yet)
  double prev_dnorm;     // ||delta||_inf of the one before (-1: none)
  double anorm;          // ||alpha||_inf after the last correction
  double err_est;        // estimated relative forward error of alpha (inf-norm; -1: not estimated)
};

}  // namespace krr

// Partitioned training data shared by the models of one krr_fit call.
struct krr_part_data {
  krr_ctx ctx = nullptr;
  void* base = nullptr;         // one allocation holding the arrays below
  int32_t p = 0, d = 0, dtype = 0;
  int64_t n = 0;
  void* X = nullptr;          // n x d grouped by partition, input dtype
  double* centroids = nullptr;  // p x d
  double* ct_t = nullptr;       // d x p (transposed, for routing)
  std::vector<int64_t> offsets; // p + 1, host copy
  int64_t* d_offsets = nullptr; // p + 1, device
  size_t bytes = 0;
  ~krr_part_data();
};

struct krr_model_s {
  krr_ctx ctx = nullptr;
  std::shared_ptr<krr_part_data> data;
  krr_fit_params params{};
  double* alpha = nullptr;      // sum_j T_j * NB padded FP64 coefficients (allocation base)
  int64_t* d_voff = nullptr;    // p + 1 padded offsets into alpha (device)
  std::vector<int64_t> voff;    // host copy
  std::vector<double> lambda_eff;
  size_t bytes = 0;
};

struct krr_timed_launch {
  const char* cls;
  hipEvent_t a, b;
  double flops;
  double bytes;
};

struct krr_timing_agg {
  int64_t count = 0;
  double ms = 0.0;       // summed launch durations
  double busy_ms = 0.0;  // time covered by at least one launch of the class (launches on several streams overlap)
  double flops = 0.0;
  double bytes = 0.0;
};

struct krr_ctx_s {
  int device = 0;
  size_t budget = 0;
  std::string last_error;
  std::map<std::string, krr::DevBuf> ws;
  size_t ws_bytes = 0;
  size_t model_bytes = 0;
  std::multimap<size_t, void*> model_cache;   // released model blocks by rounded size, for reuse
  size_t cache_bytes = 0;
  int n_models = 0;
  int n_datas = 0;
  int panel_tiles = 0;   // KRR_OPT_PANEL_TILES; 0: the precision's default (default_panel_tiles)
  int serial_fit = 0;
  int sync_check = 0;
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  int timing = 0;   // 0 off, 1 matrix-core update kernels, 2 every timed kernel class
  int noalloc = 0;  // inside a no-allocation call: no timing events
  hipStream_t cur_stream = nullptr;   // stream of the call in progress (valid while in_call)
  // Streams beside the call's stream (default priority) on which groups of
  // systems of a batch are factored at the same time (KRR_OPT_FACTOR_STREAMS);
  // every use forks from and joins back into the call's stream.
  static constexpr int kMaxFactorStreams = 4;
  hipStream_t side[kMaxFactorStreams - 1] = {};
  hipEvent_t side_ev[kMaxFactorStreams] = {};   // fork, then one join per side stream
  int factor_streams = 2;
  int column_pairs = 1;
  bool in_call = false;
  // per stream the context has queued work on: an event recorded after that
  // work (see drain)
  std::vector<std::pair<hipStream_t, hipEvent_t>> marks;
  int persistent = 0;            // factor with the persistent launch (KRR_OPT_PERSISTENT)
  int autotune = 1;              // give systems the tuned panel width of their size class
  int force_wp = 0;              // > 0: every system takes this panel width (trial fits)
  std::map<std::pair<int, int>, int> tune;   // (precision, size class) -> panel width
  int64_t persist_wait_ms = 30000;   // longest wait of one task before it gives up
  // Task plans of the persistent factorisation, uploaded once per set of
  // shapes into one of a few workspace slots (a fit at several refinement
  // levels, or graphs of several shapes, then find their plans resident).
  struct PersistPlan {
    std::vector<int> key;       // shapes the plan was built for (empty: free slot)
    void* tasks = nullptr;      // device: tasks, then the queue offsets
    size_t qoff_off = 0;
    int nq = 1, ntasks = 0;
    std::vector<int> T, act, wp;   // the plan's inputs (to upload it again for a graph replay)
    int packed = 0, tsize = 0;
    uint64_t used = 0;          // last use (least recently used slot is replaced)
  };
  struct PersistCache {
    static constexpr int kSlots = 4;
    PersistPlan slot[kSlots];
    uint64_t clock = 0;
    std::vector<int> captured;  // slots whose plans the capture in progress reads
    std::vector<int> fresh;     // slots whose upload the capture in progress recorded
  } persist;
  std::map<std::string, std::pair<void*, size_t>> pinned_bufs;   // named pinned staging
  // HIP graphs of the device phases of fits and predictions (KRR_OPT_GRAPHS):
  // a call whose key (shapes, settings, pointers, workspace epoch) was seen
  // once eagerly is captured on its next occurrence and replayed afterwards
  int graphs = 0;
  int capturing = 0;            // inside a stream capture: no synchronisation, no allocation
  uint64_t ws_epoch = 0;        // bumped whenever a workspace buffer moves
  struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    std::vector<std::pair<int, PersistPlan>> plans;   // (slot, plan) of the graph's persistent launches
  };
  std::map<std::string, GraphEntry> graph_cache;
  int64_t graph_captures = 0, graph_replays = 0;
  std::map<std::string, int> graph_seen;
  std::vector<hipEvent_t> ev_pool;
  std::vector<krr_timed_launch> pending;
  std::map<std::string, krr_timing_agg> timing_agg;
};

namespace krr {

// Workspace buffer `name` of at least `bytes`, grown (never shrunk) inside the
// context's budget.  Contents are not preserved across growth.
void* ws_get(krr_ctx ctx, const std::string& name, size_t bytes);
// Device allocation charged to the context's model memory.
void* model_alloc(krr_ctx ctx, size_t bytes);
void model_release(krr_ctx ctx, void* p, size_t bytes);
void* pinned_get(krr_ctx ctx, size_t bytes);
// Pinned host staging buffer `name`, grown (never shrunk); contents are not
// preserved across growth.
void* pinned_named(krr_ctx ctx, const std::string& name, size_t bytes);
// Runs f with the device of ctx current, translating errors into a status
// (and ctx->last_error), as every entry point does.
krr_status run_guarded(krr_ctx ctx, const std::function<void()>& f);
// Panel width for a system of m points at precision prec: the tuned one of
// its size class when tuning applies, else the context's default.
int tuned_panel(krr_ctx ctx, int prec, int64_t m);
void tune_load(krr_ctx ctx);
// Frees every workspace buffer of the context (after drain).
void ws_release_all(krr_ctx ctx);
// Runs `body` (device work on stream s only, no synchronisation, no
// allocation) eagerly, or as a replay of its HIP graph: with graphs on, the
// second call with the same key captures it, later calls replay it.  The key
// must name everything the device work depends on except the contents of
// device memory; the workspace epoch is added here.  Returns true if a graph
// was launched.
template <typename F>
bool graph_run(krr_ctx ctx, hipStream_t s, const std::string& key, F&& body);
void graph_drop_all(krr_ctx ctx);
// Byte-string key helper.
template <typename T>
inline void key_add(std::string& k, const T& v) {
  k.append(reinterpret_cast<const char*>(&v), sizeof(T));
}
// Waits until the work this context has queued is done: the current call's
// stream and the last recorded work on every other stream it has used.  Work
// of other contexts is not waited for.
void drain(krr_ctx ctx);
// Marks a call on `stream`: the context's buffers may be used by work queued
// on it until the scope ends, when an event is recorded after that work.
struct StreamScope {
  krr_ctx ctx;
  StreamScope(krr_ctx c, hipStream_t s);
  ~StreamScope();
};
void check_launch(krr_ctx ctx, hipStream_t s, const char* what);

// HIP events around one launch of kernel class `cls` (only when timing is on;
// major = 1 marks the matrix-core update kernels), with the launch's
// algorithmic flop count and algorithmic HBM bytes (the bytes the algorithm
// must move, not what the kernel moves).  Results are collected by
// krr_timing_report.
struct KernelTimer {
  krr_ctx ctx;
  hipStream_t s;
  const char* cls;
  double flops;
  double bytes;
  hipEvent_t a = nullptr, b = nullptr;
  KernelTimer(krr_ctx c, hipStream_t st, const char* name, double f, int major, double by = 0.0);
  ~KernelTimer();
};

// ---- csr.hip ----
void run_csr_to_dense(krr_ctx ctx, hipStream_t s, const int64_t* indptr, const int32_t* indices, const void* values,
                      int dtype, int64_t n, int d, int64_t nnz, void* X);

// ---- partition.hip ----
void assign_nearest(krr_ctx ctx, hipStream_t s, const void* X, int dtype, int64_t n, int d,
                    const double* C, int p, int32_t* out, const int32_t* prev, int32_t* delta,
                    const int32_t* skip);
// Stable grouping of n keys in [0, p): perm lists the points of key 0, then
// key 1, ... (each in increasing index), offsets[p + 1] the group starts.
// wsp (nullable): group_ws_bytes(n, p) bytes of device workspace to use
// instead of the context's pool.
size_t group_ws_bytes(int64_t n, int p);
void group_by_key(krr_ctx ctx, hipStream_t s, const int32_t* key, int64_t n, int p,
                  int32_t* perm, int64_t* offsets, int64_t* sizes64, const int32_t* skip, void* wsp = nullptr);
void gather_rows(krr_ctx ctx, hipStream_t s, const void* X, int dtype, int64_t n, int d,
                 const int32_t* perm, void* Xout);
void gather_vec_f64(krr_ctx ctx, hipStream_t s, const void* y, int dtype, int64_t n,
                    const int32_t* perm, double* yout);
void transpose_centroids(krr_ctx ctx, hipStream_t s, const double* C, int p, int d, double* CT);
void run_partition(krr_ctx ctx, hipStream_t s, const void* X, int dtype, int64_t n, int d, int p,
                   int method, int iters, uint64_t seed, double* C, int32_t* assign,
                   int64_t* sizes);

// Bump allocation of 256-byte aligned pieces from a fixed device region (the
// no-allocation entry points); running out is an argument error.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  void* take(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    if (used + bytes > cap)
      fail(KRR_EINVAL, "scratch of " + std::to_string(cap) + " bytes exhausted (" + std::to_string(used + bytes) +
                           " needed)");
    void* p = base + used;
    used += bytes;
    return p;
  }
};
inline size_t al256(size_t b) { return b == 0 ? 256 : (b + 255) & ~size_t(255); }
// A piece of `bytes` from the arena when there is one, else the context's
// workspace buffer `name`.
inline void* ws_or_arena(krr_ctx ctx, Arena* ar, const std::string& name, size_t bytes) {
  return ar != nullptr ? ar->take(bytes) : ws_get(ctx, name, bytes);
}

// Persistent-plan bookkeeping for graphs: the plan a captured launch reads
// must be the one on the device when the graph is replayed.
void persist_note_plan(krr_ctx ctx, krr_ctx_s::GraphEntry& e);
void persist_restore_plan(krr_ctx ctx, hipStream_t s, const krr_ctx_s::GraphEntry& e);
// Forgets the plans whose upload an abandoned capture recorded (never ran).
void persist_capture_aborted(krr_ctx ctx);

template <typename F>
bool graph_run(krr_ctx ctx, hipStream_t s, const std::string& key0, F&& body) {
  if (!ctx->graphs) {
    body();
    return false;
  }
  std::string key = key0;
  key_add(key, ctx->ws_epoch);
  key_add(key, s);
  auto it = ctx->graph_cache.find(key);
  if (it != ctx->graph_cache.end()) {
    persist_restore_plan(ctx, s, it->second);
    KRR_HIP(hipGraphLaunch(it->second.exec, s));
    ctx->graph_replays += 1;
    return true;
  }
  if (ctx->graph_seen[key] == 0) {   // first time: eager (it sizes the workspace)
    ctx->graph_seen[key] = 1;
    body();
    return false;
  }
  if (ctx->graph_seen[key] == 2) {   // its capture failed: direct launches from now on
    body();
    return false;
  }
  krr_ctx_s::GraphEntry e;
  hipGraph_t g = nullptr;
  KRR_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  ctx->capturing = 1;
  bool redo = false;
  try {
    body();
  } catch (const Error& err) {
    ctx->capturing = 0;
    hipGraph_t junk = nullptr;
    (void)hipStreamEndCapture(s, &junk);
    if (junk) (void)hipGraphDestroy(junk);
    persist_capture_aborted(ctx);
    // a step that cannot be captured (a wait, a workspace that must grow):
    // nothing recorded has run, so the call runs directly instead
    if (err.status != KRR_ESTATE) throw;
    redo = true;
  } catch (...) {
    ctx->capturing = 0;
    hipGraph_t junk = nullptr;
    (void)hipStreamEndCapture(s, &junk);
    if (junk) (void)hipGraphDestroy(junk);
    persist_capture_aborted(ctx);
    throw;
  }
  if (redo) {
    ctx->graph_seen[key] = 2;
    body();
    return false;
  }
  ctx->capturing = 0;
  KRR_HIP(hipStreamEndCapture(s, &g));
  const hipError_t ie = hipGraphInstantiate(&e.exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) fail(KRR_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
  persist_note_plan(ctx, e);
  auto& slot = ctx->graph_cache[key];
  slot = e;
  KRR_HIP(hipGraphLaunch(slot.exec, s));
  ctx->graph_captures += 1;
  return true;
}

// ---- lu.hip ----
// Systems `which` (indices into the batch; hdesc: host descriptors) solved
// by LU with partial pivoting in FP64 from the grouped points Xg (dtype) and
// labels y (FP64, grouped order); alpha (padded, at each system's v_off) is
// written.  Returns per listed system 0, or the 1-based column whose pivot
// candidates were all zero (alpha of that system is then not written).
std::vector<int32_t> lu_solve_systems(krr_ctx ctx, hipStream_t s, const std::vector<int>& which,
                                      const SysDesc* hdesc, const void* Xg, int dtype, int d, const double* y,
                                      double* alpha);

// ---- fit.hip ----
bool same_kernel_matrix(const krr_fit_params& a, const krr_fit_params& b);
// Result of a fit that creates no model (one setting): alpha of partition j is
// alpha[v_off[j], v_off[j] + m[j]) in the context's workspace, valid until the
// next fit on the context.  The partition data then lives in the workspace
// too, so no model memory is allocated or freed.
struct FitDirect {
  const double* alpha = nullptr;
  std::vector<int64_t> v_off, m;
};
void run_fit(krr_ctx ctx, hipStream_t s, const void* X, const void* y, int dtype, int64_t n, int d,
             const int32_t* assign, const double* centroids, int p, const krr_fit_params* params,
             int n_params, krr_model* models, krr_part_info* info, FitDirect* direct = nullptr);

// ---- predict.hip ----
void run_predict(krr_ctx ctx, hipStream_t s, krr_model model, const void* Xt, int dtype, int64_t k,
                 int route, double* yhat, int32_t* route_out, Arena* ar = nullptr);
// The same prediction with every temporary taken from the library's fixed
// per-device scratch array (no device allocation).
void run_predict_noalloc(krr_ctx ctx, hipStream_t s, krr_model model, const void* Xt, int dtype, int64_t k,
                         int route, double* yhat, int32_t* route_out);
// Once per device, with the device current: record the device address of the
// no-allocation scratch array.
void noalloc_scratch_init(int device);
void run_select(krr_ctx ctx, hipStream_t s, const krr_model* models, int n_models, const void* Xv,
                const void* yv, int dtype, int64_t k, int route, double* mse, int32_t* best);

}  // namespace krr
