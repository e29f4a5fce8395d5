// Autotuning of the Cholesky panel width.
//
// The panel width W (tiles per panel of the blocked factorisation) trades the
// column updates inside a panel, whose operand re-reads grow with the depth
// inside the panel, against the trailing updates, one pass over the trailing
// triangle per panel; where the balance lies depends on the system size and
// the precision path.  krr_autotune times trial fits of synthetic systems of
// one size class over a set of widths and records the fastest for (precision,
// size class); fits then give every system the width recorded for its own
// class (the persistent factorisation runs each system with its own width),
// so a system's result does not depend on the batch it is fitted in.  The
// table can be kept in a text file named by the environment variable
// KRR_TUNE_CACHE: read when a context is created, extended by every tuning.
#include "common.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <fstream>
#include <sstream>

namespace krr {

namespace {

// SplitMix64 output function: a counter-based stream of 64-bit values
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Trial data: x ~ N(0, 1) per feature (Box-Muller on two counter draws),
// y ~ N(0, 1), point i in system i / m.
__global__ void k_tune_data(float* __restrict__ X, float* __restrict__ y, int32_t* __restrict__ assign, int64_t n,
                            int d, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * (d + 1)) return;
  const uint64_t a = mix64(0x9E3779B97F4A7C15ull * (uint64_t)(2 * i + 1));
  const uint64_t b = mix64(0x9E3779B97F4A7C15ull * (uint64_t)(2 * i + 2));
  const double u1 = ((double)(a >> 11) + 1.0) * 0x1.0p-53, u2 = (double)(b >> 11) * 0x1.0p-53;
  const float v = (float)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
  if (i < n * d) {
    X[i] = v;
  } else {
    const int64_t r = i - n * d;
    y[r] = v;
    assign[r] = (int32_t)(r / m);
  }
}

__global__ void k_tune_zero(double* c, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = 0.0;
}

int size_class(int64_t T) {
  int b = 0;
  while ((int64_t(1) << b) < T) ++b;
  return b;
}

}  // namespace

int tuned_panel(krr_ctx ctx, int prec, int64_t m) {
  const int dflt = ctx->panel_tiles > 0 ? ctx->panel_tiles : default_panel_tiles(prec);
  if (!ctx->autotune || m <= 0) return dflt;
  const auto it = ctx->tune.find(std::make_pair(prec, size_class(ceil_div(m, NB))));
  return it == ctx->tune.end() ? dflt : it->second;
}

void tune_load(krr_ctx ctx) {
  const char* path = std::getenv("KRR_TUNE_CACHE");
  if (path == nullptr || *path == 0) return;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream ls(line);
    int prec = -1, cls = -1, wp = 0;
    double ms = 0;
    if (ls >> prec >> cls >> wp >> ms && prec >= 0 && prec <= 2 && cls >= 0 && cls < 40 && wp >= 1 && wp <= 64)
      ctx->tune[std::make_pair(prec, cls)] = wp;
  }
}

// Times fits of n_sys synthetic systems of m points in d dimensions at every
// candidate width and records the fastest.  The trial setting keeps the
// systems well conditioned, so every width does the same work.
int run_autotune(krr_ctx ctx, hipStream_t s, int prec, int64_t m, int d, int n_sys, double* best_ms) {
  const int64_t T = ceil_div(m, NB);
  const int64_t n = m * n_sys;
  float* X = (float*)ws_get(ctx, "tune_X", (size_t)n * d * 4);
  float* y = (float*)ws_get(ctx, "tune_y", (size_t)n * 4);
  int32_t* assign = (int32_t*)ws_get(ctx, "tune_assign", (size_t)n * 4);
  double* C = (double*)ws_get(ctx, "tune_C", (size_t)n_sys * d * 8);
  hipLaunchKernelGGL(k_tune_data, dim3((unsigned)ceil_div(n * (d + 1), 256)), dim3(256), 0, s, X, y, assign, n, d, m);
  check_launch(ctx, s, "tune_data");
  hipLaunchKernelGGL(k_tune_zero, dim3((unsigned)ceil_div((int64_t)n_sys * d, 256)), dim3(256), 0, s, C,
                     (int64_t)n_sys * d);
  check_launch(ctx, s, "tune_zero");
  krr_fit_params P{};
  P.sigma = std::sqrt(2.0 * d) / 4.0;   // off-diagonal kernel values about e^-8
  P.lambda = 1e-2;
  P.kernel = KRR_KERNEL_GAUSSIAN;
  P.prec = prec;
  P.refine_tol = 1e-6;
  P.max_refine = 10;
  std::vector<int> cand;
  for (int w : {2, 4, 6, 8, 12, 16, 20, 24, 32, 48, 64})
    if (w <= std::max<int64_t>(T, 1)) cand.push_back(w);
  hipEvent_t e0, e1;
  KRR_HIP(hipEventCreate(&e0));
  KRR_HIP(hipEventCreate(&e1));
  std::vector<krr_part_info> info(n_sys);
  int best = ctx->panel_tiles > 0 ? ctx->panel_tiles : default_panel_tiles(prec);
  double best_t = INFINITY;
  const int saved_force = ctx->force_wp, saved_timing = ctx->timing, saved_graphs = ctx->graphs;
  ctx->timing = 0;
  ctx->graphs = 0;
  try {
    for (int w : cand) {
      ctx->force_wp = w;
      FitDirect fd;
      run_fit(ctx, s, X, y, KRR_F32, n, d, assign, C, n_sys, &P, 1, nullptr, info.data(), &fd);   // warm
      std::vector<float> ts;
      for (int r = 0; r < 3; ++r) {
        KRR_HIP(hipEventRecord(e0, s));
        run_fit(ctx, s, X, y, KRR_F32, n, d, assign, C, n_sys, &P, 1, nullptr, info.data(), &fd);
        KRR_HIP(hipEventRecord(e1, s));
        KRR_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        KRR_HIP(hipEventElapsedTime(&ms, e0, e1));
        ts.push_back(ms);
      }
      std::sort(ts.begin(), ts.end());
      if (ts[1] < best_t) {
        best_t = ts[1];
        best = w;
      }
    }
  } catch (...) {
    ctx->force_wp = saved_force;
    ctx->timing = saved_timing;
    ctx->graphs = saved_graphs;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  ctx->force_wp = saved_force;
  ctx->timing = saved_timing;
  ctx->graphs = saved_graphs;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const int cls = size_class(T);
  ctx->tune[std::make_pair(prec, cls)] = best;
  if (const char* path = std::getenv("KRR_TUNE_CACHE"); path != nullptr && *path != 0) {
    std::ofstream f(path, std::ios::app);
    f << prec << " " << cls << " " << best << " " << best_t << "\n";
  }
  if (best_ms != nullptr) *best_ms = best_t;
  return best;
}

}  // namespace krr

using namespace krr;

extern "C" krr_status krr_autotune(krr_ctx ctx, hipStream_t stream, int32_t prec, int64_t m, int32_t d,
                                   int32_t n_sys, int32_t* panel_out, double* ms_out) {
  if (ctx == nullptr) return KRR_EINVAL;
  if (prec != KRR_PREC_FP64 && prec != KRR_PREC_FP32 && prec != KRR_PREC_MIXED) return KRR_EINVAL;
  if (m < 1 || m > (int64_t(1) << 20) || d < 1 || d > 4096 || n_sys < 1 || n_sys > 1024 ||
      m * n_sys >= (int64_t(1) << 31) - 1 || panel_out == nullptr)
    return KRR_EINVAL;
  return run_guarded(ctx, [&] {
    StreamScope ss(ctx, stream);
    *panel_out = run_autotune(ctx, stream, prec, m, d, n_sys, ms_out);
  });
}
