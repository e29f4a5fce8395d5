// Prediction (Eq. 7) with the routes of Sections 4.1 / 4.2 and Algorithm 5,
// and model selection by MSE (Eq. 3, Algorithm 5).
//
// NEAREST: each test point is assigned to its nearest centre with the exact
// FP64 assignment kernel (the "MyCluster" step of Algorithm 5), the points
// are grouped by partition, and every 64-point group is predicted against its
// partition's training points only.  ALL / AVERAGE: every 64-point group is
// predicted by every partition model.
//
// The fused kernel takes 64 test points against 64-point chunks of one
// partition's training points: the Gram block on FP64 matrix cores, then the
// kernel values and their contraction with alpha, so the k x m kernel matrix
// is never stored.  The Gram block does not depend on (sigma, lambda): the
// models fitted together on one partitioning (up to MAXM per launch) share it
// and only redo the exponential and the dot product.  The training chunks of
// a partition are split over `nsplit` workgroups that write partial sums;
// a second kernel adds the splits in a fixed order, so every result is
// independent of the launch shape and of the batch.
#include "common.hpp"

#include <mutex>

namespace krr {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int KCR = 32;          // features per staged block; a wave keeps its test operands of a block in registers
constexpr int KSR = KCR / 4;     // 4-deep MFMA steps per block
// training block in LDS, row-major with a row pitch of KCR + 4 doubles: the
// staging stores (consecutive features of a row) and the MFMA operand reads
// (16 rows x 4 features per instruction) both touch every bank pair at most
// twice, the minimum for 64 eight-byte accesses
constexpr int LDR = KCR + 4;
constexpr int MAXM = 8;

struct PredModels {
  const double* alpha[MAXM];
  const int64_t* voff[MAXM];
  double* out[MAXM];
  double negu[MAXM];   // the distinct kernel settings of the models (nu of them):
  double ka[MAXM];     //   Gaussian -1/(2 sigma^2); polynomial / sigmoid a, r, d
  double kr[MAXM];
  int kdeg[MAXM];
  int uidx[MAXM];      // model q uses setting uidx[q]: the kernel values are shared
  int uidx_first[MAXM];   // host bookkeeping: first model of each setting
  int nu;
  int nm;
  int kernel;
};

// KER: the call's kernel (Table 1), fixed at compile time.
template <typename TX, int KER>
__global__ __launch_bounds__(256, 2) void k_predict(const TX* __restrict__ Xt, int d, int64_t k,
                                                 const int32_t* __restrict__ tperm,
                                                 const int64_t* __restrict__ toff,
                                                 const int32_t* __restrict__ tile_start, int route,
                                                 const TX* __restrict__ Xg, const int64_t* __restrict__ xoff,
                                                 const PredModels M, int p, int cps, int64_t npos,
                                                 double* __restrict__ part_out) {
  int j;
  int64_t t0, tcnt;
  const int split = blockIdx.z;
  if (route == KRR_ROUTE_NEAREST) {
    const int b = blockIdx.x;
    if (b >= tile_start[p]) return;
    int lo = 0, hi = p;  // tile_start[lo] <= b < tile_start[lo + 1]
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (tile_start[mid] <= b) lo = mid;
      else hi = mid;
    }
    j = lo;
    t0 = toff[j] + (int64_t)(b - tile_start[j]) * NB;
    tcnt = min((int64_t)NB, toff[j + 1] - t0);
  } else {
    j = blockIdx.y;
    t0 = (int64_t)blockIdx.x * NB;
    tcnt = min((int64_t)NB, k - t0);
  }
  const int64_t x0 = xoff[j];
  const int64_t m = xoff[j + 1] - x0;
  const int64_t xbeg = (int64_t)split * cps * NB;
  const int64_t xend = min(m, xbeg + (int64_t)cps * NB);
  __shared__ double sX[NB * LDR];    // training block: sX[row * LDR + kk], zero past the features
  __shared__ double sNp[4][NB];      // training-row norms, four feature quarters
  __shared__ int64_t srow[NB];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int il = lane & 15, kl = lane >> 4;
  if (t < NB) {
    int64_t src = -1;
    if (t < tcnt) src = (route == KRR_ROUTE_NEAREST) ? (int64_t)tperm[t0 + t] : t0 + t;
    srow[t] = src;
  }
  __syncthreads();
  // this lane's test point (the B operand column) and its features 4 s + kl of a block
  const int tl = 16 * w + il;
  const int64_t trow = max(srow[tl], (int64_t)0);
  double bt[KSR];
  auto load_test = [&](int k0, int kc) {
#pragma unroll
    for (int s = 0; s < KSR; ++s) {
      const int kk = 4 * s + kl;
      const double v = (double)Xt[trow * d + k0 + min(kk, kc - 1)];   // unconditional, clamped
      bt[s] = kk < kc ? v : 0.0;
    }
  };
  double nt = 0.0;
  for (int k0 = 0; k0 < d; k0 += KCR) {
    load_test(k0, min(KCR, d - k0));
#pragma unroll
    for (int s = 0; s < KSR; ++s) nt = fma(bt[s], bt[s], nt);
  }
  nt += __shfl_xor(nt, 16, 64);
  nt += __shfl_xor(nt, 32, 64);
  const bool one_block = d <= KCR;   // the test operands stay loaded across the chunks
  // The chunks of this split and their feature blocks run as one sequence of
  // block steps; the loads of step b + 1 (training block and test operands)
  // are issued before the products of step b, so their latency overlaps the
  // matrix cores and the exponentials.
  const int nblk = (d + KCR - 1) / KCR;
  const int64_t nsteps = xend > xbeg ? ((xend - xbeg + NB - 1) / NB) * nblk : 0;
  TX lx[NB * KCR / 256];
  TX btn[KSR];       // test operands of the step's block (raw; zeroed past d when used)
  auto fetch = [&](int64_t b) {
    const int64_t xc = xbeg + (b / nblk) * NB;
    const int k0 = (int)(b % nblk) * KCR;
    const int64_t xcnt = min((int64_t)NB, xend - xc);
    const int kc = min(KCR, d - k0);
#pragma unroll
    for (int u = 0; u < NB * KCR / 256; ++u) {
      const int e = t + u * 256, row = e / KCR, kk = e - row * KCR;
      lx[u] = Xg[(x0 + xc + min((int64_t)row, xcnt - 1)) * d + k0 + min(kk, kc - 1)];
    }
    if (!one_block) {
#pragma unroll
      for (int s = 0; s < KSR; ++s) btn[s] = Xt[trow * d + k0 + min(4 * s + kl, kc - 1)];
    }
  };
  __shared__ double sA[2][MAXM][NB];   // alpha of the chunk (by chunk parity), zero past its rows
  double part[MAXM];
#pragma unroll
  for (int q = 0; q < MAXM; ++q) part[q] = 0.0;
  d4 acc[4];
  double nxp = 0.0;   // norm of training row (t & 63) over feature quarter (t >> 6) of the blocks
  if (nsteps > 0) fetch(0);
  for (int64_t b = 0; b < nsteps; ++b) {
    const int kb = (int)(b % nblk);
    const int64_t xc = xbeg + (b / nblk) * NB;
    const int64_t xcnt = min((int64_t)NB, xend - xc);
    const int k0 = kb * KCR, kc = min(KCR, d - k0);
    const int buf = (int)((b / nblk) & 1);
    if (kb == 0) {
#pragma unroll
      for (int xb = 0; xb < 4; ++xb) acc[xb] = d4{0.0, 0.0, 0.0, 0.0};
      nxp = 0.0;
    }
    __syncthreads();   // the previous block's readers are done
#pragma unroll
    for (int u = 0; u < NB * KCR / 256; ++u) {
      const int e = t + u * 256, row = e / KCR, kk = e - row * KCR;
      sX[row * LDR + kk] = kk < kc ? (double)lx[u] : 0.0;
    }
    if (kb == 0 && t < NB) {   // alpha of the chunk (read at its last block)
#pragma unroll
      for (int q = 0; q < MAXM; ++q)
        if (q < M.nm) {
          const double a = M.alpha[q][M.voff[q][j] + xc + min((int64_t)t, xcnt - 1)];
          sA[buf][q][t] = t < xcnt ? a : 0.0;
        }
    }
    if (!one_block) {
#pragma unroll
      for (int s = 0; s < KSR; ++s) bt[s] = 4 * s + kl < kc ? (double)btn[s] : 0.0;
    }
    __syncthreads();
    if (b + 1 < nsteps) fetch(b + 1);
#pragma unroll
    for (int u = 0; u < KCR / 4; ++u) {
      const double v = sX[(t & 63) * LDR + (t >> 6) * (KCR / 4) + u];
      nxp = fma(v, v, nxp);
    }
#pragma unroll
    for (int s = 0; s < KSR; ++s) {
      if (4 * s < kc) {
        const int ko = 4 * s + kl;
#pragma unroll
        for (int xb = 0; xb < 4; ++xb)
          acc[xb] = __builtin_amdgcn_mfma_f64_16x16x4f64(sX[(16 * xb + il) * LDR + ko], bt[s], acc[xb], 0, 0, 0);
      }
      if ((s & 3) == 3) __builtin_amdgcn_sched_barrier(0);   // bounds the operand loads in flight
    }
    if (kb != nblk - 1) continue;
    sNp[t >> 6][t & 63] = nxp;
    __syncthreads();
    // squared distances of the lane's 16 (training row, test point) pairs;
    // rows past the chunk carry alpha = 0 (their kernel values are finite)
    double d2[16];
#pragma unroll
    for (int xb = 0; xb < 4; ++xb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int xl = 16 * xb + kl + 4 * v;   // FP64 MFMA result row of register v
        const double nx = (sNp[0][xl] + sNp[1][xl]) + (sNp[2][xl] + sNp[3][xl]);
        d2[4 * xb + v] = fmax(0.0, (nt + nx) - 2.0 * acc[xb][v]);
      }
    // per half of the elements, one distinct sigma at a time: its 8 kernel
    // values in one branch-free block (independent exponentials the
    // scheduler interleaves), then the models that use it; every model sums
    // its elements in the same order
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll 1
      for (int u = 0; u < M.nu; ++u) {
        double kv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int el = 8 * h + e;
          const double G = acc[el >> 2][el & 3];
          if constexpr (KER == KRR_KERNEL_GAUSSIAN) kv[e] = exp(d2[el] * M.negu[u]);
          else if constexpr (KER == KRR_KERNEL_POLYNOMIAL) kv[e] = poly_kernel(G, M.ka[u], M.kr[u], M.kdeg[u]);
          else if constexpr (KER == KRR_KERNEL_SIGMOID) kv[e] = tanh(M.ka[u] * G + M.kr[u]);
          else kv[e] = G;
        }
#pragma unroll
        for (int q = 0; q < MAXM; ++q) {
          if (q < M.nm && M.uidx[q] == u) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int el = 8 * h + e;
              part[q] = fma(sA[buf][q][16 * (el >> 2) + kl + 4 * (el & 3)], kv[e], part[q]);
            }
          }
        }
      }
    }
  }
  // lanes il, il+16, il+32, il+48 hold partial sums of the same test point
#pragma unroll
  for (int q = 0; q < MAXM; ++q) {
    part[q] += __shfl_xor(part[q], 16, 64);
    part[q] += __shfl_xor(part[q], 32, 64);
  }
  if (kl == 0 && tl < tcnt) {
    const int64_t pos = (route == KRR_ROUTE_NEAREST) ? (t0 + tl) : ((t0 + tl) * p + j);
#pragma unroll
    for (int q = 0; q < MAXM; ++q)
      if (q < M.nm) part_out[((int64_t)split * npos + pos) * M.nm + q] = part[q];
  }
}

// Sum the splits in order; NEAREST positions are scattered back to the
// caller's point order.
__global__ void k_predict_reduce(const double* __restrict__ part, int nsplit, int64_t npos, const PredModels M,
                                 const int32_t* __restrict__ tperm) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= npos * M.nm) return;
  const int64_t pos = e / M.nm;
  const int q = (int)(e - pos * M.nm);
  double s = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) s += part[((int64_t)sp * npos + pos) * M.nm + q];
  const int64_t dst = (tperm != nullptr) ? (int64_t)tperm[pos] : pos;
  M.out[q][dst] = s;
}

__global__ void k_tile_prefix(const int64_t* __restrict__ toff, int p, int32_t* __restrict__ tile_start) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int32_t acc = 0;
    for (int j = 0; j < p; ++j) {
      tile_start[j] = acc;
      acc += (int32_t)((toff[j + 1] - toff[j] + NB - 1) / NB);
    }
    tile_start[p] = acc;
  }
}

__global__ void k_row_mean(const double* __restrict__ all, int64_t k, int p, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  double s = 0.0;
  for (int j = 0; j < p; ++j) s += all[i * p + j];
  out[i] = s / (double)p;
}

// Block sums of the squared errors.  yhat holds pc predictions per point
// (row-major k x pc); a point's error is the smallest over them (pc = 1: the
// plain error; pc = p: the label-based choice of Algorithm 6).
template <typename TY>
__global__ __launch_bounds__(256) void k_sqerr(const double* __restrict__ yhat, int pc, const TY* __restrict__ y,
                                               int64_t k, double* __restrict__ partial) {
  __shared__ double sred[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double e = 0.0;
  if (i < k) {
    const double yi = (double)y[i];
    double dlt = yhat[i * pc] - yi;
    e = dlt * dlt;
    for (int j = 1; j < pc; ++j) {
      dlt = yhat[i * pc + j] - yi;
      e = fmin(e, dlt * dlt);
    }
  }
  sred[threadIdx.x] = e;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sred[threadIdx.x] += sred[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sred[0];
}

__global__ void k_mse_final(const double* __restrict__ partial, int64_t nb, int64_t k, double* __restrict__ mse) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int64_t b = 0; b < nb; ++b) s += partial[b];
    *mse = s / (double)k;
  }
}

// strict "<": the first model wins ties (Algorithm 5's comparison)
__global__ void k_best(const double* __restrict__ mse, int n, int32_t* __restrict__ best) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int b = -1;
    double bv = INFINITY;
    for (int i = 0; i < n; ++i)
      if (mse[i] < bv) {
        bv = mse[i];
        b = i;
      }
    *best = b;
  }
}

struct Routing {
  int32_t* route = nullptr;
  int32_t* tperm = nullptr;
  int64_t* toff = nullptr;
  int32_t* tile_start = nullptr;
};

size_t route_ws_bytes(int64_t k, int p) {
  const size_t kb = ((size_t)k * 4 + 255) & ~size_t(255);
  return 2 * kb + (size_t)(p + 1) * 8 + (size_t)(p + 1) * 4 + 512;
}

Routing route_points(krr_ctx ctx, hipStream_t s, const krr_part_data& D, const void* Xt, int dtype, int64_t k,
                     const std::string& tag, Arena* ar = nullptr) {
  const int p = D.p;
  const size_t kb = ((size_t)k * 4 + 255) & ~size_t(255);
  char* w = (char*)ws_or_arena(ctx, ar, "route" + tag, route_ws_bytes(k, p));
  Routing R;
  R.route = (int32_t*)w;
  R.tperm = (int32_t*)(w + kb);
  R.toff = (int64_t*)(w + 2 * kb);
  R.tile_start = (int32_t*)(w + 2 * kb + (((size_t)(p + 1) * 8 + 255) & ~size_t(255)));
  assign_nearest(ctx, s, Xt, dtype, k, D.d, D.ct_t, p, R.route, nullptr, nullptr, nullptr);
  group_by_key(ctx, s, R.route, k, p, R.tperm, R.toff, nullptr, nullptr,
               ar != nullptr ? ar->take(group_ws_bytes(k, p)) : nullptr);
  hipLaunchKernelGGL(k_tile_prefix, dim3(1), dim3(64), 0, s, (const int64_t*)R.toff, p, R.tile_start);
  check_launch(ctx, s, "tile_prefix");
  return R;
}

// Launch shape of the prediction kernel: the training chunks of a partition
// are split over nsplit workgroups of cps chunks each, writing nsplit x npos
// x nm partial sums.
struct PredShape {
  int64_t nsplit, npos, base;
  int cps;
};

PredShape pred_shape(const krr_part_data& D, int64_t k, int route) {
  const int p = D.p;
  int64_t max_m = 0;
  for (int j = 0; j < p; ++j) max_m = std::max(max_m, D.offsets[j + 1] - D.offsets[j]);
  const int64_t chunks = std::max<int64_t>(1, ceil_div(max_m, NB));
  PredShape S;
  S.base = (route == KRR_ROUTE_NEAREST) ? ceil_div(k, NB) + p : ceil_div(k, NB) * p;
  S.nsplit = std::max<int64_t>(1, std::min<int64_t>(chunks, 2048 / std::max<int64_t>(S.base, 1)));
  S.cps = (int)ceil_div(chunks, S.nsplit);
  S.npos = (route == KRR_ROUTE_NEAREST) ? k : k * p;
  return S;
}

// Predict with nm (<= MAXM) models that share one partitioning.  `dst[q]`
// receives k values (NEAREST) or the k x p matrix (ALL) of model q.
void predict_group(krr_ctx ctx, hipStream_t s, const krr_model* models, int nm, const void* Xt, int dtype, int64_t k,
                   int route, const Routing& R, double* const* dst, Arena* ar = nullptr) {
  const krr_part_data& D = *models[0]->data;
  KRR_REQUIRE(dtype == D.dtype, "test inputs must have the dtype of the training inputs");
  const int p = D.p;
  PredModels M{};
  M.nm = nm;
  M.kernel = models[0]->params.kernel;
  for (int q = 0; q < nm; ++q) {
    M.alpha[q] = models[q]->alpha;
    M.voff[q] = models[q]->d_voff;
    const krr_fit_params& P = models[q]->params;
    const double ng = -1.0 / (2.0 * P.sigma * P.sigma);
    int u = 0;
    while (u < M.nu && !same_kernel_matrix(models[M.uidx_first[u]]->params, P)) ++u;
    if (u == M.nu) {
      M.negu[u] = ng;
      M.ka[u] = P.kernel_a;
      M.kr[u] = P.kernel_r;
      M.kdeg[u] = P.kernel_degree;
      M.uidx_first[u] = q;
      ++M.nu;
    }
    M.uidx[q] = u;
    M.out[q] = dst[q];
    KRR_REQUIRE(models[q]->params.kernel == M.kernel, "models of one call must share the kernel");
  }
  const PredShape S = pred_shape(D, k, route);
  const int64_t base = S.base, nsplit = S.nsplit, npos = S.npos;
  const int cps = S.cps;
  double* part = (double*)ws_or_arena(ctx, ar, "pred_part", (size_t)nsplit * npos * nm * 8);
  {
    KernelTimer kt(ctx, s, "predict", 0.0, 0);
    const dim3 grid = (route == KRR_ROUTE_NEAREST) ? dim3((unsigned)base, 1, (unsigned)nsplit)
                                                   : dim3((unsigned)ceil_div(k, NB), (unsigned)p, (unsigned)nsplit);
    const int rt = route == KRR_ROUTE_NEAREST ? route : (int)KRR_ROUTE_ALL;
    auto launch = [&](auto kern, const auto* Xtp, const auto* Xtr) {
      hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, Xtp, D.d, k, (const int32_t*)R.tperm, (const int64_t*)R.toff,
                         (const int32_t*)R.tile_start, rt, Xtr, (const int64_t*)D.d_offsets, M, p, cps, npos, part);
    };
    if (dtype == KRR_F64) {
      const double* Xtp = (const double*)Xt;
      const double* Xtr = (const double*)D.X;
      switch (M.kernel) {
        case KRR_KERNEL_GAUSSIAN: launch(k_predict<double, KRR_KERNEL_GAUSSIAN>, Xtp, Xtr); break;
        case KRR_KERNEL_POLYNOMIAL: launch(k_predict<double, KRR_KERNEL_POLYNOMIAL>, Xtp, Xtr); break;
        case KRR_KERNEL_SIGMOID: launch(k_predict<double, KRR_KERNEL_SIGMOID>, Xtp, Xtr); break;
        default: launch(k_predict<double, KRR_KERNEL_LINEAR>, Xtp, Xtr); break;
      }
    } else {
      const float* Xtp = (const float*)Xt;
      const float* Xtr = (const float*)D.X;
      switch (M.kernel) {
        case KRR_KERNEL_GAUSSIAN: launch(k_predict<float, KRR_KERNEL_GAUSSIAN>, Xtp, Xtr); break;
        case KRR_KERNEL_POLYNOMIAL: launch(k_predict<float, KRR_KERNEL_POLYNOMIAL>, Xtp, Xtr); break;
        case KRR_KERNEL_SIGMOID: launch(k_predict<float, KRR_KERNEL_SIGMOID>, Xtp, Xtr); break;
        default: launch(k_predict<float, KRR_KERNEL_LINEAR>, Xtp, Xtr); break;
      }
    }
    check_launch(ctx, s, "predict");
  }
  hipLaunchKernelGGL(k_predict_reduce, dim3((unsigned)ceil_div(npos * nm, 256)), dim3(256), 0, s,
                     (const double*)part, (int)nsplit, npos, M,
                     route == KRR_ROUTE_NEAREST ? (const int32_t*)R.tperm : nullptr);
  check_launch(ctx, s, "predict_reduce");
}

// route AVERAGE: ALL into a workspace, then the mean over the p models
void predict_models(krr_ctx ctx, hipStream_t s, const krr_model* models, int nm, const void* Xt, int dtype, int64_t k,
                    int route, const Routing& R, double* const* yhat, Arena* ar = nullptr) {
  const int p = models[0]->data->p;
  if (route != KRR_ROUTE_AVERAGE) {
    predict_group(ctx, s, models, nm, Xt, dtype, k, route, R, yhat, ar);
    return;
  }
  double* all = (double*)ws_or_arena(ctx, ar, "pred_all", (size_t)k * p * nm * 8);
  double* dst[MAXM];
  for (int q = 0; q < nm; ++q) dst[q] = all + (size_t)q * k * p;
  predict_group(ctx, s, models, nm, Xt, dtype, k, KRR_ROUTE_ALL, R, dst, ar);
  for (int q = 0; q < nm; ++q) {
    hipLaunchKernelGGL(k_row_mean, dim3((unsigned)ceil_div(k, 256)), dim3(256), 0, s, (const double*)dst[q], k, p,
                       yhat[q]);
    check_launch(ctx, s, "row_mean");
  }
}

}  // namespace

void run_predict(krr_ctx ctx, hipStream_t s, krr_model model, const void* Xt, int dtype, int64_t k, int route,
                 double* yhat, int32_t* route_out, Arena* ar) {
  KRR_REQUIRE(model->data->d > 0, "empty model");
  auto body = [&]() {
    Routing R;
    if (route == KRR_ROUTE_NEAREST || route_out != nullptr)
      R = route_points(ctx, s, *model->data, Xt, dtype, k, "", ar);
    double* dst[1] = {yhat};
    predict_models(ctx, s, &model, 1, Xt, dtype, k, route, R, dst, ar);
    if (route_out != nullptr)
      KRR_HIP(hipMemcpyAsync(route_out, R.route, (size_t)k * 4, hipMemcpyDeviceToDevice, s));
  };
  if (ar != nullptr || !ctx->graphs || s == nullptr) {
    body();
    return;
  }
  // key: the call's pointers and sizes, and what the launches take from the model
  const krr_part_data& D = *model->data;
  std::string key = "predict";
  for (const void* p : {(const void*)model, Xt, (const void*)yhat, (const void*)route_out, (const void*)model->alpha,
                        (const void*)model->d_voff, (const void*)D.X, (const void*)D.ct_t,
                        (const void*)D.d_offsets})
    key_add(key, p);
  for (int64_t v : {(int64_t)dtype, k, (int64_t)route, (int64_t)D.p, (int64_t)D.d})
    key_add(key, v);
  key_add(key, model->params);
  key.append(reinterpret_cast<const char*>(D.offsets.data()), D.offsets.size() * sizeof(int64_t));
  graph_run(ctx, s, key, body);
}

// ---------------------------------------------------------------------------
// Prediction without device allocation.  Every temporary of run_predict
// (routes, grouping counts and offsets, partial sums, the ALL matrix of the
// AVERAGE route) is carved from `scratch`, a fixed array that each GPU the
// library runs on holds until the process ends.  Its device address differs
// per GPU and is looked up once per device (noalloc_scratch_init, called when
// a context is created); host code uses only that address, never the array's
// name.  Every call on one GPU shares the array: calls that overlap on one
// GPU race.  No temporary needs to start at zero (every value read is written
// earlier in the same call), so nothing is cleared.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_SCRATCH = KRR_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[MAX_DEVICES] = {};

void noalloc_scratch_init(int device) {
  KRR_REQUIRE(device >= 0 && device < MAX_DEVICES, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device] != nullptr) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr)
    fail(KRR_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = (char*)ptr;
}

void run_predict_noalloc(krr_ctx ctx, hipStream_t s, krr_model model, const void* Xt, int dtype, int64_t k, int route,
                         double* yhat, int32_t* route_out) {
  KRR_REQUIRE(model->data->d > 0, "empty model");
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    base = g_scratch_ptr[ctx->device];
  }
  if (base == nullptr) fail(KRR_ESTATE, "scratch address of this device was not set up");
  // the call's temporaries, in the order run_predict takes them
  const krr_part_data& D = *model->data;
  size_t need = 0;
  if (route == KRR_ROUTE_NEAREST || route_out != nullptr) need += al256(route_ws_bytes(k, D.p)) + al256(group_ws_bytes(k, D.p));
  const int pr = route == KRR_ROUTE_AVERAGE ? (int)KRR_ROUTE_ALL : route;
  if (route == KRR_ROUTE_AVERAGE) need += al256((size_t)k * D.p * 8);
  const PredShape S = pred_shape(D, k, pr);
  need += al256((size_t)S.nsplit * S.npos * 8);
  if (need > NOALLOC_SCRATCH)
    fail(KRR_EINVAL, "krr_predict_noalloc: " + std::to_string(k) + " points with " + std::to_string(D.p) +
                         " partitions need " + std::to_string(need) + " bytes of scratch; the fixed scratch holds " +
                         std::to_string(NOALLOC_SCRATCH) + " bytes");
  Arena ar;
  ar.base = base;
  ar.cap = NOALLOC_SCRATCH;
  struct NoAllocScope {
    krr_ctx c;
    explicit NoAllocScope(krr_ctx x) : c(x) { c->noalloc = 1; }
    ~NoAllocScope() { c->noalloc = 0; }
  } scope(ctx);
  run_predict(ctx, s, model, Xt, dtype, k, route, yhat, route_out, &ar);
}

void run_select(krr_ctx ctx, hipStream_t s, const krr_model* models, int n_models, const void* Xv, const void* yv,
                int dtype, int64_t k, int route, double* mse, int32_t* best) {
  const int64_t nb = ceil_div(k, 256);
  const bool label = route == KRR_ROUTE_LABEL;   // every model's prediction per point, then the closest
  int pmax = 1;
  for (int i = 0; i < n_models && label; ++i) pmax = std::max(pmax, (int)models[i]->data->p);
  char* w = (char*)ws_get(ctx, "select", (size_t)k * pmax * 8 * MAXM + (size_t)nb * 8 + (size_t)n_models * 8 + 512);
  double* yh = (double*)w;
  double* partial = yh + k * pmax * MAXM;
  double* d_mse = partial + nb;
  int32_t* d_best = (int32_t*)(d_mse + n_models);
  // models fitted together share their partitioning: route the points once
  // and predict up to MAXM of them per launch
  int done = 0;
  int tag = 0;
  while (done < n_models) {
    const krr_part_data* D = models[done]->data.get();
    int nm = 0;
    while (done + nm < n_models && nm < MAXM && models[done + nm]->data.get() == D &&
           models[done + nm]->params.kernel == models[done]->params.kernel)
      ++nm;
    Routing R;
    if (route == KRR_ROUTE_NEAREST) R = route_points(ctx, s, *D, Xv, dtype, k, "_sel" + std::to_string(tag++));
    const int pc = label ? D->p : 1;
    double* dst[MAXM];
    for (int q = 0; q < nm; ++q) dst[q] = yh + (size_t)q * k * pc;
    predict_models(ctx, s, models + done, nm, Xv, dtype, k, label ? (int)KRR_ROUTE_ALL : route, R, dst);
    for (int q = 0; q < nm; ++q) {
      if (dtype == KRR_F64)
        hipLaunchKernelGGL((k_sqerr<double>), dim3((unsigned)nb), dim3(256), 0, s, (const double*)dst[q], pc,
                           (const double*)yv, k, partial);
      else
        hipLaunchKernelGGL((k_sqerr<float>), dim3((unsigned)nb), dim3(256), 0, s, (const double*)dst[q], pc,
                           (const float*)yv, k, partial);
      check_launch(ctx, s, "sqerr");
      hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, s, (const double*)partial, nb, k, d_mse + done + q);
      check_launch(ctx, s, "mse_final");
    }
    done += nm;
  }
  hipLaunchKernelGGL(k_best, dim3(1), dim3(64), 0, s, (const double*)d_mse, n_models, d_best);
  check_launch(ctx, s, "best");
  char* pin = (char*)pinned_get(ctx, (size_t)n_models * 8 + 64);
  KRR_HIP(hipMemcpyAsync(pin, d_mse, (size_t)n_models * 8 + 8, hipMemcpyDeviceToHost, s));
  KRR_HIP(hipStreamSynchronize(s));
  std::memcpy(mse, pin, (size_t)n_models * 8);
  std::memcpy(best, pin + (size_t)n_models * 8, 4);
}

}  // namespace krr
