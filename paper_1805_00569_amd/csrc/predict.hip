// Prediction (Eq. 7) with the routes of Sections 4.1 / 4.2 and Algorithm 5,
// and model selection by MSE (Eq. 3, Algorithm 5).
//
// NEAREST: each test point is assigned to its nearest centre with the exact
// FP64 assignment kernel (the "MyCluster" step of Algorithm 5), the points
// are grouped by partition, and every 64-point group is predicted by the
// fused kernel below against its partition's training points only.
// ALL / AVERAGE: every 64-point group is predicted by every partition model.
//
// The fused kernel computes, for 64 test points against chunks of 64
// training points, the Gram block on FP64 matrix cores, turns it into kernel
// values and contracts them with alpha, so the k x m kernel matrix is never
// stored.  Every sum has a fixed order (results do not depend on the batch).
#include "common.hpp"

namespace krr {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int KC = 32;
constexpr int LDX = NB + 1;

template <typename TX>
__global__ __launch_bounds__(256) void k_predict(const TX* __restrict__ Xt, int d, int64_t k,
                                                 const int32_t* __restrict__ tperm,
                                                 const int64_t* __restrict__ toff,
                                                 const int32_t* __restrict__ tile_start, int route,
                                                 const TX* __restrict__ Xg, const int64_t* __restrict__ xoff,
                                                 const double* __restrict__ alpha, const int64_t* __restrict__ voff,
                                                 double neg_inv_2s2, int kernel, int p, double* __restrict__ out) {
  int j, tt;
  int64_t t0, tcnt;
  if (route == KRR_ROUTE_NEAREST) {
    const int b = blockIdx.x;
    if (b >= tile_start[p]) return;
    int lo = 0, hi = p;  // find j with tile_start[j] <= b < tile_start[j+1]
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (tile_start[mid] <= b) lo = mid;
      else hi = mid;
    }
    j = lo;
    tt = b - tile_start[j];
    t0 = toff[j] + (int64_t)tt * NB;
    tcnt = min((int64_t)NB, toff[j + 1] - t0);
  } else {
    j = blockIdx.y;
    tt = blockIdx.x;
    t0 = (int64_t)tt * NB;
    tcnt = min((int64_t)NB, k - t0);
  }
  const int64_t x0 = xoff[j];
  const int64_t m = xoff[j + 1] - x0;
  const double* al = alpha + voff[j];
  __shared__ double sT[KC * LDX];
  __shared__ double sX[KC * LDX];
  __shared__ double sNt[NB], sNx[NB];
  __shared__ int64_t srow[NB];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int il = lane & 15, kl = lane >> 4;
  if (t < NB) {
    int64_t src = -1;
    if (t < tcnt) src = (route == KRR_ROUTE_NEAREST) ? (int64_t)tperm[t0 + t] : t0 + t;
    srow[t] = src;
  }
  __syncthreads();
  double part = 0.0;
  for (int64_t xc = 0; xc < m; xc += NB) {
    const int64_t xcnt = min((int64_t)NB, m - xc);
    d4 acc[4];
#pragma unroll
    for (int xb = 0; xb < 4; ++xb) acc[xb] = d4{0.0, 0.0, 0.0, 0.0};
    double nrm = 0.0;
    for (int k0 = 0; k0 < d; k0 += KC) {
      const int kc = min(KC, d - k0);
      __syncthreads();
      for (int e = t; e < NB * KC; e += 256) {
        const int row = e / KC, kk = e - row * KC;
        double vt = 0.0, vx = 0.0;
        if (kk < kc) {
          const int64_t sr = srow[row];
          if (sr >= 0) vt = (double)Xt[sr * d + k0 + kk];
          if (row < xcnt) vx = (double)Xg[(x0 + xc + row) * d + k0 + kk];
        }
        sT[kk * LDX + row] = vt;
        sX[kk * LDX + row] = vx;
      }
      __syncthreads();
      if (t < NB) {
        for (int kk = 0; kk < kc; ++kk) nrm = fma(sX[kk * LDX + t], sX[kk * LDX + t], nrm);
      } else if (t < 2 * NB && xc == 0) {
        for (int kk = 0; kk < kc; ++kk) nrm = fma(sT[kk * LDX + t - NB], sT[kk * LDX + t - NB], nrm);
      }
      for (int kb = 0; kb < kc; kb += 4) {
        const int ko = (kb + kl) * LDX;
        const double bt = sT[ko + 16 * w + il];
#pragma unroll
        for (int xb = 0; xb < 4; ++xb)
          acc[xb] = __builtin_amdgcn_mfma_f64_16x16x4f64(sX[ko + 16 * xb + il], bt, acc[xb], 0, 0, 0);
      }
    }
    if (t < NB) sNx[t] = nrm;
    else if (t < 2 * NB && xc == 0) sNt[t - NB] = nrm;
    __syncthreads();
    const int tl = 16 * w + il;
    const double nt = sNt[tl];
#pragma unroll
    for (int xb = 0; xb < 4; ++xb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int xl = 16 * xb + kl + 4 * v;
        if (xl < xcnt) {
          const double G = acc[xb][v];
          double kv;
          if (kernel == KRR_KERNEL_GAUSSIAN) kv = exp(fmax(0.0, (nt + sNx[xl]) - 2.0 * G) * neg_inv_2s2);
          else kv = G;
          part = fma(al[xc + xl], kv, part);
        }
      }
  }
  // lanes il, il+16, il+32, il+48 hold partial sums of the same test point
  part += __shfl_xor(part, 16, 64);
  part += __shfl_xor(part, 32, 64);
  const int tl = 16 * w + il;
  if (kl == 0 && tl < tcnt) {
    if (route == KRR_ROUTE_NEAREST) out[srow[tl]] = part;
    else out[(t0 + tl) * p + j] = part;
  }
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

template <typename TY>
__global__ __launch_bounds__(256) void k_sqerr(const double* __restrict__ yhat, const TY* __restrict__ y, int64_t k,
                                               double* __restrict__ partial) {
  __shared__ double sred[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double e = 0.0;
  if (i < k) {
    const double dlt = yhat[i] - (double)y[i];
    e = dlt * dlt;
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
  int32_t* route;
  int32_t* tperm;
  int64_t* toff;
  int32_t* tile_start;
};

Routing route_points(krr_ctx ctx, hipStream_t s, krr_model model, const void* Xt, int dtype, int64_t k,
                     const std::string& tag) {
  const int p = model->data->p;
  const size_t kb = ((size_t)k * 4 + 255) & ~size_t(255);
  char* w = (char*)ws_get(ctx, "route" + tag, 2 * kb + (size_t)(p + 1) * 8 + (size_t)(p + 1) * 4 + 512);
  Routing R;
  R.route = (int32_t*)w;
  R.tperm = (int32_t*)(w + kb);
  R.toff = (int64_t*)(w + 2 * kb);
  R.tile_start = (int32_t*)(w + 2 * kb + (((size_t)(p + 1) * 8 + 255) & ~size_t(255)));
  assign_nearest(ctx, s, Xt, dtype, k, model->data->d, model->data->ct_t, p, R.route, nullptr, nullptr, nullptr);
  group_by_key(ctx, s, R.route, k, p, R.tperm, R.toff, nullptr, nullptr);
  hipLaunchKernelGGL(k_tile_prefix, dim3(1), dim3(64), 0, s, (const int64_t*)R.toff, p, R.tile_start);
  check_launch(ctx, s, "tile_prefix");
  return R;
}

template <typename TX>
void predict_launch(krr_ctx ctx, hipStream_t s, krr_model model, const TX* Xt, int64_t k, int route,
                    const Routing* R, double* out) {
  const krr_part_data& D = *model->data;
  const double neg = -1.0 / (2.0 * model->params.sigma * model->params.sigma);
  const int p = D.p;
  if (route == KRR_ROUTE_NEAREST) {
    const unsigned nblk = (unsigned)(ceil_div(k, NB) + p);
    hipLaunchKernelGGL((k_predict<TX>), dim3(nblk), dim3(256), 0, s, Xt, D.d, k, (const int32_t*)R->tperm,
                       (const int64_t*)R->toff, (const int32_t*)R->tile_start, route, (const TX*)D.X,
                       (const int64_t*)D.d_offsets, (const double*)model->alpha, (const int64_t*)model->d_voff, neg,
                       model->params.kernel, p, out);
  } else {
    hipLaunchKernelGGL((k_predict<TX>), dim3((unsigned)ceil_div(k, NB), (unsigned)p), dim3(256), 0, s, Xt, D.d, k,
                       nullptr, nullptr, nullptr, KRR_ROUTE_ALL, (const TX*)D.X, (const int64_t*)D.d_offsets,
                       (const double*)model->alpha, (const int64_t*)model->d_voff, neg, model->params.kernel, p,
                       out);
  }
  check_launch(ctx, s, "predict");
}

void predict_into(krr_ctx ctx, hipStream_t s, krr_model model, const void* Xt, int dtype, int64_t k, int route,
                  const Routing* R, double* yhat) {
  const int p = model->data->p;
  KRR_REQUIRE(dtype == model->data->dtype, "test inputs must have the dtype of the training inputs");
  double* dst = yhat;
  if (route == KRR_ROUTE_AVERAGE) dst = (double*)ws_get(ctx, "pred_all", (size_t)k * p * 8);
  if (dtype == KRR_F64)
    predict_launch<double>(ctx, s, model, (const double*)Xt, k, route, R, dst);
  else
    predict_launch<float>(ctx, s, model, (const float*)Xt, k, route, R, dst);
  if (route == KRR_ROUTE_AVERAGE) {
    hipLaunchKernelGGL(k_row_mean, dim3((unsigned)ceil_div(k, 256)), dim3(256), 0, s, (const double*)dst, k, p,
                       yhat);
    check_launch(ctx, s, "row_mean");
  }
}

}  // namespace

void run_predict(krr_ctx ctx, hipStream_t s, krr_model model, const void* Xt, int dtype, int64_t k, int route,
                 double* yhat, int32_t* route_out) {
  KRR_REQUIRE(model->data->d > 0, "empty model");
  Routing R{};
  if (route == KRR_ROUTE_NEAREST || route_out != nullptr) R = route_points(ctx, s, model, Xt, dtype, k, "");
  predict_into(ctx, s, model, Xt, dtype, k, route, &R, yhat);
  if (route_out != nullptr)
    KRR_HIP(hipMemcpyAsync(route_out, R.route, (size_t)k * 4, hipMemcpyDeviceToDevice, s));
}

void run_select(krr_ctx ctx, hipStream_t s, const krr_model* models, int n_models, const void* Xv, const void* yv,
                int dtype, int64_t k, int route, double* mse, int32_t* best) {
  const int64_t nb = ceil_div(k, 256);
  char* w = (char*)ws_get(ctx, "select", (size_t)k * 8 + (size_t)nb * 8 + (size_t)n_models * 8 + 512);
  double* yhat = (double*)w;
  double* partial = yhat + k;
  double* d_mse = partial + nb;
  int32_t* d_best = (int32_t*)(d_mse + n_models);
  // models fitted together share their partition: route the points once
  std::map<const krr_part_data*, Routing> routes;
  for (int i = 0; i < n_models; ++i) {
    const krr_model M = models[i];
    Routing R{};
    if (route == KRR_ROUTE_NEAREST) {
      auto it = routes.find(M->data.get());
      if (it == routes.end()) {
        R = route_points(ctx, s, M, Xv, dtype, k, "_sel" + std::to_string(routes.size()));
        routes[M->data.get()] = R;
      } else {
        R = it->second;
      }
    }
    predict_into(ctx, s, M, Xv, dtype, k, route, &R, yhat);
    if (dtype == KRR_F64)
      hipLaunchKernelGGL((k_sqerr<double>), dim3((unsigned)nb), dim3(256), 0, s, (const double*)yhat,
                         (const double*)yv, k, partial);
    else
      hipLaunchKernelGGL((k_sqerr<float>), dim3((unsigned)nb), dim3(256), 0, s, (const double*)yhat,
                         (const float*)yv, k, partial);
    check_launch(ctx, s, "sqerr");
    hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, s, (const double*)partial, nb, k, d_mse + i);
    check_launch(ctx, s, "mse_final");
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
