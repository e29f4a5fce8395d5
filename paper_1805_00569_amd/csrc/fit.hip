// krr_fit: group the training points by partition, form every system
// A_s = K_s + lambda_s I (Table 1 Gaussian or linear kernel, Eq. 6), factor
// the whole batch (cholesky.hip), solve for alpha (solve.hip), refine in
// mixed precision, and hand out one model per (sigma, lambda) setting
// (Algorithm 5: p local models per setting).
#include "common.hpp"

#include <algorithm>
#include <cmath>
#include <exception>

namespace krr {

bool cholesky_factor(krr_ctx ctx, hipStream_t s, int prec, const SysDesc* desc, SysStatus* st, int n_sys, int Tmax,
                     void* A, void* Wt, int level, bool bf16, const SysDesc* hdesc, void* pack, double* zfwd);
int64_t pack_slot_elems(int T, int Wp);
void trsv_forward(krr_ctx ctx, hipStream_t s, int prec, const SysDesc* desc, const SysStatus* st, int n_sys,
                  int Tmax, int64_t v_tot, const void* A, const void* Wt, const double* b, double* z,
                  int skip_converged);
void trsv_backward(krr_ctx ctx, hipStream_t s, int prec, const SysDesc* desc, const SysStatus* st, int n_sys,
                   int Tmax, int64_t v_tot, const void* A, const void* Wt, const double* z, double* x,
                   double* alpha_acc, int skip_converged);
void pivot_range(krr_ctx ctx, hipStream_t s, int prec, const SysDesc* desc, SysStatus* st, int n_sys, const void* A,
                 int level);
void correction_norms(krr_ctx ctx, hipStream_t s, const SysDesc* desc, SysStatus* st, int n_sys, const double* delta,
                      const double* alpha);
void residual_check(krr_ctx ctx, hipStream_t s, const SysDesc* desc, SysStatus* st, int n_sys, int p, int n_groups,
                    const int32_t* grp_first, const int32_t* grp_next, int Tmax, const double* K64,
                    const double* alpha, const double* y, double* r, double* P, const int64_t* p_off, double* rn,
                    double* yn, const int64_t* n_off, double tol, int will_refine, int32_t* active, double* Pabs,
                    double* glo, double* ghi);

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int TILE = NB * NB;
constexpr int KC = 32;        // feature chunk staged in LDS
constexpr int LDX = NB + 1;   // padded LDS row (doubles)

__device__ __forceinline__ int64_t tile_index(int i, int j) { return (int64_t)i * (i + 1) / 2 + j; }

// Kernel formation for partition j = blockIdx.y, tile (ti, tj) = triangle
// index blockIdx.x.  The Gram block G = X_ti X_tj^T is computed once in FP64
// on matrix cores (v_mfma_f64_16x16x4f64) and reused by every setting of the
// partition: A_s(r, c) = exp(-(|x_r|^2 + |x_c|^2 - 2 G(r, c)) / (2 sigma_s^2)),
// the diagonal set to exactly 1 + lambda_s; rows/columns past m are the
// identity.  STORE: 0 -> FP64 tiles; 1 -> FP32 tiles; 2 -> FP32 tiles plus the
// FP64 kernel tiles K (without the shift), written once for every group of
// settings of the partition that share the kernel and sigma (settings that
// differ only in lambda share K; the refinement residual adds each shift).
// Settings are visited by group (grp_first[g], then grp_next[...]): the
// kernel values are computed once per group and written to every setting of
// the group with its own shift.
// GENERAL: the batch has polynomial or sigmoid settings (without it the
// code holds only the Gaussian and linear kernels, and fewer registers).
// Four workgroups per CU (registers capped at 128): the exponentials and the
// stores of one workgroup overlap the loads and MFMAs of the others.
template <typename TX, int STORE, bool GENERAL>
__global__ __launch_bounds__(256, 4) void k_form(const TX* __restrict__ Xg, int d, const SysDesc* __restrict__ desc,
                                              int p, int n_groups, const int32_t* __restrict__ grp_first,
                                              const int32_t* __restrict__ grp_next, void* __restrict__ Aout,
                                              double* __restrict__ K64) {
  const int j = blockIdx.y;
  const SysDesc D0 = desc[j];
  const int T = D0.T;
  if (T == 0) return;
  const int bx = blockIdx.x;
  int ti = (int)((sqrt(8.0 * (double)bx + 1.0) - 1.0) * 0.5);
  while ((int64_t)ti * (ti + 1) / 2 > bx) --ti;
  while ((int64_t)(ti + 1) * (ti + 2) / 2 <= bx) ++ti;
  const int tj = bx - ti * (ti + 1) / 2;
  if (ti >= T) return;
  const int m = D0.m;
  __shared__ double sXi[KC * LDX + 1];   // + a spare slot for staged values past d
  __shared__ double sXj[KC * LDX + 1];
  __shared__ double sNi[NB], sNj[NB];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int r0 = 32 * (w & 1), c0 = 32 * (w >> 1);
  const int il = lane & 15, kl = lane >> 4;
  const int rows_i = min(NB, m - ti * NB), rows_j = min(NB, m - tj * NB);
  const TX* Xi = Xg + (D0.x_off + (int64_t)ti * NB) * d;
  const TX* Xj = Xg + (D0.x_off + (int64_t)tj * NB) * d;
  d4 acc[2][2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) acc[cb][rb] = d4{0.0, 0.0, 0.0, 0.0};
  double nrm = 0.0;  // thread t < 64: |x_i(t)|^2, 64 <= t < 128: |x_j(t-64)|^2
  for (int k0 = 0; k0 < d; k0 += KC) {
    const int kc = min(KC, d - k0);
    __syncthreads();
    // unconditional loads from clamped addresses, then select and store
    TX li[NB * KC / 256], lj[NB * KC / 256];
#pragma unroll
    for (int u = 0; u < NB * KC / 256; ++u) {
      const int e = t + u * 256;
      const int row = e / KC, kk = min(e - row * KC, kc - 1);
      li[u] = Xi[(int64_t)min(row, rows_i - 1) * d + k0 + kk];
      lj[u] = Xj[(int64_t)min(row, rows_j - 1) * d + k0 + kk];
    }
    // stored unconditionally: rows past m only feed entries that the
    // epilogue overrides; the k slots past d read by the last 4-wide MFMA
    // step are zeroed below (selecting on a loaded value would turn into a
    // branch around the load)
#pragma unroll
    for (int u = 0; u < NB * KC / 256; ++u) {
      const int e = t + u * 256;
      const int row = e / KC, kk = e - row * KC;
      const int slot = (kk < kc) ? kk * LDX + row : KC * LDX;   // past d: the spare slot
      sXi[slot] = (double)li[u];
      sXj[slot] = (double)lj[u];
    }
    const int kc4 = (kc + 3) & ~3;
    for (int e = t; e < (kc4 - kc) * NB; e += 256) {
      const int kk = kc + e / NB, row = e % NB;
      sXi[kk * LDX + row] = 0.0;
      sXj[kk * LDX + row] = 0.0;
    }
    __syncthreads();
    if (t < NB) {
      for (int kk = 0; kk < kc; ++kk) nrm = fma(sXi[kk * LDX + t], sXi[kk * LDX + t], nrm);
    } else if (t < 2 * NB) {
      for (int kk = 0; kk < kc; ++kk) nrm = fma(sXj[kk * LDX + t - NB], sXj[kk * LDX + t - NB], nrm);
    }
    for (int kb = 0; kb < kc; kb += 4) {
      const int ko = (kb + kl) * LDX;
      double a[2], b[2];
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) a[cb] = sXj[ko + c0 + 16 * cb + il];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) b[rb] = sXi[ko + r0 + 16 * rb + il];
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
          acc[cb][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[cb], b[rb], acc[cb][rb], 0, 0, 0);
    }
  }
  if (t < NB) sNi[t] = nrm;
  else if (t < 2 * NB) sNj[t - NB] = nrm;
  __syncthreads();
  const int64_t toff = tile_index(ti, tj) * TILE;
  for (int g = 0; g < n_groups; ++g) {
    int q = grp_first[g];
    const SysDesc Dg = desc[q * p + j];
    double kv[2][2][4];   // kernel values of the group (identity past m)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = c0 + 16 * cb + kl + 4 * v;   // FP64 MFMA result row of register v
          const int r = r0 + 16 * rb + il;
          const int gr = ti * NB + r, gc = tj * NB + c;
          const double G = acc[cb][rb][v];
          double k;
          if (gr >= m || gc >= m) k = (gr == gc) ? 1.0 : 0.0;
          else if (Dg.kernel == KRR_KERNEL_GAUSSIAN)
            k = (gr == gc) ? 1.0 : exp(fmax(0.0, (sNi[r] + sNj[c]) - 2.0 * G) * Dg.neg_inv_2s2);
          else if (GENERAL && Dg.kernel == KRR_KERNEL_POLYNOMIAL) k = poly_kernel(G, Dg.ka, Dg.kr, Dg.kdeg);
          else if (GENERAL && Dg.kernel == KRR_KERNEL_SIGMOID) k = tanh(Dg.ka * G + Dg.kr);
          else k = G;
          kv[cb][rb][v] = k;
          if (STORE == 2) K64[Dg.k_off + toff + c * NB + r] = k;
        }
    for (; q >= 0; q = grp_next[q]) {
      const SysDesc Dq = desc[q * p + j];
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int c = c0 + 16 * cb + kl + 4 * v;
            const int r = r0 + 16 * rb + il;
            const int gr = ti * NB + r, gc = tj * NB + c;
            const double val = (gr == gc && gr < m) ? kv[cb][rb][v] + Dq.lambda : kv[cb][rb][v];
            const int64_t e = Dq.a_off + toff + c * NB + r;
            if (STORE == 0) reinterpret_cast<double*>(Aout)[e] = val;
            else reinterpret_cast<float*>(Aout)[e] = (float)val;
          }
    }
  }
}

// Padded right-hand sides: b[v_off + r] = y_grouped[x_off + r] for r < m, else 0.
__global__ void k_pad_rhs(const SysDesc* __restrict__ desc, int n_sys, const double* __restrict__ yg,
                          double* __restrict__ b) {
  const int s = blockIdx.y;
  const SysDesc D = desc[s];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D.T * NB) return;
  b[D.v_off + r] = (r < D.m) ? yg[D.x_off + r] : 0.0;
}

__global__ void k_zero_status(SysStatus* st, int n) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) {
    st[s].status = 0;
    st[s].failed_pivot = 0;
    st[s].refine_iters = 0;
    st[s].converged = 0;
    st[s].stalled = 0;
    st[s].corr = 0;
    st[s].rel_residual = -1.0;
    st[s].prev_rel = -1.0;
    st[s].ynorm = 0.0;
    st[s].kappa_l = 1.0;
    st[s].kappa_u = -1.0;
    st[s].dnorm = -1.0;
    st[s].prev_dnorm = -1.0;
    st[s].anorm = 0.0;
    st[s].err_est = -1.0;
  }
}

// Systems escalated to `level`: clear their failure / refinement state (the
// refinement step count is kept); k_restore_tiles rebuilds their FP32 tiles
// from the shared FP64 kernel tiles plus the system's shift (the values
// k_form wrote), since the failed factorisation overwrote them.
__global__ void k_reset_level(const SysDesc* __restrict__ desc, SysStatus* __restrict__ st, int n, int level) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n && desc[s].level == level) {
    st[s].status = 0;
    st[s].failed_pivot = 0;
    st[s].converged = 0;
    st[s].stalled = 0;
    st[s].prev_rel = -1.0;
    st[s].corr = 0;
    st[s].kappa_l = 1.0;
    st[s].dnorm = -1.0;
    st[s].prev_dnorm = -1.0;
    st[s].err_est = -1.0;
  }
}

__global__ __launch_bounds__(256) void k_restore_tiles(const SysDesc* __restrict__ desc, const double* __restrict__ K64,
                                                       float* __restrict__ A, int level) {
  const int s = blockIdx.y;
  const SysDesc D = desc[s];
  if (D.level != level) return;
  const int bx = blockIdx.x;
  int ti = (int)((sqrt(8.0 * (double)bx + 1.0) - 1.0) * 0.5);
  while ((int64_t)ti * (ti + 1) / 2 > bx) --ti;
  while ((int64_t)(ti + 1) * (ti + 2) / 2 <= bx) ++ti;
  const int tj = bx - ti * (ti + 1) / 2;
  if (ti >= D.T) return;
  const int64_t toff = tile_index(ti, tj) * TILE;
  for (int e = threadIdx.x; e < TILE; e += 256) {
    const int c = e >> 6, r = e & 63;
    const int gr = ti * NB + r, gc = tj * NB + c;
    const double kv = K64[D.k_off + toff + e];
    A[D.a_off + toff + e] = (float)((gr == gc && gr < D.m) ? kv + D.lambda : kv);
  }
}

__global__ void k_zero_f64(double* a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

__global__ void k_zero_i32(int32_t* a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

template <typename TX, bool GENERAL>
void launch_form_k(hipStream_t s, int prec, dim3 grid, const TX* X, int d, const SysDesc* desc, int p, int n_groups,
                   const int32_t* grp_first, const int32_t* grp_next, void* A, double* K64) {
  if (prec == KRR_PREC_FP64)
    hipLaunchKernelGGL((k_form<TX, 0, GENERAL>), grid, dim3(256), 0, s, X, d, desc, p, n_groups, grp_first,
                       grp_next, A, K64);
  else if (prec == KRR_PREC_FP32)
    hipLaunchKernelGGL((k_form<TX, 1, GENERAL>), grid, dim3(256), 0, s, X, d, desc, p, n_groups, grp_first,
                       grp_next, A, K64);
  else
    hipLaunchKernelGGL((k_form<TX, 2, GENERAL>), grid, dim3(256), 0, s, X, d, desc, p, n_groups, grp_first,
                       grp_next, A, K64);
}

template <typename TX>
void launch_form(krr_ctx ctx, hipStream_t s, int prec, const void* Xg, int d, const SysDesc* desc, int p,
                 int n_groups, const int32_t* grp_first, const int32_t* grp_next, int Tmax, void* A, double* K64,
                 bool general) {
  const int64_t ntri = (int64_t)Tmax * (Tmax + 1) / 2;
  if (ntri == 0) return;
  const dim3 grid((unsigned)ntri, (unsigned)p);
  const TX* X = (const TX*)Xg;
  KernelTimer kt(ctx, s, "form_kernel", 0.0, 0);
  if (general)
    launch_form_k<TX, true>(s, prec, grid, X, d, desc, p, n_groups, grp_first, grp_next, A, K64);
  else
    launch_form_k<TX, false>(s, prec, grid, X, d, desc, p, n_groups, grp_first, grp_next, A, K64);
  check_launch(ctx, s, "form");
}

}  // namespace

// Settings whose kernel matrices are equal: the same kernel with the same
// sigma (Gaussian) or a, r, d (polynomial; a, r for the sigmoid).
bool same_kernel_matrix(const krr_fit_params& a, const krr_fit_params& b) {
  if (a.kernel != b.kernel) return false;
  switch (a.kernel) {
    case KRR_KERNEL_GAUSSIAN: return a.sigma == b.sigma;
    case KRR_KERNEL_POLYNOMIAL:
      return a.kernel_a == b.kernel_a && a.kernel_r == b.kernel_r && a.kernel_degree == b.kernel_degree;
    case KRR_KERNEL_SIGMOID: return a.kernel_a == b.kernel_a && a.kernel_r == b.kernel_r;
    default: return true;
  }
}

// A persistent factorisation that gave up waiting marks its systems
// KRR_EDEVICE: the whole call fails.
static void check_gave_up(const SysStatus* st_h, int n_sys) {
  for (int i = 0; i < n_sys; ++i)
    if (st_h[i].status == KRR_EDEVICE)
      fail(KRR_EDEVICE, "the persistent factorisation gave up waiting for a stage (KRR_OPT_PERSIST_WAIT_MS)");
}

void run_fit(krr_ctx ctx, hipStream_t s, const void* X, const void* y, int dtype, int64_t n, int d,
             const int32_t* assign, const double* centroids, int p, const krr_fit_params* params, int n_params,
             krr_model* models, krr_part_info* info, FitDirect* direct) {
  KRR_REQUIRE(direct == nullptr || n_params == 1, "a direct fit takes one setting");
  const int prec = params[0].prec;
  const size_t xes = (dtype == KRR_F64) ? 8 : 4;
  const size_t aes = (prec == KRR_PREC_FP64) ? 8 : 4;

  // 1. stable grouping by partition
  char* g = (char*)ws_get(ctx, "fit_group", (size_t)n * 4 + (size_t)(p + 1) * 8 + 64);
  int32_t* perm = (int32_t*)g;
  int64_t* off_d = (int64_t*)(g + (((size_t)n * 4 + 15) & ~size_t(15)));
  group_by_key(ctx, s, assign, n, p, perm, off_d, nullptr, nullptr);
  int64_t* off_h = (int64_t*)pinned_get(ctx, (size_t)(p + 1) * 8 + 4096);
  KRR_HIP(hipMemcpyAsync(off_h, off_d, (size_t)(p + 1) * 8, hipMemcpyDeviceToHost, s));
  KRR_HIP(hipStreamSynchronize(s));
  std::vector<int64_t> off(off_h, off_h + p + 1);

  // 2. partition data owned by the models
  auto data = std::make_shared<krr_part_data>();
  const size_t xbytes = ((size_t)n * d * xes + 255) & ~size_t(255);
  const size_t cbytes = ((size_t)p * d * 8 + 255) & ~size_t(255);
  const size_t obytes = ((size_t)(p + 1) * 8 + 255) & ~size_t(255);
  data->bytes = xbytes + 2 * cbytes + obytes;
  if (direct != nullptr) {
    data->base = ws_get(ctx, "fit_direct_data", data->bytes);   // not owned: ctx stays null
  } else {
    data->base = model_alloc(ctx, data->bytes);
    data->ctx = ctx;
    ctx->n_datas += 1;
  }
  // on an error below, wait for the queued work that reads or writes the
  // partition data before it is released (the guard unwinds before `data`)
  struct SyncOnUnwind {
    hipStream_t st;
    int n0 = std::uncaught_exceptions();
    ~SyncOnUnwind() {
      if (std::uncaught_exceptions() > n0) (void)hipStreamSynchronize(st);
    }
  } unwind_sync{s};
  data->p = p;
  data->d = d;
  data->dtype = dtype;
  data->n = n;
  data->X = data->base;
  data->centroids = (double*)((char*)data->base + xbytes);
  data->ct_t = (double*)((char*)data->base + xbytes + cbytes);
  data->d_offsets = (int64_t*)((char*)data->base + xbytes + 2 * cbytes);
  data->offsets = off;
  KRR_HIP(hipMemcpyAsync(data->centroids, centroids, (size_t)p * d * 8, hipMemcpyDeviceToDevice, s));
  transpose_centroids(ctx, s, centroids, p, d, data->ct_t);
  KRR_HIP(hipMemcpyAsync(data->d_offsets, off_d, (size_t)(p + 1) * 8, hipMemcpyDeviceToDevice, s));
  // graphs on a stream other than the legacy default one: the grouped inputs
  // go to a workspace buffer (a stable address for the replays) and are
  // copied into the partition data afterwards
  const bool use_graph = ctx->graphs && s != nullptr && !ctx->serial_fit;
  void* Xg = use_graph ? ws_get(ctx, "fit_xg", xbytes) : data->X;

  // 3. system descriptors
  const int n_sys = n_params * p;
  std::vector<SysDesc> desc(n_sys);
  std::vector<int64_t> p_off(n_sys), n_off(n_sys);
  int64_t a_tot = 0, w_tot = 0, v_tot = 0, p_tot = 0, n_tot = 0, pk_tot = 0;
  // mixed precision: FP64 kernel tiles per (partition, group of settings with
  // the same kernel matrix: same kernel and sigma, or a, r, d); grp_first /
  // grp_next list each group's settings
  std::vector<int32_t> grp_of(n_params), grp_first, grp_next(n_params, -1);
  for (int q = 0; q < n_params; ++q) {
    int g = -1;
    for (int h = 0; h < (int)grp_first.size() && g < 0; ++h) {
      const krr_fit_params& P0 = params[grp_first[h]];
      if (same_kernel_matrix(P0, params[q])) g = h;
    }
    if (g < 0) {
      g = (int)grp_first.size();
      grp_first.push_back(q);
    } else {
      int last = grp_first[g];
      while (grp_next[last] >= 0) last = grp_next[last];
      grp_next[last] = q;
    }
    grp_of[q] = g;
  }
  const int n_groups = (int)grp_first.size();
  std::vector<int64_t> k_off((size_t)n_groups * p);
  int64_t k_tot = 0;
  for (int g = 0; g < n_groups; ++g)
    for (int jp = 0; jp < p; ++jp) {
      k_off[(size_t)g * p + jp] = k_tot;
      k_tot += tri(ceil_div(off[jp + 1] - off[jp], NB)) * TILE;
    }
  int Tmax = 0;
  for (int q = 0; q < n_params; ++q)
    for (int jp = 0; jp < p; ++jp) {
      SysDesc& D = desc[q * p + jp];
      const int64_t m = off[jp + 1] - off[jp];
      D.m = (int32_t)m;
      D.T = (int32_t)ceil_div(m, NB);
      D.part = jp;
      D.param = q;
      D.a_off = a_tot;
      D.w_off = w_tot;
      D.v_off = v_tot;
      D.x_off = off[jp];
      D.neg_inv_2s2 = -1.0 / (2.0 * params[q].sigma * params[q].sigma);
      D.lambda = params[q].lambda_times_m ? params[q].lambda * (double)m : params[q].lambda;
      D.kernel = params[q].kernel;
      D.ka = params[q].kernel_a;
      D.kr = params[q].kernel_r;
      D.kdeg = params[q].kernel_degree;
      D.wp = ctx->force_wp > 0 ? ctx->force_wp : tuned_panel(ctx, prec, m);
      D.level = 0;
      D.pk_off = pk_tot;
      pk_tot += (prec == KRR_PREC_MIXED) ? pack_slot_elems(D.T, D.wp) : 0;
      D.k_off = k_off[(int64_t)grp_of[q] * p + jp];
      D.g_sys = grp_first[grp_of[q]] * p + jp;
      D.pad_ = 0;
      a_tot += tri(D.T) * TILE;
      w_tot += (int64_t)D.T * TILE;
      v_tot += (int64_t)D.T * NB;
      p_off[q * p + jp] = p_tot;
      n_off[q * p + jp] = n_tot;
      p_tot += (int64_t)D.T * D.T * NB;
      n_tot += D.T;
      Tmax = std::max(Tmax, (int)D.T);
    }
  const bool mixed = prec == KRR_PREC_MIXED;

  // 4. workspace (grown inside the HBM budget, reused across calls)
  void* A = ws_get(ctx, "fit_A", (size_t)std::max<int64_t>(a_tot, 1) * aes);
  void* Wt = ws_get(ctx, "fit_W", (size_t)std::max<int64_t>(w_tot, 1) * aes);
  double* K64 = mixed ? (double*)ws_get(ctx, "fit_K64", (size_t)std::max<int64_t>(k_tot, 1) * 8) : nullptr;
  void* pack = mixed ? ws_get(ctx, "fit_pack", (size_t)std::max<int64_t>(pk_tot, 1) * 2) : nullptr;
  const size_t vb = (size_t)std::max<int64_t>(v_tot, 1) * 8;
  char* vecs = (char*)ws_get(ctx, "fit_vec", 5 * vb);
  double* yg = (double*)ws_get(ctx, "fit_yg", (size_t)n * 8);
  double* rhs = (double*)vecs;
  double* alpha = (double*)(vecs + vb);
  double* zb = (double*)(vecs + 2 * vb);
  double* rb = (double*)(vecs + 3 * vb);
  double* db = (double*)(vecs + 4 * vb);
  const size_t meta = (size_t)n_sys * (sizeof(SysDesc) + sizeof(SysStatus) + 16) + 64;
  char* mb = (char*)ws_get(ctx, "fit_meta", meta);
  SysDesc* d_desc = (SysDesc*)mb;
  SysStatus* d_st = (SysStatus*)(mb + (size_t)n_sys * sizeof(SysDesc));
  int64_t* d_poff = (int64_t*)(mb + (size_t)n_sys * (sizeof(SysDesc) + sizeof(SysStatus)));
  int64_t* d_noff = d_poff + n_sys;
  int32_t* d_active = (int32_t*)(d_noff + n_sys);
  double* P = nullptr;
  double* Pabs = nullptr;
  double* rn = nullptr;
  double* yn = nullptr;
  double* glo = nullptr;
  double* ghi = nullptr;
  if (mixed) {
    P = (double*)ws_get(ctx, "fit_P", (size_t)std::max<int64_t>(p_tot, 1) * 8);
    Pabs = (double*)ws_get(ctx, "fit_Pabs", (size_t)std::max<int64_t>(p_tot, 1) * 8);
    const int64_t nt1 = std::max<int64_t>(n_tot, 1);
    char* nb = (char*)ws_get(ctx, "fit_norms", (size_t)nt1 * 32);
    rn = (double*)nb;
    yn = rn + nt1;
    glo = yn + nt1;
    ghi = glo + nt1;
  }

  // host -> device descriptors through pinned staging (kept until the sync below)
  const size_t up_bytes = (size_t)n_sys * (sizeof(SysDesc) + 16);
  const size_t dn_bytes = (size_t)n_sys * sizeof(SysStatus);
  // groups: grp_first[n_groups], grp_next[n_params], then {0, -1}: the one-setting
  // group that the plain per-system sequence forms each system with
  const size_t grp_bytes = (size_t)(n_groups + n_params + 2) * 4;
  int32_t* d_grp = (int32_t*)ws_get(ctx, "fit_groups", grp_bytes + 64);
  char* pin = (char*)pinned_get(ctx, up_bytes + dn_bytes + 4096 + grp_bytes);
  int32_t* gpin = (int32_t*)(pin + up_bytes + dn_bytes + 4096);
  std::memcpy(gpin, grp_first.data(), (size_t)n_groups * 4);
  std::memcpy(gpin + n_groups, grp_next.data(), (size_t)n_params * 4);
  gpin[n_groups + n_params] = 0;
  gpin[n_groups + n_params + 1] = -1;
  KRR_HIP(hipMemcpyAsync(d_grp, gpin, grp_bytes, hipMemcpyHostToDevice, s));
  std::memcpy(pin, desc.data(), (size_t)n_sys * sizeof(SysDesc));
  std::memcpy(pin + (size_t)n_sys * sizeof(SysDesc), p_off.data(), (size_t)n_sys * 8);
  std::memcpy(pin + (size_t)n_sys * (sizeof(SysDesc) + 8), n_off.data(), (size_t)n_sys * 8);
  KRR_HIP(hipMemcpyAsync(d_desc, pin, (size_t)n_sys * sizeof(SysDesc), hipMemcpyHostToDevice, s));
  KRR_HIP(hipMemcpyAsync(d_poff, pin + (size_t)n_sys * sizeof(SysDesc), (size_t)n_sys * 16, hipMemcpyHostToDevice,
                         s));

  // 5-8. grouped inputs, padded right-hand sides, form, factor, solve, and
  // (mixed precision) the first refinement steps: the device phase of the
  // fit, which a graph replay may stand in for
  bool general = false;   // polynomial or sigmoid settings in the batch
  for (int q = 0; q < n_params; ++q)
    general |= params[q].kernel == KRR_KERNEL_POLYNOMIAL || params[q].kernel == KRR_KERNEL_SIGMOID;
  auto form = [&](const SysDesc* dd, int pp, int ng, const int32_t* gf, const int32_t* gn, int tmax) {
    if (dtype == KRR_F64)
      launch_form<double>(ctx, s, prec, Xg, d, dd, pp, ng, gf, gn, tmax, A, K64, general);
    else
      launch_form<float>(ctx, s, prec, Xg, d, dd, pp, ng, gf, gn, tmax, A, K64, general);
  };
  const bool mixed_ref = mixed && Tmax > 0;
  const int maxr = params[0].max_refine;
  const double tol = params[0].refine_tol;
  // refinement step `it` without a host check: the residual and convergence
  // test, then a correction of the systems still refining (the kernels skip
  // the others); returns whether the step went on past the test
  auto refine_step = [&](int it) {
    const int will = it < maxr ? 1 : 0;
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, d_active, 1);
    check_launch(ctx, s, "zero_active");
    residual_check(ctx, s, d_desc, d_st, n_sys, p, n_groups, d_grp, d_grp + n_groups, Tmax, K64, alpha, rhs, rb, P,
                   d_poff, rn, yn, d_noff, tol, will, d_active, Pabs, glo, ghi);
    return will != 0;
  };
  auto correct = [&]() {
    trsv_forward(ctx, s, prec, d_desc, d_st, n_sys, Tmax, v_tot, A, Wt, rb, zb, 1);
    trsv_backward(ctx, s, prec, d_desc, d_st, n_sys, Tmax, v_tot, A, Wt, zb, db, alpha, 1);
    correction_norms(ctx, s, d_desc, d_st, n_sys, db, alpha);
  };
  // refinement steps taken inside the device phase (graphs only; the host
  // cannot look at the active count there, the kernels of a step whose
  // systems have all stopped do nothing)
  const int graph_steps = (use_graph && mixed_ref) ? std::min(maxr, 2) : 0;
  auto device_phase = [&]() {
    if (use_graph) gather_rows(ctx, s, X, dtype, n, d, perm, Xg);
    hipLaunchKernelGGL(k_zero_status, dim3((unsigned)ceil_div(n_sys, 128)), dim3(128), 0, s, d_st, n_sys);
    check_launch(ctx, s, "zero_status");
    gather_vec_f64(ctx, s, y, dtype, n, perm, yg);
    if (Tmax > 0) {
      hipLaunchKernelGGL(k_pad_rhs, dim3((unsigned)ceil_div((int64_t)Tmax * NB, 256), (unsigned)n_sys), dim3(256),
                         0, s, (const SysDesc*)d_desc, n_sys, (const double*)yg, rhs);
      check_launch(ctx, s, "pad_rhs");
    }
    form(d_desc, p, n_groups, d_grp, d_grp + n_groups, Tmax);
    // mixed precision: the BF16 packed factorisation carries the forward solve along (zb = rhs on entry)
    if (mixed) KRR_HIP(hipMemcpyAsync(zb, rhs, vb, hipMemcpyDeviceToDevice, s));
    if (!cholesky_factor(ctx, s, prec, d_desc, d_st, n_sys, Tmax, A, Wt, 0, mixed, desc.data(), pack,
                         mixed ? zb : nullptr))
      trsv_forward(ctx, s, prec, d_desc, d_st, n_sys, Tmax, v_tot, A, Wt, rhs, zb, 0);
    pivot_range(ctx, s, prec, d_desc, d_st, n_sys, A, 0);
    trsv_backward(ctx, s, prec, d_desc, d_st, n_sys, Tmax, v_tot, A, Wt, zb, alpha, nullptr, 0);
    for (int it = 0; it < graph_steps; ++it)
      if (refine_step(it)) correct();
  };
  if (!ctx->serial_fit) {
    if (!use_graph) {
      gather_rows(ctx, s, X, dtype, n, d, perm, Xg);
      device_phase();
    } else {
      // key: everything the device phase reads from the host side
      std::string key = "fit";
      for (const void* ptr : {X, y, (const void*)assign, (const void*)Xg})
        key_add(key, ptr);
      for (int64_t v : {n, (int64_t)d, (int64_t)p, (int64_t)dtype, (int64_t)prec, (int64_t)Tmax, v_tot,
                        (int64_t)ctx->panel_tiles, (int64_t)ctx->persistent, (int64_t)graph_steps})
        key_add(key, v);
      key.append(reinterpret_cast<const char*>(params), sizeof(krr_fit_params) * n_params);
      key.append(reinterpret_cast<const char*>(desc.data()), sizeof(SysDesc) * desc.size());
      key.append(reinterpret_cast<const char*>(grp_first.data()), sizeof(int32_t) * grp_first.size());
      key.append(reinterpret_cast<const char*>(grp_next.data()), sizeof(int32_t) * grp_next.size());
      graph_run(ctx, s, key, device_phase);
    }
  } else {
    gather_rows(ctx, s, X, dtype, n, d, perm, Xg);
    hipLaunchKernelGGL(k_zero_status, dim3((unsigned)ceil_div(n_sys, 128)), dim3(128), 0, s, d_st, n_sys);
    check_launch(ctx, s, "zero_status");
    gather_vec_f64(ctx, s, y, dtype, n, perm, yg);
    if (Tmax > 0) {
      hipLaunchKernelGGL(k_pad_rhs, dim3((unsigned)ceil_div((int64_t)Tmax * NB, 256), (unsigned)n_sys), dim3(256),
                         0, s, (const SysDesc*)d_desc, n_sys, (const double*)yg, rhs);
      check_launch(ctx, s, "pad_rhs");
    }
    // plain per-system sequence: every system formed, factored and solved
    // by its own launches, one after another
    for (int sidx = 0; sidx < n_sys; ++sidx) {
      if (desc[sidx].T == 0) continue;
      form(d_desc + sidx, 1, 1, d_grp + n_groups + n_params, d_grp + n_groups + n_params + 1, desc[sidx].T);
      cholesky_factor(ctx, s, prec, d_desc + sidx, d_st + sidx, 1, desc[sidx].T, A, Wt, 0, mixed,
                      desc.data() + sidx, pack, nullptr);
      pivot_range(ctx, s, prec, d_desc + sidx, d_st + sidx, 1, A, 0);
      trsv_forward(ctx, s, prec, d_desc + sidx, d_st + sidx, 1, desc[sidx].T, v_tot, A, Wt, rhs, zb, 0);
      trsv_backward(ctx, s, prec, d_desc + sidx, d_st + sidx, 1, desc[sidx].T, v_tot, A, Wt, zb, alpha, nullptr,
                    0);
    }
  }

  // 9. mixed precision: refine alpha with an FP64 residual; systems whose
  // BF16-updated factor is not positive definite or whose refinement stalls
  // are re-formed from the FP64 kernel and refactored with FP32 updates.
  SysStatus* st_h = (SysStatus*)(pin + up_bytes);
  std::vector<int> fallback(n_sys, 0);
  if (mixed_ref) {
    int32_t* act_h = (int32_t*)(pin + up_bytes + dn_bytes);
    // steps [it0, ...) with a look at the active count after each test
    auto refine = [&](int it0) {
      for (int it = it0;; ++it) {
        if (!refine_step(it)) break;
        KRR_HIP(hipMemcpyAsync(act_h, d_active, 4, hipMemcpyDeviceToHost, s));
        KRR_HIP(hipStreamSynchronize(s));
        if (*act_h == 0) break;
        correct();
      }
    };
    refine(graph_steps);
    KRR_HIP(hipMemcpyAsync(st_h, d_st, dn_bytes, hipMemcpyDeviceToHost, s));
    KRR_HIP(hipStreamSynchronize(s));
    check_gave_up(st_h, n_sys);
    int n_esc = 0;
    for (int sidx = 0; sidx < n_sys; ++sidx)
      if (desc[sidx].T > 0 && !st_h[sidx].converged) {
        desc[sidx].level = 1;
        fallback[sidx] = 1;
        ++n_esc;
      }
    if (n_esc > 0) {
      std::memcpy(pin, desc.data(), (size_t)n_sys * sizeof(SysDesc));
      KRR_HIP(hipMemcpyAsync(d_desc, pin, (size_t)n_sys * sizeof(SysDesc), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_reset_level, dim3((unsigned)ceil_div(n_sys, 128)), dim3(128), 0, s,
                         (const SysDesc*)d_desc, d_st, n_sys, 1);
      check_launch(ctx, s, "reset_level");
      hipLaunchKernelGGL(k_restore_tiles, dim3((unsigned)tri(Tmax), (unsigned)n_sys), dim3(256), 0, s,
                         (const SysDesc*)d_desc, (const double*)K64, (float*)A, 1);
      check_launch(ctx, s, "restore_tiles");
      cholesky_factor(ctx, s, prec, d_desc, d_st, n_sys, Tmax, A, Wt, 1, false, desc.data(), pack, nullptr);
      pivot_range(ctx, s, prec, d_desc, d_st, n_sys, A, 1);
      trsv_forward(ctx, s, prec, d_desc, d_st, n_sys, Tmax, v_tot, A, Wt, rhs, zb, 1);
      trsv_backward(ctx, s, prec, d_desc, d_st, n_sys, Tmax, v_tot, A, Wt, zb, alpha, nullptr, 1);
      refine(0);
    }
  }

  // 10. status to host
  KRR_HIP(hipMemcpyAsync(st_h, d_st, dn_bytes, hipMemcpyDeviceToHost, s));
  KRR_HIP(hipStreamSynchronize(s));
  check_gave_up(st_h, n_sys);
  // systems Cholesky rejected, of settings that ask for it: Gaussian
  // elimination (LU with partial pivoting) of the FP64 system
  std::vector<int> lu_sys;
  for (int sidx = 0; sidx < n_sys; ++sidx)
    if (desc[sidx].T > 0 && st_h[sidx].status == KRR_ENOTSPD && params[desc[sidx].param].indefinite)
      lu_sys.push_back(sidx);
  std::vector<int32_t> lu_bad = lu_solve_systems(ctx, s, lu_sys, desc.data(), Xg, dtype, d, yg, alpha);
  std::vector<int> solver(n_sys, 0);
  for (size_t i = 0; i < lu_sys.size(); ++i) {
    solver[lu_sys[i]] = 1;
    if (lu_bad[i] == 0) st_h[lu_sys[i]].status = KRR_OK;
  }
  for (int q = 0; q < n_params; ++q)
    for (int jp = 0; jp < p; ++jp) {
      const int sidx = q * p + jp;
      krr_part_info& I = info[sidx];
      const SysStatus& S = st_h[sidx];
      I.partition = jp;
      I.param = q;
      I.m = desc[sidx].m;
      I.status = S.status;
      I.failed_pivot = S.failed_pivot;
      I.refine_iters = S.refine_iters;
      I.fallback = fallback[sidx];
      I.solver = solver[sidx];
      const bool chol = solver[sidx] == 0;
      I.rel_residual = mixed && chol ? S.rel_residual : -1.0;
      I.kappa_est = S.kappa_l;
      I.kappa_bound = mixed && chol ? S.kappa_u : -1.0;
      I.err_est = mixed && chol ? S.err_est : -1.0;
      if (mixed && chol && S.status == 0 && !S.converged && desc[sidx].T > 0) I.status = KRR_ENOCONV;
    }

  if (use_graph && Xg != data->X)
    KRR_HIP(hipMemcpyAsync(data->X, Xg, (size_t)n * d * xes, hipMemcpyDeviceToDevice, s));
  if (direct != nullptr) {
    direct->alpha = alpha;
    direct->v_off.resize(p);
    direct->m.resize(p);
    for (int jp = 0; jp < p; ++jp) {
      direct->v_off[jp] = desc[jp].v_off;
      direct->m[jp] = desc[jp].m;
    }
    return;
  }

  // 11. models: alpha of setting q is the contiguous range of its p systems;
  // their offset tables go up from one pinned slice per model (one wait)
  int64_t* voff_pin = (int64_t*)pinned_get(ctx, (size_t)n_params * (p + 1) * 8);
  std::vector<krr_model> made;
  for (int q = 0; q < n_params; ++q) {
    krr_model M = new krr_model_s();
    M->ctx = ctx;
    M->data = data;
    M->params = params[q];
    const int64_t v0 = desc[q * p].v_off;
    const int64_t v1 = (q + 1 < n_params) ? desc[(q + 1) * p].v_off : v_tot;
    const size_t abytes = (((size_t)(v1 - v0) * 8 + 255) & ~size_t(255));
    M->bytes = abytes + (size_t)(p + 1) * 8;
    try {
      M->alpha = (double*)model_alloc(ctx, M->bytes);
    } catch (...) {
      // no model is handed out: release the ones made so far (their queued
      // copies and uploads finish first) and clear the output handles
      delete M;
      (void)hipStreamSynchronize(s);
      for (krr_model P : made) {
        model_release(ctx, P->alpha, P->bytes);
        ctx->n_models -= 1;
        delete P;
      }
      for (int q2 = 0; q2 < n_params; ++q2) models[q2] = nullptr;
      throw;
    }
    made.push_back(M);
    ctx->n_models += 1;
    M->d_voff = (int64_t*)((char*)M->alpha + abytes);
    M->voff.resize(p + 1);
    for (int jp = 0; jp < p; ++jp) M->voff[jp] = desc[q * p + jp].v_off - v0;
    M->voff[p] = v1 - v0;
    M->lambda_eff.resize(p);
    for (int jp = 0; jp < p; ++jp) M->lambda_eff[jp] = desc[q * p + jp].lambda;
    if (v1 > v0)
      KRR_HIP(hipMemcpyAsync(M->alpha, alpha + v0, (size_t)(v1 - v0) * 8, hipMemcpyDeviceToDevice, s));
    int64_t* vp = voff_pin + (size_t)q * (p + 1);
    std::memcpy(vp, M->voff.data(), (size_t)(p + 1) * 8);
    KRR_HIP(hipMemcpyAsync(M->d_voff, vp, (size_t)(p + 1) * 8, hipMemcpyHostToDevice, s));
    models[q] = M;
  }
  KRR_HIP(hipStreamSynchronize(s));   // the pinned slices are reused by the next call
}

}  // namespace krr
