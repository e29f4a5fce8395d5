// Solve of the systems (K + lambda I) alpha = y that are not positive
// definite (the sigmoid kernel of Table 1 is not positive semi-definite in
// general, so Eq. 6 may meet a non-positive Cholesky pivot): LU
// factorisation with partial pivoting in FP64, on a dense copy of each such
// system, all of them in one batch.
//
// For every column k: one workgroup per system finds the pivot (the largest
// |A(r, k)|, r >= k, lowest r on ties), swaps rows k and the pivot row (and
// the right-hand side entries), forms the multipliers A(r, k) / A(k, k) and
// eliminates them from the right-hand side; then the trailing rank-one update
// A(r, c) -= A(r, k) A(k, c) runs over the whole device.  A back substitution
// with U (one workgroup per system) gives alpha.  This path is taken only on
// request (krr_fit_params.indefinite) for the systems the Cholesky
// factorisation rejects; it is O(m^3) memory traffic per system, not a
// tuned kernel.
#include "common.hpp"

#include <algorithm>
#include <cmath>

namespace krr {

namespace {

// One failed system: where its data, dense copy and vectors are.
struct LuSys {
  int32_t m;
  int32_t sys;          // index of the system in the batch
  int64_t x_off;        // first row of its partition in the grouped inputs
  int64_t a_off;        // element offset of its dense m x m copy (row-major)
  int64_t v_off;        // offset of its padded vectors (rhs, alpha)
  double neg_inv_2s2, lambda, ka, kr;
  int32_t kernel, kdeg;
};

// A(r, c) = k(x_r, x_c) + lambda [r = c], FP64 (Table 1 kernels; squared
// distances by direct difference).
template <typename TX>
__global__ void k_lu_form(const TX* __restrict__ Xg, int d, const LuSys* __restrict__ ls, double* __restrict__ A) {
  const LuSys L = ls[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)L.m * L.m) return;
  const int r = (int)(e / L.m), c = (int)(e - (int64_t)r * L.m);
  const TX* xr = Xg + (L.x_off + r) * d;
  const TX* xc = Xg + (L.x_off + c) * d;
  double v;
  if (L.kernel == KRR_KERNEL_GAUSSIAN) {
    double s = 0.0;
    for (int f = 0; f < d; ++f) {
      const double t = (double)xr[f] - (double)xc[f];
      s = fma(t, t, s);
    }
    v = (r == c) ? 1.0 : exp(s * L.neg_inv_2s2);
  } else {
    double g = 0.0;
    for (int f = 0; f < d; ++f) g = fma((double)xr[f], (double)xc[f], g);
    if (L.kernel == KRR_KERNEL_POLYNOMIAL) v = poly_kernel(g, L.ka, L.kr, L.kdeg);
    else if (L.kernel == KRR_KERNEL_SIGMOID) v = tanh(L.ka * g + L.kr);
    else v = g;
  }
  if (r == c) v += L.lambda;
  A[L.a_off + e] = v;
}

__global__ void k_lu_rhs(const LuSys* __restrict__ ls, const double* __restrict__ y, double* __restrict__ b) {
  const LuSys L = ls[blockIdx.y];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < L.m) b[L.v_off + r] = y[L.x_off + r];
}

constexpr int LU_T = 256;

// Column k: pivot, row swap, multipliers, forward elimination of b.
__global__ __launch_bounds__(LU_T) void k_lu_pivot(const LuSys* __restrict__ ls, double* __restrict__ A,
                                                   double* __restrict__ b, int32_t* __restrict__ bad, int k) {
  const LuSys L = ls[blockIdx.x];
  if (k >= L.m || bad[blockIdx.x]) return;
  const int m = L.m, t = threadIdx.x;
  double* Ab = A + L.a_off;
  __shared__ double sv[LU_T];
  __shared__ int si[LU_T];
  double best = -1.0;
  int bi = m;
  for (int r = k + t; r < m; r += LU_T) {
    const double v = fabs(Ab[(int64_t)r * m + k]);
    if (v > best) {   // rows in increasing order per thread: the first maximum is kept
      best = v;
      bi = r;
    }
  }
  sv[t] = best;
  si[t] = bi;
  __syncthreads();
  for (int w = LU_T / 2; w > 0; w >>= 1) {
    if (t < w) {
      const double o = sv[t + w];
      const int oi = si[t + w];
      if (o > sv[t] || (o == sv[t] && oi < si[t])) {
        sv[t] = o;
        si[t] = oi;
      }
    }
    __syncthreads();
  }
  const int p = si[0];
  const double pv = Ab[(int64_t)p * m + k];
  if (!(sv[0] > 0.0)) {   // a zero column below the diagonal: numerically singular
    if (t == 0) bad[blockIdx.x] = k + 1;
    return;
  }
  if (p != k) {
    for (int c = t; c < m; c += LU_T) {
      const double u = Ab[(int64_t)k * m + c], w = Ab[(int64_t)p * m + c];
      Ab[(int64_t)k * m + c] = w;
      Ab[(int64_t)p * m + c] = u;
    }
    if (t == 0) {
      const double u = b[L.v_off + k];
      b[L.v_off + k] = b[L.v_off + p];
      b[L.v_off + p] = u;
    }
  }
  __syncthreads();
  const double bk = b[L.v_off + k];
  for (int r = k + 1 + t; r < m; r += LU_T) {
    const double l = Ab[(int64_t)r * m + k] / pv;
    Ab[(int64_t)r * m + k] = l;
    b[L.v_off + r] = fma(-l, bk, b[L.v_off + r]);
  }
}

// Trailing update of column k: A(r, c) -= A(r, k) A(k, c), r, c > k.  Block
// (bx, by) covers rows k + 1 + 16 bx .. +15 and columns k + 1 + 64 by .. +63.
__global__ __launch_bounds__(256) void k_lu_update(const LuSys* __restrict__ ls, double* __restrict__ A,
                                                    const int32_t* __restrict__ bad, int k) {
  const LuSys L = ls[blockIdx.z];
  if (k + 1 >= L.m || bad[blockIdx.z]) return;
  const int m = L.m;
  const int r = k + 1 + 16 * blockIdx.x + (threadIdx.x >> 4);
  const int c0 = k + 1 + 64 * blockIdx.y + 4 * (threadIdx.x & 15);
  if (r >= m || c0 >= m) return;
  double* Ab = A + L.a_off;
  const double l = Ab[(int64_t)r * m + k];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = c0 + u;
    if (c < m) Ab[(int64_t)r * m + c] = fma(-l, Ab[(int64_t)k * m + c], Ab[(int64_t)r * m + c]);
  }
}

// Back substitution with U, one workgroup per system; alpha past m is zero.
__global__ __launch_bounds__(1024) void k_lu_back(const LuSys* __restrict__ ls, const double* __restrict__ A,
                                                  const double* __restrict__ b, double* __restrict__ x,
                                                  const int32_t* __restrict__ bad, int vpad) {
  const LuSys L = ls[blockIdx.x];
  if (bad[blockIdx.x]) return;
  const int m = L.m, t = threadIdx.x;
  const double* Ab = A + L.a_off;
  double* xs = x + L.v_off;
  __shared__ double red[1024];
  for (int i = m + t; i < vpad; i += 1024) xs[i] = 0.0;
  for (int k = m - 1; k >= 0; --k) {
    double acc = 0.0;
    for (int j = k + 1 + t; j < m; j += 1024) acc = fma(Ab[(int64_t)k * m + j], xs[j], acc);
    red[t] = acc;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
      if (t < w) red[t] += red[t + w];
      __syncthreads();
    }
    if (t == 0) xs[k] = (b[L.v_off + k] - red[0]) / Ab[(int64_t)k * m + k];
    __syncthreads();
  }
}

}  // namespace

// Solves the systems `which` (indices into the batch, hdesc their host
// descriptors) by LU with partial pivoting from their inputs: grouped
// points Xg (dtype) and labels y (FP64, grouped order); writes alpha
// (padded, at each system's v_off).  Returns, per listed system, 0 or the 1-based column
// at which it was found numerically singular.
std::vector<int32_t> lu_solve_systems(krr_ctx ctx, hipStream_t s, const std::vector<int>& which,
                                      const SysDesc* hdesc, const void* Xg, int dtype, int d, const double* y,
                                      double* alpha) {
  const int nl = (int)which.size();
  std::vector<int32_t> out(nl, 0);
  if (nl == 0) return out;
  std::vector<LuSys> ls(nl);
  int64_t dense = 0, mmax = 0;
  int64_t vtot = 0;
  for (int i = 0; i < nl; ++i) {
    const SysDesc& D = hdesc[which[i]];
    LuSys& L = ls[i];
    L.m = D.m;
    L.sys = which[i];
    L.x_off = D.x_off;
    L.a_off = dense;
    L.v_off = D.v_off;
    L.neg_inv_2s2 = D.neg_inv_2s2;
    L.lambda = D.lambda;
    L.ka = D.ka;
    L.kr = D.kr;
    L.kernel = D.kernel;
    L.kdeg = D.kdeg;
    dense += (int64_t)D.m * D.m;
    mmax = std::max<int64_t>(mmax, D.m);
    vtot = std::max<int64_t>(vtot, D.v_off + (int64_t)D.T * NB);
  }
  double* A = (double*)ws_get(ctx, "lu_A", (size_t)std::max<int64_t>(dense, 1) * 8);
  double* b = (double*)ws_get(ctx, "lu_b", (size_t)std::max<int64_t>(vtot, 1) * 8);
  char* meta = (char*)ws_get(ctx, "lu_meta", (size_t)nl * (sizeof(LuSys) + 4) + 64);
  LuSys* d_ls = (LuSys*)meta;
  int32_t* bad = (int32_t*)(meta + (size_t)nl * sizeof(LuSys));
  char* pin = (char*)pinned_named(ctx, "lu", (size_t)nl * (sizeof(LuSys) + 4) + 64);
  std::memcpy(pin, ls.data(), (size_t)nl * sizeof(LuSys));
  std::memset(pin + (size_t)nl * sizeof(LuSys), 0, (size_t)nl * 4);
  KRR_HIP(hipMemcpyAsync(meta, pin, (size_t)nl * (sizeof(LuSys) + 4), hipMemcpyHostToDevice, s));
  const dim3 gform((unsigned)ceil_div(mmax * mmax, 256), (unsigned)nl);
  if (dtype == KRR_F64)
    hipLaunchKernelGGL(k_lu_form<double>, gform, dim3(256), 0, s, (const double*)Xg, d, (const LuSys*)d_ls, A);
  else
    hipLaunchKernelGGL(k_lu_form<float>, gform, dim3(256), 0, s, (const float*)Xg, d, (const LuSys*)d_ls, A);
  check_launch(ctx, s, "lu_form");
  hipLaunchKernelGGL(k_lu_rhs, dim3((unsigned)ceil_div(mmax, 256), (unsigned)nl), dim3(256), 0, s,
                     (const LuSys*)d_ls, y, b);
  check_launch(ctx, s, "lu_rhs");
  for (int k = 0; k < mmax; ++k) {
    hipLaunchKernelGGL(k_lu_pivot, dim3((unsigned)nl), dim3(LU_T), 0, s, (const LuSys*)d_ls, A, b, bad, k);
    check_launch(ctx, s, "lu_pivot");
    const int64_t rem = mmax - k - 1;
    if (rem > 0) {
      hipLaunchKernelGGL(k_lu_update, dim3((unsigned)ceil_div(rem, 16), (unsigned)ceil_div(rem, 64), (unsigned)nl),
                         dim3(256), 0, s, (const LuSys*)d_ls, A, (const int32_t*)bad, k);
      check_launch(ctx, s, "lu_update");
    }
  }
  // padded length of each system's vectors: T * NB (the same for all here: pass the largest and let each
  // system zero its own tail up to its own T * NB)
  for (int i = 0; i < nl; ++i) {
    const SysDesc& D = hdesc[which[i]];
    hipLaunchKernelGGL(k_lu_back, dim3(1), dim3(1024), 0, s, (const LuSys*)(d_ls + i), (const double*)A,
                       (const double*)b, alpha, (const int32_t*)(bad + i), D.T * NB);
    check_launch(ctx, s, "lu_back");
  }
  KRR_HIP(hipMemcpyAsync(pin + (size_t)nl * sizeof(LuSys), bad, (size_t)nl * 4, hipMemcpyDeviceToHost, s));
  KRR_HIP(hipStreamSynchronize(s));
  std::memcpy(out.data(), pin + (size_t)nl * sizeof(LuSys), (size_t)nl * 4);
  return out;
}

}  // namespace krr
