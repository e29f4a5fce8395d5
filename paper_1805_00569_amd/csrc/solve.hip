// Triangular solves L z = b, L^T x = z for the factored batch (Section 2.3,
// Eq. 6 solved by Cholesky), and the FP64 residual r = y - (K + lambda I) alpha
// that drives iterative refinement in mixed precision.
//
// One workgroup per system walks its tile rows in order.  A tile row's
// off-diagonal part is a GEMV over tiles already solved; the diagonal block is
// applied through the inverse Winv(i) = L(i,i)^-1 kept by the factorisation,
// so the whole solve is a sequence of dense tile GEMVs.  All sums run in a
// fixed order: results do not depend on the launch or on the batch.
#include "common.hpp"

namespace krr {

namespace {

constexpr int TILE = NB * NB;

__device__ __forceinline__ int64_t tile_index(int i, int j) { return (int64_t)i * (i + 1) / 2 + j; }

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ bool skip_system(const SysStatus& S, int skip_converged) {
  return S.status != 0 || (skip_converged && (S.converged || S.stalled));
}

// z = L^-1 b.  Thread (r = t % 64, g = t / 64) handles row r and the column
// subset c = g + 4q of every tile.
template <typename TS>
__global__ __launch_bounds__(256) void k_trsv_fwd(const SysDesc* __restrict__ desc, const SysStatus* __restrict__ st,
                                                  const TS* __restrict__ A, const TS* __restrict__ Wt,
                                                  const double* __restrict__ b, double* __restrict__ z,
                                                  int skip_converged) {
  const int s = blockIdx.x;
  const SysDesc D = desc[s];
  if (skip_system(st[s], skip_converged)) return;
  __shared__ double sred[4][NB];
  __shared__ double sv[NB];
  const int t = threadIdx.x, r = t & 63, g = t >> 6;
  const TS* Ab = A + D.a_off;
  const double* bb = b + D.v_off;
  double* zz = z + D.v_off;
  for (int i = 0; i < D.T; ++i) {
    double acc = 0.0;
    for (int j = 0; j < i; ++j) {
      const TS* L = Ab + tile_index(i, j) * TILE;
      const double* zj = zz + j * NB;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int c = g + 4 * q;
        acc = fma((double)L[c * NB + r], zj[c], acc);
      }
    }
    sred[g][r] = acc;
    __syncthreads();
    if (t < NB) sv[r] = bb[i * NB + r] - ((sred[0][r] + sred[1][r]) + (sred[2][r] + sred[3][r]));
    __syncthreads();
    const TS* W = Wt + D.w_off + (int64_t)i * TILE;
    double acc2 = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = g + 4 * q;
      acc2 = fma((double)W[c * NB + r], sv[c], acc2);
    }
    sred[g][r] = acc2;
    __syncthreads();
    if (t < NB) zz[i * NB + r] = (sred[0][r] + sred[1][r]) + (sred[2][r] + sred[3][r]);
    __syncthreads();
  }
}

// x = L^-T z (and alpha += x when `alpha_acc` is given).  For the transposed
// tiles every thread keeps one partial per column c = g + 4q and the 64 rows
// are summed across the wavefront once per tile row.
template <typename TS>
__global__ __launch_bounds__(256) void k_trsv_bwd(const SysDesc* __restrict__ desc, const SysStatus* __restrict__ st,
                                                  const TS* __restrict__ A, const TS* __restrict__ Wt,
                                                  const double* __restrict__ z, double* __restrict__ x,
                                                  double* __restrict__ alpha_acc, int skip_converged) {
  const int s = blockIdx.x;
  const SysDesc D = desc[s];
  if (skip_system(st[s], skip_converged)) return;
  __shared__ double su[NB];
  const int t = threadIdx.x, lane = t & 63, g = t >> 6;
  const TS* Ab = A + D.a_off;
  const double* zz = z + D.v_off;
  double* xx = x + D.v_off;
  for (int i = D.T - 1; i >= 0; --i) {
    double part[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) part[q] = 0.0;
    for (int j = i + 1; j < D.T; ++j) {
      const TS* L = Ab + tile_index(j, i) * TILE;   // (L^T)(i,j) = L(j,i)^T
      const double xj = xx[j * NB + lane];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int c = g + 4 * q;
        part[q] = fma((double)L[c * NB + lane], xj, part[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const double v = wave_sum(part[q]);
      if (lane == 0) {
        const int c = g + 4 * q;
        su[c] = zz[i * NB + c] - v;
      }
    }
    __syncthreads();
    // x_i = Winv(i)^T u: x_i[c] = sum_r W(r, c) u[r], W(r, c) at c * NB + r
    const TS* W = Wt + D.w_off + (int64_t)i * TILE;
    const double ul = su[lane];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = g + 4 * q;
      const double v = wave_sum((double)W[c * NB + lane] * ul);
      if (lane == 0) {
        xx[i * NB + c] = v;
        if (alpha_acc != nullptr) alpha_acc[D.v_off + i * NB + c] += v;
      }
    }
    __syncthreads();
  }
}

// Residual partials: tile (i, j) of the symmetric matrix (lower tiles only
// stored) contributes K(i,j) alpha_j to row block i and, off the diagonal,
// K(i,j)^T alpha_i to row block j.  Partials go to P[(row block, col block)]
// and are summed in column-block order by k_resid_reduce.
__global__ __launch_bounds__(256) void k_resid_tiles(const SysDesc* __restrict__ desc,
                                                     const SysStatus* __restrict__ st,
                                                     const double* __restrict__ K, const double* __restrict__ alpha,
                                                     double* __restrict__ P, const int64_t* __restrict__ p_off) {
  const int s = blockIdx.y;
  const SysDesc D = desc[s];
  if (skip_system(st[s], 1)) return;
  const int bx = blockIdx.x;
  int ii = (int)((sqrt(8.0 * (double)bx + 1.0) - 1.0) * 0.5);
  while ((int64_t)ii * (ii + 1) / 2 > bx) --ii;
  while ((int64_t)(ii + 1) * (ii + 2) / 2 <= bx) ++ii;
  const int jj = bx - ii * (ii + 1) / 2;
  if (ii >= D.T) return;
  __shared__ double sred[4][NB];
  const int t = threadIdx.x, lane = t & 63, g = t >> 6;
  const double* Kt = K + D.a_off + tile_index(ii, jj) * TILE;
  const double* aj = alpha + D.v_off + jj * NB;
  const double* ai = alpha + D.v_off + ii * NB;
  double* Pb = P + p_off[s];
  // K(i,j) alpha_j
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int c = g + 4 * q;
    acc = fma(Kt[c * NB + lane], aj[c], acc);
  }
  sred[g][lane] = acc;
  __syncthreads();
  if (t < NB) Pb[((int64_t)ii * D.T + jj) * NB + lane] = (sred[0][lane] + sred[1][lane]) + (sred[2][lane] + sred[3][lane]);
  if (ii != jj) {
    const double al = ai[lane];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = g + 4 * q;
      const double v = wave_sum(Kt[c * NB + lane] * al);
      if (lane == 0) Pb[((int64_t)jj * D.T + ii) * NB + c] = v;
    }
  }
}

// r_i = y_i - sum_j P(i, j) (fixed j order) and per-tile-row sums of r^2, y^2.
__global__ __launch_bounds__(64) void k_resid_reduce(const SysDesc* __restrict__ desc, const SysStatus* __restrict__ st,
                                                     const double* __restrict__ y, const double* __restrict__ P,
                                                     const int64_t* __restrict__ p_off, double* __restrict__ r,
                                                     double* __restrict__ rn, double* __restrict__ yn,
                                                     const int64_t* __restrict__ n_off) {
  const int s = blockIdx.y;
  const SysDesc D = desc[s];
  if (skip_system(st[s], 1)) return;
  const int i = blockIdx.x;
  if (i >= D.T) return;
  const int lane = threadIdx.x;
  const double* Pb = P + p_off[s] + (int64_t)i * D.T * NB;
  double acc = 0.0;
  for (int j = 0; j < D.T; ++j) acc += Pb[j * NB + lane];
  const double yv = y[D.v_off + i * NB + lane];
  const double rv = yv - acc;
  r[D.v_off + i * NB + lane] = rv;
  const double r2 = wave_sum(rv * rv);
  const double y2 = wave_sum(yv * yv);
  if (lane == 0) {
    rn[n_off[s] + i] = r2;
    yn[n_off[s] + i] = y2;
  }
}

// Per system: ||r|| / ||y||, convergence flag, and the refinement step count.
__global__ void k_ir_check(const SysDesc* __restrict__ desc, SysStatus* __restrict__ st, int n_sys,
                           const double* __restrict__ rn, const double* __restrict__ yn,
                           const int64_t* __restrict__ n_off, double tol, int will_refine,
                           int32_t* __restrict__ active) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sys) return;
  SysStatus& S = st[s];
  if (S.status != 0 || S.converged || S.stalled) return;
  const SysDesc D = desc[s];
  double r2 = 0.0, y2 = 0.0;
  for (int i = 0; i < D.T; ++i) {
    r2 += rn[n_off[s] + i];
    y2 += yn[n_off[s] + i];
  }
  const double rel = (y2 > 0.0) ? sqrt(r2) / sqrt(y2) : sqrt(r2);
  const double prev = S.prev_rel;
  S.rel_residual = rel;
  S.prev_rel = rel;
  S.ynorm = sqrt(y2);
  if (rel <= tol) {
    S.converged = 1;
  } else if (prev >= 0.0 && !(rel <= 0.5 * prev)) {
    S.stalled = 1;  // a step that does not halve the residual: escalate precision
  } else if (will_refine) {
    S.refine_iters += 1;
    atomicAdd(active, 1);
  }
}

}  // namespace

void trsv_forward(krr_ctx ctx, hipStream_t s, int prec, const SysDesc* desc, const SysStatus* st, int n_sys,
                  const void* A, const void* Wt, const double* b, double* z, int skip_converged) {
  KernelTimer kt(ctx, s, "trsv_forward", 0.0, 0);
  if (prec == KRR_PREC_FP64)
    hipLaunchKernelGGL((k_trsv_fwd<double>), dim3(n_sys), dim3(256), 0, s, desc, st, (const double*)A,
                       (const double*)Wt, b, z, skip_converged);
  else
    hipLaunchKernelGGL((k_trsv_fwd<float>), dim3(n_sys), dim3(256), 0, s, desc, st, (const float*)A,
                       (const float*)Wt, b, z, skip_converged);
  check_launch(ctx, s, "trsv_fwd");
}

void trsv_backward(krr_ctx ctx, hipStream_t s, int prec, const SysDesc* desc, const SysStatus* st, int n_sys,
                   const void* A, const void* Wt, const double* z, double* x, double* alpha_acc, int skip_converged) {
  KernelTimer kt(ctx, s, "trsv_backward", 0.0, 0);
  if (prec == KRR_PREC_FP64)
    hipLaunchKernelGGL((k_trsv_bwd<double>), dim3(n_sys), dim3(256), 0, s, desc, st, (const double*)A,
                       (const double*)Wt, z, x, alpha_acc, skip_converged);
  else
    hipLaunchKernelGGL((k_trsv_bwd<float>), dim3(n_sys), dim3(256), 0, s, desc, st, (const float*)A,
                       (const float*)Wt, z, x, alpha_acc, skip_converged);
  check_launch(ctx, s, "trsv_bwd");
}

void residual_check(krr_ctx ctx, hipStream_t s, const SysDesc* desc, SysStatus* st, int n_sys, int Tmax,
                    const double* K64, const double* alpha, const double* y, double* r, double* P,
                    const int64_t* p_off, double* rn, double* yn, const int64_t* n_off, double tol,
                    int will_refine, int32_t* active) {
  const int64_t ntri = (int64_t)Tmax * (Tmax + 1) / 2;
  KernelTimer kt(ctx, s, "ir_residual", 0.0, 0);
  hipLaunchKernelGGL(k_resid_tiles, dim3((unsigned)ntri, (unsigned)n_sys), dim3(256), 0, s, desc,
                     (const SysStatus*)st, K64, alpha, P, p_off);
  check_launch(ctx, s, "resid_tiles");
  hipLaunchKernelGGL(k_resid_reduce, dim3((unsigned)Tmax, (unsigned)n_sys), dim3(64), 0, s, desc,
                     (const SysStatus*)st, y, (const double*)P, p_off, r, rn, yn, n_off);
  check_launch(ctx, s, "resid_reduce");
  hipLaunchKernelGGL(k_ir_check, dim3((unsigned)ceil_div(n_sys, 64)), dim3(64), 0, s, desc, st, n_sys,
                     (const double*)rn, (const double*)yn, n_off, tol, will_refine, active);
  check_launch(ctx, s, "ir_check");
}

}  // namespace krr
