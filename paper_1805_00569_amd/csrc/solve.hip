// Triangular solves L z = b, L^T x = z for the factored batch (Section 2.3,
// Eq. 6 solved by Cholesky), and the FP64 residual r = y - (K + lambda I) alpha
// that drives iterative refinement in mixed precision.
//
// One workgroup per system walks its tile rows in order (systems of more than
// TRSV_XL_MAXT tile rows: band by band, with the contributions of a solved
// band to the other rows spread over many workgroups).  A tile row's
// off-diagonal part is a GEMV over tiles already solved; the diagonal block is
// applied through the inverse Winv(i) = L(i,i)^-1 kept by the factorisation,
// so the whole solve is a sequence of dense tile GEMVs.  All sums run in a
// fixed order that depends on the system alone: results do not depend on the
// launch or on the batch.
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

// Thread layout of both solves: a workgroup of TRSV_G groups of 256 threads
// per system; group g reads the tiles j = g, g + TRSV_G, ... of a tile row,
// and thread t of a group owns rows 4 (t & 15) .. +3 and columns
// (t >> 4) + 16 q (q < 4) of every tile it reads, with four 4-row vector
// loads per tile and TRSV_JB tiles in flight, so that one workgroup keeps
// enough loads outstanding to stream its factor at a useful share of HBM
// bandwidth.  Partial sums are combined in LDS in a fixed order.
// tiles in flight per thread: FP32 tiles 4, FP64 tiles 2 (128 registers per thread)
template <typename TS>
struct TrsvJB {
  static constexpr int value = sizeof(TS) == 4 ? 4 : 2;
};
constexpr int TRSV_G = 4;
constexpr int TRSV_THREADS = 256 * TRSV_G;

__device__ __forceinline__ void load4(const float* __restrict__ p, float (&o)[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x;
  o[1] = v.y;
  o[2] = v.z;
  o[3] = v.w;
}
__device__ __forceinline__ void load4(const double* __restrict__ p, double (&o)[4]) {
  const double2 a = reinterpret_cast<const double2*>(p)[0];
  const double2 b = reinterpret_cast<const double2*>(p)[1];
  o[0] = a.x;
  o[1] = a.y;
  o[2] = b.x;
  o[3] = b.y;
}

// sum over the 16 lanes that share (t >> 4) (fixed butterfly order)
__device__ __forceinline__ double quad16_sum(double v) {
  for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Systems with T <= TRSV_XL_MAXT are solved whole by one workgroup each;
// larger ones band by band (TRSV_BAND tile rows at absolute multiples of
// TRSV_BAND, from the first): one workgroup per system solves the band's rows
// against the band, and k_trsv_fwd_upd subtracts the band's contribution from
// every tile row below it into a working copy bw of b (the path depends on the
// system's own T only).
// Threshold measured on the 96-system batch of m = 4,096 (T = 64): the band
// path takes the backward solve from 0.85 to 0.79 ms, as its band updates
// spread the factor over the whole chip while the whole-system path keeps it
// on one CU per system.
constexpr int TRSV_XL_MAXT = 32;
constexpr int TRSV_BAND = 16;

// z = L^-1 b over tile rows [lo, hi): u = b_i - sum_{lo<=j<i} L(i,j) z_j, then
// z_i = Winv(i) u.  BAND = false: the whole system (lo = 0, hi = T); BAND =
// true: the band starting at i0, right-hand side b for the first band, else bw.
template <typename TS, bool BAND>
__global__ __launch_bounds__(TRSV_THREADS) void k_trsv_fwd(const SysDesc* __restrict__ desc,
                                                           const SysStatus* __restrict__ st,
                                                           const TS* __restrict__ A, const TS* __restrict__ Wt,
                                                           const double* __restrict__ b,
                                                           const double* __restrict__ bw, double* __restrict__ z,
                                                           int skip_converged, int i0) {
  constexpr int TRSV_JB = TrsvJB<TS>::value;
  const int s = blockIdx.x;
  const SysDesc D = desc[s];
  if (BAND ? (D.T <= TRSV_XL_MAXT || i0 >= D.T) : D.T > TRSV_XL_MAXT) return;
  if (skip_system(st[s], skip_converged)) return;
  const int lo = BAND ? i0 : 0, hi = BAND ? min(i0 + TRSV_BAND, D.T) : D.T;
  __shared__ double sred[TRSV_G * 16][NB];
  __shared__ double sv[NB];
  const int t = threadIdx.x, grp = t >> 8, rq = t & 15, cg = (t >> 4) & 15;
  const TS* Ab = A + D.a_off;
  const double* bb = ((BAND && lo > 0) ? bw : b) + D.v_off;
  double* zz = z + D.v_off;
  for (int i = lo; i < hi; ++i) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const TS* row = Ab + tile_index(i, 0) * TILE;   // tiles (i, 0 .. i-1) are contiguous
    int j = lo + grp;
    for (; j + TRSV_G * (TRSV_JB - 1) < i; j += TRSV_G * TRSV_JB) {
      TS lv[TRSV_JB][4][4];
      double zv[TRSV_JB][4];
#pragma unroll
      for (int u = 0; u < TRSV_JB; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int c = cg + 16 * q;
          load4(row + (int64_t)(j + TRSV_G * u) * TILE + c * NB + 4 * rq, lv[u][q]);
          zv[u][q] = zz[(j + TRSV_G * u) * NB + c];
        }
#pragma unroll
      for (int u = 0; u < TRSV_JB; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int k = 0; k < 4; ++k) acc[k] = fma((double)lv[u][q][k], zv[u][q], acc[k]);
    }
    for (; j < i; j += TRSV_G) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = cg + 16 * q;
        TS lv[4];
        load4(row + (int64_t)j * TILE + c * NB + 4 * rq, lv);
        const double zc = zz[j * NB + c];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = fma((double)lv[k], zc, acc[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) sred[grp * 16 + cg][4 * rq + k] = acc[k];
    __syncthreads();
    if (t < NB) {
      double sum = 0.0;
#pragma unroll 16
      for (int g = 0; g < TRSV_G * 16; ++g) sum += sred[g][t];
      sv[t] = bb[i * NB + t] - sum;
    }
    __syncthreads();
    if (grp == 0) {
      const TS* W = Wt + D.w_off + (int64_t)i * TILE;
      double acc2[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = cg + 16 * q;
        TS wv[4];
        load4(W + c * NB + 4 * rq, wv);
        const double uc = sv[c];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc2[k] = fma((double)wv[k], uc, acc2[k]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) sred[cg][4 * rq + k] = acc2[k];
    }
    __syncthreads();
    if (t < NB) {
      double sum = 0.0;
#pragma unroll
      for (int g = 0; g < 16; ++g) sum += sred[g][t];
      zz[i * NB + t] = sum;
    }
    __syncthreads();
  }
}

// Band update of the forward solve: for tile row i >= i0 + TRSV_BAND of a
// system on the band path (i = i0 + TRSV_BAND + blockIdx.x), bw_i = (b_i for
// the first band, else bw_i) - sum_{i0<=j<i1} L(i,j) z_j.  One workgroup per
// (i, system); thread t owns rows 4 (t & 15) .. +3 and columns (t >> 4) + 16 q
// of each tile; fixed order (over the lanes of a wave, then the four waves).
template <typename TS>
__global__ __launch_bounds__(256) void k_trsv_fwd_upd(const SysDesc* __restrict__ desc,
                                                      const SysStatus* __restrict__ st, const TS* __restrict__ A,
                                                      const double* __restrict__ b, double* __restrict__ bw,
                                                      const double* __restrict__ z, int skip_converged, int i0) {
  const int s = blockIdx.y;
  const SysDesc D = desc[s];
  const int i = i0 + TRSV_BAND + (int)blockIdx.x;
  if (D.T <= TRSV_XL_MAXT || i >= D.T) return;
  if (skip_system(st[s], skip_converged)) return;
  const int i1 = i0 + TRSV_BAND;
  __shared__ double sred[4][NB];
  const int t = threadIdx.x, rq = t & 15, cg = t >> 4, w = t >> 6;
  const TS* row = A + D.a_off + tile_index(i, 0) * TILE;
  const double* zz = z + D.v_off;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int j = i0; j < i1; j += 4) {
    TS lv[4][4][4];
    double zv[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = cg + 16 * q;
        load4(row + (int64_t)(j + u) * TILE + c * NB + 4 * rq, lv[u][q]);
        zv[u][q] = zz[(j + u) * NB + c];
      }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = fma((double)lv[u][q][k], zv[u][q], acc[k]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double v = acc[k];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if ((t & 63) < 16) sred[w][4 * rq + k] = v;
  }
  __syncthreads();
  if (t < NB) {
    const double sum = (sred[0][t] + sred[1][t]) + (sred[2][t] + sred[3][t]);
    const double src = (i0 == 0 ? b : bw)[D.v_off + (int64_t)i * NB + t];
    bw[D.v_off + (int64_t)i * NB + t] = src - sum;
  }
}

// x = L^-T z (and alpha += x when `alpha_acc` is given), tile row i from the
// last: u = z_i - sum_{j>i} L(j,i)^T x_j, then x_i = Winv(i)^T u.
// Systems with T <= TRSV_XL_MAXT are solved whole by one workgroup each with x
// in LDS.  Larger systems go band by band (TRSV_BAND tile rows, bands at
// absolute multiples of TRSV_BAND, from the last): one workgroup per system
// solves the band's rows against the band only, and k_trsv_bwd_upd then
// subtracts the band's contribution from every tile row above it, one
// workgroup per (tile row, system), into a working copy zw of z.  Which path a
// system takes depends on its own T only, so results do not depend on the batch.
// Tile rows [lo, hi) from the last: BAND = false, the whole system (lo = 0,
// hi = T, right-hand side z); BAND = true, the band starting at i0 (right-hand
// side z for the last band, else zw).  Winv(i) comes from LDS: groups 1..3 load
// the next step's block into the other half of a double buffer while group 0
// forms x_i; the rows' x stay in LDS and are written out at the end.
template <typename TS, bool BAND>
__global__ __launch_bounds__(TRSV_THREADS) void k_trsv_bwd(const SysDesc* __restrict__ desc,
                                                           const SysStatus* __restrict__ st,
                                                           const TS* __restrict__ A, const TS* __restrict__ Wt,
                                                           const double* __restrict__ z,
                                                           const double* __restrict__ zw, double* __restrict__ x,
                                                           double* __restrict__ alpha_acc, int skip_converged,
                                                           int i0) {
  constexpr int TRSV_JB = TrsvJB<TS>::value;
  const int s = blockIdx.x;
  const SysDesc D = desc[s];
  if (BAND ? (D.T <= TRSV_XL_MAXT || i0 >= D.T) : D.T > TRSV_XL_MAXT) return;
  if (skip_system(st[s], skip_converged)) return;
  const int lo = BAND ? i0 : 0, hi = BAND ? min(i0 + TRSV_BAND, D.T) : D.T;
  __shared__ double sp[TRSV_G][NB];
  __shared__ double su[NB];
  extern __shared__ double dyn[];
  TS* sW = reinterpret_cast<TS*>(dyn);             // [2][TILE]
  double* sx = dyn + (2 * TILE * sizeof(TS)) / 8;   // [(hi - lo) * NB]: x of rows lo ..
  const int t = threadIdx.x, grp = t >> 8, rq = t & 15, cg = (t >> 4) & 15;
  const TS* Ab = A + D.a_off;
  const double* zz = ((BAND && hi < D.T) ? zw : z) + D.v_off;
  double* xx = x + D.v_off;
  // Winv of the last tile row into buffer (hi - 1) & 1
  if (hi > lo) {
    const TS* W = Wt + D.w_off + (int64_t)(hi - 1) * TILE;
    for (int e = 4 * t; e < TILE; e += 4 * TRSV_THREADS) {
      TS v[4];
      load4(W + e, v);
#pragma unroll
      for (int k = 0; k < 4; ++k) sW[((hi - 1) & 1) * TILE + e + k] = v[k];
    }
  }
  __syncthreads();
  for (int i = hi - 1; i >= lo; --i) {
    double part[4] = {0.0, 0.0, 0.0, 0.0};
    int j = i + 1 + grp;
    for (; j + TRSV_G * (TRSV_JB - 1) < hi; j += TRSV_G * TRSV_JB) {
      TS lv[TRSV_JB][4][4];
      double xv[TRSV_JB][4];
#pragma unroll
      for (int u = 0; u < TRSV_JB; ++u) {
        const TS* L = Ab + tile_index(j + TRSV_G * u, i) * TILE;   // (L^T)(i,j) = L(j,i)^T
#pragma unroll
        for (int q = 0; q < 4; ++q) load4(L + (cg + 16 * q) * NB + 4 * rq, lv[u][q]);
#pragma unroll
        for (int k = 0; k < 4; ++k) xv[u][k] = sx[(j + TRSV_G * u - lo) * NB + 4 * rq + k];
      }
#pragma unroll
      for (int u = 0; u < TRSV_JB; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int k = 0; k < 4; ++k) part[q] = fma((double)lv[u][q][k], xv[u][k], part[q]);
    }
    for (; j < hi; j += TRSV_G) {
      const TS* L = Ab + tile_index(j, i) * TILE;
      double xv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) xv[k] = sx[(j - lo) * NB + 4 * rq + k];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        TS lv[4];
        load4(L + (cg + 16 * q) * NB + 4 * rq, lv);
#pragma unroll
        for (int k = 0; k < 4; ++k) part[q] = fma((double)lv[k], xv[k], part[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double v = quad16_sum(part[q]);
      if (rq == 0) sp[grp][cg + 16 * q] = v;
    }
    __syncthreads();
    if (t < NB) {
      double sum = 0.0;
#pragma unroll
      for (int g = 0; g < TRSV_G; ++g) sum += sp[g][t];
      su[t] = zz[i * NB + t] - sum;
    }
    __syncthreads();
    if (grp == 0) {
      // x_i[c] = sum_r W(r, c) u[r], W(r, c) at c * NB + r
      const TS* W = sW + (i & 1) * TILE;
      double ur[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) ur[k] = su[4 * rq + k];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = cg + 16 * q;
        double p = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) p = fma((double)W[c * NB + 4 * rq + k], ur[k], p);
        const double v = quad16_sum(p);
        if (rq == 0) sx[(i - lo) * NB + c] = v;
      }
    } else if (i > lo) {
      // the next step's Winv into the other buffer
      const TS* W = Wt + D.w_off + (int64_t)(i - 1) * TILE;
      for (int e = 4 * (t - 256); e < TILE; e += 4 * (TRSV_THREADS - 256)) {
        TS v[4];
        load4(W + e, v);
#pragma unroll
        for (int k = 0; k < 4; ++k) sW[((i - 1) & 1) * TILE + e + k] = v[k];
      }
    }
    __syncthreads();
  }
  for (int e = t; e < (hi - lo) * NB; e += TRSV_THREADS) {
    const double v = sx[e];
    xx[lo * NB + e] = v;
    if (alpha_acc != nullptr) alpha_acc[D.v_off + lo * NB + e] += v;
  }
}

// Band update of the backward solve: for tile row i < i0 of a system on the
// band path, zw_i = (z_i for the last band, else zw_i) - sum_{i0<=j<i1}
// L(j,i)^T x_j.  One workgroup per (i, system); thread t owns rows
// 4 (t & 15) .. +3 and columns (t >> 4) + 16 q of each tile; fixed order.
template <typename TS>
__global__ __launch_bounds__(256) void k_trsv_bwd_upd(const SysDesc* __restrict__ desc,
                                                      const SysStatus* __restrict__ st, const TS* __restrict__ A,
                                                      const double* __restrict__ z, double* __restrict__ zw,
                                                      const double* __restrict__ x, int skip_converged, int i0) {
  const int i = blockIdx.x, s = blockIdx.y;
  const SysDesc D = desc[s];
  if (D.T <= TRSV_XL_MAXT || i0 >= D.T || i >= i0) return;
  if (skip_system(st[s], skip_converged)) return;
  const int i1 = min(i0 + TRSV_BAND, D.T);
  const int t = threadIdx.x, rq = t & 15, cg = t >> 4;
  const TS* Ab = A + D.a_off;
  const double* xx = x + D.v_off;
  double part[4] = {0.0, 0.0, 0.0, 0.0};
  int j = i0;
  for (; j + 3 < i1; j += 4) {
    TS lv[4][4][4];
    double xv[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const TS* L = Ab + tile_index(j + u, i) * TILE;
#pragma unroll
      for (int q = 0; q < 4; ++q) load4(L + (cg + 16 * q) * NB + 4 * rq, lv[u][q]);
#pragma unroll
      for (int k = 0; k < 4; ++k) xv[u][k] = xx[(j + u) * NB + 4 * rq + k];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k) part[q] = fma((double)lv[u][q][k], xv[u][k], part[q]);
  }
  for (; j < i1; ++j) {
    const TS* L = Ab + tile_index(j, i) * TILE;
    double xv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) xv[k] = xx[j * NB + 4 * rq + k];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      TS lv[4];
      load4(L + (cg + 16 * q) * NB + 4 * rq, lv);
#pragma unroll
      for (int k = 0; k < 4; ++k) part[q] = fma((double)lv[k], xv[k], part[q]);
    }
  }
  const double* src = (i1 == D.T ? z : zw) + D.v_off + (int64_t)i * NB;
  double* dst = zw + D.v_off + (int64_t)i * NB;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double v = quad16_sum(part[q]);
    if (rq == 0) dst[cg + 16 * q] = src[cg + 16 * q] - v;
  }
}

// Residual partials for the settings of one group (same kernel and sigma)
// of partition j: blockIdx.y = group * p + j, tile (i, j) = triangle index
// blockIdx.x.  The group's FP64 kernel tile K is read once (thread t holds
// the 4 x 4 block of rows 4 (t >> 4) + k, columns 4 (t & 15) + l); each
// setting adds its shift on the diagonal of its m x m system.  Tile (i, j)
// contributes A(i,j) alpha_j to row block i and, off the diagonal,
// A(i,j)^T alpha_i to row block j; partials go to P[(row block, col block)]
// of the system and are summed in column-block order by k_resid_reduce.
// Each thread sums its 4 x 4 block along rows and along columns; the 16
// threads' partials of one row (column) meet in LDS, where wave 0 adds the
// row partials and wave 1 the column partials in a fixed order (lane
// shuffles for these sums had made the kernel bound by LDS permutes).
__global__ __launch_bounds__(256) void k_resid_tiles(const SysDesc* __restrict__ desc,
                                                     const SysStatus* __restrict__ st, int p,
                                                     const int32_t* __restrict__ grp_first,
                                                     const int32_t* __restrict__ grp_next,
                                                     const double* __restrict__ K64,
                                                     const double* __restrict__ alpha, double* __restrict__ P,
                                                     const int64_t* __restrict__ p_off, double* __restrict__ Pabs) {
  const int j = blockIdx.y % p, grp = blockIdx.y / p;
  int q = grp_first[grp];
  const SysDesc D0 = desc[q * p + j];
  const int bx = blockIdx.x;
  int ii = (int)((sqrt(8.0 * (double)bx + 1.0) - 1.0) * 0.5);
  while ((int64_t)ii * (ii + 1) / 2 > bx) --ii;
  while ((int64_t)(ii + 1) * (ii + 2) / 2 <= bx) ++ii;
  const int jj = bx - ii * (ii + 1) / 2;
  if (ii >= D0.T) return;
  // sr[c][r]: row r's partial from column group c; sc[r][c]: column c's
  // partial from row group r (rows padded to 66 doubles)
  __shared__ __align__(16) double sr[16][NB + 2];
  __shared__ __align__(16) double sc[16][NB + 2];
  const int t = threadIdx.x, cbk = t & 15, rbk = t >> 4, w = t >> 6, lane = t & 63;
  const double* Kt = K64 + D0.k_off + tile_index(ii, jj) * TILE;
  double K[4][4];   // K[l][k] = K(4 rbk + k, 4 cbk + l)
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const double2* src = reinterpret_cast<const double2*>(Kt + (4 * cbk + l) * NB + 4 * rbk);
    const double2 u0 = src[0], u1 = src[1];
    K[l][0] = u0.x;
    K[l][1] = u0.y;
    K[l][2] = u1.x;
    K[l][3] = u1.y;
  }
  const bool diag_tile = ii == jj;
  // the thread's row and column partials into LDS, then the fixed-order sums
  // of wave 0 (rows, into row block ii, column block jj) and wave 1 (columns,
  // into row block jj, column block ii; off the diagonal only)
  auto reduce_out = [&](const double (&rs)[4], const double (&cs)[4], double* out, int T) {
    *reinterpret_cast<double2*>(&sr[cbk][4 * rbk]) = make_double2(rs[0], rs[1]);
    *reinterpret_cast<double2*>(&sr[cbk][4 * rbk + 2]) = make_double2(rs[2], rs[3]);
    *reinterpret_cast<double2*>(&sc[rbk][4 * cbk]) = make_double2(cs[0], cs[1]);
    *reinterpret_cast<double2*>(&sc[rbk][4 * cbk + 2]) = make_double2(cs[2], cs[3]);
    __syncthreads();
    if (w == 0) {
      double a = 0.0;
#pragma unroll
      for (int c = 0; c < 16; ++c) a += sr[c][lane];
      out[((int64_t)ii * T + jj) * NB + lane] = a;
    } else if (w == 1 && !diag_tile) {
      double a = 0.0;
#pragma unroll
      for (int r = 0; r < 16; ++r) a += sc[r][lane];
      out[((int64_t)jj * T + ii) * NB + lane] = a;
    }
    __syncthreads();   // before the next use of sr / sc
  };
  // partials of |K| times ones (row sums of |K| for Gershgorin's bounds):
  // the shift only moves the diagonal, so they are formed once for the
  // settings that share K, while any of them has no kappa bound yet, into
  // the slot of the group's first system
  bool need_abs = false;
  if (Pabs != nullptr)
    for (int q2 = q; q2 >= 0 && !need_abs; q2 = grp_next[q2]) need_abs = st[q2 * p + j].kappa_u < 0.0;
  if (need_abs) {   // uniform over the workgroup
    double rs[4], cs[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double acc = 0.0;
#pragma unroll
      for (int l = 0; l < 4; ++l) acc += fabs(K[l][k]);
      rs[k] = acc;
    }
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) acc += fabs(K[l][k]);
      cs[l] = acc;
    }
    reduce_out(rs, cs, Pabs + p_off[q * p + j], D0.T);
  }
  for (; q >= 0; q = grp_next[q]) {
    const int s = q * p + j;
    if (skip_system(st[s], 1)) continue;   // uniform over the workgroup: the residual only for the systems still refining
    const SysDesc D = desc[s];
    const double* aj = alpha + D.v_off + jj * NB + 4 * cbk;
    const double* ai = alpha + D.v_off + ii * NB + 4 * rbk;
    double av[4], bv[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) av[l] = aj[l];
#pragma unroll
    for (int k = 0; k < 4; ++k) bv[k] = ai[k];
    // rows: (K + lambda I)(i,j) alpha_j; columns: K(i,j)^T alpha_i (no shift off the diagonal)
    double rs[4], cs[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double acc = 0.0;
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        double kv = K[l][k];
        if (diag_tile && rbk == cbk && k == l && ii * NB + 4 * rbk + k < D.m) kv += D.lambda;
        acc = fma(kv, av[l], acc);
      }
      rs[k] = acc;
    }
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) acc = fma(K[l][k], bv[k], acc);
      cs[l] = acc;
    }
    reduce_out(rs, cs, P + p_off[s], D.T);
  }
}

// r_i = y_i - sum_j P(i, j) (fixed j order) and per-tile-row sums of r^2, y^2.
// First pass (Pabs non-null): per tile row, Gershgorin's bounds over its
// rows i < m: min_i (2 A_ii - sum_j |A_ij|) into glo and max_i sum_j |A_ij|
// into ghi.
__global__ __launch_bounds__(64) void k_resid_reduce(const SysDesc* __restrict__ desc, const SysStatus* __restrict__ st,
                                                     const double* __restrict__ y, const double* __restrict__ P,
                                                     const int64_t* __restrict__ p_off, double* __restrict__ r,
                                                     double* __restrict__ rn, double* __restrict__ yn,
                                                     const int64_t* __restrict__ n_off,
                                                     const double* __restrict__ Pabs, const double* __restrict__ K64,
                                                     double* __restrict__ glo, double* __restrict__ ghi) {
  const int s = blockIdx.y;
  const SysDesc D = desc[s];
  const bool need_abs = Pabs != nullptr && st[s].kappa_u < 0.0;
  const bool do_res = !skip_system(st[s], 1);
  if (!need_abs && !do_res) return;
  const int i = blockIdx.x;
  if (i >= D.T) return;
  const int lane = threadIdx.x;
  if (do_res) {
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
  if (need_abs) {
    // row sums of |K| of the settings sharing K (the group's first system), with the diagonal moved by the shift
    const double* Ab = Pabs + p_off[D.g_sys] + (int64_t)i * D.T * NB;
    double sk = 0.0;
    for (int j = 0; j < D.T; ++j) sk += Ab[j * NB + lane];
    const double kii = K64[D.k_off + tile_index(i, i) * TILE + lane * NB + lane];
    const double aii = kii + D.lambda;
    const double sa = sk - fabs(kii) + fabs(aii);
    const bool in = i * NB + lane < D.m;
    double lo = in ? 2.0 * aii - sa : INFINITY, hi = in ? sa : 0.0;
    for (int off = 32; off > 0; off >>= 1) {
      lo = fmin(lo, __shfl_xor(lo, off, 64));
      hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    if (lane == 0) {
      glo[n_off[s] + i] = lo;
      ghi[n_off[s] + i] = hi;
    }
  }
}

// Per system: ||r|| / ||y||, the forward-error estimate of alpha, the
// convergence flag and the refinement step count.
//
// The target `tol` bounds the relative error of alpha as well as the
// relative residual.  Through the residual the error is at most
// kappa(A) ||r|| / ||y||, with kappa_u, an upper bound of kappa_2(A) for the
// FP64 system the residual measures, in place of kappa: Gershgorin's discs
// give lambda_max <= max_i sum_j |A_ij| and lambda_min >= min_i (2 A_ii -
// sum_j |A_ij|), and for a positive semi-definite kernel (Gaussian, linear,
// polynomial with a, r >= 0) lambda_min >= lambda as well (computed once, on
// the first pass).  Once corrections have been applied, their sizes estimate
// the error directly: refinement contracts the error by rho per step (the
// ratio of the last two corrections), so about ||delta|| rho / (1 - rho) is
// left after the last one (||delta|| itself after the first, or when the
// corrections no longer shrink by half: the error then sits at the level of
// their fluctuation, the accuracy the FP64 residual allows).  A system
// converges when its residual and one of the two estimates are within tol.
// A step that does not halve the residual otherwise stalls it (the caller
// escalates its precision), and so does a BF16-updated factor whose pivot
// ratio kappa_l (a lower bound of kappa_2) exceeds 128: its error of order
// kappa u_bf16 (u_bf16 = 2^-8) would not contract.
__global__ void k_ir_check(const SysDesc* __restrict__ desc, SysStatus* __restrict__ st, int n_sys,
                           const double* __restrict__ rn, const double* __restrict__ yn,
                           const int64_t* __restrict__ n_off, double tol, int will_refine,
                           int32_t* __restrict__ active, const double* __restrict__ glo,
                           const double* __restrict__ ghi) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sys) return;
  SysStatus& S = st[s];
  const SysDesc D = desc[s];
  if (glo != nullptr && S.kappa_u < 0.0 && D.T > 0) {
    double lo = INFINITY, hi = 0.0;
    for (int i = 0; i < D.T; ++i) {
      lo = fmin(lo, glo[n_off[s] + i]);
      hi = fmax(hi, ghi[n_off[s] + i]);
    }
    const bool psd = D.kernel == KRR_KERNEL_GAUSSIAN || D.kernel == KRR_KERNEL_LINEAR ||
                     (D.kernel == KRR_KERNEL_POLYNOMIAL && D.ka >= 0.0 && D.kr >= 0.0);
    if (psd) lo = fmax(lo, D.lambda);
    S.kappa_u = lo > 0.0 ? hi / lo : INFINITY;
  }
  if (S.status != 0 || S.converged || S.stalled) return;
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
  const double kest = (S.kappa_u < 0.0 ? INFINITY : fmax(1.0, S.kappa_u)) * rel;
  double est = kest;
  if (S.corr >= 1) {
    const double e = S.dnorm / fmax(S.anorm, 1e-300);
    est = e;
    if (S.corr >= 2 && S.prev_dnorm > 0.0) {
      const double rho = S.dnorm / S.prev_dnorm;
      if (rho < 0.5) est = e * (rho / (1.0 - rho));
    }
  }
  S.err_est = fmin(est, kest);
  if (rel <= tol && S.err_est <= tol) {
    S.converged = 1;
  } else if ((prev >= 0.0 && !(rel <= 0.5 * prev)) || (D.level == 0 && S.corr == 0 && S.kappa_l > 128.0)) {
    S.stalled = 1;  // escalate precision
  } else if (will_refine) {
    S.refine_iters += 1;
    atomicAdd(active, 1);
  }
}

// kappa_l of the systems factored at `level`: the extreme diagonal entries of
// their factors (one wave per system).
template <typename TS>
__global__ __launch_bounds__(64) void k_pivot_range(const SysDesc* __restrict__ desc, SysStatus* __restrict__ st,
                                                    const TS* __restrict__ A, int level) {
  const int s = blockIdx.x;
  const SysDesc D = desc[s];
  if (D.level != level || D.m == 0 || st[s].status != 0) return;
  double lo = INFINITY, hi = 0.0;
  for (int i = threadIdx.x; i < D.m; i += 64) {
    const int k = i >> 6, r = i & 63;
    const double v = fabs((double)A[D.a_off + tile_index(k, k) * TILE + r * NB + r]);
    lo = fmin(lo, v);
    hi = fmax(hi, v);
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
  }
  if (threadIdx.x == 0) st[s].kappa_l = lo > 0.0 ? (hi / lo) * (hi / lo) : INFINITY;
}

// After a correction alpha += delta of the systems still refining: the
// infinity norms of delta and of the new alpha (one wave per system).
__global__ __launch_bounds__(64) void k_corr_norms(const SysDesc* __restrict__ desc, SysStatus* __restrict__ st,
                                                   const double* __restrict__ delta,
                                                   const double* __restrict__ alpha) {
  const int s = blockIdx.x;
  if (skip_system(st[s], 1)) return;
  const SysDesc D = desc[s];
  double dm = 0.0, am = 0.0;
  for (int i = threadIdx.x; i < D.m; i += 64) {
    dm = fmax(dm, fabs(delta[D.v_off + i]));
    am = fmax(am, fabs(alpha[D.v_off + i]));
  }
  for (int off = 32; off > 0; off >>= 1) {
    dm = fmax(dm, __shfl_xor(dm, off, 64));
    am = fmax(am, __shfl_xor(am, off, 64));
  }
  if (threadIdx.x == 0) {
    SysStatus& S = st[s];
    S.prev_dnorm = S.dnorm;
    S.dnorm = dm;
    S.anorm = am;
    S.corr += 1;
  }
}

}  // namespace

void trsv_forward(krr_ctx ctx, hipStream_t s, int prec, const SysDesc* desc, const SysStatus* st, int n_sys,
                  int Tmax, int64_t v_tot, const void* A, const void* Wt, const double* b, double* z,
                  int skip_converged) {
  KernelTimer kt(ctx, s, "trsv_forward", 0.0, 0);
  const bool f64 = prec == KRR_PREC_FP64;
  if (f64)
    hipLaunchKernelGGL((k_trsv_fwd<double, false>), dim3(n_sys), dim3(TRSV_THREADS), 0, s, desc, st,
                       (const double*)A, (const double*)Wt, b, (const double*)nullptr, z, skip_converged, 0);
  else
    hipLaunchKernelGGL((k_trsv_fwd<float, false>), dim3(n_sys), dim3(TRSV_THREADS), 0, s, desc, st,
                       (const float*)A, (const float*)Wt, b, (const double*)nullptr, z, skip_converged, 0);
  check_launch(ctx, s, "trsv_fwd");
  if (Tmax <= TRSV_XL_MAXT) return;
  // band path of the systems with T > TRSV_XL_MAXT
  double* bw = (double*)ws_get(ctx, "trsv_bw", (size_t)std::max<int64_t>(v_tot, 1) * 8);
  for (int i0 = 0; i0 < Tmax; i0 += TRSV_BAND) {
    if (f64)
      hipLaunchKernelGGL((k_trsv_fwd<double, true>), dim3(n_sys), dim3(TRSV_THREADS), 0, s, desc, st,
                         (const double*)A, (const double*)Wt, b, (const double*)bw, z, skip_converged, i0);
    else
      hipLaunchKernelGGL((k_trsv_fwd<float, true>), dim3(n_sys), dim3(TRSV_THREADS), 0, s, desc, st,
                         (const float*)A, (const float*)Wt, b, (const double*)bw, z, skip_converged, i0);
    check_launch(ctx, s, "trsv_fwd_band");
    const int below = Tmax - (i0 + TRSV_BAND);
    if (below <= 0) break;
    if (f64)
      hipLaunchKernelGGL((k_trsv_fwd_upd<double>), dim3((unsigned)below, (unsigned)n_sys), dim3(256), 0, s, desc,
                         st, (const double*)A, b, bw, (const double*)z, skip_converged, i0);
    else
      hipLaunchKernelGGL((k_trsv_fwd_upd<float>), dim3((unsigned)below, (unsigned)n_sys), dim3(256), 0, s, desc,
                         st, (const float*)A, b, bw, (const double*)z, skip_converged, i0);
    check_launch(ctx, s, "trsv_fwd_upd");
  }
}

void trsv_backward(krr_ctx ctx, hipStream_t s, int prec, const SysDesc* desc, const SysStatus* st, int n_sys,
                   int Tmax, int64_t v_tot, const void* A, const void* Wt, const double* z, double* x,
                   double* alpha_acc, int skip_converged) {
  KernelTimer kt(ctx, s, "trsv_backward", 0.0, 0);
  const size_t ts = prec == KRR_PREC_FP64 ? sizeof(double) : sizeof(float);
  const bool f64 = prec == KRR_PREC_FP64;
  const size_t lds_xl = 2 * TILE * ts + (size_t)std::max(std::min(Tmax, TRSV_XL_MAXT), 1) * NB * sizeof(double);
  if (f64)
    hipLaunchKernelGGL((k_trsv_bwd<double, false>), dim3(n_sys), dim3(TRSV_THREADS), lds_xl, s, desc, st,
                       (const double*)A, (const double*)Wt, z, (const double*)nullptr, x, alpha_acc, skip_converged,
                       0);
  else
    hipLaunchKernelGGL((k_trsv_bwd<float, false>), dim3(n_sys), dim3(TRSV_THREADS), lds_xl, s, desc, st,
                       (const float*)A, (const float*)Wt, z, (const double*)nullptr, x, alpha_acc, skip_converged,
                       0);
  check_launch(ctx, s, "trsv_bwd");
  if (Tmax <= TRSV_XL_MAXT) return;
  // band path of the systems with T > TRSV_XL_MAXT
  double* zw = (double*)ws_get(ctx, "trsv_zw", (size_t)std::max<int64_t>(v_tot, 1) * 8);
  const size_t lds_band = 2 * TILE * ts + (size_t)TRSV_BAND * NB * sizeof(double);
  for (int b = ceil_div(Tmax, TRSV_BAND) - 1; b >= 0; --b) {
    const int i0 = b * TRSV_BAND;
    if (f64)
      hipLaunchKernelGGL((k_trsv_bwd<double, true>), dim3(n_sys), dim3(TRSV_THREADS), lds_band, s, desc, st,
                         (const double*)A, (const double*)Wt, z, (const double*)zw, x, alpha_acc, skip_converged,
                         i0);
    else
      hipLaunchKernelGGL((k_trsv_bwd<float, true>), dim3(n_sys), dim3(TRSV_THREADS), lds_band, s, desc, st,
                         (const float*)A, (const float*)Wt, z, (const double*)zw, x, alpha_acc, skip_converged,
                         i0);
    check_launch(ctx, s, "trsv_bwd_band");
    if (i0 == 0) break;
    if (f64)
      hipLaunchKernelGGL((k_trsv_bwd_upd<double>), dim3((unsigned)i0, (unsigned)n_sys), dim3(256), 0, s, desc, st,
                         (const double*)A, z, zw, (const double*)x, skip_converged, i0);
    else
      hipLaunchKernelGGL((k_trsv_bwd_upd<float>), dim3((unsigned)i0, (unsigned)n_sys), dim3(256), 0, s, desc, st,
                         (const float*)A, z, zw, (const double*)x, skip_converged, i0);
    check_launch(ctx, s, "trsv_bwd_upd");
  }
}

void pivot_range(krr_ctx ctx, hipStream_t s, int prec, const SysDesc* desc, SysStatus* st, int n_sys, const void* A,
                 int level) {
  if (prec == KRR_PREC_FP64)
    hipLaunchKernelGGL((k_pivot_range<double>), dim3(n_sys), dim3(64), 0, s, desc, st, (const double*)A, level);
  else
    hipLaunchKernelGGL((k_pivot_range<float>), dim3(n_sys), dim3(64), 0, s, desc, st, (const float*)A, level);
  check_launch(ctx, s, "pivot_range");
}

void correction_norms(krr_ctx ctx, hipStream_t s, const SysDesc* desc, SysStatus* st, int n_sys, const double* delta,
                      const double* alpha) {
  hipLaunchKernelGGL(k_corr_norms, dim3(n_sys), dim3(64), 0, s, desc, st, delta, alpha);
  check_launch(ctx, s, "corr_norms");
}

// Pabs (nullable): on the first pass, the |A| partials and Gershgorin's
// bounds per tile row (glo, ghi) are formed beside the residual.
void residual_check(krr_ctx ctx, hipStream_t s, const SysDesc* desc, SysStatus* st, int n_sys, int p, int n_groups,
                    const int32_t* grp_first, const int32_t* grp_next, int Tmax, const double* K64,
                    const double* alpha, const double* y, double* r, double* P, const int64_t* p_off, double* rn,
                    double* yn, const int64_t* n_off, double tol, int will_refine, int32_t* active, double* Pabs,
                    double* glo, double* ghi) {
  const int64_t ntri = (int64_t)Tmax * (Tmax + 1) / 2;
  KernelTimer kt(ctx, s, "ir_residual", 0.0, 0);
  hipLaunchKernelGGL(k_resid_tiles, dim3((unsigned)ntri, (unsigned)(n_groups * p)), dim3(256), 0, s, desc,
                     (const SysStatus*)st, p, grp_first, grp_next, K64, alpha, P, p_off, Pabs);
  check_launch(ctx, s, "resid_tiles");
  hipLaunchKernelGGL(k_resid_reduce, dim3((unsigned)Tmax, (unsigned)n_sys), dim3(64), 0, s, desc,
                     (const SysStatus*)st, y, (const double*)P, p_off, r, rn, yn, n_off, (const double*)Pabs, K64,
                     glo, ghi);
  check_launch(ctx, s, "resid_reduce");
  hipLaunchKernelGGL(k_ir_check, dim3((unsigned)ceil_div(n_sys, 64)), dim3(64), 0, s, desc, st, n_sys,
                     (const double*)rn, (const double*)yn, n_off, tol, will_refine, active,
                     Pabs != nullptr ? (const double*)glo : nullptr, (const double*)ghi);
  check_launch(ctx, s, "ir_check");
}

}  // namespace krr
