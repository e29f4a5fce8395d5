// Batched ragged Cholesky factorisation A_s = L_s L_s^T of the systems
// (K_s + lambda_s I) of one fit (Section 2.3, Eq. 6: the paper solves these
// SPD systems by Cholesky, Section 5.5).
//
// Storage: every system keeps its lower triangle as T(T+1)/2 packed NB x NB
// tiles (column-major inside a tile, see common.hpp).  The factorisation is
// blocked right-looking with a panel of `W` tile columns:
//
//   for each panel [K0, K0+W):
//     for k in the panel:
//       column update   A(i,k) -= sum_{q in [K0,k)} L(i,q) L(k,q)^T   (i >= k)
//       diagonal block  A(k,k) = L(k,k) L(k,k)^T in FP64, and Winv(k) = L(k,k)^-1
//       panel solve     L(i,k) = A(i,k) Winv(k)^T                      (i > k)
//     trailing update   A(i,j) -= sum_{q in panel} L(i,q) L(j,q)^T     (i >= j >= K0+W)
//
// Every launch covers all systems of the batch (blockIdx.y = system); tiles
// beyond a system's own size exit at once, so one launch sequence serves a
// ragged batch.  The products run on matrix cores: FP64 MFMA for FP64
// storage, FP32 MFMA for FP32 storage, and BF16 MFMA with FP32 accumulation
// for the mixed-precision trailing updates.  Diagonal blocks are always
// factored and inverted in FP64.
#include "common.hpp"

#include <type_traits>

namespace krr {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int TILE = NB * NB;
constexpr int FRAG = 512;   // BF16 elements per packed MFMA operand fragment (16 rows x 32 columns)

__device__ __forceinline__ int64_t tile_index(int i, int j) { return (int64_t)i * (i + 1) / 2 + j; }

// acc[cb][rb] -= sum over the packed fragment columns ks in [ks0, ks1) of
// P(rbj + cb, ks) P(rbi + rb, ks)^T with v_mfma_f32_16x16x32_bf16 (FP32
// accumulation; the subtraction flips the sign of one BF16 operand, which is
// exact).  P points at the system's pack plus lane * 8; one 16-byte load per
// lane and fragment.  The fragments of PK_DEPTH steps are in flight in a
// register ring, so the loads of a step are issued several steps before its
// MFMAs (the ring's refills past ks1 re-read the last step and are unused).
// Output element (cb, rb, v) of a lane is row 16 rb + (lane & 15), column
// 16 cb + 4 (lane >> 4) + v of the 16 x 64-column block.
template <int NCB, int PK_DEPTH>
__device__ __forceinline__ void packed_sub(f4 (&acc)[NCB][4], const __bf16* __restrict__ P, int rbi, int rbj,
                                           int KSW, int ks0, int ks1) {
  if (ks0 >= ks1) return;
  typedef unsigned u4v __attribute__((ext_vector_type(4)));
  const u4v sgn{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  bf8 pa[PK_DEPTH][4], qv[PK_DEPTH][NCB];
  auto load = [&](int u, int ks) {
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
      pa[u][rb] = *reinterpret_cast<const bf8*>(P + ((int64_t)(rbi + rb) * KSW + ks) * FRAG);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
      qv[u][cb] = *reinterpret_cast<const bf8*>(P + ((int64_t)(rbj + cb) * KSW + ks) * FRAG);
  };
#pragma unroll
  for (int u = 0; u < PK_DEPTH; ++u) load(u, min(ks0 + u, ks1 - 1));
  for (int ks = ks0; ks < ks1; ks += PK_DEPTH) {
#pragma unroll
    for (int u = 0; u < PK_DEPTH; ++u) {
      if (ks + u < ks1) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const bf8 nq = __builtin_bit_cast(bf8, __builtin_bit_cast(u4v, qv[u][cb]) ^ sgn);
#pragma unroll
          for (int rb = 0; rb < 4; ++rb)
            acc[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nq, pa[u][rb], acc[cb][rb], 0, 0, 0);
        }
      }
      load(u, min(ks + u + PK_DEPTH, ks1 - 1));
    }
  }
}

// ---------------------------------------------------------------------------
// Diagonal block: A(k,k) = L L^T in FP64 and Winv(k) = L^-1, one workgroup of
// two waves per system, with the matrix held in registers.  The block is
// factored as A = U D^-1 U^T (U = L D^1/2: the columns of the successive
// Schur complements, D the pivots), so a column step needs one reciprocal
// and no square root on its dependency chain; L = U D^-1/2 and
// L^-1 = D^-1/2 U~^-1 (U~ = U D^-1, unit lower triangular) are formed at the
// end.
//   Wave 0 (factor): lane r holds row r of the working matrix.  Step j takes
//   the pivot d_j from lane j (computed by that lane at the end of step j-1),
//   publishes column j of the Schur complement (u, zero at and above the
//   diagonal) and 1/d_j through LDS, and applies a(r, c) -= (u_r / d_j) u_c.
//   Wave 1 (inverse): lane t holds column t of X = U~^-1 as the right-hand
//   side e_t of U~ x = e_t and runs the unit forward substitution step j
//   right after the barrier that publishes column j (a ring of two LDS slots,
//   one barrier per step).
// The 64 steps run as 8 straight-line groups of 8; group g keeps only the
// live columns [8g, 64) in registers (index c - 8g), so register indices are
// compile-time constants and no step touches a finished column.
// A pivot that is not positive (or NaN) marks the system failed with the
// LAPACK-style 1-based global column index.
// ---------------------------------------------------------------------------
constexpr int DIAG_THREADS = 128;
constexpr int SW_LD = NB + 1;   // padded LDS column of the staged results

__device__ __forceinline__ double read_lane(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// 1 / d: hardware reciprocal estimate refined by two Newton steps
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

struct DiagShared {
  double slot[2][NB + 2];   // slot[b][c] = u_c of step j (j % 2 == b), 0 for c <= j; slot[b][NB] = 1 / d_j
  double sU[NB * SW_LD];    // sU[j * SW_LD + r] = u_r of step j (0 above the diagonal)
  double sX[NB * SW_LD];    // sX[t * SW_LD + j] = X(j, t)
  double sd[NB];            // pivots, then 1 / sqrt(pivot)
  int fail;
};

// Steps [J0, J0 + 8) with J0 = NB - W; v[c] holds column J0 + c.
template <int W>
__device__ __forceinline__ void diag_group(bool factor_wave, int lane, double (&v)[W], double& piv,
                                           DiagShared& sh) {
  constexpr int J0 = NB - W;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int j = J0 + q;
    double* sl = sh.slot[q & 1];
    double s = 0.0;
    if (factor_wave) {
      if (!(piv > 0.0)) {
        if (lane == 0) sh.fail = j + 1;
      } else {
        const double rcp = recip(piv);
        const double u = v[q];
        s = lane > j ? u * rcp : 0.0;
        sl[lane] = lane > j ? u : 0.0;
        sh.sU[j * SW_LD + lane] = lane >= j ? u : 0.0;
        if (lane == 0) {
          sl[NB] = rcp;
          sh.sd[j] = piv;
        }
        if (q + 1 < W) piv = read_lane(fma(-s, u, v[q + 1]), j + 1);   // next pivot, owned by lane j+1
      }
    }
    __syncthreads();
    if (sh.fail) return;
    if (!factor_wave) {
      const double x = v[q];   // X(j, t)
      sh.sX[lane * SW_LD + j] = x;
      s = x * sl[NB];
    }
    // a(., c) -= s * u_c for the columns c > j of the group's window
    const double* col = sl + J0;
#pragma unroll
    for (int c = (q + 1) & ~1; c < W; c += 2) {
      const double2 b = *reinterpret_cast<const double2*>(col + c);
      if (c > q) v[c] = fma(-s, b.x, v[c]);
      v[c + 1] = fma(-s, b.y, v[c + 1]);
    }
  }
}

// drop the group's 8 finished columns
template <int W>
__device__ __forceinline__ void diag_shift(const double (&v)[W], double (&w)[W - 8]) {
#pragma unroll
  for (int c = 0; c < W - 8; ++c) w[c] = v[c + 8];
}

// With a BF16 panel pack (Pk != null, FP32 storage) and k > K0, the block
// first receives its column update A(k,k) -= sum_{q in [K0,k)} L(k,q) L(k,q)^T
// from the packed fragments (each wave 32 of the 64 columns), staged in LDS.
// Wpk (nullable): Winv(k) is also written as BF16 high/low operand
// fragments for the BF16 panel solve (see k_panel_col).
template <typename TS>
__global__ __launch_bounds__(DIAG_THREADS) void k_potrf_diag(const SysDesc* __restrict__ desc,
                                                             SysStatus* __restrict__ st, TS* __restrict__ A,
                                                             TS* __restrict__ Wt, int k, int level,
                                                             const __bf16* __restrict__ Pk, int K0, int Wp,
                                                             __bf16* __restrict__ Wpk) {
  const int s = blockIdx.x;
  const SysDesc D = desc[s];
  if (k >= D.T || st[s].status != 0 || D.level != level) return;
  __shared__ __align__(16) DiagShared sh;
  TS* tile = A + D.a_off + tile_index(k, k) * TILE;
  const int lane = threadIdx.x & 63;
  const bool factor_wave = threadIdx.x < 64;
  const bool fused = std::is_same<TS, float>::value && Pk != nullptr && k > K0;
  if (fused) {
    const int w = threadIdx.x >> 6, il = lane & 15, kg = lane >> 4;
    f4 acc[2][4];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[cb][rb][v] = (float)tile[(16 * (2 * w + cb) + 4 * kg + v) * NB + 16 * rb + il];
    packed_sub<2, 2>(acc, Pk + D.pk_off + lane * 8, (k - K0) * 4, (k - K0) * 4 + 2 * w, 2 * Wp, 0, 2 * (k - K0));
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          sh.sX[(16 * (2 * w + cb) + 4 * kg + v) * SW_LD + 16 * rb + il] = (double)acc[cb][rb][v];
    __syncthreads();
  }
  double v64[NB];
  if (factor_wave) {
    // row `lane` of A(k,k); entries above the diagonal are never consumed
    if (fused) {
#pragma unroll
      for (int c = 0; c < NB; ++c) v64[c] = sh.sX[c * SW_LD + lane];
    } else {
#pragma unroll
      for (int c = 0; c < NB; ++c) v64[c] = (double)tile[c * NB + lane];
    }
  } else {
#pragma unroll
    for (int c = 0; c < NB; ++c) v64[c] = (c == lane) ? 1.0 : 0.0;
  }
  if (threadIdx.x == 0) sh.fail = 0;
  __syncthreads();
  double piv = factor_wave ? read_lane(v64[0], 0) : 0.0;
  do {
    diag_group<64>(factor_wave, lane, v64, piv, sh);
    if (sh.fail) break;
    double v56[56];
    diag_shift<64>(v64, v56);
    diag_group<56>(factor_wave, lane, v56, piv, sh);
    if (sh.fail) break;
    double v48[48];
    diag_shift<56>(v56, v48);
    diag_group<48>(factor_wave, lane, v48, piv, sh);
    if (sh.fail) break;
    double v40[40];
    diag_shift<48>(v48, v40);
    diag_group<40>(factor_wave, lane, v40, piv, sh);
    if (sh.fail) break;
    double v32[32];
    diag_shift<40>(v40, v32);
    diag_group<32>(factor_wave, lane, v32, piv, sh);
    if (sh.fail) break;
    double v24[24];
    diag_shift<32>(v32, v24);
    diag_group<24>(factor_wave, lane, v24, piv, sh);
    if (sh.fail) break;
    double v16[16];
    diag_shift<24>(v24, v16);
    diag_group<16>(factor_wave, lane, v16, piv, sh);
    if (sh.fail) break;
    double v8[8];
    diag_shift<16>(v16, v8);
    diag_group<8>(factor_wave, lane, v8, piv, sh);
  } while (false);
  if (sh.fail) {
    if (threadIdx.x == 0) {
      st[s].status = KRR_ENOTSPD;
      st[s].failed_pivot = k * NB + sh.fail;
    }
    return;
  }
  __syncthreads();
  if (threadIdx.x < NB) sh.sd[threadIdx.x] = 1.0 / sqrt(sh.sd[threadIdx.x]);
  __syncthreads();
  // L(r, c) = u_r(c) / sqrt(d_c); W(r, c) = X(r, c) / sqrt(d_r)
  TS* wt = Wt + D.w_off + (int64_t)k * TILE;
  for (int e = threadIdx.x; e < TILE; e += DIAG_THREADS) {
    const int c = e >> 6, r = e & 63;
    tile[e] = (TS)(sh.sU[c * SW_LD + r] * sh.sd[c]);
    wt[e] = (TS)((r >= c) ? sh.sX[c * SW_LD + r] * sh.sd[r] : 0.0);
  }
  if (Wpk != nullptr) {
    // fragment f = 2 cb + ks, part hl (0 high, 1 low): lane l holds Winv(16 cb + (l & 15), 32 ks + 8 (l >> 4) + e)
    // split from its FP32 value: hi = bf16(w), lo = bf16(w - hi)
    __bf16* base = Wpk + ((int64_t)s * Wp + (k - K0)) * 16 * FRAG;
    for (int task = threadIdx.x; task < 8 * 64; task += DIAG_THREADS) {
      const int f = task >> 6, l = task & 63;
      const int cb = f >> 1, ks = f & 1;
      const int row = 16 * cb + (l & 15);
      bf8 hi, lo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int col = 32 * ks + 8 * (l >> 4) + e;
        const float w = (float)((row >= col) ? sh.sX[col * SW_LD + row] * sh.sd[row] : 0.0);
        const __bf16 h = (__bf16)w;
        hi[e] = h;
        lo[e] = (__bf16)(w - (float)h);
      }
      *reinterpret_cast<bf8*>(base + (int64_t)(2 * f) * FRAG + l * 8) = hi;
      *reinterpret_cast<bf8*>(base + (int64_t)(2 * f + 1) * FRAG + l * 8) = lo;
    }
  }
}

// ---------------------------------------------------------------------------
// Tile products C = sum_q P_q Q_q^T on matrix cores, with P_q, Q_q, C packed
// column-major NB x NB tiles.  The MFMA computes D' = Q P^T so that a lane's
// result index along 16 consecutive lanes walks down a tile column (unit
// stride in memory).  Wave w owns rows [32(w&1), +32) and columns
// [32(w>>1), +32) of the output tile.
//   MODE_TRSM:   C(i,k) <- A(i,k) Winv(k)^T         i = i0 + bx, j = k
//   MODE_COL:    C(i,k) <- C(i,k) - sum_{q0<=q<q1} L(i,q) L(k,q)^T, i = i0 + bx
//   MODE_TRI:    C(i,j) <- C(i,j) - sum_{q0<=q<q1} L(i,q) L(j,q)^T for the
//                lower triangle j0 <= j <= i (bx = linear triangle index)
// ---------------------------------------------------------------------------
enum { MODE_TRSM = 0, MODE_COL = 1, MODE_TRI = 2 };

__device__ __forceinline__ void mfma_step(d4& acc, double a, double b) {
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}
__device__ __forceinline__ void mfma_step(f4& acc, float a, float b) {
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}
// row of register v of a lane's 16x16 block result
__device__ __forceinline__ int out_row(double*, int lane, int v) { return (lane >> 4) + 4 * v; }
__device__ __forceinline__ int out_row(float*, int lane, int v) { return 4 * (lane >> 4) + v; }

template <typename TS>
struct AccT;
template <>
struct AccT<double> {
  typedef d4 type;
};
template <>
struct AccT<float> {
  typedef f4 type;
};

__device__ __forceinline__ bool locate(int mode, int bx, int i0, int jc, int T, int& i, int& j) {
  if (mode == MODE_TRI) {
    // bx = ii (ii + 1) / 2 + jj, 0 <= jj <= ii
    int ii = (int)((sqrt(8.0 * (double)bx + 1.0) - 1.0) * 0.5);
    while ((int64_t)ii * (ii + 1) / 2 > bx) --ii;
    while ((int64_t)(ii + 1) * (ii + 2) / 2 <= bx) ++ii;
    const int jj = bx - ii * (ii + 1) / 2;
    i = i0 + ii;
    j = i0 + jj;
  } else {
    i = i0 + bx;
    j = jc;
  }
  return i < T;
}

template <typename TS, int MODE>
__global__ __launch_bounds__(256) void k_tile_gemm(const SysDesc* __restrict__ desc,
                                                   const SysStatus* __restrict__ st, TS* __restrict__ A,
                                                   const TS* __restrict__ Wt, int i0, int jc, int q0, int q1,
                                                   int level) {
  typedef typename AccT<TS>::type acc_t;
  const int s = blockIdx.y;
  const SysDesc D = desc[s];
  if (st[s].status != 0 || D.level != level) return;
  int i, j;
  if (!locate(MODE, blockIdx.x, i0, jc, D.T, i, j)) return;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int r0 = 32 * (w & 1);
  const int c0 = 32 * (w >> 1);
  TS* Ab = A + D.a_off;
  TS* C = Ab + tile_index(i, j) * TILE;
  acc_t acc[2][2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[cb][rb][v] = 0;
  const int kl = lane >> 4;   // k offset of this lane inside a 4-step
  const int il = lane & 15;   // row offset inside a 16-block
  int qa = q0, qb = q1;
  if (MODE == MODE_TRSM) {
    qa = 0;
    qb = 1;
  }
  for (int q = qa; q < qb; ++q) {
    const TS* P;
    const TS* Q;
    if (MODE == MODE_TRSM) {
      P = C;
      Q = Wt + D.w_off + (int64_t)jc * TILE;
    } else {
      P = Ab + tile_index(i, q) * TILE;
      Q = Ab + tile_index(j, q) * TILE;
    }
#pragma unroll 4
    for (int kb = 0; kb < NB; kb += 4) {
      const int koff = (kb + kl) * NB;
      TS pa[2], qv[2];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) pa[rb] = P[koff + r0 + 16 * rb + il];
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) qv[cb] = Q[koff + c0 + 16 * cb + il];
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) mfma_step(acc[cb][rb], qv[cb], pa[rb]);
    }
  }
  if (MODE == MODE_TRSM) __syncthreads();  // C aliases P: every wave must finish reading
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = c0 + 16 * cb + out_row((TS*)nullptr, lane, v);
        const int r = r0 + 16 * rb + il;
        const int e = c * NB + r;
        if (MODE == MODE_TRSM)
          C[e] = (TS)acc[cb][rb][v];
        else
          C[e] = (TS)(C[e] - acc[cb][rb][v]);
      }
}

// ---------------------------------------------------------------------------
// Mixed precision trailing/column updates: FP32 tiles, operands rounded to
// BF16, products accumulated in FP32 on v_mfma_f32_16x16x32_bf16.  Operands
// are staged through LDS row-major (32 consecutive k per row as BF16) so
// that a lane reads its 8 consecutive k values with one 16-byte load.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void k_tile_gemm_bf16(const SysDesc* __restrict__ desc,
                                                        const SysStatus* __restrict__ st, float* __restrict__ A,
                                                        int i0, int jc, int q0, int q1, int level) {
  const int s = blockIdx.y;
  const SysDesc D = desc[s];
  if (st[s].status != 0 || D.level != level) return;
  int i, j;
  if (!locate(MODE, blockIdx.x, i0, jc, D.T, i, j)) return;
  constexpr int KC = NB;         // k per stage
  constexpr int LDR = KC + 8;    // padded row length (bf16 elements)
  __shared__ __attribute__((aligned(16))) __bf16 sP[NB * LDR];
  __shared__ __attribute__((aligned(16))) __bf16 sQ[NB * LDR];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int r0 = 32 * (w & 1);
  const int c0 = 32 * (w >> 1);
  float* Ab = A + D.a_off;
  float* C = Ab + tile_index(i, j) * TILE;
  f4 acc[2][2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[cb][rb][v] = 0.f;
  const int il = lane & 15;
  const int kg = lane >> 4;  // 8-wide k group
  for (int q = q0; q < q1; ++q) {
    const float* P = Ab + tile_index(i, q) * TILE;
    const float* Q = Ab + tile_index(j, q) * TILE;
    for (int k0 = 0; k0 < NB; k0 += KC) {
      // stage: element (row, k) of the chunk; consecutive threads walk rows
      // (unit stride in the column-major tile)
      __syncthreads();
#pragma unroll
      for (int e = t; e < NB * KC; e += 256) {
        const int row = e & 63;
        const int kk = e >> 6;
        sP[row * LDR + kk] = (__bf16)P[(k0 + kk) * NB + row];
        sQ[row * LDR + kk] = (__bf16)Q[(k0 + kk) * NB + row];
      }
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < KC; ks += 32) {
        bf8 pa[2], qv[2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
          pa[rb] = *reinterpret_cast<const bf8*>(&sP[(r0 + 16 * rb + il) * LDR + ks + 8 * kg]);
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          qv[cb] = *reinterpret_cast<const bf8*>(&sQ[(c0 + 16 * cb + il) * LDR + ks + 8 * kg]);
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
          for (int rb = 0; rb < 2; ++rb)
            acc[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qv[cb], pa[rb], acc[cb][rb], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = c0 + 16 * cb + 4 * (lane >> 4) + v;
        const int r = r0 + 16 * rb + il;
        const int e = c * NB + r;
        C[e] = C[e] - acc[cb][rb][v];
      }
}

// ---------------------------------------------------------------------------
// Mixed precision updates with pre-packed BF16 operands.
// The pack of a system holds the current panel [K0, K0 + W) as
// v_mfma_f32_16x16x32_bf16 operand fragments: fragment (rb, ks) covers rows
// [K0*64 + 16 rb, +16) and panel columns [32 ks, +32) (ks < 2W); lane l holds
// row 16 rb + (l & 15) and columns 32 ks + 8 (l >> 4) + e (e = 0..7): 16
// contiguous bytes per lane, 1 KiB per fragment.  Column k of the panel is
// packed (rows below the diagonal block) by k_panel_col right after its
// panel solve.
// ---------------------------------------------------------------------------

// Column k of the panel [K0, K0 + Wp), tile rows i > k, one 64 x 64 tile per
// wavefront (waves are independent: no barrier):
//   C(i,k) -= sum_{q in [K0,k)} L(i,q) L(k,q)^T   BF16 packed operands, FP32 accumulation,
//                                                 starting from the C tile in registers
//   L(i,k)  = C(i,k) Winv(k)^T                    FP32 matrix cores, C through the wave's LDS
//   L(i,k) -> the FP32 tile, and (do_pack) BF16 fragments of the pack
constexpr int PC_LD = NB + 1;
__global__ __launch_bounds__(256) void k_panel_col(const SysDesc* __restrict__ desc, const SysStatus* __restrict__ st,
                                                   float* __restrict__ A, const __bf16* __restrict__ Wpk,
                                                   __bf16* __restrict__ Pk, int K0, int k, int Wp, int level,
                                                   int do_pack) {
  const int s = blockIdx.z;
  const SysDesc D = desc[s];
  if (st[s].status != 0 || D.level != level) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = k + 1 + 4 * blockIdx.x + w;
  if (i >= D.T) return;
  __shared__ float sC[4][NB * PC_LD];
  float* sc = sC[w];
  const int KSW = 2 * Wp;
  const int il = lane & 15, kg = lane >> 4;
  // Winv(k) fragments first: their latency overlaps the column update
  const __bf16* Wf = Wpk + ((int64_t)s * Wp + (k - K0)) * 16 * FRAG + lane * 8;
  bf8 whi[4][2], wlo[4][2];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
      if (ks == 0 || cb >= 2) {
        whi[cb][ks] = *reinterpret_cast<const bf8*>(Wf + (int64_t)(2 * (2 * cb + ks)) * FRAG);
        wlo[cb][ks] = *reinterpret_cast<const bf8*>(Wf + (int64_t)(2 * (2 * cb + ks) + 1) * FRAG);
      }
  float* C = A + D.a_off + tile_index(i, k) * TILE;
  f4 acc[4][4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[cb][rb][v] = C[(16 * cb + 4 * kg + v) * NB + 16 * rb + il];
  if (k > K0) packed_sub<4, 4>(acc, Pk + D.pk_off + lane * 8, (i - K0) * 4, (k - K0) * 4, KSW, 0, 2 * (k - K0));
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) sc[(16 * cb + 4 * kg + v) * PC_LD + 16 * rb + il] = acc[cb][rb][v];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // out(r, c) = sum_{t <= c} C(r, t) Winv(c, t) on BF16 matrix cores with
  // high/low splits of both operands (three products, FP32 accumulation:
  // about 16 significant bits per product, below the error of the BF16
  // updates and corrected by the FP64 refinement); blocks of Winv above its
  // diagonal are zero and skipped.  A operand: Winv fragments (cb, ks);
  // B operand: C(16 rb + (lane & 15), 32 ks + 8 (lane >> 4) + e) from LDS.
  f4 o[4][4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) o[cb][rb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      bf8 chi, clo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float cv = sc[(32 * ks + 8 * kg + e) * PC_LD + 16 * rb + il];
        const __bf16 h = (__bf16)cv;
        chi[e] = h;
        clo[e] = (__bf16)(cv - (float)h);
      }
#pragma unroll
      for (int cb = 2 * ks; cb < 4; ++cb) {
        o[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wlo[cb][ks], chi, o[cb][rb], 0, 0, 0);
        o[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(whi[cb][ks], clo, o[cb][rb], 0, 0, 0);
        o[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(whi[cb][ks], chi, o[cb][rb], 0, 0, 0);
      }
    }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // MFMA result: register v of a lane is column 4 (lane >> 4) + v, row lane & 15 of its 16 x 16 block
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = 16 * cb + 4 * kg + v, r = 16 * rb + il;
        C[c * NB + r] = o[cb][rb][v];
        sc[c * PC_LD + r] = o[cb][rb][v];
      }
  if (!do_pack) return;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  __bf16* Pout = Pk + D.pk_off + lane * 8;
#pragma unroll
  for (int rbl = 0; rbl < 4; ++rbl)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = 16 * rbl + il, cl = 32 * h + 8 * kg;
      bf8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (__bf16)sc[(cl + e) * PC_LD + r];
      const int rb = (i - K0) * 4 + rbl, ks = 2 * (k - K0) + h;
      *reinterpret_cast<bf8*>(Pout + ((int64_t)rb * KSW + ks) * FRAG) = v;
    }
}

// Trailing update A(i,j) -= sum_{q in panel} L(i,q) L(j,q)^T for the lower
// triangle i >= j >= i0, from the packed fragment columns [ks0, ks1): 128 x 128
// super-tiles (blockIdx.x = triangle index), one 64 x 64 tile per wavefront,
// accumulators starting from the C tile; systems along blockIdx.z.
__global__ __launch_bounds__(256) void k_packed_trailing(const SysDesc* __restrict__ desc,
                                                         const SysStatus* __restrict__ st, float* __restrict__ A,
                                                         const __bf16* __restrict__ Pk, int K0, int ks0, int ks1,
                                                         int i0, int Wp, int level) {
  const int s = blockIdx.z;
  const SysDesc D = desc[s];
  if (st[s].status != 0 || D.level != level) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int R = D.T - i0;
  if (R <= 0) return;
  const int NS = (R + 1) / 2;
  const int bx = blockIdx.x;
  int I = (int)((sqrt(8.0 * (double)bx + 1.0) - 1.0) * 0.5);
  while (I * (I + 1) / 2 > bx) --I;
  while ((I + 1) * (I + 2) / 2 <= bx) ++I;
  const int J = bx - I * (I + 1) / 2;
  if (I >= NS) return;
  const int i = i0 + 2 * I + (w & 1);
  const int j = i0 + 2 * J + (w >> 1);
  if (i >= D.T || j > i) return;       // waves are independent: no barrier follows
  float* C = A + D.a_off + tile_index(i, j) * TILE;
  const int il = lane & 15, kg = lane >> 4;
  f4 acc[4][4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[cb][rb][v] = C[(16 * cb + 4 * kg + v) * NB + 16 * rb + il];
  packed_sub<4, 2>(acc, Pk + D.pk_off + lane * 8, (i - K0) * 4, (j - K0) * 4, 2 * Wp, ks0, ks1);
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) C[(16 * cb + 4 * kg + v) * NB + 16 * rb + il] = acc[cb][rb][v];
}

template <typename TS>
void launch_update(krr_ctx ctx, hipStream_t s, bool bf16, int mode, const SysDesc* desc, SysStatus* st, TS* A,
                   const TS* Wt, int n_sys, int64_t nblk, int i0, int jc, int q0, int q1, int level) {
  if (nblk <= 0) return;
  const dim3 grid((unsigned)nblk, (unsigned)n_sys);
  if constexpr (std::is_same<TS, float>::value) {
    if (bf16 && mode != MODE_TRSM) {
      if (mode == MODE_COL)
        hipLaunchKernelGGL((k_tile_gemm_bf16<MODE_COL>), grid, dim3(256), 0, s, desc, st, A, i0, jc, q0, q1, level);
      else
        hipLaunchKernelGGL((k_tile_gemm_bf16<MODE_TRI>), grid, dim3(256), 0, s, desc, st, A, i0, jc, q0, q1, level);
      check_launch(ctx, s, "tile_gemm_bf16");
      return;
    }
  }
  const SysStatus* cst = st;
  if (mode == MODE_TRSM)
    hipLaunchKernelGGL((k_tile_gemm<TS, MODE_TRSM>), grid, dim3(256), 0, s, desc, cst, A, Wt, i0, jc, q0, q1, level);
  else if (mode == MODE_COL)
    hipLaunchKernelGGL((k_tile_gemm<TS, MODE_COL>), grid, dim3(256), 0, s, desc, cst, A, Wt, i0, jc, q0, q1, level);
  else
    hipLaunchKernelGGL((k_tile_gemm<TS, MODE_TRI>), grid, dim3(256), 0, s, desc, cst, A, Wt, i0, jc, q0, q1, level);
  check_launch(ctx, s, "tile_gemm");
}

template <typename TS>
void factor_t(krr_ctx ctx, hipStream_t s, const SysDesc* desc, SysStatus* st, int n_sys, int Tmax, TS* A, TS* Wt,
              bool bf16, int Wp, int level, const SysDesc* hdesc, __bf16* Pk) {
  // algorithmic flops of each launch (timing only), from the real sizes m
  auto each = [&](auto&& f) {
    double tot = 0.0;
    if (ctx->timing == 0 || hdesc == nullptr) return 0.0;
    for (int i = 0; i < n_sys; ++i)
      if (hdesc[i].level == level) tot += f((double)hdesc[i].m);
    return tot;
  };
  const bool f64 = std::is_same<TS, double>::value;
  const char* trail_name = bf16 ? "chol_trailing_bf16" : (f64 ? "chol_trailing_f64" : "chol_trailing_f32");
  const char* col_name = bf16 ? "chol_column_bf16" : (f64 ? "chol_column_f64" : "chol_column_f32");
  const char* trsm_name = f64 ? "chol_trsm_f64" : "chol_trsm_f32";
  const bool packed = std::is_same<TS, float>::value && bf16 && Pk != nullptr;
  auto diag_trsm = [&](int k) {
    {
      KernelTimer kt(ctx, s, "chol_diag", each([&](double m) {
        const double b = std::min<double>(NB, m - k * NB);
        return b > 0 ? 2.0 * b * b * b / 3.0 : 0.0;
      }), 0);
      hipLaunchKernelGGL((k_potrf_diag<TS>), dim3(n_sys), dim3(DIAG_THREADS), 0, s, desc, st, A, Wt, k, level,
                         (const __bf16*)nullptr, 0, 1, (__bf16*)nullptr);
      check_launch(ctx, s, "potrf_diag");
    }
    if (k + 1 < Tmax) {
      KernelTimer kt(ctx, s, trsm_name, each([&](double m) {
        const double rows = m - (k + 1) * NB;
        return rows > 0 ? rows * (double)NB * NB : 0.0;
      }), 1);
      launch_update<TS>(ctx, s, false, MODE_TRSM, desc, st, A, Wt, n_sys, Tmax - k - 1, k + 1, k, 0, 1, level);
    }
  };
  if (packed) {
    // Two launches per panel column: the diagonal block with its own column
    // update, then the fused column update + panel solve + BF16 packing of
    // the tiles below it; after the panel, one trailing update.  Wpk: BF16
    // high/low fragments of the panel's inverse diagonal blocks.
    __bf16* Wpk = (__bf16*)ws_get(ctx, "chol_wpk", (size_t)n_sys * Wp * 16 * FRAG * sizeof(__bf16));
    for (int K0 = 0; K0 < Tmax; K0 += Wp) {
      const int K1 = std::min(K0 + Wp, Tmax);
      for (int k = K0; k < K1; ++k) {
        {
          KernelTimer kt(ctx, s, "chol_diag", each([&](double m) {
            const double b = std::min<double>(NB, m - k * NB);
            return b > 0 ? 2.0 * b * b * b / 3.0 : 0.0;
          }), 0);
          hipLaunchKernelGGL((k_potrf_diag<TS>), dim3(n_sys), dim3(DIAG_THREADS), 0, s, desc, st, A, Wt, k, level,
                             (const __bf16*)Pk, K0, Wp, Wpk);
          check_launch(ctx, s, "potrf_diag");
        }
        if (k + 1 < Tmax) {
          // credited: the column update of the tiles below the diagonal and their panel solve;
          // algorithmic bytes: read those tiles and write their factor (FP32)
          KernelTimer kt(ctx, s, col_name, each([&](double m) {
            const double rows = m - (k + 1) * NB;
            return rows > 0 ? 2.0 * rows * NB * (k - K0) * NB + rows * (double)NB * NB : 0.0;
          }), 1, each([&](double m) {
            const double rows = m - (k + 1) * NB;
            return rows > 0 ? 2.0 * rows * NB * sizeof(float) : 0.0;
          }));
          const int do_pack = (k + 1 < K1 || K1 < Tmax) ? 1 : 0;
          hipLaunchKernelGGL(k_panel_col, dim3((unsigned)ceil_div(Tmax - k - 1, 4), 1, (unsigned)n_sys), dim3(256), 0,
                             s, desc, (const SysStatus*)st, (float*)A, (const __bf16*)Wpk, (__bf16*)Pk, K0, k, Wp,
                             level, do_pack);
          check_launch(ctx, s, "panel_col");
        }
      }
      if (K1 < Tmax) {
        const int64_t R = Tmax - K1;
        // algorithmic bytes: read and write the lower trailing triangle (FP32)
        KernelTimer kt(ctx, s, trail_name, each([&](double m) {
          const double n = m - K1 * NB;
          const double kk = std::min<double>(K1 * NB, m) - K0 * NB;
          return n > 0 ? n * (n + 1.0) * kk : 0.0;
        }), 1, each([&](double m) {
          const double n = m - K1 * NB;
          return n > 0 ? n * (n + 1.0) * sizeof(float) : 0.0;
        }));
        const int64_t NS = (R + 1) / 2;
        hipLaunchKernelGGL(k_packed_trailing, dim3((unsigned)(NS * (NS + 1) / 2), 1, (unsigned)n_sys), dim3(256), 0,
                           s, desc, (const SysStatus*)st, (float*)A, (const __bf16*)Pk, K0, 0, 2 * (K1 - K0), K1, Wp,
                           level);
        check_launch(ctx, s, "packed_trailing");
      }
    }
    return;
  }
  for (int K0 = 0; K0 < Tmax; K0 += Wp) {
    const int K1 = std::min(K0 + Wp, Tmax);
    for (int k = K0; k < K1; ++k) {
      if (k > K0) {
        KernelTimer kt(ctx, s, col_name, each([&](double m) {
          const double rows = m - k * NB;
          return rows > 0 ? 2.0 * rows * std::min<double>(NB, rows) * (k - K0) * NB : 0.0;
        }), 1);
        launch_update<TS>(ctx, s, bf16, MODE_COL, desc, st, A, Wt, n_sys, Tmax - k, k, k, K0, k, level);
      }
      diag_trsm(k);
    }
    if (K1 < Tmax) {
      const int64_t R = Tmax - K1;
      KernelTimer kt(ctx, s, trail_name, each([&](double m) {
        const double n = m - K1 * NB;
        const double kk = std::min<double>(K1 * NB, m) - K0 * NB;
        return n > 0 ? n * (n + 1.0) * kk : 0.0;
      }), 1);
      launch_update<TS>(ctx, s, bf16, MODE_TRI, desc, st, A, Wt, n_sys, R * (R + 1) / 2, K1, 0, K0, K1, level);
    }
  }
}

}  // namespace

// Factor, in place, the systems of the batch whose descriptor carries
// `level` (the others are left untouched).  prec: KRR_PREC_FP64 -> A, Wt are
// double; FP32 / MIXED -> float.  bf16: BF16 trailing and column updates
// (MIXED first pass); otherwise FP32 (or FP64) matrix-core updates.  hdesc:
// host copy of desc (used for the flop counts of timed launches; nullable).
void cholesky_factor(krr_ctx ctx, hipStream_t s, int prec, const SysDesc* desc, SysStatus* st, int n_sys, int Tmax,
                     void* A, void* Wt, int level, bool bf16, const SysDesc* hdesc, void* pack) {
  const int Wp = ctx->panel_tiles;
  if (prec == KRR_PREC_FP64)
    factor_t<double>(ctx, s, desc, st, n_sys, Tmax, (double*)A, (double*)Wt, false, Wp, level, hdesc, nullptr);
  else
    factor_t<float>(ctx, s, desc, st, n_sys, Tmax, (float*)A, (float*)Wt, bf16, Wp, level, hdesc, (__bf16*)pack);
}

// BF16 elements of the panel pack slot of a system with T tile rows (the
// first panel, rows [0, T*64) x 2W fragment columns, is the largest).
int64_t pack_slot_elems(int T, int Wp) {
  return (int64_t)T * 4 * 2 * (int64_t)Wp * FRAG;
}

}  // namespace krr
