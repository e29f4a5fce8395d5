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
#include "persist_plan.hpp"

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
// The loop runs whole rounds of the ring with no condition and the remaining
// steps follow it (WHOLE: the step count is a multiple of PK_DEPTH and there
// are none): MFMAs under a branch inside the loop let the compiler move the
// prefetched loads into the branch, next to their use.  Scheduling
// barriers keep the ring order (prologue) and each step's operand handling
// inside its step, so that a step waits only for its own loads.
// Output element (cb, rb, v) of a lane is row 16 rb + (lane & 15), column
// 16 cb + 4 (lane >> 4) + v of the 16 x 64-column block.
template <int NCB, int PK_DEPTH, bool WHOLE = false>
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
  auto step = [&](int u) {
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const bf8 nq = __builtin_bit_cast(bf8, __builtin_bit_cast(u4v, qv[u][cb]) ^ sgn);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
        acc[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nq, pa[u][rb], acc[cb][rb], 0, 0, 0);
    }
  };
#pragma unroll
  for (int u = 0; u < PK_DEPTH; ++u) {
    load(u, min(ks0 + u, ks1 - 1));
    __builtin_amdgcn_sched_barrier(0);
  }
  const int rounds = (ks1 - ks0) / PK_DEPTH, rest = (ks1 - ks0) - rounds * PK_DEPTH;
  int ks = ks0;
  for (int g = 0; g < rounds; ++g, ks += PK_DEPTH) {
#pragma unroll
    for (int u = 0; u < PK_DEPTH; ++u) {
      step(u);
      load(u, min(ks + u + PK_DEPTH, ks1 - 1));
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  if constexpr (!WHOLE) {   // WHOLE: the caller guarantees rest == 0
#pragma unroll
    for (int u = 0; u < PK_DEPTH - 1; ++u)
      if (u < rest) step(u);
  }
}

// ---------------------------------------------------------------------------
// Diagonal block: A(k,k) = L L^T in FP64 and Winv(k) = L^-1, one workgroup of
// four waves per system, with the block held in LDS in FP64.  The block is
// factored blockwise in 16 x 16 sub-blocks (right-looking):
//   * a sub-block S_bb is factored by one wave as S_bb = U D^-1 U^T (U = the
//     columns of the successive Schur complements, D the pivots), so a column
//     step needs one reciprocal and no square root on its dependency chain;
//     the same wave carries the inverse of the unit factor U~ = U D^-1 along
//     (row operations applied to the identity), giving L_bb = U D^-1/2 and
//     L_bb^-1 = D^-1/2 U~^-1.  Lane 4 r + q holds S(r, 4 q + e), e < 4; the
//     column and inverse row of a step go through LDS inside the wave.
//   * the sub-blocks below follow on FP64 matrix cores: L_ib = S_ib L_bb^-T
//     and S_ij -= L_ib L_jb^T, formed by each wave that needs them.
//   * L^-1 below its diagonal sub-blocks, W_ij = -L_ii^-1 sum_{j<=q<i} L_iq W_qj,
//     is formed by the waves that are idle while wave 0 updates and factors the
//     next diagonal sub-block, as soon as its inputs are final.
// A pivot that is not positive (or NaN) marks the system failed with the
// LAPACK-style 1-based global column index of the first such pivot.
// ---------------------------------------------------------------------------
constexpr int DIAG_THREADS = 256;
constexpr int DIAG_PK_DEPTH = 4;   // fragment steps in flight in the fused column update
constexpr int DG_LD = NB + 1;      // padded LDS column (doubles)

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

// LDS of the diagonal block (66.7 KB, so that the column kernel that carries
// it keeps two workgroups per CU).  Sub-blocks (16 x 16) are addressed by
// their top-left element; S[c * DG_LD + r] is element (r, c).
//   S: the working matrix (successive Schur complements); a diagonal
//      sub-block of S is replaced by its factor L_bb once factored, and two
//      consumed sub-blocks park partial sums of the last block row of L^-1.
//   W: L^-1 in its lower sub-blocks; the factor's off-diagonal sub-blocks
//      L_ij (i > j) in the unused upper sub-block (j, i), untransposed
//      (element (r, c) of L_ij at W[(16 i + c) * DG_LD + 16 j + r]); before
//      all that, the FP32 partial sums of the fused column update.
struct DiagLds {
  double S[NB * DG_LD];
  double W[NB * DG_LD];
  double col[16];         // column j of the sub-block being factored (0 at and above the diagonal)
  double xrow[16];        // row j of its running inverse
  double zv[NB];          // right-hand side block of the fused forward solve
  int fail;
};

// Orders LDS traffic between the lanes of one wave: no compiler reordering
// across it, and every lane has reached it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Sub-block b (rows and columns [16 b, 16 b + 16)) by one wave: L_bb in
// place of S_bb, L_bb^-1 into sh.W.  Returns 0 or the 1-based local column of the
// first pivot that is not positive.
__device__ __forceinline__ int diag_sub(DiagLds& sh, int b, int lane) {
  const int r = lane >> 2, q = lane & 3, o = 16 * b;
  double a[4], x[4], dc[4], dr = 1.0;
  int fail = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    a[e] = sh.S[(o + 4 * q + e) * DG_LD + o + r];
    x[e] = (r == 4 * q + e) ? 1.0 : 0.0;
    dc[e] = 1.0;
  }
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int jq = j >> 2, je = j & 3;
    // publish column j of the Schur complement (below the pivot) and row j of the inverse
    if (q == jq) sh.col[r] = (r > j) ? a[je] : 0.0;
    if (r == j) {
#pragma unroll
      for (int e = 0; e < 4; ++e) sh.xrow[4 * q + e] = x[e];
    }
    wave_sync();
    const double2 c01 = *reinterpret_cast<const double2*>(&sh.col[4 * q]);
    const double2 c23 = *reinterpret_cast<const double2*>(&sh.col[4 * q + 2]);
    const double2 x01 = *reinterpret_cast<const double2*>(&sh.xrow[4 * q]);
    const double2 x23 = *reinterpret_cast<const double2*>(&sh.xrow[4 * q + 2]);
    const double cr = sh.col[r];
    const double d = read_lane(a[je], 4 * j + jq);   // pivot S(j, j)
    fail = (fail == 0 && !(d > 0.0)) ? j + 1 : fail;
    const double sr = cr * recip(d);                  // U~(r, j), 0 for r <= j
    a[0] = fma(-sr, c01.x, a[0]);
    a[1] = fma(-sr, c01.y, a[1]);
    a[2] = fma(-sr, c23.x, a[2]);
    a[3] = fma(-sr, c23.y, a[3]);
    x[0] = fma(-sr, x01.x, x[0]);
    x[1] = fma(-sr, x01.y, x[1]);
    x[2] = fma(-sr, x23.x, x[2]);
    x[3] = fma(-sr, x23.y, x[3]);
    if (q == jq) dc[je] = d;
    if (r == j) dr = d;
    wave_sync();
  }
  if (fail) return fail;
  const double rr = 1.0 / sqrt(dr);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int c = 4 * q + e;
    const double rc = 1.0 / sqrt(dc[e]);
    sh.S[(o + c) * DG_LD + o + r] = (r >= c) ? a[e] * rc : 0.0;
    sh.W[(o + c) * DG_LD + o + r] = (r >= c) ? x[e] * rr : 0.0;
  }
  return 0;
}

// The 16 x 16 products below leave lane l holding Z(kl + 4 v, il) of their
// result Z (il = l & 15, kl = l >> 4), which is also the operand layout of
// the right factor of a following product.
// L_ib (i > b) as L_bb^-1 S_ib^T: lane l holds L_ib(il, kl + 4 v)
__device__ __forceinline__ d4 sub_panel(const DiagLds& sh, int i, int b, int il, int kl) {
  d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int t = 16 * b + 4 * kk + kl;
    acc = mfma64(sh.W[t * DG_LD + 16 * b + il], sh.S[t * DG_LD + 16 * i + il], acc);
  }
  return acc;
}

// S_ij -= L_ib L_jb^T
__device__ __forceinline__ void sub_update(DiagLds& sh, int i, int j, const d4& Li, const d4& Lj, int il, int kl) {
  d4 acc;
#pragma unroll
  for (int v = 0; v < 4; ++v) acc[v] = sh.S[(16 * j + il) * DG_LD + 16 * i + kl + 4 * v];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) acc = mfma64(-Li[kk], Lj[kk], acc);
#pragma unroll
  for (int v = 0; v < 4; ++v) sh.S[(16 * j + il) * DG_LD + 16 * i + kl + 4 * v] = acc[v];
}

// L_ib into the upper sub-block (b, i) of W
__device__ __forceinline__ void store_panel(DiagLds& sh, int i, int b, const d4& Li, int il, int kl) {
#pragma unroll
  for (int v = 0; v < 4; ++v) sh.W[(16 * i + kl + 4 * v) * DG_LD + 16 * b + il] = Li[v];
}

// acc += s X Y for 16 x 16 blocks of LDS arrays (top-left corners (xr, xc), (yr, yc))
__device__ __forceinline__ d4 mm_ss(d4 acc, double s, const double* X, int xr, int xc, const double* Y, int yr, int yc,
                                    int il, int kl) {
#pragma unroll
  for (int kk = 0; kk < 4; ++kk)
    acc = mfma64(s * X[(xc + 4 * kk + kl) * DG_LD + xr + il], Y[(yc + il) * DG_LD + yr + 4 * kk + kl], acc);
  return acc;
}

// acc += s X Y with Y a product result held as described above
__device__ __forceinline__ d4 mm_sr(d4 acc, double s, const double* X, int xr, int xc, const d4& Y, int il, int kl) {
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) acc = mfma64(s * X[(xc + 4 * kk + kl) * DG_LD + xr + il], Y[kk], acc);
  return acc;
}

__device__ __forceinline__ void st_blk(double* P, int zr, int zc, const d4& Z, int il, int kl) {
#pragma unroll
  for (int v = 0; v < 4; ++v) P[(zc + il) * DG_LD + zr + kl + 4 * v] = Z[v];
}

__device__ __forceinline__ d4 ld_blk(const double* P, int zr, int zc, int il, int kl) {
  d4 z;
#pragma unroll
  for (int v = 0; v < 4; ++v) z[v] = P[(zc + il) * DG_LD + zr + kl + 4 * v];
  return z;
}

__device__ __forceinline__ void load4(const float* p, double (&v)[4]) {
  const float4 f = *reinterpret_cast<const float4*>(p);
  v[0] = f.x;
  v[1] = f.y;
  v[2] = f.z;
  v[3] = f.w;
}
__device__ __forceinline__ void load4(const double* p, double (&v)[4]) {
  const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
  v[0] = a.x;
  v[1] = a.y;
  v[2] = b.x;
  v[3] = b.y;
}
__device__ __forceinline__ void store4(float* p, const double (&v)[4]) {
  *reinterpret_cast<float4*>(p) = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
}
__device__ __forceinline__ void store4(double* p, const double (&v)[4]) {
  reinterpret_cast<double2*>(p)[0] = make_double2(v[0], v[1]);
  reinterpret_cast<double2*>(p)[1] = make_double2(v[2], v[3]);
}

// With a BF16 panel pack (Pk != null, FP32 storage) and k > K0, the block
// first receives its column update A(k,k) -= sum_{q in [K0,k)} L(k,q) L(k,q)^T
// from the packed fragments (waves: two column halves x two halves of the
// fragment steps, summed in LDS).  Wpk (nullable): Winv(k) is also written as
// BF16 high/low operand fragments for the BF16 panel solve (see k_panel_col).
// The diagonal block k of system s by the DIAG_THREADS threads of a
// workgroup (thread t); D = desc[s], already checked to be factored in this
// pass with k < D.T.
// zf (nullable, FP64 vectors at D.v_off): forward solve carried along the
// factorisation; on entry block k holds b_k - sum_{j<k} L(k,j) z_j, and it
// is replaced by z_k = L(k,k)^-1 (that).
template <typename TS>
__device__ __forceinline__ void diag_block(const SysDesc& D, int s, SysStatus* __restrict__ st, TS* __restrict__ A,
                                           TS* __restrict__ Wt, int k, const __bf16* __restrict__ Pk, int K0, int Wp, int wps,
                                           __bf16* __restrict__ Wpk, double* __restrict__ zf, DiagLds& sh, int t) {
  TS* tile = A + D.a_off + tile_index(k, k) * TILE;
  const int lane = t & 63, w = t >> 6;
  const int il = lane & 15, kl = lane >> 4;
  const bool fused = std::is_same<TS, float>::value && Pk != nullptr && k > K0;
  if (fused) {
    const int ch = w & 1, kh = w >> 1, half = k - K0;
    f4 acc[2][4];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          acc[cb][rb][v] = kh ? 0.f : (float)tile[(16 * (2 * ch + cb) + 4 * kl + v) * NB + 16 * rb + il];
    packed_sub<2, DIAG_PK_DEPTH>(acc, Pk + D.pk_off + lane * 8, half * 4, half * 4 + 2 * ch, 2 * Wp, kh * half,
                                 (kh + 1) * half);
    float* part = reinterpret_cast<float*>(sh.W);
    if (kh) {
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int v = 0; v < 4; ++v) part[(16 * (2 * ch + cb) + 4 * kl + v) * NB + 16 * rb + il] = acc[cb][rb][v];
    }
    __syncthreads();
    if (!kh) {
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int c = 16 * (2 * ch + cb) + 4 * kl + v, r = 16 * rb + il;
            sh.S[c * DG_LD + r] = (double)(acc[cb][rb][v] + part[c * NB + r]);
          }
    }
  } else {
    double v[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) load4(tile + 4 * (t + DIAG_THREADS * i), v[i]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = 4 * (t + DIAG_THREADS * i), c = e >> 6, r = e & 63;
#pragma unroll
      for (int u = 0; u < 4; ++u) sh.S[c * DG_LD + r + u] = v[i][u];
    }
  }
  if (t == 0) sh.fail = 0;
  __syncthreads();
  if (w == 0) {
    const int f = diag_sub(sh, 0, lane);
    if (f && lane == 0) sh.fail = f;
  }
  __syncthreads();
  // Block steps b = 0, 1, 2: wave 0 updates diagonal sub-block b + 1 and
  // factors it at once; the other waves update the rest of the trailing
  // sub-blocks and form the blocks of L^-1 whose inputs are final.
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    if (sh.fail) break;
    const d4 z = {0.0, 0.0, 0.0, 0.0};
    if (w == 0) {
      const d4 Ln = sub_panel(sh, b + 1, b, il, kl);
      sub_update(sh, b + 1, b + 1, Ln, Ln, il, kl);
      store_panel(sh, b + 1, b, Ln, il, kl);
      wave_sync();
      const int f = diag_sub(sh, b + 1, lane);
      if (f && lane == 0) sh.fail = 16 * (b + 1) + f;
    } else if (b == 0) {
      if (w == 1) {
        const d4 L2 = sub_panel(sh, 2, 0, il, kl), L1 = sub_panel(sh, 1, 0, il, kl);
        sub_update(sh, 2, 2, L2, L2, il, kl);
        sub_update(sh, 2, 1, L2, L1, il, kl);
        store_panel(sh, 2, 0, L2, il, kl);
      } else if (w == 2) {
        const d4 L3 = sub_panel(sh, 3, 0, il, kl), L1 = sub_panel(sh, 1, 0, il, kl);
        sub_update(sh, 3, 3, L3, L3, il, kl);
        sub_update(sh, 3, 1, L3, L1, il, kl);
        store_panel(sh, 3, 0, L3, il, kl);
      } else {
        const d4 L3 = sub_panel(sh, 3, 0, il, kl), L2 = sub_panel(sh, 2, 0, il, kl);
        sub_update(sh, 3, 2, L3, L2, il, kl);
      }
    } else if (b == 1) {
      if (w == 1) {
        const d4 L3 = sub_panel(sh, 3, 1, il, kl), L2 = sub_panel(sh, 2, 1, il, kl);
        sub_update(sh, 3, 2, L3, L2, il, kl);
      } else if (w == 2) {
        const d4 L3 = sub_panel(sh, 3, 1, il, kl);
        sub_update(sh, 3, 3, L3, L3, il, kl);
        store_panel(sh, 3, 1, L3, il, kl);
      } else {
        const d4 y = mm_ss(z, 1.0, sh.W, 0, 16, sh.W, 0, 0, il, kl);            // L_10 W_00
        st_blk(sh.W, 16, 0, mm_sr(z, -1.0, sh.W, 16, 16, y, il, kl), il, kl);   // W_10
      }
    } else {
      if (w == 1) {
        const d4 y = mm_ss(z, 1.0, sh.W, 16, 32, sh.W, 16, 16, il, kl);         // L_21 W_11
        st_blk(sh.W, 32, 16, mm_sr(z, -1.0, sh.W, 32, 32, y, il, kl), il, kl);  // W_21
      } else if (w == 2) {
        d4 y = mm_ss(z, 1.0, sh.W, 0, 32, sh.W, 0, 0, il, kl);                  // L_20 W_00
        y = mm_ss(y, 1.0, sh.W, 16, 32, sh.W, 16, 0, il, kl);                   //  + L_21 W_10
        st_blk(sh.W, 32, 0, mm_sr(z, -1.0, sh.W, 32, 32, y, il, kl), il, kl);   // W_20
      } else {
        // the terms of the last block row that do not involve block 2, parked
        // in the consumed sub-blocks (1, 0) and (2, 0) of S
        d4 y = mm_ss(z, 1.0, sh.W, 0, 48, sh.W, 0, 0, il, kl);                  // L_30 W_00
        y = mm_ss(y, 1.0, sh.W, 16, 48, sh.W, 16, 0, il, kl);                   //  + L_31 W_10
        st_blk(sh.S, 16, 0, y, il, kl);
        st_blk(sh.S, 32, 0, mm_ss(z, 1.0, sh.W, 16, 48, sh.W, 16, 16, il, kl), il, kl);   // L_31 W_11
      }
    }
    __syncthreads();
  }
  if (sh.fail) {
    if (t == 0) {
      st[s].status = KRR_ENOTSPD;
      st[s].failed_pivot = k * NB + sh.fail;
    }
    return;
  }
  if (w < 3) {
    // last block row, column block jb: W_3jb = -L_33^-1 (parked terms + L_32 W_2jb)
    const d4 z = {0.0, 0.0, 0.0, 0.0};
    const int jb = 2 - w;
    const d4 y0 = (w == 0) ? z : ld_blk(sh.S, 16 * (jb + 1), 0, il, kl);
    const d4 y = mm_ss(y0, 1.0, sh.W, 32, 48, sh.W, 32, 16 * jb, il, kl);
    st_blk(sh.W, 48, 16 * jb, mm_sr(z, -1.0, sh.W, 48, 48, y, il, kl), il, kl);
  }
  if (zf != nullptr && t < NB) sh.zv[t] = zf[D.v_off + (int64_t)k * NB + t];
  __syncthreads();
  if (zf != nullptr) {
    // z_k(r) = sum_{c <= r} L^-1(r, c) b(c): four threads per row, 16 columns each
    const int r = t >> 2, q = t & 3;
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int c = 16 * q + u;
      const double w0 = sh.W[c * DG_LD + r];   // unconditional load; the upper part holds L
      acc = fma(c <= r ? w0 : 0.0, sh.zv[c], acc);
    }
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    if (q == 0) zf[D.v_off + (int64_t)k * NB + r] = acc;
  }
  // L into the tile, L^-1 into Wt (zero above the diagonal)
  TS* wt = Wt + D.w_off + (int64_t)k * TILE;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int e = 4 * (t + DIAG_THREADS * i), c = e >> 6, r = e & 63;
    double lv[4], wv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int rr = r + u, bi = rr >> 4, bj = c >> 4;
      // unconditional loads: diagonal sub-blocks of L from S, the others from the upper part of W
      const double ld = sh.S[c * DG_LD + rr];
      const double lo = sh.W[(16 * bi + (c & 15)) * DG_LD + 16 * bj + (rr & 15)];
      const double w0 = sh.W[c * DG_LD + rr];
      lv[u] = bi > bj ? lo : (bi == bj ? ld : 0.0);
      wv[u] = (bi > bj || (bi == bj && rr >= c)) ? w0 : 0.0;
    }
    store4(tile + e, lv);
    store4(wt + e, wv);
  }
  if (Wpk != nullptr) {
    // fragment f = 2 cb + ks, part hl (0 high, 1 low): lane l holds Winv(16 cb + (l & 15), 32 ks + 8 (l >> 4) + e)
    // split from its FP32 value: hi = bf16(w), lo = bf16(w - hi)
    __bf16* base = Wpk + ((int64_t)s * wps + (k - K0)) * 16 * FRAG;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int task = t + DIAG_THREADS * it;
      const int f = task >> 6, l = task & 63;
      const int cb = f >> 1, ks = f & 1;
      const int row = 16 * cb + (l & 15);
      bf8 hi, lo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int col = 32 * ks + 8 * (l >> 4) + e;
        const double w0 = sh.W[col * DG_LD + row];
        const float wv = (row >= col) ? (float)w0 : 0.f;
        const __bf16 h = (__bf16)wv;
        hi[e] = h;
        lo[e] = (__bf16)(wv - (float)h);
      }
      *reinterpret_cast<bf8*>(base + (int64_t)(2 * f) * FRAG + l * 8) = hi;
      *reinterpret_cast<bf8*>(base + (int64_t)(2 * f + 1) * FRAG + l * 8) = lo;
    }
  }
}

template <typename TS>
__global__ __launch_bounds__(DIAG_THREADS) void k_potrf_diag(const SysDesc* __restrict__ desc,
                                                             SysStatus* __restrict__ st, TS* __restrict__ A,
                                                             TS* __restrict__ Wt, int k, int level,
                                                             const __bf16* __restrict__ Pk, int K0, int Wp,
                                                             __bf16* __restrict__ Wpk, double* __restrict__ zf) {
  const int s = blockIdx.x;
  const SysDesc D = desc[s];
  const int status = st[s].status;
  if (k >= D.T || status != 0 || D.level != level) return;
  __shared__ __align__(16) DiagLds sh;
  diag_block<TS>(D, s, st, A, Wt, k, Pk, K0, Wp, Wp, Wpk, zf, sh, threadIdx.x);
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

// One output tile (i, j) of a k_tile_gemm launch (see above), by the 256
// threads of a workgroup.
template <typename TS, int MODE>
__device__ __forceinline__ void tile_gemm_body(const SysDesc& D, TS* __restrict__ A, const TS* __restrict__ Wt,
                                               int i, int j, int jc, int q0, int q1) {
  typedef typename AccT<TS>::type acc_t;
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

template <typename TS, int MODE>
__global__ __launch_bounds__(256) void k_tile_gemm(const SysDesc* __restrict__ desc,
                                                   const SysStatus* __restrict__ st, TS* __restrict__ A,
                                                   const TS* __restrict__ Wt, int i0, int jc, int q0, int q1,
                                                   int level) {
  const int s = blockIdx.y;
  const SysDesc D = desc[s];
  if (st[s].status != 0 || D.level != level) return;
  int i, j;
  if (!locate(MODE, blockIdx.x, i0, jc, D.T, i, j)) return;
  tile_gemm_body<TS, MODE>(D, A, Wt, i, j, jc, q0, q1);
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
// Workgroups go to the chip's 8 XCDs in turn (workgroup b to XCD b % 8), and
// each XCD has its own L2.  The update kernels place all workgroups of
// system s on XCD s % 8 (slot b / 8 of that XCD), so that the operands a
// system's workgroups share are fetched into one L2.  Grids hold
// 8 * ceil(n_sys / 8) * (workgroups per system); the padding exits at once.
// A batch of fewer than 8 systems would leave XCDs idle that way, and so
// would a ragged batch whose largest systems hold most of the work (one XCD
// each): those launches ("spread") keep the plain order, a system's
// workgroups spread over all XCDs.
constexpr int NXCD = 8;

// Winv(k) as BF16 high/low operand fragments (cb, ks) of the panel solve;
// the blocks above Winv's diagonal (cb < 2, ks = 1) are zero and not loaded.
struct WinvFrags {
  bf8 hi[4][2], lo[4][2];
};

__device__ __forceinline__ void load_winv(const __bf16* __restrict__ Wpk, int s, int wps, int K0, int k, int lane,
                                          WinvFrags& W) {
  const __bf16* Wf = Wpk + ((int64_t)s * wps + (k - K0)) * 16 * FRAG + lane * 8;
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
      if (ks == 0 || cb >= 2) {
        W.hi[cb][ks] = *reinterpret_cast<const bf8*>(Wf + (int64_t)(2 * (2 * cb + ks)) * FRAG);
        W.lo[cb][ks] = *reinterpret_cast<const bf8*>(Wf + (int64_t)(2 * (2 * cb + ks) + 1) * FRAG);
      }
}

// element (16 cb + 4 kg + v, 16 rb + il) of the tile C: a scalar base per
// column block cb, one per-lane offset lo = 4 kg NB + il, the rest immediate
__device__ __forceinline__ void load_ctile(const float* __restrict__ C, int lo, f4 (&acc)[4][4]) {
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const float* Cc = C + 16 * cb * NB;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[cb][rb][v] = Cc[lo + v * NB + 16 * rb];
  }
}

__device__ __forceinline__ void store_ctile(float* __restrict__ C, int lo, const f4 (&acc)[4][4]) {
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    float* Cc = C + 16 * cb * NB;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) Cc[lo + v * NB + 16 * rb] = acc[cb][rb][v];
  }
}

__device__ __forceinline__ void lds_wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The panel solve of tile (i, k) from its updated value in acc:
// L(i,k) = C(i,k) Winv(k)^T into the FP32 tile C and the wave's LDS tile sc
// (left there for the caller), and (do_pack) BF16 fragments of the pack;
// zf: b_i -= L(i,k) z_k.
__device__ __forceinline__ void tile_solve(const SysDesc& D, int i, int lane, float* __restrict__ C, int lo,
                                           const WinvFrags& W, __bf16* __restrict__ Pk, int K0, int k, int KSW,
                                           int do_pack, double* __restrict__ zf, float* __restrict__ sc,
                                           const f4 (&acc)[4][4]) {
  const int il = lane & 15, kg = lane >> 4;
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) sc[(16 * cb + 4 * kg + v) * PC_LD + 16 * rb + il] = acc[cb][rb][v];
  lds_wave_fence();
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
        o[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.lo[cb][ks], chi, o[cb][rb], 0, 0, 0);
        o[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.hi[cb][ks], clo, o[cb][rb], 0, 0, 0);
        o[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.hi[cb][ks], chi, o[cb][rb], 0, 0, 0);
      }
    }
  lds_wave_fence();
  // MFMA result: register v of a lane is column 4 (lane >> 4) + v, row lane & 15 of its 16 x 16 block
  int lo2;   // the offset recomputed here, not held in registers across the products
  asm volatile("" : "=v"(lo2) : "0"(lo));
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    float* Cc = C + 16 * cb * NB;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = 16 * cb + 4 * kg + v, r = 16 * rb + il;
        Cc[lo2 + v * NB + 16 * rb] = o[cb][rb][v];
        sc[c * PC_LD + r] = o[cb][rb][v];
      }
  }
  if (zf != nullptr) {
    // forward solve: b_i -= L(i,k) z_k (FP64 sums of the stored FP32 factor)
    const double* zk = zf + D.v_off + (int64_t)k * NB;
    double zc[4][4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) zc[cb][v] = zk[16 * cb + 4 * kg + v];
    double pr[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      double a = 0.0;
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) a = fma((double)o[cb][rb][v], zc[cb][v], a);
      a += __shfl_xor(a, 16, 64);
      a += __shfl_xor(a, 32, 64);
      pr[rb] = a;
    }
    if (kg == 0) {
      double* bi = zf + D.v_off + (int64_t)i * NB;
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) bi[16 * rb + il] -= pr[rb];
    }
  }
  if (!do_pack) return;
  lds_wave_fence();
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

__device__ __forceinline__ void panel_col_tile(const SysDesc& D, int s, int i, int lane, float* __restrict__ A,
                                               const __bf16* __restrict__ Wpk, __bf16* __restrict__ Pk, int K0, int k,
                                               int Wp, int wps, int do_pack, double* __restrict__ zf,
                                               float* __restrict__ sc) {
  const int KSW = 2 * Wp;
  // Winv(k) fragments first: their latency overlaps the column update
  WinvFrags W;
  load_winv(Wpk, s, wps, K0, k, lane, W);
  float* C = A + D.a_off + tile_index(i, k) * TILE;
  const int lo = 4 * (lane >> 4) * NB + (lane & 15);
  f4 acc[4][4];
  load_ctile(C, lo, acc);
  if (k > K0) packed_sub<4, 2, true>(acc, Pk + D.pk_off + lane * 8, (i - K0) * 4, (k - K0) * 4, KSW, 0, 2 * (k - K0));
  tile_solve(D, i, lane, C, lo, W, Pk, K0, k, KSW, do_pack, zf, sc, acc);
}

// acc0 -= sum_{ks in [ks0, ks1)} P(rbj0 + cb, ks) P(rbi + rb, ks)^T and acc1
// the same with rbj1: one pass over the row fragments (rbi) for two panel
// columns.  Each accumulator takes exactly the MFMAs packed_sub would give
// it, in the same order; (ks1 - ks0) is a multiple of PK_DEPTH.
template <int PK_DEPTH>
__device__ __forceinline__ void packed_sub2(f4 (&acc0)[4][4], f4 (&acc1)[4][4], const __bf16* __restrict__ P,
                                            int rbi, int rbj0, int rbj1, int KSW, int ks0, int ks1) {
  if (ks0 >= ks1) return;
  typedef unsigned u4v __attribute__((ext_vector_type(4)));
  const u4v sgn{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  bf8 pa[PK_DEPTH][4], q0[PK_DEPTH][4], q1[PK_DEPTH][4];
  auto load = [&](int u, int ks) {
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
      pa[u][rb] = *reinterpret_cast<const bf8*>(P + ((int64_t)(rbi + rb) * KSW + ks) * FRAG);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      q0[u][cb] = *reinterpret_cast<const bf8*>(P + ((int64_t)(rbj0 + cb) * KSW + ks) * FRAG);
      q1[u][cb] = *reinterpret_cast<const bf8*>(P + ((int64_t)(rbj1 + cb) * KSW + ks) * FRAG);
    }
  };
  auto step = [&](int u) {
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const bf8 n0 = __builtin_bit_cast(bf8, __builtin_bit_cast(u4v, q0[u][cb]) ^ sgn);
      const bf8 n1 = __builtin_bit_cast(bf8, __builtin_bit_cast(u4v, q1[u][cb]) ^ sgn);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        acc0[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(n0, pa[u][rb], acc0[cb][rb], 0, 0, 0);
        acc1[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(n1, pa[u][rb], acc1[cb][rb], 0, 0, 0);
      }
    }
  };
#pragma unroll
  for (int u = 0; u < PK_DEPTH; ++u) {
    load(u, min(ks0 + u, ks1 - 1));
    __builtin_amdgcn_sched_barrier(0);
  }
  for (int ks = ks0; ks < ks1; ks += PK_DEPTH) {
#pragma unroll
    for (int u = 0; u < PK_DEPTH; ++u) {
      step(u);
      load(u, min(ks + u + PK_DEPTH, ks1 - 1));
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// Tile row i of columns c and c + 1 of the panel in one pass over the row's
// fragments: both columns' updates over the panel columns [K0, c), the
// panel solve of column c, then column c + 1's last term L(i,c) L(c+1,c)^T
// (operands: BF16 of L(i,c) from the wave's LDS, equal to what the pack
// holds, and L(c+1,c) from the pack) and its panel solve.  Results equal
// two single-column passes bit for bit.  Column c is always packed (column
// c + 1 reads it); pack1 for column c + 1.
__device__ __forceinline__ void pair_tile(const SysDesc& D, int s, int i, int lane, float* __restrict__ A,
                                          const __bf16* __restrict__ Wpk, __bf16* __restrict__ Pk, int K0, int c,
                                          int Wp, int wps, int pack1, double* __restrict__ zf, float* __restrict__ sc) {
  const int KSW = 2 * Wp, il = lane & 15, kg = lane >> 4;
  WinvFrags W;
  load_winv(Wpk, s, wps, K0, c, lane, W);
  float* C0 = A + D.a_off + tile_index(i, c) * TILE;
  float* C1 = C0 + TILE;   // tile (i, c + 1)
  const int lo = 4 * kg * NB + il;
  f4 acc0[4][4], acc1[4][4];
  load_ctile(C0, lo, acc0);
  load_ctile(C1, lo, acc1);
  const __bf16* P = Pk + D.pk_off + lane * 8;
  const int rbi = (i - K0) * 4, rbj = (c - K0) * 4;
  packed_sub2<1>(acc0, acc1, P, rbi, rbj, rbj + 4, KSW, 0, 2 * (c - K0));
  tile_solve(D, i, lane, C0, lo, W, Pk, K0, c, KSW, 1, zf, sc, acc0);
  lds_wave_fence();
  {
    typedef unsigned u4v __attribute__((ext_vector_type(4)));
    const u4v sgn{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int ks = 2 * (c - K0) + h, cl = 32 * h + 8 * kg;
      bf8 pa[4], qv[4];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) qv[cb] = *reinterpret_cast<const bf8*>(P + ((int64_t)(rbj + 4 + cb) * KSW + ks) * FRAG);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int e = 0; e < 8; ++e) pa[rb][e] = (__bf16)sc[(cl + e) * PC_LD + 16 * rb + il];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const bf8 nq = __builtin_bit_cast(bf8, __builtin_bit_cast(u4v, qv[cb]) ^ sgn);
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
          acc1[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nq, pa[rb], acc1[cb][rb], 0, 0, 0);
      }
    }
  }
  lds_wave_fence();
  load_winv(Wpk, s, wps, K0, c + 1, lane, W);
  tile_solve(D, i, lane, C1, lo, W, Pk, K0, c + 1, KSW, pack1, zf, sc, acc1);
}

union PcolLds {
  float sC[4][NB * PC_LD];   // per wave: the tile being solved
  DiagLds dg;
};

// Tile-row group g of column k (rows k + 1 + 4 g + w, one per wave w), then
// for diag_next and g = 0 the diagonal block k + 1 (see k_panel_col).
__device__ __forceinline__ void pcol_body(const SysDesc& D, int s, SysStatus* __restrict__ st, float* __restrict__ A,
                                          float* __restrict__ Wt, __bf16* __restrict__ Wpk, __bf16* __restrict__ Pk,
                                          int K0, int k, int Wp, int wps, int do_pack, int diag_next, int g,
                                          double* __restrict__ zf, PcolLds& lds) {
  // wave-uniform wave index: the tile bases stay in scalar registers
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int i = k + 1 + 4 * g + w;
  if (i < D.T) panel_col_tile(D, s, i, lane, A, Wpk, Pk, K0, k, Wp, wps, do_pack, zf, lds.sC[w]);
  if (diag_next && g == 0 && k + 1 < D.T) {
    __syncthreads();   // tile row k + 1 (factor and pack) complete; LDS free
    diag_block<float>(D, s, st, A, Wt, k + 1, Pk, K0, Wp, wps, Wpk, zf, lds.dg, threadIdx.x);
  }
}

// diag_next: the first workgroup of each system (tile rows k+1 .. k+4,
// dispatched before the other workgroups) then factors diagonal block k + 1
// with its column update over the panel columns [K0, k] (diag_block), which
// needs only tile row k + 1 of this column; its latency hides behind the
// other workgroups' tiles.  ng = tile groups of four rows per system; on
// each XCD the slots hold first group 0 of its U = ceil(n_sys / 8) systems,
// then the other groups system by system.
__global__ __launch_bounds__(256) void k_panel_col(const SysDesc* __restrict__ desc, SysStatus* __restrict__ st,
                                                   float* __restrict__ A, float* __restrict__ Wt,
                                                   __bf16* __restrict__ Wpk, __bf16* __restrict__ Pk, int K0, int k,
                                                   int Wp, int level, int do_pack, int diag_next, int n_sys, int ng,
                                                   double* __restrict__ zf, int spread) {
  int s, g;
  if (spread) {
    // workgroups in turn over all XCDs (group 0 of every system first)
    if ((int)blockIdx.x >= n_sys * ng) return;
    g = blockIdx.x / n_sys;
    s = blockIdx.x % n_sys;
  } else {
    const int xcd = blockIdx.x % NXCD, slot = blockIdx.x / NXCD, U = (n_sys + NXCD - 1) / NXCD;
    int u;
    if (slot < U) {
      u = slot;
      g = 0;
    } else {
      u = (slot - U) / (ng - 1);
      g = 1 + (slot - U) % (ng - 1);
    }
    s = xcd + NXCD * u;
    if (s >= n_sys) return;
  }
  const SysDesc D = desc[s];
  if (st[s].status != 0 || D.level != level) return;
  __shared__ __align__(16) PcolLds lds;
  pcol_body(D, s, st, A, Wt, Wpk, Pk, K0, k, Wp, Wp, do_pack, diag_next, g, zf, lds);
}

// Rows c + 2 (waves 0, 1) and c + 3 (waves 2, 3) of columns c and c + 1 for
// the chain workgroup of a column-pair launch, each row split over two waves
// by column-block halves (wave parity hf: column blocks 2 hf and 2 hf + 1 of
// the tiles), the row's tile shared through its LDS tile.  With `park`, row
// c + 3's waves also sum tile (c+3, c+2)'s update over the panel columns
// before c and leave it in the FP32 tile.  Every element takes the
// operations of pair_tile in the same order (its MFMAs; the forward-solve sum
// over the whole tile, read back from LDS, by one wave), so the results are
// the same bit for bit.  All four waves pass the same barriers.
__device__ __forceinline__ void chain_rows(const SysDesc& D, int s, int w, int lane, float* __restrict__ A,
                                           const __bf16* __restrict__ Wpk, __bf16* __restrict__ Pk, int K0, int c,
                                           int Wp, int wps, int pack1, bool park, double* __restrict__ zf,
                                           PcolLds& lds) {
  typedef unsigned u4v __attribute__((ext_vector_type(4)));
  const u4v sgn{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  const int ri = w >> 1, hf = w & 1, i = c + 2 + ri;
  const bool valid = i < D.T, dopark = valid && park && ri == 1;
  const int KSW = 2 * Wp, il = lane & 15, kg = lane >> 4, lo = 4 * kg * NB + il;
  float* sc = lds.sC[ri];
  float* C0 = A + D.a_off + tile_index(valid ? i : c + 1, c) * TILE;   // (c+1, c) stands in when row i is absent
  float* C1 = C0 + TILE;
  float* CP = A + D.a_off + tile_index(c + 3, c + 2) * TILE;
  const __bf16* P = Pk + D.pk_off + lane * 8;
  const int rbi = (i - K0) * 4, rbj = (c - K0) * 4, rbp = (c + 2 - K0) * 4;
  f4 a0[2][4], a1[2][4], ap[2][4];
  auto load_half = [&](const float* C, f4 (&acc)[2][4]) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const float* Cc = C + 16 * (2 * hf + u) * NB;
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][rb][v] = Cc[lo + v * NB + 16 * rb];
    }
  };
  if (valid) {
    load_half(C0, a0);
    load_half(C1, a1);
    if (dopark) load_half(CP, ap);
    // the update over the panel columns before c: row i's fragments once for
    // both columns (and the parked tile), each accumulator's steps in order;
    // a two-step operand ring (the step count is even) keeps the next step's
    // loads in flight during a step's products, the refill past the end
    // re-reading the last step
    const int nks = 2 * (c - K0);
    bf8 pa[2][4], q0[2][2], q1[2][2], qp[2][2];
    auto load = [&](int b, int ks) {
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
        pa[b][rb] = *reinterpret_cast<const bf8*>(P + ((int64_t)(rbi + rb) * KSW + ks) * FRAG);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int cb = 2 * hf + u;
        q0[b][u] = *reinterpret_cast<const bf8*>(P + ((int64_t)(rbj + cb) * KSW + ks) * FRAG);
        q1[b][u] = *reinterpret_cast<const bf8*>(P + ((int64_t)(rbj + 4 + cb) * KSW + ks) * FRAG);
        if (dopark) qp[b][u] = *reinterpret_cast<const bf8*>(P + ((int64_t)(rbp + cb) * KSW + ks) * FRAG);
      }
    };
    auto step = [&](int b) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const bf8 n0 = __builtin_bit_cast(bf8, __builtin_bit_cast(u4v, q0[b][u]) ^ sgn);
        const bf8 n1 = __builtin_bit_cast(bf8, __builtin_bit_cast(u4v, q1[b][u]) ^ sgn);
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
          a0[u][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(n0, pa[b][rb], a0[u][rb], 0, 0, 0);
          a1[u][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(n1, pa[b][rb], a1[u][rb], 0, 0, 0);
        }
        if (dopark) {
          const bf8 np = __builtin_bit_cast(bf8, __builtin_bit_cast(u4v, qp[b][u]) ^ sgn);
#pragma unroll
          for (int rb = 0; rb < 4; ++rb)
            ap[u][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(np, pa[b][rb], ap[u][rb], 0, 0, 0);
        }
      }
    };
    if (nks > 0) {
      load(0, 0);
      __builtin_amdgcn_sched_barrier(0);
      for (int ks = 0; ks < nks; ks += 2) {
        load(1, ks + 1);
        __builtin_amdgcn_sched_barrier(0);
        step(0);
        load(0, min(ks + 2, nks - 1));
        __builtin_amdgcn_sched_barrier(0);
        step(1);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (dopark) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        float* Cc = CP + 16 * (2 * hf + u) * NB;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int v = 0; v < 4; ++v) Cc[lo + v * NB + 16 * rb] = ap[u][rb][v];
      }
    }
  }
  // the panel solve of column k (acc: this wave's column blocks of the
  // updated tile): the tile in LDS, then out(r, c') = sum_{t <= c'} C(r, t)
  // Winv(c', t) for this wave's column blocks (tile_solve's products), L to
  // the tile and LDS, the forward-solve update of row i by wave hf = 0, and
  // this wave's half of the BF16 pack
  auto solve_half = [&](int k, float* C, f4 (&acc)[2][4], int do_pack) {
    if (valid) {
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int v = 0; v < 4; ++v) sc[(16 * (2 * hf + u) + 4 * kg + v) * PC_LD + 16 * rb + il] = acc[u][rb][v];
    }
    __syncthreads();
    f4 o[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) o[u][rb] = f4{0.f, 0.f, 0.f, 0.f};
    if (valid) {
      // Winv(k) fragments of this wave's column blocks (blocks 0, 1 take only ks = 0)
      const __bf16* Wf = Wpk + ((int64_t)s * wps + (k - K0)) * 16 * FRAG + lane * 8;
      bf8 whi[2][2], wlo[2][2];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
          if (ks <= hf) {
            const int cb = 2 * hf + u;
            whi[u][ks] = *reinterpret_cast<const bf8*>(Wf + (int64_t)(2 * (2 * cb + ks)) * FRAG);
            wlo[u][ks] = *reinterpret_cast<const bf8*>(Wf + (int64_t)(2 * (2 * cb + ks) + 1) * FRAG);
          }
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          if (ks > hf) continue;
          bf8 chi, clo;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const float cv = sc[(32 * ks + 8 * kg + e) * PC_LD + 16 * rb + il];
            const __bf16 h = (__bf16)cv;
            chi[e] = h;
            clo[e] = (__bf16)(cv - (float)h);
          }
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            o[u][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wlo[u][ks], chi, o[u][rb], 0, 0, 0);
            o[u][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(whi[u][ks], clo, o[u][rb], 0, 0, 0);
            o[u][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(whi[u][ks], chi, o[u][rb], 0, 0, 0);
          }
        }
    }
    __syncthreads();   // every read of the updated tile is done
    if (valid) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int cb = 2 * hf + u;
        float* Cc = C + 16 * cb * NB;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            Cc[lo + v * NB + 16 * rb] = o[u][rb][v];
            sc[(16 * cb + 4 * kg + v) * PC_LD + 16 * rb + il] = o[u][rb][v];
          }
      }
    }
    __syncthreads();
    if (valid && zf != nullptr && hf == 0) {
      const double* zk = zf + D.v_off + (int64_t)k * NB;
      double pr[4];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        double a = 0.0;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            a = fma((double)sc[(16 * cb + 4 * kg + v) * PC_LD + 16 * rb + il], zk[16 * cb + 4 * kg + v], a);
        a += __shfl_xor(a, 16, 64);
        a += __shfl_xor(a, 32, 64);
        pr[rb] = a;
      }
      if (kg == 0) {
        double* bi = zf + D.v_off + (int64_t)i * NB;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) bi[16 * rb + il] -= pr[rb];
      }
    }
    if (valid && do_pack) {
      __bf16* Pout = Pk + D.pk_off + lane * 8;
#pragma unroll
      for (int rbl = 0; rbl < 4; ++rbl) {
        const int r = 16 * rbl + il, cl = 32 * hf + 8 * kg;
        bf8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (__bf16)sc[(cl + e) * PC_LD + r];
        *reinterpret_cast<bf8*>(Pout + ((int64_t)(rbi + rbl) * KSW + 2 * (k - K0) + hf) * FRAG) = v;
      }
    }
  };
  solve_half(c, C0, a0, 1);
  // column c + 1's last term L(i,c) L(c+1,c)^T: BF16 of L(i,c) from LDS (what
  // the pack holds) and row c + 1's fragments of column c from the pack
  if (valid) {
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2) {
      const int ks = 2 * (c - K0) + h2, cl = 32 * h2 + 8 * kg;
      bf8 pa[4], qv[2];
#pragma unroll
      for (int u = 0; u < 2; ++u)
        qv[u] = *reinterpret_cast<const bf8*>(P + ((int64_t)(rbj + 4 + 2 * hf + u) * KSW + ks) * FRAG);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int e = 0; e < 8; ++e) pa[rb][e] = (__bf16)sc[(cl + e) * PC_LD + 16 * rb + il];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const bf8 nq = __builtin_bit_cast(bf8, __builtin_bit_cast(u4v, qv[u]) ^ sgn);
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
          a1[u][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nq, pa[rb], a1[u][rb], 0, 0, 0);
      }
    }
  }
  __syncthreads();   // L(i,c) read from LDS by both waves of the row
  solve_half(c + 1, C1, a1, pack1);
}

// Tile (i, k) of the diagonal chain (i = k + 1) once diagonal block k is
// factored, by the four waves of the workgroup, wave w owning column block w:
// the last NUPD fragment steps of its update (tile (c+3, c+2) of a column
// pair: panel columns c and c + 1, its earlier columns already summed in the
// FP32 tile; a panel head's tile (K0+1, K0): none), its panel solve, the
// forward-solve update of row i (wave 0, from LDS) and the pack.  Every
// element takes the operations of panel_col_tile in the same order.
template <int NUPD>
__device__ __forceinline__ void chain_tile(const SysDesc& D, int s, int w, int lane, float* __restrict__ C,
                                           const __bf16* __restrict__ Wpk, __bf16* __restrict__ Pk, int K0, int k,
                                           int Wp, int wps, double* __restrict__ zf, float* __restrict__ sc) {
  typedef unsigned u4v __attribute__((ext_vector_type(4)));
  const u4v sgn{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  const int KSW = 2 * Wp, il = lane & 15, kg = lane >> 4, lo = 4 * kg * NB + il;
  const int i = k + 1, cb = w;
  const __bf16* P = Pk + D.pk_off + lane * 8;
  const int rbi = (i - K0) * 4, rbk = (k - K0) * 4;
  f4 acc[4];
  const float* Cc = C + 16 * cb * NB;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[rb][v] = Cc[lo + v * NB + 16 * rb];
  // its last NUPD steps, all loads issued first
  const int ks0 = 2 * (k - K0) - NUPD;
  bf8 pa[NUPD > 0 ? NUPD : 1][4], qv[NUPD > 0 ? NUPD : 1];
#pragma unroll
  for (int u = 0; u < NUPD; ++u) {
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
      pa[u][rb] = *reinterpret_cast<const bf8*>(P + ((int64_t)(rbi + rb) * KSW + ks0 + u) * FRAG);
    qv[u] = *reinterpret_cast<const bf8*>(P + ((int64_t)(rbk + cb) * KSW + ks0 + u) * FRAG);
  }
#pragma unroll
  for (int u = 0; u < NUPD; ++u) {
    const bf8 nq = __builtin_bit_cast(bf8, __builtin_bit_cast(u4v, qv[u]) ^ sgn);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nq, pa[u][rb], acc[rb], 0, 0, 0);
  }
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) sc[(16 * cb + 4 * kg + v) * PC_LD + 16 * rb + il] = acc[rb][v];
  __syncthreads();
  // out(r, c') for this wave's column block (tile_solve's products)
  const __bf16* Wf = Wpk + ((int64_t)s * wps + (k - K0)) * 16 * FRAG + lane * 8;
  const int nks = cb >= 2 ? 2 : 1;
  bf8 whi[2], wlo[2];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks)
    if (ks < nks) {
      whi[ks] = *reinterpret_cast<const bf8*>(Wf + (int64_t)(2 * (2 * cb + ks)) * FRAG);
      wlo[ks] = *reinterpret_cast<const bf8*>(Wf + (int64_t)(2 * (2 * cb + ks) + 1) * FRAG);
    }
  f4 o[4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    o[rb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      if (ks >= nks) continue;
      bf8 chi, clo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float cv = sc[(32 * ks + 8 * kg + e) * PC_LD + 16 * rb + il];
        const __bf16 h = (__bf16)cv;
        chi[e] = h;
        clo[e] = (__bf16)(cv - (float)h);
      }
      o[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wlo[ks], chi, o[rb], 0, 0, 0);
      o[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(whi[ks], clo, o[rb], 0, 0, 0);
      o[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(whi[ks], chi, o[rb], 0, 0, 0);
    }
  }
  __syncthreads();   // every read of the updated tile is done
  float* Cw = C + 16 * cb * NB;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Cw[lo + v * NB + 16 * rb] = o[rb][v];
      sc[(16 * cb + 4 * kg + v) * PC_LD + 16 * rb + il] = o[rb][v];
    }
  __syncthreads();
  if (zf != nullptr && w == 0) {
    const double* zk = zf + D.v_off + (int64_t)k * NB;
    double pr[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      double a = 0.0;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          a = fma((double)sc[(16 * cc + 4 * kg + v) * PC_LD + 16 * rb + il], zk[16 * cc + 4 * kg + v], a);
      a += __shfl_xor(a, 16, 64);
      a += __shfl_xor(a, 32, 64);
      pr[rb] = a;
    }
    if (kg == 0) {
      double* bi = zf + D.v_off + (int64_t)i * NB;
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) bi[16 * rb + il] -= pr[rb];
    }
  }
  // pack: wave w writes row block w of both column halves
  __bf16* Pout = Pk + D.pk_off + lane * 8;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = 16 * w + il, cl = 32 * h + 8 * kg;
    bf8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (__bf16)sc[(cl + e) * PC_LD + r];
    *reinterpret_cast<bf8*>(Pout + ((int64_t)(rbi + w) * KSW + 2 * (k - K0) + h) * FRAG) = v;
  }
}

// System s and tile-row group g of workgroup blockIdx.x in the placement of
// k_panel_col (ng groups per system); false for the grid's padding.
__device__ __forceinline__ bool group_of(int spread, int n_sys, int ng, int& s, int& g) {
  if (spread) {
    if ((int)blockIdx.x >= n_sys * ng) return false;
    g = blockIdx.x / n_sys;
    s = blockIdx.x % n_sys;
    return true;
  }
  const int xcd = blockIdx.x % NXCD, slot = blockIdx.x / NXCD, U = (n_sys + NXCD - 1) / NXCD;
  int u;
  if (slot < U) {
    u = slot;
    g = 0;
  } else {
    u = (slot - U) / (ng - 1);
    g = 1 + (slot - U) % (ng - 1);
  }
  s = xcd + NXCD * u;
  return s < n_sys;
}

// Columns c and c + 1 of the panel [K0, K0 + Wp) in one launch, for the tile
// rows below c + 1 (pair_tile, one row per wave).  On entry the columns
// before c are final for every row, and so are the diagonal blocks c and
// c + 1 (Winv fragments, z), and L(c+1, c).  Group 0 (rows c + 2, c + 3)
// carries the diagonal chain two columns ahead, so that the next launch
// finds the same: rows c + 2 and c + 3 on all four waves (chain_rows, which
// also sums tile (c+3, c+2)'s update over the columns before c and parks it
// in the FP32 tile), diagonal block c + 2 (its update reads row c + 2's
// fragments of columns c and c + 1, just packed), the rest of tile
// (c+3, c+2) (chain_tile), then diagonal block c + 3.  Every tile and block
// takes the operations of the single-column sequence in the same order, so
// the factor is the same bit for bit.
__device__ __forceinline__ void ppair_body(const SysDesc& D, int s, SysStatus* __restrict__ st, float* __restrict__ A,
                                           float* __restrict__ Wt, __bf16* __restrict__ Wpk, __bf16* __restrict__ Pk,
                                           int K0, int c, int Wp, int wps, int pack1, int g, double* __restrict__ zf,
                                           PcolLds& lds) {
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (g > 0) {
    const int i = c + 4 * g + w;
    if (i < D.T) pair_tile(D, s, i, lane, A, Wpk, Pk, K0, c, Wp, wps, pack1, zf, lds.sC[w]);
    return;
  }
  const int kend = min(K0 + Wp, (int)D.T);
  const bool d2 = c + 2 < kend, d3 = c + 3 < kend;   // uniform over the workgroup
  float* C32 = A + D.a_off + tile_index(c + 3, c + 2) * TILE;
  chain_rows(D, s, w, lane, A, Wpk, Pk, K0, c, Wp, wps, pack1, d3 && c > K0, zf, lds);
  if (!d2) return;
  __syncthreads();   // rows c + 2 and c + 3 packed, the parked sum stored; LDS free
  diag_block<float>(D, s, st, A, Wt, c + 2, Pk, K0, Wp, wps, Wpk, zf, lds.dg, threadIdx.x);
  if (!d3) return;
  __syncthreads();
  if (lds.dg.fail) return;   // the system failed at block c + 2 (status set)
  __syncthreads();           // every wave has read the flag before the LDS is reused
  chain_tile<4>(D, s, w, lane, C32, Wpk, Pk, K0, c + 2, Wp, wps, zf, lds.sC[0]);
  __syncthreads();
  diag_block<float>(D, s, st, A, Wt, c + 3, Pk, K0, Wp, wps, Wpk, zf, lds.dg, threadIdx.x);
}

// Columns c, c + 1 of the panel (ppair_body); ng = tile-row groups of four
// per system (group 0: rows c + 2, c + 3), placed as in k_panel_col.
__global__ __launch_bounds__(256, 2) void k_panel_pair(const SysDesc* __restrict__ desc, SysStatus* __restrict__ st,
                                                    float* __restrict__ A, float* __restrict__ Wt,
                                                    __bf16* __restrict__ Wpk, __bf16* __restrict__ Pk, int K0, int c,
                                                    int Wp, int level, int pack1, int n_sys, int ng,
                                                    double* __restrict__ zf, int spread) {
  int s, g;
  if (!group_of(spread, n_sys, ng, s, g)) return;
  const SysDesc D = desc[s];
  if (st[s].status != 0 || D.level != level) return;
  __shared__ __align__(16) PcolLds lds;
  ppair_body(D, s, st, A, Wt, Wpk, Pk, K0, c, Wp, Wp, pack1, g, zf, lds);
}

// The head of a panel that runs as column pairs, one workgroup per system:
// diagonal block K0, tile (K0+1, K0) (its panel solve; no update inside the
// panel yet), diagonal block K0 + 1.
__device__ __forceinline__ void phead_body(const SysDesc& D, int s, SysStatus* __restrict__ st, float* __restrict__ A,
                                           float* __restrict__ Wt, __bf16* __restrict__ Wpk, __bf16* __restrict__ Pk,
                                           int K0, int Wp, int wps, double* __restrict__ zf, PcolLds& lds) {
  diag_block<float>(D, s, st, A, Wt, K0, Pk, K0, Wp, wps, Wpk, zf, lds.dg, threadIdx.x);
  if (K0 + 1 >= D.T || K0 + 1 >= K0 + Wp) return;
  __syncthreads();
  if (lds.dg.fail) return;
  __syncthreads();
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  chain_tile<0>(D, s, w, lane, A + D.a_off + tile_index(K0 + 1, K0) * TILE, Wpk, Pk, K0, K0, Wp, wps, zf, lds.sC[0]);
  __syncthreads();
  diag_block<float>(D, s, st, A, Wt, K0 + 1, Pk, K0, Wp, wps, Wpk, zf, lds.dg, threadIdx.x);
}

__global__ __launch_bounds__(256) void k_panel_head(const SysDesc* __restrict__ desc, SysStatus* __restrict__ st,
                                                    float* __restrict__ A, float* __restrict__ Wt,
                                                    __bf16* __restrict__ Wpk, __bf16* __restrict__ Pk, int K0, int Wp,
                                                    int level, double* __restrict__ zf) {
  const int s = blockIdx.x;
  const SysDesc D = desc[s];
  if (K0 >= D.T || st[s].status != 0 || D.level != level) return;
  __shared__ __align__(16) PcolLds lds;
  phead_body(D, s, st, A, Wt, Wpk, Pk, K0, Wp, Wp, zf, lds);
}

// Super-tile order of the trailing update: bands of TRAIL_BAND super-rows,
// column by column inside a band (rows ascending).  A band's row fragments
// stay in L2 while its columns stream past, and each column's fragments are
// read by consecutive workgroups; in row-major order a column's fragments
// are evicted before the next super-row reuses them.  Returns false past the
// system's NS (NS + 1) / 2 super-tiles.
constexpr int TRAIL_BAND = 8;
__device__ __forceinline__ bool trail_decode(int bx, int NS, int& I, int& J) {
  if (bx >= NS * (NS + 1) / 2) return false;
  int lo = 0, hi = min(NS, TRAIL_BAND);
  for (;;) {
    const int cnt = (hi * (hi + 1) - lo * (lo + 1)) / 2;
    if (bx < cnt) break;
    bx -= cnt;
    lo = hi;
    hi = min(NS, lo + TRAIL_BAND);
  }
  const int h = hi - lo;
  if (bx < lo * h) {   // columns left of the band: h super-tiles each
    J = bx / h;
    I = lo + bx % h;
    return true;
  }
  bx -= lo * h;        // columns inside the band: column J has hi - J super-tiles
  J = lo;
  while (bx >= hi - J) {
    bx -= hi - J;
    ++J;
  }
  I = J + bx;
  return true;
}

// Trailing update A(i,j) -= sum_{q in panel} L(i,q) L(j,q)^T for the lower
// triangle i >= j >= i0, from the packed fragment columns [ks0, ks1): 128 x 128
// super-tiles (blockIdx.x = position in the banded order of trail_decode), one
// 64 x 64 tile per wavefront, accumulators starting from the C tile;
// workgroups placed by system on the XCDs (NXCD).  A step's operands are the
// fragments of the super-tile's four tile rows (ib, ib + 1, jb, jb + 1; four
// row blocks each): the workgroup loads them once (four 16-byte loads per
// thread, TR_RD steps ahead into registers), writes them to one of two LDS
// stages, and each wave reads the eight it multiplies, so that a fragment is
// fetched from L2 once per workgroup instead of once per wave.  The step
// count 2 (K1 - K0) is a multiple of TR_RD.
constexpr int TR_RD = 2;
__device__ __forceinline__ void trail_body(const SysDesc& D, int bxs, float* __restrict__ A,
                                           const __bf16* __restrict__ Pk, int K0, int ks0, int ks1, int i0, int Wp,
                                           bf8 (&sF)[2][16][64]);
__global__ __launch_bounds__(256, 2) void k_packed_trailing(const SysDesc* __restrict__ desc,
                                                         const SysStatus* __restrict__ st, float* __restrict__ A,
                                                         const __bf16* __restrict__ Pk, int K0, int ks0, int ks1,
                                                         int i0, int Wp, int level, int n_sys, int ntri, int spread) {
  // XCD placement (see NXCD): slot = system-major (system, super-tile)
  int s, bxs;
  if (spread) {   // workgroups in turn over all XCDs
    if ((int)blockIdx.x >= n_sys * ntri) return;
    s = blockIdx.x / ntri;
    bxs = blockIdx.x % ntri;
  } else {
    const int xcd = blockIdx.x % NXCD, slot = blockIdx.x / NXCD;
    s = xcd + NXCD * (slot / ntri);
    if (s >= n_sys) return;
    bxs = slot % ntri;
  }
  const SysDesc D = desc[s];
  if (st[s].status != 0 || D.level != level) return;
  __shared__ __align__(16) bf8 sF[2][16][64];   // [stage][4 * row set + row block][lane]
  trail_body(D, bxs, A, Pk, K0, ks0, ks1, i0, Wp, sF);
}

// Super-tile bxs (banded order) of the packed trailing update of system D
// (see k_packed_trailing), by the 256 threads of a workgroup.
__device__ __forceinline__ void trail_body(const SysDesc& D, int bxs, float* __restrict__ A,
                                           const __bf16* __restrict__ Pk, int K0, int ks0, int ks1, int i0, int Wp,
                                           bf8 (&sF)[2][16][64]) {
  const int T = D.T;
  const int R = T - i0;
  if (R <= 0) return;
  const int NS = (R + 1) / 2;
  int I, J;
  if (!trail_decode(bxs, NS, I, J)) return;   // uniform: the whole workgroup leaves
  // the wave index as a wave-uniform value: tile and fragment bases stay in
  // scalar registers and the addresses need one per-lane offset each
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int ib = i0 + 2 * I, jb = i0 + 2 * J;
  const int i = ib + (w & 1), j = jb + (w >> 1);
  const bool act = i < T && j <= i;
  // C tile (clamped to a valid tile for the idle waves, which store nothing)
  const int ic = min(i, T - 1);
  float* C = A + D.a_off + tile_index(ic, min(j, ic)) * TILE;
  // element (16 cb + 4 (lane >> 4) + v, 16 rb + (lane & 15)) of the tile: a
  // scalar base per column block cb, one per-lane offset, the rest immediate
  const int lo = 4 * (lane >> 4) * NB + (lane & 15);
  f4 acc[4][4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const float* Cc = C + 16 * cb * NB;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[cb][rb][v] = Cc[lo + v * NB + 16 * rb];
  }
  // this thread loads row block w of row set q (0: ib, 1: ib + 1, 2: jb, 3: jb + 1; clamped to T - 1)
  const int KSW = 2 * Wp;
  const __bf16* src[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = min((q < 2 ? ib : jb) + (q & 1), T - 1);
    src[q] = Pk + D.pk_off + lane * 8 + ((int64_t)((row - K0) * 4 + w) * KSW) * FRAG;
  }
  typedef unsigned u4v __attribute__((ext_vector_type(4)));
  const u4v sgn{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  bf8 rg[TR_RD][4];
#pragma unroll
  for (int u = 0; u < TR_RD; ++u) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      rg[u][q] = *reinterpret_cast<const bf8*>(src[q] + (int64_t)min(ks0 + u, ks1 - 1) * FRAG);
    __builtin_amdgcn_sched_barrier(0);
  }
  const int fi = 4 * (w & 1), fj = 8 + 4 * (w >> 1);
  for (int ks = ks0; ks < ks1; ks += TR_RD) {
#pragma unroll
    for (int u = 0; u < TR_RD; ++u) {
      // stage u & 1: its readers of two steps ago passed the previous barrier
#pragma unroll
      for (int q = 0; q < 4; ++q) sF[u & 1][4 * q + w][lane] = rg[u][q];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q)
        rg[u][q] = *reinterpret_cast<const bf8*>(src[q] + (int64_t)min(ks + u + TR_RD, ks1 - 1) * FRAG);
      if (act) {
        bf8 pa[4], qv[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) pa[rb] = sF[u & 1][fi + rb][lane];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
          qv[cb] = __builtin_bit_cast(bf8, __builtin_bit_cast(u4v, sF[u & 1][fj + cb][lane]) ^ sgn);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
          for (int rb = 0; rb < 4; ++rb)
            acc[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qv[cb], pa[rb], acc[cb][rb], 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  if (!act) return;
  int lo2;   // the offset recomputed here, not held in registers across the loop
  asm volatile("" : "=v"(lo2) : "0"(lo));
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    float* Cc = C + 16 * cb * NB;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) Cc[lo2 + v * NB + 16 * rb] = acc[cb][rb][v];
  }
}

// ---------------------------------------------------------------------------
// Persistent factorisation: one launch runs every stage of every system of
// the batch from the device queues of a PPlan (persist_plan.hpp).  The grid
// holds as many workgroups as the device keeps resident; workgroup b works
// from queue b % nq first (the queue of its XCD) and then from the others.
// A task waits (one lane polling, with sleeps) until its system has finished
// `need` tasks, runs the same body as the corresponding workgroup of the
// multi-launch sequence -- so the results are identical bit for bit -- and
// then counts itself done (every wave's stores released at agent scope
// before the count, the waiter acquiring after it).  Every wait is bounded:
// past `wait_ticks` of the device's constant-rate clock, or once another
// workgroup has given up, the workgroup sets the give-up flag and leaves;
// the caller then marks the systems failed.  A system that turns out not
// positive definite is skipped by its later tasks, which still count.
// ctr: [0, nq) queue heads, [nq, nq + n_sys) tasks done per system,
// [nq + n_sys] the give-up flag; all zero at launch.
// ---------------------------------------------------------------------------
union PersistLds {
  PcolLds pc;
  bf8 sF[2][16][64];
};

// The task bodies as separate (not inlined) functions: each is register-
// allocated on its own, like the kernel of the multi-launch sequence it comes
// from, instead of the persistent kernel holding the union of their register
// needs.  The workgroup's LDS arrives as an LDS-space pointer, so the bodies
// keep their LDS instructions.
typedef __attribute__((address_space(3))) PersistLds* lds_ptr;

__device__ __noinline__ void persist_diag_packed(const SysDesc* __restrict__ desc, int s, SysStatus* __restrict__ st,
                                                 float* __restrict__ A, float* __restrict__ Wt, int k, int K0,
                                                 __bf16* __restrict__ Pk, int wps, __bf16* __restrict__ Wpk,
                                                 double* __restrict__ zf, lds_ptr lp) {
  PersistLds& lds = *(PersistLds*)lp;
  const SysDesc D = desc[s];
  diag_block<float>(D, s, st, A, Wt, k, Pk, K0, D.wp, wps, Wpk, zf, lds.pc.dg, threadIdx.x);
}

__device__ __noinline__ void persist_pcol(const SysDesc* __restrict__ desc, int s, SysStatus* __restrict__ st,
                                          float* __restrict__ A, float* __restrict__ Wt, __bf16* __restrict__ Wpk,
                                          __bf16* __restrict__ Pk, int K0, int k, int wps, int do_pack, int diag_next,
                                          int g, double* __restrict__ zf, lds_ptr lp) {
  PersistLds& lds = *(PersistLds*)lp;
  const SysDesc D = desc[s];
  pcol_body(D, s, st, A, Wt, Wpk, Pk, K0, k, D.wp, wps, do_pack, diag_next, g, zf, lds.pc);
}

__device__ __noinline__ void persist_phead(const SysDesc* __restrict__ desc, int s, SysStatus* __restrict__ st,
                                           float* __restrict__ A, float* __restrict__ Wt, __bf16* __restrict__ Wpk,
                                           __bf16* __restrict__ Pk, int K0, int wps, double* __restrict__ zf,
                                           lds_ptr lp) {
  PersistLds& lds = *(PersistLds*)lp;
  const SysDesc D = desc[s];
  phead_body(D, s, st, A, Wt, Wpk, Pk, K0, D.wp, wps, zf, lds.pc);
}

__device__ __noinline__ void persist_ppair(const SysDesc* __restrict__ desc, int s, SysStatus* __restrict__ st,
                                           float* __restrict__ A, float* __restrict__ Wt, __bf16* __restrict__ Wpk,
                                           __bf16* __restrict__ Pk, int K0, int c, int wps, int pack1, int g,
                                           double* __restrict__ zf, lds_ptr lp) {
  PersistLds& lds = *(PersistLds*)lp;
  const SysDesc D = desc[s];
  ppair_body(D, s, st, A, Wt, Wpk, Pk, K0, c, D.wp, wps, pack1, g, zf, lds.pc);
}

__device__ __noinline__ void persist_trail(const SysDesc* __restrict__ desc, int s, float* __restrict__ A,
                                           const __bf16* __restrict__ Pk, int K0, int K1, int b, lds_ptr lp) {
  PersistLds& lds = *(PersistLds*)lp;
  const SysDesc D = desc[s];
  trail_body(D, b, A, Pk, K0, 0, 2 * (K1 - K0), K1, D.wp, lds.sF);
}

template <typename TS>
__device__ __noinline__ void persist_diag(const SysDesc* __restrict__ desc, int s, SysStatus* __restrict__ st,
                                          TS* __restrict__ A, TS* __restrict__ Wt, int k, lds_ptr lp) {
  PersistLds& lds = *(PersistLds*)lp;
  const SysDesc D = desc[s];
  diag_block<TS>(D, s, st, A, Wt, k, (const __bf16*)nullptr, 0, 1, 1, (__bf16*)nullptr, (double*)nullptr, lds.pc.dg,
                 threadIdx.x);
}

template <typename TS, int MODE>
__device__ __noinline__ void persist_tile(const SysDesc* __restrict__ desc, int s, TS* __restrict__ A,
                                          const TS* __restrict__ Wt, int i, int j, int jc, int q0, int q1) {
  const SysDesc D = desc[s];
  tile_gemm_body<TS, MODE>(D, A, Wt, i, j, jc, q0, q1);
}

__device__ __forceinline__ int ld_agent(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Index of the XCD (accelerator complex die) the calling wave runs on.
__device__ __forceinline__ int xcd_id() {
  unsigned x;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(x));
  return (int)(x & (NXCD - 1));
}

// Counter block of a persistent launch (int32, zeroed before it):
// [nq queue heads][n_sys tasks done per system][give-up flag][nq queue owners]
inline int persist_ctr_count(int nq, int n_sys) { return 2 * nq + n_sys + 1; }

// The persistent factorisation: workgroups take tasks from the plan's
// queues and run each once its system has finished `need` tasks.
//
// local = 1 (one queue per XCD): every queue is served by the workgroups of
// a single XCD (the queue's owner: its own XCD, claimed at first use, or
// another XCD that has drained its own queues and finds it unclaimed), and a
// system's tasks all sit in one queue, so every dependency stays inside one
// XCD and its shared L2: a task publishes its results by waiting for its
// stores to reach the L2 before it counts itself done (no L2 write-back),
// and a waiting task drops the stale lines of its compute unit's L1 before
// it reads them.
// local = 0 (one shared queue): any workgroup takes any task; results cross
// XCDs, so every task ends with an agent-scope release (L2 write-back) and
// starts with an agent-scope acquire (L2 invalidation).
template <typename TS, bool PACKED>
__global__ __launch_bounds__(256, 2) void k_chol_persist(const SysDesc* __restrict__ desc, SysStatus* __restrict__ st,
                                                      TS* __restrict__ A, TS* __restrict__ Wt,
                                                      __bf16* __restrict__ Wpk, __bf16* __restrict__ Pk, int wps,
                                                      double* __restrict__ zf, const PTask* __restrict__ tasks,
                                                      const int32_t* __restrict__ qoff, int nq,
                                                      int32_t* __restrict__ ctr, int n_sys, long long wait_ticks,
                                                      int local) {
  __shared__ __align__(16) PersistLds lds;
  __shared__ int s_task, s_go;
  int32_t* done = ctr + nq;
  int32_t* giveup = ctr + nq + n_sys;
  int32_t* owner = ctr + nq + n_sys + 1;
  const int t = threadIdx.x;
  const int me = local ? xcd_id() : 0;
  const int home = local ? me % nq : (int)(blockIdx.x % (unsigned)nq);
  unsigned exhausted = 0;   // thread 0: queues found empty (or owned by another XCD)
  for (;;) {
    if (t == 0) {
      int task = -1;
      if (!ld_agent(giveup)) {
        for (int u = 0; u < nq && task < 0; ++u) {
          const int q = (home + u) % nq;
          if (exhausted & (1u << q)) continue;
          if (local) {
            int o = ld_agent(owner + q);
            if (o == 0) {
              int expect = 0;
              o = __hip_atomic_compare_exchange_strong(owner + q, &expect, me + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT)
                      ? me + 1
                      : expect;
            }
            if (o != me + 1) {
              exhausted |= 1u << q;
              continue;
            }
          }
          const int x = __hip_atomic_fetch_add(&ctr[q], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (x < qoff[q + 1] - qoff[q]) task = qoff[q] + x;
          else exhausted |= 1u << q;
        }
      }
      int go = 0;
      if (task >= 0) {
        const PTask T = tasks[task];
        int v = ld_agent(done + T.s);
        if (v >= T.need) {
          go = 1;
        } else {
          const long long t0 = wall_clock64();
          for (;;) {
            __builtin_amdgcn_s_sleep(2);
            v = ld_agent(done + T.s);
            if (v >= T.need) {
              go = 1;
              break;
            }
            if (ld_agent(giveup) || wall_clock64() - t0 > wait_ticks) {
              __hip_atomic_store(giveup, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              break;
            }
          }
        }
        if (go) {
          if (!local) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          // a system found not positive definite: its later tasks only count
          if (ld_agent(&st[T.s].status) != 0) go = 2;
        }
      }
      s_task = task;
      s_go = go;
    }
    __syncthreads();
    const int task = s_task, go = s_go;
    if (task < 0 || go == 0) break;
    const PTask T = tasks[task];
    // drop this compute unit's L1 copies of what the earlier tasks wrote (a
    // workgroup-scope invalidation leaves the L1 alone outside thread-group
    // split mode, so the agent-scope one is taken; it keeps dirty L2 lines)
    if (local && go == 1) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (go == 1) {
      const lds_ptr lp = (lds_ptr)&lds;
      if constexpr (PACKED) {
        if (T.kind == PT_DIAG)
          persist_diag_packed(desc, T.s, st, (float*)A, (float*)Wt, T.a, T.b, Pk, wps, Wpk, zf, lp);
        else if (T.kind == PT_PCOL)
          persist_pcol(desc, T.s, st, (float*)A, (float*)Wt, Wpk, Pk, T.c, T.a, wps, T.flags & PF_PACK,
                       (T.flags & PF_DIAG_NEXT) ? 1 : 0, T.b, zf, lp);
        else if (T.kind == PT_PTRAIL)
          persist_trail(desc, T.s, (float*)A, Pk, T.a, T.c, T.b, lp);
        else if (T.kind == PT_PHEAD)
          persist_phead(desc, T.s, st, (float*)A, (float*)Wt, Wpk, Pk, T.a, wps, zf, lp);
        else if (T.kind == PT_PPAIR)
          persist_ppair(desc, T.s, st, (float*)A, (float*)Wt, Wpk, Pk, T.c, T.a, wps, T.flags & PF_PACK, T.b, zf, lp);
      } else {
        if (T.kind == PT_DIAG) {
          persist_diag<TS>(desc, T.s, st, A, Wt, T.a, lp);
        } else if (T.kind == PT_COL) {
          persist_tile<TS, MODE_COL>(desc, T.s, A, Wt, T.a, T.b, T.b, T.c, T.b);
        } else if (T.kind == PT_TRSM) {
          persist_tile<TS, MODE_TRSM>(desc, T.s, A, Wt, T.a, T.b, T.b, 0, 1);
        } else if (T.kind == PT_TRI) {
          int ii = (int)((sqrt(8.0 * (double)T.a + 1.0) - 1.0) * 0.5);
          while ((int64_t)ii * (ii + 1) / 2 > T.a) --ii;
          while ((int64_t)(ii + 1) * (ii + 2) / 2 <= T.a) ++ii;
          const int jj = T.a - ii * (ii + 1) / 2;
          persist_tile<TS, MODE_TRI>(desc, T.s, A, Wt, T.c + ii, T.c + jj, 0, T.b, T.c);
        }
      }
    }
    // every wave's stores have reached the L2 before the task counts as done
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (t == 0) {
      if (local)
        __hip_atomic_fetch_add(done + T.s, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      else
        __hip_atomic_fetch_add(done + T.s, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// After a persistent launch: if a workgroup gave up waiting, every system
// factored in this pass is marked failed (KRR_EDEVICE).
__global__ void k_persist_check(const int32_t* __restrict__ giveup, const SysDesc* __restrict__ desc,
                                SysStatus* __restrict__ st, int n_sys, int level) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n_sys && *giveup && desc[s].level == level) st[s].status = KRR_EDEVICE;
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

__global__ void k_zero_ctr(int32_t* a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

// Resident workgroups of the persistent kernel on the context's device.
template <typename TS, bool PACKED>
int persist_grid(krr_ctx ctx) {
  int per_cu = 0, cus = 0;
  KRR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_chol_persist<TS, PACKED>, 256, 0));
  KRR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
  return std::max(1, per_cu) * std::max(1, cus);
}

// Slot of the context's plan cache holding the PPlan of these shapes,
// uploaded unless resident.  force_slot >= 0: upload into that slot (graph
// replays re-install the plan their launch reads).  Replacing a slot's plan
// waits for the context's queued work, which may still read it; inside a
// graph capture that is an error (ESTATE), so only a free slot is taken there.
// mode: 0 the matrix-core path, 1 the packed path, 2 the packed path in
// column-pair stages.
int persist_upload(krr_ctx ctx, hipStream_t s, const std::vector<int>& T, const std::vector<int>& act,
                   const std::vector<int>& Wp, int mode, int tsize, int force_slot) {
  std::vector<int> key = T;
  key.insert(key.end(), act.begin(), act.end());
  key.insert(key.end(), Wp.begin(), Wp.end());
  key.push_back(mode);
  key.push_back(tsize);
  auto& pc = ctx->persist;
  constexpr int NS = krr_ctx_s::PersistCache::kSlots;
  int slot = force_slot;
  if (slot < 0) {
    for (int i = 0; i < NS; ++i)
      if (pc.slot[i].key == key) {
        pc.slot[i].used = ++pc.clock;
        return i;
      }
    slot = 0;
    for (int i = 0; i < NS; ++i) {
      if (pc.slot[i].key.empty()) {
        slot = i;
        break;
      }
      if (pc.slot[i].used < pc.slot[slot].used) slot = i;
    }
  } else if (pc.slot[slot].key == key) {
    pc.slot[slot].used = ++pc.clock;
    return slot;
  }
  auto& pl = pc.slot[slot];
  if (!pl.key.empty()) {
    if (ctx->capturing) fail(KRR_ESTATE, "persistent plan cache full inside a graph capture");
    drain(ctx);   // queued work may still read this slot's plan or its staging buffer
  }
  const PPlan P = build_plan(T, act, Wp, mode != 0, NXCD, mode == 2);
  const size_t tb = P.tasks.size() * sizeof(PTask), qb = P.qoff.size() * sizeof(int32_t);
  const std::string name = "persist_plan" + std::to_string(slot);
  char* dev = (char*)ws_get(ctx, name, std::max<size_t>(tb + qb + 256, 512));
  void* h = pinned_named(ctx, name, tb + qb + 256);
  std::memcpy(h, P.tasks.data(), tb);
  std::memcpy((char*)h + tb, P.qoff.data(), qb);
  KRR_HIP(hipMemcpyAsync(dev, h, tb + qb, hipMemcpyHostToDevice, s));
  if (ctx->capturing) pc.fresh.push_back(slot);
  pl.key = key;
  pl.tasks = dev;
  pl.qoff_off = tb;
  pl.nq = P.nq;
  pl.ntasks = (int)P.tasks.size();
  pl.T = T;
  pl.act = act;
  pl.wp = Wp;
  pl.packed = mode;
  pl.tsize = tsize;
  pl.used = ++pc.clock;
  return slot;
}

// The persistent factorisation of the systems at `level` (the PPlan is kept
// on the context and rebuilt only when the shapes change).
// Wp: panel width of the matrix-core path; the packed path takes each
// system's own width (SysDesc::wp), with wps the stride of the inverse
// diagonal fragments (Wpk) per system.
template <typename TS>
void factor_persistent(krr_ctx ctx, hipStream_t s, const SysDesc* desc, SysStatus* st, int n_sys, TS* A, TS* Wt,
                       bool packed, int Wp, int wps, int level, const SysDesc* hdesc, __bf16* Pk, __bf16* Wpk,
                       double* zf, double flops, double bytes, const char* cls) {
  std::vector<int> T(n_sys), act(n_sys), wp(n_sys);
  for (int i = 0; i < n_sys; ++i) {
    T[i] = hdesc[i].T;
    act[i] = hdesc[i].level == level ? 1 : 0;
    wp[i] = hdesc[i].wp;
  }
  const int slot = persist_upload(ctx, s, T, act, wp, packed ? (ctx->column_pairs ? 2 : 1) : 0, (int)sizeof(TS), -1);
  const auto& pc = ctx->persist.slot[slot];
  if (ctx->capturing) ctx->persist.captured.push_back(slot);
  if (pc.ntasks == 0) return;
  const int nctr = persist_ctr_count(pc.nq, n_sys);
  int32_t* ctr = (int32_t*)ws_get(ctx, "persist_ctr", (size_t)nctr * 4);
  const int local = pc.nq == NXCD ? 1 : 0;
  hipLaunchKernelGGL(k_zero_ctr, dim3((unsigned)ceil_div(nctr, 256)), dim3(256), 0, s, ctr, nctr);
  check_launch(ctx, s, "zero_ctr");
  int khz = 0;
  KRR_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device));
  const long long ticks = (long long)std::max(1, khz) * (long long)std::max<int64_t>(ctx->persist_wait_ms, 0);
  const PTask* tasks = (const PTask*)pc.tasks;
  const int32_t* qoff = (const int32_t*)((const char*)pc.tasks + pc.qoff_off);
  {
    KernelTimer kt(ctx, s, cls, flops, 1, bytes);
    if (packed) {
      const int grid = std::min(persist_grid<float, true>(ctx), (int)ceil_div(pc.ntasks, NXCD) * NXCD);
      hipLaunchKernelGGL((k_chol_persist<float, true>), dim3((unsigned)grid), dim3(256), 0, s, desc, st, (float*)A,
                         (float*)Wt, Wpk, Pk, wps, zf, tasks, qoff, pc.nq, ctr, n_sys, ticks, local);
    } else {
      const int grid = std::min(persist_grid<TS, false>(ctx), (int)ceil_div(pc.ntasks, NXCD) * NXCD);
      hipLaunchKernelGGL((k_chol_persist<TS, false>), dim3((unsigned)grid), dim3(256), 0, s, desc, st, A, Wt,
                         (__bf16*)nullptr, (__bf16*)nullptr, Wp, (double*)nullptr, tasks, qoff, pc.nq, ctr, n_sys,
                         ticks, local);
    }
    check_launch(ctx, s, "chol_persist");
  }
  hipLaunchKernelGGL(k_persist_check, dim3((unsigned)ceil_div(n_sys, 128)), dim3(128), 0, s,
                     (const int32_t*)(ctr + pc.nq + n_sys), desc, st, n_sys, level);
  check_launch(ctx, s, "persist_check");
}

// grp: -1 for a whole batch; >= 0 for one group of systems of a batch split
// over streams (the call then takes neither the persistent path nor a split).
template <typename TS>
void factor_t(krr_ctx ctx, hipStream_t s, const SysDesc* desc, SysStatus* st, int n_sys, int Tmax, TS* A, TS* Wt,
              bool bf16, int Wp, int level, const SysDesc* hdesc, __bf16* Pk, double* zf, int grp = -1) {
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
  // tasks of the persistent plan: a plan of more than PERSIST_MAX_TASKS (one
  // system of tens of thousands of rows, say) is not built; its stages run as
  // launches (the same bodies, the same results), which for so large a
  // system keep the device as busy
  constexpr int64_t PERSIST_MAX_TASKS = int64_t(1) << 23;
  auto plan_tasks = [&]() {
    int64_t tot = 0;
    for (int i = 0; i < n_sys && hdesc != nullptr; ++i) {
      if (hdesc[i].level != level) continue;
      const int64_t T = hdesc[i].T, w = std::max(1, hdesc[i].wp);
      for (int64_t K0 = 0; K0 < T; K0 += w) {
        const int64_t K1 = std::min(K0 + w, T), R = T - K1;
        if (packed) {
          tot += 1 + (K1 - K0) * ((T - K0) / 4 + 1);
          tot += ((R + 1) / 2) * ((R + 1) / 2 + 1) / 2;
        } else {
          tot += (K1 - K0) * (2 * (T - K0) + 1) + R * (R + 1) / 2;
        }
      }
    }
    return tot;
  };
  // the launch sequence takes one width for the whole batch: the systems' own
  // when they share it
  int uniform = -1;
  for (int i = 0; i < n_sys && hdesc != nullptr; ++i) {
    if (hdesc[i].level != level) continue;
    if (uniform < 0) uniform = hdesc[i].wp;
    else if (uniform != hdesc[i].wp) uniform = 0;
  }
  if (grp < 0 && hdesc != nullptr && (packed || !bf16) &&
      ((ctx->persistent && plan_tasks() <= PERSIST_MAX_TASKS) || uniform == 0)) {
    // one launch: m^3/3 per system credited; bytes: read and write the lower triangle once
    const double fl = each([](double m) { return m * m * m / 3.0; });
    const double by = each([](double m) { return m * (m + 1.0) * sizeof(TS); });
    const char* cls = packed ? "chol_persist_bf16" : (f64 ? "chol_persist_f64" : "chol_persist_f32");
    int wps = 1;
    for (int i = 0; i < n_sys; ++i) wps = std::max(wps, hdesc[i].wp);
    __bf16* Wpk = packed ? (__bf16*)ws_get(ctx, "chol_wpk", (size_t)n_sys * wps * 16 * FRAG * sizeof(__bf16)) : nullptr;
    factor_persistent<TS>(ctx, s, desc, st, n_sys, A, Wt, packed, Wp, wps, level, hdesc, Pk, Wpk, zf, fl, by, cls);
    return;
  }
  if (uniform > 0) Wp = uniform;
  // Groups of consecutive systems of about equal work (m^3), at least NXCD
  // systems each, factored at the same time on the call's stream and the
  // context's side streams: one group's launches that are bound by the
  // latency of the diagonal chain leave CUs idle, which the other groups'
  // launches fill.  Each system's arithmetic is unchanged.
  if (grp < 0 && hdesc != nullptr && ctx->factor_streams > 1) {
    std::vector<double> w(n_sys, 0.0);
    double tot = 0.0;
    int n_act = 0;
    for (int i = 0; i < n_sys; ++i)
      if (hdesc[i].level == level && hdesc[i].T > 0) {
        w[i] = std::pow((double)hdesc[i].T, 3.0);
        tot += w[i];
        ++n_act;
      }
    const int G = std::min(ctx->factor_streams, n_act / NXCD);
    if (G > 1) {
      std::vector<int> cut{0};
      double acc = 0.0;
      for (int i = 0; i < n_sys && (int)cut.size() < G; ++i) {
        acc += w[i];
        if (acc >= tot * (double)cut.size() / G && i + 1 < n_sys) cut.push_back(i + 1);
      }
      cut.push_back(n_sys);
      const int ng = (int)cut.size() - 1;
      KRR_HIP(hipEventRecord(ctx->side_ev[0], s));
      for (int g = 1; g < ng; ++g) KRR_HIP(hipStreamWaitEvent(ctx->side[g - 1], ctx->side_ev[0], 0));
      for (int g = 0; g < ng; ++g) {
        const int lo = cut[g], cnt = cut[g + 1] - cut[g];
        int tg = 0;
        for (int i = lo; i < lo + cnt; ++i)
          if (hdesc[i].level == level) tg = std::max(tg, (int)hdesc[i].T);
        if (tg == 0) continue;
        factor_t<TS>(ctx, g == 0 ? s : ctx->side[g - 1], desc + lo, st + lo, cnt, tg, A, Wt, bf16, Wp, level,
                     hdesc + lo, Pk, zf, g);
      }
      for (int g = 1; g < ng; ++g) {
        KRR_HIP(hipEventRecord(ctx->side_ev[g], ctx->side[g - 1]));
        KRR_HIP(hipStreamWaitEvent(s, ctx->side_ev[g], 0));
      }
      return;
    }
  }
  auto diag_trsm = [&](int k) {
    {
      KernelTimer kt(ctx, s, "chol_diag", each([&](double m) {
        const double b = std::min<double>(NB, m - k * NB);
        return b > 0 ? 2.0 * b * b * b / 3.0 : 0.0;
      }), 0);
      hipLaunchKernelGGL((k_potrf_diag<TS>), dim3(n_sys), dim3(DIAG_THREADS), 0, s, desc, st, A, Wt, k, level,
                         (const __bf16*)nullptr, 0, 1, (__bf16*)nullptr, (double*)nullptr);
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
    // One launch per panel column: the fused column update + panel solve +
    // BF16 packing of the tiles below the diagonal, which also factors the
    // next diagonal block of the panel; the panel's first diagonal block
    // (after the trailing update) has a launch of its own.  After the panel,
    // one trailing update.  Wpk: BF16 high/low fragments of the panel's
    // inverse diagonal blocks.  zf (nullable): the forward solve z = L^-1 b in
    // place, carried column by column (the column launches subtract
    // L(i,k) z_k from the blocks below, each diagonal block forms its z_k).
    // one buffer per group of a split batch (the groups run at the same time)
    __bf16* Wpk = (__bf16*)ws_get(ctx, grp > 0 ? "chol_wpk" + std::to_string(grp) : std::string("chol_wpk"),
                                  (size_t)n_sys * Wp * 16 * FRAG * sizeof(__bf16));
    // placement (see NXCD): spread over all XCDs for fewer than 8 systems, or
    // when the largest system is more than twice the median one (ragged: the
    // largest systems hold most of the work); else one XCD per system
    int spread = n_sys < NXCD ? 1 : 0;
    if (!spread && hdesc != nullptr) {
      std::vector<int> ts;
      for (int i = 0; i < n_sys; ++i)
        if (hdesc[i].level == level && hdesc[i].T > 0) ts.push_back(hdesc[i].T);
      if (!ts.empty()) {
        std::nth_element(ts.begin(), ts.begin() + ts.size() / 2, ts.end());
        if (Tmax > 2 * ts[ts.size() / 2]) spread = 1;
      }
    }
    for (int K0 = 0; K0 < Tmax; K0 += Wp) {
      const int K1 = std::min(K0 + Wp, Tmax);
      auto diag_flops = [&](int k) {
        return each([&](double m) {
          const double b = std::min<double>(NB, m - k * NB);
          return b > 0 ? 2.0 * b * b * b / 3.0 : 0.0;
        });
      };
      // credited to the launch of column k: the column update of the tiles
      // below the diagonal and their panel solve, and the next diagonal block
      // inside the panel (its factorisation); algorithmic bytes: read those
      // tiles and write their factor, read the next diagonal tile and write
      // its factor and inverse (FP32)
      auto col_flops = [&](int k) {
        const bool nd = k + 1 < K1;
        return each([&](double m) {
          const double rows = m - (k + 1) * NB, b = std::min<double>(NB, rows);
          return rows > 0 ? 2.0 * rows * NB * (k - K0) * NB + rows * (double)NB * NB + (nd ? 2.0 * b * b * b / 3.0 : 0.0)
                          : 0.0;
        });
      };
      auto col_bytes = [&](int k) {
        const bool nd = k + 1 < K1;
        return each([&](double m) {
          const double rows = m - (k + 1) * NB;
          return rows > 0 ? 2.0 * rows * NB * sizeof(float) + (nd ? 3.0 * NB * NB * sizeof(float) : 0.0) : 0.0;
        });
      };
      auto single_column = [&](int k) {
        const bool nd = k + 1 < K1;
        KernelTimer kt(ctx, s, col_name, col_flops(k), 1, col_bytes(k));
        const int do_pack = (k + 1 < K1 || K1 < Tmax) ? 1 : 0;
        const int ng = ceil_div(Tmax - k - 1, 4);
        hipLaunchKernelGGL(k_panel_col, dim3((unsigned)(NXCD * ceil_div(n_sys, NXCD) * ng)), dim3(256), 0, s, desc,
                           st, (float*)A, (float*)Wt, Wpk, (__bf16*)Pk, K0, k, Wp, level, do_pack, nd ? 1 : 0, n_sys, ng,
                           zf, spread);
        check_launch(ctx, s, "panel_col");
      };
      if (ctx->column_pairs && K1 - K0 >= 2) {
        // column pairs: the head (diagonal blocks K0 and K0 + 1), then columns
        // (K0, K0 + 1), (K0 + 2, K0 + 3), ... two per launch; an odd width's
        // last column on its own
        {
          KernelTimer kt(ctx, s, "chol_diag", diag_flops(K0), 0);
          hipLaunchKernelGGL(k_panel_head, dim3(n_sys), dim3(256), 0, s, desc, st, (float*)A, (float*)Wt, Wpk,
                             (__bf16*)Pk, K0, Wp, level, zf);
          check_launch(ctx, s, "panel_head");
        }
        int c = K0;
        for (; c + 1 < K1 && c + 2 < Tmax; c += 2) {
          KernelTimer kt(ctx, s, col_name, col_flops(c) + col_flops(c + 1), 1, col_bytes(c) + col_bytes(c + 1));
          const int pack1 = (c + 2 < K1 || K1 < Tmax) ? 1 : 0;
          const int ng = 1 + ceil_div(Tmax - c - 4, 4);
          hipLaunchKernelGGL(k_panel_pair, dim3((unsigned)(NXCD * ceil_div(n_sys, NXCD) * ng)), dim3(256), 0, s, desc,
                             st, (float*)A, (float*)Wt, Wpk, (__bf16*)Pk, K0, c, Wp, level, pack1, n_sys, ng, zf, spread);
          check_launch(ctx, s, "panel_pair");
        }
        if ((K1 - K0) % 2 == 1 && K1 < Tmax) single_column(K1 - 1);
      } else {
        for (int k = K0; k < K1; ++k) {
          if (k == K0) {
            KernelTimer kt(ctx, s, "chol_diag", diag_flops(k), 0);
            hipLaunchKernelGGL((k_potrf_diag<TS>), dim3(n_sys), dim3(DIAG_THREADS), 0, s, desc, st, A, Wt, k, level,
                               (const __bf16*)Pk, K0, Wp, Wpk, zf);
            check_launch(ctx, s, "potrf_diag");
          }
          if (k + 1 < Tmax) single_column(k);
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
        const int ntri = (int)(NS * (NS + 1) / 2);
        hipLaunchKernelGGL(k_packed_trailing, dim3((unsigned)(NXCD * ceil_div(n_sys, NXCD) * ntri)), dim3(256), 0, s,
                           desc, (const SysStatus*)st, (float*)A, (const __bf16*)Pk, K0, 0, 2 * (K1 - K0), K1, Wp,
                           level, n_sys, ntri, spread);
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

void persist_note_plan(krr_ctx ctx, krr_ctx_s::GraphEntry& e) {
  auto& pc = ctx->persist;
  for (int sl : pc.captured) e.plans.emplace_back(sl, pc.slot[sl]);
  pc.captured.clear();
  pc.fresh.clear();
}

void persist_capture_aborted(krr_ctx ctx) {
  auto& pc = ctx->persist;
  for (int sl : pc.fresh) pc.slot[sl] = krr_ctx_s::PersistPlan{};
  pc.fresh.clear();
  pc.captured.clear();
}

void persist_restore_plan(krr_ctx ctx, hipStream_t s, const krr_ctx_s::GraphEntry& e) {
  for (const auto& [sl, pl] : e.plans) {
    if (ctx->persist.slot[sl].key == pl.key) continue;
    persist_upload(ctx, s, pl.T, pl.act, pl.wp, pl.packed, pl.tsize, sl);
    if (ctx->persist.slot[sl].tasks != pl.tasks)
      fail(KRR_ESTATE, "the persistent plan of a captured graph could not be restored");
  }
}

// Factor, in place, the systems of the batch whose descriptor carries
// `level` (the others are left untouched).  prec: KRR_PREC_FP64 -> A, Wt are
// double; FP32 / MIXED -> float.  bf16: BF16 trailing and column updates
// (MIXED first pass); otherwise FP32 (or FP64) matrix-core updates.  hdesc:
// host copy of desc (used for the flop counts of timed launches; nullable).
//
// zfwd (nullable): FP64 vectors (one T*NB block per system at v_off) holding
// the right-hand sides b; with the BF16 packed path (bf16 and pack) they are
// replaced by z = L^-1 b during the factorisation and the call returns true;
// otherwise they are left untouched and the call returns false.
bool cholesky_factor(krr_ctx ctx, hipStream_t s, int prec, const SysDesc* desc, SysStatus* st, int n_sys, int Tmax,
                     void* A, void* Wt, int level, bool bf16, const SysDesc* hdesc, void* pack, double* zfwd) {
  // the multi-launch path's width
  const int Wp = ctx->force_wp > 0 ? ctx->force_wp : (ctx->panel_tiles > 0 ? ctx->panel_tiles : default_panel_tiles(prec));
  if (prec == KRR_PREC_FP64) {
    factor_t<double>(ctx, s, desc, st, n_sys, Tmax, (double*)A, (double*)Wt, false, Wp, level, hdesc, nullptr, nullptr);
    return false;
  }
  const bool packed = bf16 && pack != nullptr;
  factor_t<float>(ctx, s, desc, st, n_sys, Tmax, (float*)A, (float*)Wt, bf16, Wp, level, hdesc, (__bf16*)pack,
                  packed ? zfwd : nullptr);
  return packed && zfwd != nullptr;
}

// BF16 elements of the panel pack slot of a system with T tile rows (the
// first panel, rows [0, T*64) x 2W fragment columns, is the largest).
int64_t pack_slot_elems(int T, int Wp) {
  return (int64_t)T * 4 * 2 * (int64_t)Wp * FRAG;
}

}  // namespace krr
