// Partitioning kernels: exact nearest-centre assignment, stable grouping by
// partition, k-means++ seeding, Lloyd mean updates (Section 2.4, Algorithm 2)
// and the K-balance capacity-constrained greedy pass (Section 4.3,
// Algorithm 4).
//
// Every distance here is the FP64 squared Euclidean distance accumulated
// sequentially over the feature index with separately rounded subtract,
// multiply and add (no contraction into fused multiply-add), so assignments
// are reproducible bit for bit.  Comparisons use
// the squared value; the strict "<" over ascending centre index sends ties to
// the lowest index, as in Algorithm 4.
#include "common.hpp"
#include "exact_sum.hpp"

#include <cmath>

namespace krr {

namespace {

constexpr int GROUP_BLOCK = 256;
constexpr int KPP_BLOCK = 256;   // k-means++ cumulative-weight block
constexpr int ACH = 4;           // centres per register chunk in assignment
constexpr int AROWS = 64;        // rows per assignment block (one per lane)

// Plain operators: the library is compiled with -ffp-contract=off (and the
// pragma keeps it off here), so every operation is rounded on its own.  The
// __d*_rn intrinsics give the same results but compile to strict-FP
// operations that the scheduler will not move loads across.
__device__ __forceinline__ double sqdiff_acc(double acc, double a, double b) {
#pragma clang fp contract(off)
  const double t = a - b;
  return acc + t * t;
}

__device__ __forceinline__ double add_sep(double a, double b) {
#pragma clang fp contract(off)
  return a + b;
}

__device__ __forceinline__ double mul_sep(double a, double b) {
#pragma clang fp contract(off)
  return a * b;
}

// Sequential sum over the features (the additions stay in order; the
// unrolling only lets the loads of eight features issue together).
template <typename TX>
__device__ __forceinline__ double dist2_rows(const TX* __restrict__ a, const TX* __restrict__ b, int d) {
  double acc = 0.0;
#pragma unroll 8
  for (int k = 0; k < d; ++k) acc = sqdiff_acc(acc, (double)a[k], (double)b[k]);
  return acc;
}

__device__ __forceinline__ int first_active_lane() {
  return __ffsll((unsigned long long)__ballot(1)) - 1;
}

// ---------------------------------------------------------------------------
// Assignment of rows of X to the nearest of p centres (CT is d x p, i.e. the
// centres transposed, so that the p values of one feature are contiguous).
// MODE 0: argmin index (+ change count against `prev`); MODE 1: all p squared
// distances into D (n x p).  A block stages 64 rows in LDS feature-major
// (lane = row); its 4 waves take the centre chunks [4c, 4c + 4) with
// c = wave, wave + 4, ..., so that a wave's centre values are uniform and
// each SIMD holds several waves.  CTL: the centres are staged in LDS too
// (p d doubles; the inner loop then issues only LDS loads, which return in
// order, instead of scalar loads, whose waits drain every LDS load in
// flight); otherwise they are read with scalar loads.  The per-wave minima
// are combined with the rule of the sequential scan: lowest value, then
// lowest index.
// ---------------------------------------------------------------------------
template <typename TX, int MODE, bool CTL>
__global__ __launch_bounds__(256) void k_assign(const TX* __restrict__ X, int64_t n, int d,
                                                const double* __restrict__ CT, int p,
                                                int32_t* __restrict__ out, double* __restrict__ D,
                                                const int32_t* __restrict__ prev,
                                                int32_t* __restrict__ delta,
                                                const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip) return;
  extern __shared__ unsigned char smem_raw[];
  TX* sX = reinterpret_cast<TX*>(smem_raw);
  double* sCT = reinterpret_cast<double*>(smem_raw + ((((size_t)d * (AROWS + 1) + 1) * sizeof(TX) + 15) & ~size_t(15)));
  __shared__ double sbest[4][AROWS];
  __shared__ int32_t sidx[4][AROWS];
  constexpr int ld = AROWS + 1;
  const int64_t row0 = (int64_t)blockIdx.x * AROWS;
  const int rows = (int)min((int64_t)AROWS, n - row0);
  const TX* src = X + row0 * d;
  const int tot = rows * d;
  // batches of 8 unconditional loads from clamped addresses, then the stores;
  // (row, feature) of element e0 + 256 u follow from those of e0 by steps of
  // 256 = sq d + sr (one division per batch)
  const int sq = 256 / d, sr = 256 - sq * d;
  for (int e0 = threadIdx.x; e0 < tot; e0 += 8 * 256) {
    TX v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[min(e0 + u * 256, tot - 1)];
    int r = e0 / d, k = e0 - r * d;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256;
      // out-of-range elements go to a spare LDS slot instead of a conditional store
      sX[(e < tot) ? (k * ld + r) : d * ld] = v[u];
      k += sr;
      r += sq;
      if (k >= d) {
        k -= d;
        ++r;
      }
    }
  }
  if (CTL)
    for (int e = threadIdx.x; e < d * p; e += 256) sCT[e] = CT[e];
  __syncthreads();
  const int r = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool valid = r < rows;
  const int64_t i = row0 + min(r, rows - 1);
  double best = INFINITY;
  int bj = -1;
  for (int j0 = ACH * w; j0 < p; j0 += 4 * ACH) {
    const int nj = min(ACH, p - j0);
    double acc[ACH];
#pragma unroll
    for (int q = 0; q < ACH; ++q) acc[q] = 0.0;
    if (nj == ACH) {
      for (int k = 0; k < d; ++k) {
        const double xk = (double)sX[k * ld + r];
        const double* c = (CTL ? sCT : CT) + (int64_t)k * p + j0;
#pragma unroll
        for (int q = 0; q < ACH; ++q) acc[q] = sqdiff_acc(acc[q], xk, c[q]);
      }
    } else {
      for (int k = 0; k < d; ++k) {
        const double xk = (double)sX[k * ld + r];
        const double* c = (CTL ? sCT : CT) + (int64_t)k * p + j0;
#pragma unroll
        for (int q = 0; q < ACH; ++q)
          if (q < nj) acc[q] = sqdiff_acc(acc[q], xk, c[q]);
      }
    }
    if (MODE == 1) {
      if (valid)
        for (int q = 0; q < nj; ++q) D[i * p + j0 + q] = acc[q];
    } else {
      for (int q = 0; q < nj; ++q)
        if (acc[q] < best) {
          best = acc[q];
          bj = j0 + q;
        }
    }
  }
  if (MODE == 0) {
    sbest[w][r] = best;
    sidx[w][r] = bj;
    __syncthreads();
    if (w == 0) {
      double bv = INFINITY;
      int bi = -1;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int ju = sidx[u][r];
        const double vu = sbest[u][r];
        if (ju >= 0 && (vu < bv || (vu == bv && (bi < 0 || ju < bi)))) {
          bv = vu;
          bi = ju;
        }
      }
      if (bi < 0) bi = 0;  // every distance +inf: first centre, as the sequential scan does
      if (valid) out[i] = bi;
      if (delta != nullptr) {
        const bool changed = valid && ((prev == nullptr) || (prev[i] != bi));
        const unsigned long long b = __ballot(changed);
        if (r == 0) atomicAdd(delta, (int32_t)__popcll(b));
      }
    }
  }
}

// Unstaged variant for very wide rows (LDS cannot hold a block of rows).
template <typename TX, int MODE>
__global__ __launch_bounds__(256) void k_assign_wide(const TX* __restrict__ X, int64_t n, int d,
                                                     const double* __restrict__ CT, int p,
                                                     int32_t* __restrict__ out, double* __restrict__ D,
                                                     const int32_t* __restrict__ prev,
                                                     int32_t* __restrict__ delta,
                                                     const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const TX* x = X + i * d;
  double best = INFINITY;
  int bj = -1;
  for (int j = 0; j < p; ++j) {
    double acc = 0.0;
    for (int k = 0; k < d; ++k) acc = sqdiff_acc(acc, (double)x[k], CT[(int64_t)k * p + j]);
    if (MODE == 1) {
      D[i * p + j] = acc;
    } else if (acc < best) {
      best = acc;
      bj = j;
    }
  }
  if (MODE == 0) {
    if (bj < 0) bj = 0;
    out[i] = bj;
    if (delta != nullptr) {
      const bool changed = (prev == nullptr) || (prev[i] != bj);
      const unsigned long long b = __ballot(changed);
      if ((int)(threadIdx.x & 63) == first_active_lane()) atomicAdd(delta, (int32_t)__popcll(b));
    }
  }
}

__global__ void k_transpose(const double* __restrict__ C, int p, int d, double* __restrict__ CT) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p * d) return;
  const int j = e / d, k = e - j * d;
  CT[(int64_t)k * p + j] = C[e];
}

// ---------------------------------------------------------------------------
// Stable grouping of n keys in [0, p): perm lists the indices of key 0 in
// increasing order, then key 1, ...; offsets[j] is where key j starts.
// ---------------------------------------------------------------------------
// Rank of each key among the earlier keys of its block that are equal, and
// the block's count per key: inside a wave one ballot per distinct key, then
// the counts of the earlier waves (LDS, [wave][key]).
__global__ __launch_bounds__(GROUP_BLOCK) void k_group_local(const int32_t* __restrict__ key, int64_t n,
                                                             int p, int32_t* __restrict__ local_rank,
                                                             int32_t* __restrict__ blockcounts,
                                                             const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip) return;
  constexpr int NWV = GROUP_BLOCK / 64;
  extern __shared__ int32_t wc[];   // [NWV][p]
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int e = threadIdx.x; e < NWV * p; e += GROUP_BLOCK) wc[e] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * GROUP_BLOCK + threadIdx.x;
  const int kv = (i < n) ? key[i] : -1;
  int rw = 0;
  unsigned long long todo = __ballot(kv >= 0);
  while (todo != 0ull) {
    const int leader = __ffsll(todo) - 1;
    const int kk = __shfl(kv, leader, 64);
    const unsigned long long m = __ballot(kv == kk);
    if (kv == kk) rw = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == leader) wc[w * p + kk] = __popcll(m);
    todo &= ~m;
  }
  __syncthreads();
  if (kv >= 0) {
    int r = rw;
    for (int u = 0; u < w; ++u) r += wc[u * p + kv];
    local_rank[i] = r;
  }
  for (int j = threadIdx.x; j < p; j += GROUP_BLOCK) {
    int c = 0;
    for (int u = 0; u < NWV; ++u) c += wc[u * p + j];
    blockcounts[(int64_t)blockIdx.x * p + j] = c;
  }
}

// Per key j: exclusive prefix of the per-block counts (block offsets) and the
// total; one wave per key (lane l takes a contiguous run of blocks, then a
// 64-lane scan of the run sums).  Then the key offsets in key order.
__global__ __launch_bounds__(1024) void k_group_scan(const int32_t* __restrict__ blockcounts, int64_t nblocks,
                                                     int p, int32_t* __restrict__ blockoffs,
                                                     int64_t* __restrict__ offsets,
                                                     int64_t* __restrict__ sizes64,
                                                     const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip) return;
  extern __shared__ int64_t tot[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int64_t per = (nblocks + 63) / 64;
  const int64_t b0 = min(nblocks, lane * per), b1 = min(nblocks, b0 + per);
  constexpr int SCAN_REG = 8;   // a lane's counts kept in registers when it has at most this many
  for (int j = w; j < p; j += nw) {
    int32_t cr[SCAN_REG];
    int64_t sum = 0;
    if (per <= SCAN_REG) {
#pragma unroll
      for (int u = 0; u < SCAN_REG; ++u) cr[u] = (b0 + u < b1) ? blockcounts[(b0 + u) * p + j] : 0;
#pragma unroll
      for (int u = 0; u < SCAN_REG; ++u) sum += cr[u];
    } else {
      for (int64_t b = b0; b < b1; ++b) sum += blockcounts[b * p + j];
    }
    int64_t x = sum;   // inclusive scan over the lanes
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    int64_t run = x - sum;
    if (per <= SCAN_REG) {
#pragma unroll
      for (int u = 0; u < SCAN_REG; ++u)
        if (b0 + u < b1) {
          blockoffs[(b0 + u) * p + j] = (int32_t)run;
          run += cr[u];
        }
    } else {
      for (int64_t b = b0; b < b1; ++b) {
        const int32_t c = blockcounts[b * p + j];
        blockoffs[b * p + j] = (int32_t)run;
        run += c;
      }
    }
    if (lane == 63) {
      tot[j] = x;
      if (sizes64 != nullptr) sizes64[j] = x;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t o = 0;
    for (int j = 0; j < p; ++j) {
      offsets[j] = o;
      o += tot[j];
    }
    offsets[p] = o;
  }
}

__global__ __launch_bounds__(GROUP_BLOCK) void k_group_scatter(const int32_t* __restrict__ key, int64_t n,
                                                               int p, const int32_t* __restrict__ local_rank,
                                                               const int32_t* __restrict__ blockoffs,
                                                               const int64_t* __restrict__ offsets,
                                                               int32_t* __restrict__ perm,
                                                               const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * GROUP_BLOCK + threadIdx.x;
  if (i >= n) return;
  const int kv = key[i];
  perm[offsets[kv] + blockoffs[(int64_t)blockIdx.x * p + kv] + local_rank[i]] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// Means of the grouped members (Algorithm 2's mean step): C[j][f] = (exactly
// rounded sum of the member values) / count_j in FP64; an empty partition
// keeps its centre.  The sums are integer sums of the values' units
// (exact_sum.hpp), which take the members in any order: workgroup (j, slice,
// split) adds the member rows [cnt split / rs, cnt (split + 1) / rs) of
// partition j (in the stable grouping perm) for the MS_W features of slice
// `slice`: it stages up to MS_CH member indices in LDS (one coalesced pass),
// then thread (feature fl, row subset rr) adds rows rr, rr + RR, ... into its
// own limbs in LDS (B rows' loads issued together, then one LDS atomic add per
// term), and the workgroup writes the per-feature limb sums of its rows to P.  k_means_round adds the rs partial limb sets of each (j, f), rounds once
// and divides by the count.  Lloyd passes: `skip` is this pass's "fixed point
// reached" flag; k_means_round's first thread writes the next pass's flag (set
// when this pass was skipped or changed no assignment), so no workgroup of a
// launch reads a flag that the same launch writes.  CT (nullable) receives the
// centres transposed (d x p).
// ---------------------------------------------------------------------------
constexpr int MS_W = 16;      // features per workgroup
constexpr int MS_CH = 1024;   // member indices a workgroup stages in LDS at once

template <typename TX>
struct MeansCfg {
  static constexpr int THREADS = sizeof(TX) == 4 ? 256 : 64;   // FP64: 66 limbs per thread in LDS
  static constexpr int RR = THREADS / MS_W;                     // row subsets of a workgroup
  static constexpr int B = sizeof(TX) == 4 ? 16 : 8;            // rows per thread whose loads issue together
};

template <typename TX>
__global__ __launch_bounds__(MeansCfg<TX>::THREADS) void k_means_acc(const TX* __restrict__ X, int d, int nsl, int rs,
                                                                      const int32_t* __restrict__ perm,
                                                                      const int64_t* __restrict__ offsets,
                                                                      int64_t* __restrict__ P,
                                                                      const int32_t* __restrict__ skip) {
  constexpr int NL = ExactSum<TX>::NL, NT = MeansCfg<TX>::THREADS, RR = MeansCfg<TX>::RR, B = MeansCfg<TX>::B;
  constexpr int NORM_EVERY = ExactSum<TX>::ADDS;
  static_assert(NORM_EVERY % B == 0, "normalisation at whole batches");
  if (skip != nullptr && *skip) return;
  const int split = blockIdx.x % rs, js = blockIdx.x / rs;
  const int j = js / nsl, slice = js - j * nsl;
  const int64_t base = offsets[j], cnt = offsets[j + 1] - base;
  const int64_t r0 = cnt * split / rs, r1 = cnt * (split + 1) / rs;
  __shared__ int64_t acc[NL * NT];   // acc[k * NT + t]: thread t's limb k
  __shared__ int32_t sP[MS_CH];
  const int t = threadIdx.x, fl = t % MS_W, rr = t / MS_W;
  const int f = slice * MS_W + fl;
  const bool live = f < d;
  const int fc = min(f, d - 1);   // lanes past d load a valid value and add zero
  int64_t* mine = acc + t;
  for (int k = 0; k < NL; ++k) mine[k * NT] = 0;
  auto get = [&](int k) { return mine[k * NT]; };
  auto set = [&](int k, int64_t v) { mine[k * NT] = v; };
  int since = 0;
  for (int64_t c0 = r0; c0 < r1; c0 += MS_CH) {
    const int nr = (int)min<int64_t>(MS_CH, r1 - c0);
    for (int q = t; q < MS_CH; q += NT) sP[q] = perm[base + c0 + min(q, nr - 1)];
    __syncthreads();
    for (int q0 = rr; q0 < nr; q0 += RR * B) {
      TX v[B];
#pragma unroll
      for (int u = 0; u < B; ++u) v[u] = X[(int64_t)sP[min(q0 + RR * u, nr - 1)] * d + fc];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const bool ok = live && q0 + RR * u < nr;
        const XsTerms tm = xs_terms(v[u]);
        atomicAdd(reinterpret_cast<unsigned long long*>(mine + tm.l0 * NT), (unsigned long long)(ok ? tm.c0 : 0));
        if (sizeof(TX) == 8)
          atomicAdd(reinterpret_cast<unsigned long long*>(mine + tm.l1 * NT), (unsigned long long)(ok ? tm.c1 : 0));
      }
      since += B;
      if (since == NORM_EVERY) {
        xs_normalise<NL>(get, set);
        since = 0;
      }
    }
    __syncthreads();   // every read of sP done before the next chunk's indices
  }
  xs_normalise<NL>(get, set);
  __syncthreads();
  // per (feature, limb): the sum over the row subsets (each limb below 2^32
  // but the signed top one, so the sum stays far from overflow)
  int64_t* out = P + (int64_t)blockIdx.x * MS_W * NL;
  for (int e = t; e < MS_W * NL; e += NT) {
    const int f2 = e / NL, k = e - f2 * NL;
    int64_t s = 0;
#pragma unroll
    for (int q = 0; q < RR; ++q) s += acc[k * NT + q * MS_W + f2];
    out[e] = s;
  }
}

// Workgroup of 256 threads: RoundCfg::PAIRS (partition, feature) pairs; thread
// (pair, limb) adds that limb over the row splits, then one thread per pair
// rounds.
template <typename TX>
struct RoundCfg {
  static constexpr int PAIRS = 256 / ExactSum<TX>::NL;
};

template <typename TX>
__global__ __launch_bounds__(256) void k_means_round(int d, int nsl, int rs, int p,
                                                     const int64_t* __restrict__ offsets,
                                                     const int64_t* __restrict__ P, double* __restrict__ C,
                                                     double* __restrict__ CT, const int32_t* __restrict__ skip,
                                                     const int32_t* __restrict__ delta,
                                                     int32_t* __restrict__ done_next) {
  constexpr int NL = ExactSum<TX>::NL, PAIRS = RoundCfg<TX>::PAIRS;
  const int skipped = (skip != nullptr) ? *skip : 0;
  if (done_next != nullptr && blockIdx.x == 0 && threadIdx.x == 0)
    *done_next = (skipped || *delta == 0) ? 1 : 0;
  if (skipped) return;
  __shared__ int64_t sL[PAIRS * NL];
  const int t = threadIdx.x;
  const int64_t pd = (int64_t)p * d;
  if (t < PAIRS * NL) {
    const int64_t id = (int64_t)blockIdx.x * PAIRS + t / NL;
    const int k = t % NL;
    int64_t s = 0;
    if (id < pd) {
      const int j = (int)(id / d), f = (int)(id - (int64_t)j * d);
      const int slice = f / MS_W, fl = f - slice * MS_W;
      const int64_t* src = P + ((int64_t)(j * nsl + slice) * rs * MS_W + fl) * NL + k;
      for (int q = 0; q < rs; ++q) s += src[(int64_t)q * MS_W * NL];
    }
    sL[t] = s;
  }
  __syncthreads();
  if (t >= PAIRS) return;
  const int64_t id = (int64_t)blockIdx.x * PAIRS + t;
  if (id >= pd) return;
  const int j = (int)(id / d), f = (int)(id - (int64_t)j * d);
  const int64_t cnt = offsets[j + 1] - offsets[j];
  if (cnt == 0) return;
  int64_t limb[NL];
  for (int k = 0; k < NL; ++k) limb[k] = sL[t * NL + k];
  const double val = xs_round<TX>(limb) / (double)cnt;
  C[(int64_t)j * d + f] = val;
  if (CT != nullptr) CT[(int64_t)f * p + j] = val;
}

// ---------------------------------------------------------------------------
// k-means++ seeding with the cumulative D^2 weight formed in blocks of 256
// points: sequential inside a block, block totals summed sequentially, and one
// add of the block offset.  Centre t is the first point whose cumulative
// weight exceeds u_t times the total.
// ---------------------------------------------------------------------------
template <typename TX>
__global__ __launch_bounds__(KPP_BLOCK) void k_kpp_update(const TX* __restrict__ X, int64_t n, int d,
                                                          const int64_t* __restrict__ cidx, int t,
                                                          double* __restrict__ D2, double* __restrict__ P,
                                                          double* __restrict__ Tb) {
  __shared__ double sd[KPP_BLOCK];
  const int64_t i = (int64_t)blockIdx.x * KPP_BLOCK + threadIdx.x;
  const int64_t c = cidx[t];
  double v = 0.0;
  if (i < n) {
    const double dd = dist2_rows(X + i * d, X + c * d, d);
    if (t == 0) {
      v = dd;
    } else {
      const double old = D2[i];
      v = (dd < old) ? dd : old;
    }
    D2[i] = v;
  }
  sd[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    // sequential prefix in point order, 16 loads at a time; past the block's
    // points the weights are 0 and leave the sum unchanged
    double acc = sd[0];
#pragma unroll 1
    for (int q0 = 0; q0 < KPP_BLOCK; q0 += 16) {
      double x[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) x[u] = sd[q0 + u];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        if (q0 + u > 0) acc = add_sep(acc, x[u]);
        x[u] = acc;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) sd[q0 + u] = x[u];
    }
    Tb[blockIdx.x] = acc;
  }
  __syncthreads();
  if (i < n) P[i] = sd[threadIdx.x];
}

// Selection of centre t.  Thread 0 forms the block offsets (sequential sum
// of the block totals, loads batched) into LDS; every thread then scans its
// share of the blocks for the first whose end weight exceeds the threshold,
// and the first such block is searched point by point.  The offsets live in
// LDS when nblk <= KPP_MAXBLK, else in the global buffer gOb.
constexpr int KPP_MAXBLK = 4096;

template <typename TX>
__global__ __launch_bounds__(KPP_BLOCK) void k_kpp_select(const double* __restrict__ P,
                                                          const double* __restrict__ Tb, int64_t nblk,
                                                          int64_t n, double u, const TX* __restrict__ X, int d,
                                                          int64_t* __restrict__ cidx, int t,
                                                          double* __restrict__ C, double* __restrict__ gOb) {
  extern __shared__ double shOb[];   // nblk block offsets (when gOb is null)
  double* sOb = gOb != nullptr ? gOb : shOb;
  __shared__ double s_total;
  __shared__ int64_t s_idx[KPP_BLOCK];
  if (gOb == nullptr) {
    // offsets in LDS: the block totals come in with one coalesced load, then
    // thread 0 turns them into the exclusive prefix in place (same order)
    for (int64_t b = threadIdx.x; b < nblk; b += KPP_BLOCK) shOb[b] = Tb[b];
    __syncthreads();
    if (threadIdx.x == 0) {
      double o = 0.0;
      for (int64_t b = 0; b < nblk; ++b) {
        const double tv = shOb[b];
        shOb[b] = o;
        o = add_sep(o, tv);
      }
      s_total = o;
    }
  } else if (threadIdx.x == 0) {
    double o = 0.0;
    int64_t b = 0;
    for (; b + 8 <= nblk; b += 8) {
      double tv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) tv[q] = Tb[b + q];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        sOb[b + q] = o;
        o = add_sep(o, tv[q]);
      }
    }
    for (; b < nblk; ++b) {
      const double tv = Tb[b];
      sOb[b] = o;
      o = add_sep(o, tv);
    }
    s_total = o;
  }
  __syncthreads();
  const double total = s_total;
  int64_t idx;
  if (!(total > 0.0)) {
    idx = (int64_t)floor(mul_sep(u, (double)n));
    if (idx > n - 1) idx = n - 1;
  } else {
    const double thr = mul_sep(u, total);
    int64_t cand = INT64_MAX;
    for (int64_t b = threadIdx.x; b < nblk; b += KPP_BLOCK)
      if (add_sep(sOb[b], Tb[b]) > thr) {
        cand = b;
        break;
      }
    s_idx[threadIdx.x] = cand;
    __syncthreads();
    for (int w = KPP_BLOCK / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) s_idx[threadIdx.x] = min(s_idx[threadIdx.x], s_idx[threadIdx.x + w]);
      __syncthreads();
    }
    const int64_t blk = s_idx[0];
    __syncthreads();
    if (blk == INT64_MAX) {
      idx = 0;  // no cumulative weight above the threshold: the first point
    } else {
      const int64_t i = blk * KPP_BLOCK + threadIdx.x;
      s_idx[threadIdx.x] = (i < n && add_sep(sOb[blk], P[i]) > thr) ? i : INT64_MAX;
      __syncthreads();
      for (int w = KPP_BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s_idx[threadIdx.x] = min(s_idx[threadIdx.x], s_idx[threadIdx.x + w]);
        __syncthreads();
      }
      idx = s_idx[0];
    }
  }
  if (threadIdx.x == 0) cidx[t] = idx;
  for (int f = threadIdx.x; f < d; f += KPP_BLOCK) C[(int64_t)t * d + f] = (double)X[idx * d + f];
}

template <typename TX>
__global__ void k_kpp_first(int64_t n, double u0, const TX* __restrict__ X, int d,
                            int64_t* __restrict__ cidx, double* __restrict__ C) {
  int64_t idx = (int64_t)floor(mul_sep(u0, (double)n));
  if (idx > n - 1) idx = n - 1;
  if (threadIdx.x == 0) cidx[0] = idx;
  for (int f = threadIdx.x; f < d; f += blockDim.x) C[f] = (double)X[idx * d + f];
}

// ---------------------------------------------------------------------------
// K-balance greedy pass (Algorithm 4), one wavefront.  Points are visited in
// input order; each takes the nearest centre whose count is below `cap`.
// Chunks of 64 points are decided in parallel from the set of centres open at
// the chunk start; when no centre would pass `cap` inside the chunk, that is
// exactly the sequential result (a point's choice is minimal over a superset
// that still contains it).  Otherwise the chunk is replayed point by point.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_argmin(double& v, int& j) {
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off, 64);
    const int oj = __shfl_xor(j, off, 64);
    if (ov < v || (ov == v && oj < j)) {
      v = ov;
      j = oj;
    }
  }
}

// Segment q = blockIdx.x of nseg covers the samples [floor(q n / nseg),
// floor((q + 1) n / nseg)) and runs the greedy pass on them alone with
// capacity `cap` (cap <= 0: ceil(segment size / p)).  One segment is
// Algorithm 4's pass; p segments with cap <= 0 are the approximate parallel
// K-balance of Section 4.3 (one segment per node, n / p^2 per node and centre).
__global__ __launch_bounds__(64) void k_kbalance(const double* __restrict__ D, const int32_t* __restrict__ a0,
                                                 int64_t n, int p, int nseg, int64_t cap_in,
                                                 int32_t* __restrict__ MB) {
  extern __shared__ int32_t sh[];
  int32_t* cs = sh;        // p counts
  int32_t* hist = sh + p;  // p per-chunk counts
  const int lane = threadIdx.x;
  const int64_t lo = (int64_t)blockIdx.x * n / nseg, hi = ((int64_t)blockIdx.x + 1) * n / nseg;
  const int64_t cap = cap_in > 0 ? cap_in : (hi - lo + p - 1) / p;
  for (int j = lane; j < p; j += 64) {
    cs[j] = 0;
    hist[j] = 0;
  }
  __builtin_amdgcn_wave_barrier();
  int next_a = (lo + lane < hi) ? a0[lo + lane] : 0;
  for (int64_t c0 = lo; c0 < hi; c0 += 64) {
    const int64_t i = c0 + lane;
    const bool valid = i < hi;
    const int cur_a = next_a;
    if (c0 + 64 + lane < hi) next_a = a0[c0 + 64 + lane];   // prefetch the next chunk
    int bj = -1;
    if (valid) {
      bj = cur_a;
      if (cs[bj] >= cap) {  // nearest centre already full: search the open ones
        double bd = INFINITY;
        bj = -1;
        for (int j = 0; j < p; ++j) {
          if (cs[j] < cap) {
            const double v = D[i * p + j];
            if (v < bd) {
              bd = v;
              bj = j;
            }
          }
        }
        if (bj < 0) bj = 0;
      }
      atomicAdd(&hist[bj], 1);
    }
    __builtin_amdgcn_wave_barrier();
    bool ok = true;
    for (int j = lane; j < p; j += 64)
      if ((int64_t)cs[j] + hist[j] > cap) ok = false;
    ok = __all(ok);
    __builtin_amdgcn_wave_barrier();
    if (ok) {
      if (valid) MB[i] = bj;
      for (int j = lane; j < p; j += 64) {
        cs[j] += hist[j];
        hist[j] = 0;
      }
      __builtin_amdgcn_wave_barrier();
    } else {
      for (int j = lane; j < p; j += 64) hist[j] = 0;
      __builtin_amdgcn_wave_barrier();
      const int cnt = (int)min((int64_t)64, hi - c0);
      for (int l = 0; l < cnt; ++l) {
        const int64_t ii = c0 + l;
        double v = INFINITY;
        int jj = INT32_MAX;
        for (int j = lane; j < p; j += 64) {
          if (cs[j] < cap) {
            const double dv = D[ii * p + j];
            if (dv < v) {
              v = dv;
              jj = j;
            }
          }
        }
        wave_argmin(v, jj);
        if (jj == INT32_MAX) jj = 0;
        if (lane == 0) {
          MB[ii] = jj;
          cs[jj] += 1;
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
  }
}

// Event-driven K-balance (same result as the sequential pass).  The set of
// full centres only grows, and between two "a centre becomes full" events
// every point takes the plain argmin over the open centres.  A round computes
// the choices of all points from `start` on in parallel (k_kbal_choose), then
// finds the first point that fills a centre (k_kbal_event): the choices up to
// it are final, that centre closes, and the next round starts after it.
// At most p + 1 rounds; rounds after the last event exit at once (`done`).
// State: st[0] = start, st[1] = done; counts cs[p], full[p].
constexpr int KB_BLOCK = 256;
constexpr int KB_MAXP = 256;    // event kernel: one thread per centre

__global__ __launch_bounds__(KB_BLOCK) void k_kbal_choose(const double* __restrict__ D, int64_t n, int p,
                                                          const int32_t* __restrict__ full,
                                                          const int64_t* __restrict__ st, int32_t* __restrict__ MB,
                                                          int32_t* __restrict__ bc) {
  if (st[1]) return;
  extern __shared__ int32_t hist[];
  for (int j = threadIdx.x; j < p; j += KB_BLOCK) hist[j] = 0;
  __syncthreads();
  const int64_t start = st[0];
  const int64_t i = (int64_t)blockIdx.x * KB_BLOCK + threadIdx.x;
  if (i >= start && i < n) {
    double bd = INFINITY;
    int bj = -1;
    for (int j = 0; j < p; ++j) {
      if (!full[j]) {
        const double v = D[i * p + j];
        if (v < bd) {
          bd = v;
          bj = j;
        }
      }
    }
    if (bj < 0) bj = 0;   // no open centre at a finite distance: centre 0, as the sequential pass does
    MB[i] = bj;
    atomicAdd(&hist[bj], 1);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < p; j += KB_BLOCK) bc[(int64_t)blockIdx.x * p + j] = hist[j];
}

__global__ __launch_bounds__(KB_MAXP) void k_kbal_event(const int32_t* __restrict__ MB, const int32_t* __restrict__ bc,
                                                        int64_t nblk, int64_t n, int p, int64_t cap,
                                                        int32_t* __restrict__ cs, int32_t* __restrict__ full,
                                                        int64_t* __restrict__ st) {
  if (st[1]) return;
  __shared__ int64_t spos[KB_MAXP];
  const int j = threadIdx.x;
  const int64_t start = st[0];
  // position of the point that would fill centre j, if any
  int64_t pos = INT64_MAX;
  if (j < p && !full[j]) {
    const int64_t need = cap - cs[j];
    int64_t cum = 0, b = start / KB_BLOCK;
    for (; b < nblk; ++b) {
      const int c = bc[b * p + j];
      if (cum + c >= need) break;
      cum += c;
    }
    if (b < nblk) {
      const int64_t i0 = max(start, b * KB_BLOCK), i1 = min(n, (b + 1) * KB_BLOCK);
      for (int64_t i = i0; i < i1; ++i)
        if (MB[i] == j && ++cum == need) {
          pos = i;
          break;
        }
    }
  }
  spos[j] = pos;
  __syncthreads();
  for (int off = KB_MAXP / 2; off > 0; off >>= 1) {
    if (j < off) spos[j] = min(spos[j], spos[j + off]);
    __syncthreads();
  }
  const int64_t istar = spos[0];
  const int64_t last = (istar == INT64_MAX) ? n - 1 : istar;   // choices in [start, last] are final
  if (j < p) {
    // counts of the final choices in [start, last]
    int64_t cnt = 0;
    const int64_t bl = last / KB_BLOCK;
    for (int64_t b = start / KB_BLOCK; b < bl; ++b) cnt += bc[b * p + j];
    for (int64_t i = max(start, bl * KB_BLOCK); i <= last; ++i) cnt += (MB[i] == j);
    cs[j] += (int32_t)cnt;
  }
  __syncthreads();
  if (j == 0) {
    if (istar == INT64_MAX || istar + 1 >= n) {
      st[1] = 1;
    } else {
      full[MB[istar]] = 1;
      st[0] = istar + 1;
    }
  }
}

// The same event step for p <= 16 centres with the whole workgroup: thread
// t = 16 j + q serves centre j and block slot q.  Blocks are taken 16 at a
// time; a 16-lane scan of their counts finds, per centre, the block in which
// it reaches its need (cap - cs[j]), and the first such block over the open
// centres holds the event.  Inside it, per-centre ranks of the block's
// choices (ballots per wave, wave totals in LDS) give the first point whose
// choice reaches its centre's need.  Result identical to k_kbal_event.
constexpr int KB_SMALLP = 16;
__global__ __launch_bounds__(KB_BLOCK) void k_kbal_event16(const int32_t* __restrict__ MB,
                                                           const int32_t* __restrict__ bc, int64_t nblk, int64_t n,
                                                           int p, int64_t cap, int32_t* __restrict__ cs,
                                                           int32_t* __restrict__ full, int64_t* __restrict__ st) {
  if (st[1]) return;
  __shared__ int64_t s_min[KB_BLOCK / 64];
  __shared__ int64_t s_cum[KB_SMALLP];     // per centre: choices in [start, event block)
  __shared__ int64_t s_need[KB_SMALLP];    // per centre: choices still needed to fill it (huge: closed)
  __shared__ int32_t s_wc[KB_BLOCK / 64][KB_SMALLP];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int j = t >> 4, q = t & 15;
  const int64_t start = st[0];
  const bool open = j < p && !full[j];
  const int64_t need = open ? cap - cs[j] : INT64_MAX / 2;
  if (q == 0) s_need[j] = need;
  // block-wide minimum of an int64 (every thread gets it)
  auto wg_min = [&](int64_t v) {
    for (int off = 32; off > 0; off >>= 1) v = min(v, (int64_t)__shfl_xor(v, off, 64));
    __syncthreads();
    if (lane == 0) s_min[wv] = v;
    __syncthreads();
    int64_t r = s_min[0];
    for (int w = 1; w < KB_BLOCK / 64; ++w) r = min(r, s_min[w]);
    return r;
  };
  // 1. the event block
  int64_t cum = 0, B = INT64_MAX;
  for (int64_t b = start / KB_BLOCK; b < nblk; b += 16) {
    const int64_t bb = b + q;
    const int64_t c = (j < p && bb < nblk) ? bc[bb * p + j] : 0;
    int64_t x = c;   // inclusive scan over the 16 slots of centre j
    for (int off = 1; off < 16; off <<= 1) {
      const int64_t y = __shfl_up(x, off, 16);
      if (q >= off) x += y;
    }
    const int64_t incl = cum + x, excl = incl - c;
    const bool reached = open && bb < nblk && excl < need && incl >= need;
    B = wg_min(reached ? bb : INT64_MAX);
    if (B != INT64_MAX) {
      if (bb == B && j < p) s_cum[j] = excl;   // the slot of block B: choices of j in [start, B)
      break;
    }
    cum += __shfl(x, 15, 16);
  }
  if (B == INT64_MAX) {
    // no centre fills: every remaining choice is final
    if (q == 0 && j < p) cs[j] += (int32_t)cum;
    if (t == 0) st[1] = 1;
    return;
  }
  __syncthreads();
  // 2. inside block B: point i = 256 B + t, its choice jt
  const int64_t i = B * KB_BLOCK + t;
  const int jt = (i >= start && i < n) ? MB[i] : -1;
  for (int jj = 0; jj < p; ++jj) {
    const uint64_t m = __ballot(jt == jj);
    if (lane == 0) s_wc[wv][jj] = __popcll(m);
  }
  __syncthreads();
  int64_t cand = INT64_MAX;
  {
    // rank of point i among the choices of its centre in [start, i]
    int64_t rank = 0;
    for (int jj = 0; jj < p; ++jj) {
      const uint64_t m = __ballot(jt == jj);
      if (jt == jj) {
        rank = __popcll(m & ((2ull << lane) - 1));
        for (int w = 0; w < wv; ++w) rank += s_wc[w][jj];
      }
    }
    if (jt >= 0 && s_cum[jt] + rank == s_need[jt]) cand = i;
  }
  const int64_t istar = wg_min(cand);   // exists: some centre fills inside B
  // 3. final choices in [start, istar]: the counts before B plus those in B up to istar
  for (int jj = 0; jj < p; ++jj) {
    const uint64_t m = __ballot(jt == jj && i <= istar);
    if (lane == 0) s_wc[wv][jj] = __popcll(m);
  }
  __syncthreads();
  if (t < p) {
    int64_t c = s_cum[t];
    for (int w = 0; w < KB_BLOCK / 64; ++w) c += s_wc[w][t];
    cs[t] += (int32_t)c;
  }
  if (t == 0) {
    if (istar + 1 >= n) {
      st[1] = 1;
    } else {
      full[MB[istar]] = 1;
      st[0] = istar + 1;
    }
  }
}

__global__ void k_kbal_init(int32_t* __restrict__ cs, int32_t* __restrict__ full, int p, int64_t* __restrict__ st) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < p) {
    cs[j] = 0;
    full[j] = 0;
  }
  if (j == 0) {
    st[0] = 0;
    st[1] = 0;
  }
}

__global__ void k_fill_i32(int32_t* __restrict__ a, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_cast_rows(const void* __restrict__ X, int dtype, const int32_t* __restrict__ perm,
                            int64_t n, int d, void* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * d) return;
  const int64_t r = e / d, k = e - r * d;
  const int64_t src = (int64_t)perm[r] * d + k;
  if (dtype == KRR_F64)
    reinterpret_cast<double*>(out)[e] = reinterpret_cast<const double*>(X)[src];
  else
    reinterpret_cast<float*>(out)[e] = reinterpret_cast<const float*>(X)[src];
}

__global__ void k_gather_vec(const void* __restrict__ y, int dtype, const int32_t* __restrict__ perm,
                             int64_t n, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int64_t src = perm[e];
  out[e] = (dtype == KRR_F64) ? reinterpret_cast<const double*>(y)[src]
                              : (double)reinterpret_cast<const float*>(y)[src];
}

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): state advances by the golden
// gamma; the output mixes the state with two xor-shift-multiply rounds.
struct SplitMix64 {
  uint64_t state;
  uint64_t next() {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }
};

// DC-KRR divide step (Algorithm 3): the rows are shuffled and handed out
// evenly.  The shuffle is a keyed pseudo-random permutation that every point
// evaluates on its own: a balanced Feistel network of SHUFFLE_ROUNDS rounds on
// 2h-bit values (2^2h >= n), round r mapping (L, R) to (R, L xor F_r(R)) with
// F_r(R) = the low h bits of the SplitMix64 output function of K_r + R (K_r =
// the r-th SplitMix64 output of the seed), restricted to [0, n) by
// cycle-walking (Black and Rogaway, CT-RSA 2002): an image outside [0, n) is
// mapped again.  The walk ends because the point's own cycle returns to it.
// Shuffled row pos belongs to partition j = ceil((pos + 1) p / n) - 1, i.e.
// floor(j n / p) <= pos < floor((j + 1) n / p).
constexpr int SHUFFLE_ROUNDS = 8;
struct ShuffleKeys {
  uint64_t k[SHUFFLE_ROUNDS];
};

__device__ __forceinline__ uint64_t splitmix_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_random_assign(int64_t n, int p, int h, const ShuffleKeys K,
                                                       int32_t* __restrict__ assign) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t mask = (1ull << h) - 1ull;
  uint64_t v = (uint64_t)i;
  do {
    uint64_t left = v >> h, right = v & mask;
#pragma unroll
    for (int r = 0; r < SHUFFLE_ROUNDS; ++r) {
      const uint64_t t = left ^ (splitmix_out(K.k[r] + right) & mask);
      left = right;
      right = t;
    }
    v = (left << h) | right;
  } while (v >= (uint64_t)n);
  assign[i] = (int32_t)((((int64_t)v + 1) * p + n - 1) / n - 1);
}

template <typename TX>
void assign_t(krr_ctx ctx, hipStream_t s, const TX* X, int64_t n, int d, const double* CT, int p,
              int32_t* out, double* D, const int32_t* prev, int32_t* delta, const int32_t* skip,
              bool all) {
  // 64 rows per block staged in LDS (plus a spare slot); very wide rows use the unstaged kernel
  const size_t lds = ((size_t)d * (AROWS + 1) + 1) * sizeof(TX);
  const size_t lds_ct = ((lds + 15) & ~size_t(15)) + (size_t)p * d * sizeof(double);   // with the centres
  const int64_t nblk = ceil_div(n, AROWS);
  KernelTimer kt(ctx, s, "assign", 0.0, 0);
  if (lds_ct <= 48 * 1024) {
    if (all)
      hipLaunchKernelGGL((k_assign<TX, 1, true>), dim3(nblk), dim3(256), lds_ct, s, X, n, d, CT, p, out, D, prev,
                         delta, skip);
    else
      hipLaunchKernelGGL((k_assign<TX, 0, true>), dim3(nblk), dim3(256), lds_ct, s, X, n, d, CT, p, out, D, prev,
                         delta, skip);
  } else if (lds <= 96 * 1024) {
    if (all)
      hipLaunchKernelGGL((k_assign<TX, 1, false>), dim3(nblk), dim3(256), lds, s, X, n, d, CT, p, out, D, prev,
                         delta, skip);
    else
      hipLaunchKernelGGL((k_assign<TX, 0, false>), dim3(nblk), dim3(256), lds, s, X, n, d, CT, p, out, D, prev,
                         delta, skip);
  } else {
    const int64_t nb = ceil_div(n, 256);
    if (all)
      hipLaunchKernelGGL((k_assign_wide<TX, 1>), dim3(nb), dim3(256), 0, s, X, n, d, CT, p, out, D, prev,
                         delta, skip);
    else
      hipLaunchKernelGGL((k_assign_wide<TX, 0>), dim3(nb), dim3(256), 0, s, X, n, d, CT, p, out, D, prev,
                         delta, skip);
  }
  check_launch(ctx, s, "assign");
}

template <typename TX>
void means_t(krr_ctx ctx, hipStream_t s, const TX* X, int d, const int32_t* perm, const int64_t* offsets,
             double* C, double* CT, int p, const int32_t* skip, const int32_t* delta, int32_t* done_next) {
  KernelTimer kt(ctx, s, "lloyd_means", 0.0, 0);
  constexpr int NL = ExactSum<TX>::NL;
  const int nsl = (int)ceil_div(d, MS_W);
  // row splits: about 1,024 workgroups in all
  const int rs = (int)std::max<int64_t>(1, std::min<int64_t>(64, ceil_div(1024, (int64_t)p * nsl)));
  int64_t* P = (int64_t*)ws_get(ctx, "means_part", (size_t)p * nsl * rs * MS_W * NL * sizeof(int64_t));
  hipLaunchKernelGGL((k_means_acc<TX>), dim3((unsigned)(p * nsl * rs)), dim3(MeansCfg<TX>::THREADS), 0, s, X, d, nsl,
                     rs, perm, offsets, P, skip);
  check_launch(ctx, s, "means_acc");
  hipLaunchKernelGGL((k_means_round<TX>), dim3((unsigned)ceil_div((int64_t)p * d, RoundCfg<TX>::PAIRS)), dim3(256), 0,
                     s, d, nsl, rs, p, offsets, (const int64_t*)P, C, CT, skip, delta, done_next);
  check_launch(ctx, s, "means_round");
}

template <typename TX>
void kmeanspp_t(krr_ctx ctx, hipStream_t s, const TX* X, int64_t n, int d, int k, uint64_t seed,
                double* C) {
  const int64_t nblk = ceil_div(n, KPP_BLOCK);
  char* w = (char*)ws_get(ctx, "kpp", (size_t)(3 * n + 2 * nblk + 8) * 8 + (size_t)k * 8);
  double* D2 = (double*)w;
  double* P = D2 + n;
  double* Tb = P + n;
  double* Ob = Tb + nblk;
  int64_t* cidx = (int64_t*)(Ob + nblk + 8);
  KernelTimer kt(ctx, s, "kmeanspp", 0.0, 0);
  SplitMix64 g{seed};
  std::vector<double> u(k);
  for (int t = 0; t < k; ++t) u[t] = g.uniform();
  hipLaunchKernelGGL((k_kpp_first<TX>), dim3(1), dim3(128), 0, s, n, u[0], X, d, cidx, C);
  check_launch(ctx, s, "kpp_first");
  for (int t = 1; t < k; ++t) {
    hipLaunchKernelGGL((k_kpp_update<TX>), dim3(nblk), dim3(KPP_BLOCK), 0, s, X, n, d,
                       (const int64_t*)cidx, t - 1, D2, P, Tb);
    check_launch(ctx, s, "kpp_update");
    const bool lds = nblk <= KPP_MAXBLK;
    hipLaunchKernelGGL((k_kpp_select<TX>), dim3(1), dim3(KPP_BLOCK), lds ? (size_t)nblk * 8 : 0, s,
                       (const double*)P, (const double*)Tb, nblk, n, u[t], X, d, cidx, t, C, lds ? nullptr : Ob);
    check_launch(ctx, s, "kpp_select");
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host entry points used by the other modules
// ---------------------------------------------------------------------------
void transpose_centroids(krr_ctx ctx, hipStream_t s, const double* C, int p, int d, double* CT) {
  const int tot = p * d;
  hipLaunchKernelGGL(k_transpose, dim3(ceil_div(tot, 256)), dim3(256), 0, s, C, p, d, CT);
  check_launch(ctx, s, "transpose");
}

void assign_nearest(krr_ctx ctx, hipStream_t s, const void* X, int dtype, int64_t n, int d,
                    const double* CT, int p, int32_t* out, const int32_t* prev, int32_t* delta,
                    const int32_t* skip) {
  if (dtype == KRR_F64)
    assign_t(ctx, s, (const double*)X, n, d, CT, p, out, nullptr, prev, delta, skip, false);
  else
    assign_t(ctx, s, (const float*)X, n, d, CT, p, out, nullptr, prev, delta, skip, false);
}

size_t group_ws_bytes(int64_t n, int p) { return (size_t)n * 4 + (size_t)ceil_div(n, GROUP_BLOCK) * p * 8 + 64; }

void group_by_key(krr_ctx ctx, hipStream_t s, const int32_t* key, int64_t n, int p, int32_t* perm,
                  int64_t* offsets, int64_t* sizes64, const int32_t* skip, void* wsp) {
  const int64_t nblk = ceil_div(n, GROUP_BLOCK);
  KernelTimer kt(ctx, s, "group", 0.0, 0);
  char* w = wsp != nullptr ? (char*)wsp : (char*)ws_get(ctx, "group", group_ws_bytes(n, p));
  int32_t* rank = (int32_t*)w;
  int32_t* bc = rank + n;
  int32_t* bo = bc + nblk * p;
  hipLaunchKernelGGL(k_group_local, dim3(nblk), dim3(GROUP_BLOCK), (size_t)(GROUP_BLOCK / 64) * p * 4, s, key, n, p,
                     rank, bc,
                     skip);
  check_launch(ctx, s, "group_local");
  hipLaunchKernelGGL(k_group_scan, dim3(1), dim3(std::min(1024, 64 * p)), (size_t)p * 8, s,
                     (const int32_t*)bc, nblk, p, bo, offsets, sizes64, skip);
  check_launch(ctx, s, "group_scan");
  hipLaunchKernelGGL(k_group_scatter, dim3(nblk), dim3(GROUP_BLOCK), 0, s, key, n, p, (const int32_t*)rank,
                     (const int32_t*)bo, (const int64_t*)offsets, perm, skip);
  check_launch(ctx, s, "group_scatter");
}

void gather_rows(krr_ctx ctx, hipStream_t s, const void* X, int dtype, int64_t n, int d,
                 const int32_t* perm, void* Xout) {
  const int64_t tot = n * d;
  hipLaunchKernelGGL(k_cast_rows, dim3(ceil_div(tot, 256)), dim3(256), 0, s, X, dtype, perm, n, d, Xout);
  check_launch(ctx, s, "gather_rows");
}

void gather_vec_f64(krr_ctx ctx, hipStream_t s, const void* y, int dtype, int64_t n, const int32_t* perm,
                    double* yout) {
  hipLaunchKernelGGL(k_gather_vec, dim3(ceil_div(n, 256)), dim3(256), 0, s, y, dtype, perm, n, yout);
  check_launch(ctx, s, "gather_vec");
}

template <typename TX>
static void partition_t(krr_ctx ctx, hipStream_t s, const TX* X, int64_t n, int d, int p, int method,
                        int iters, uint64_t seed, double* C, int32_t* assign, int64_t* sizes) {
  double* CT = (double*)ws_get(ctx, "part_ct", (size_t)p * d * 8);
  if (method == KRR_PART_RANDOM) {
    // Algorithm 3: shuffled even split; centres = member means (for routing)
    ShuffleKeys K;
    SplitMix64 g{seed};
    for (int r = 0; r < SHUFFLE_ROUNDS; ++r) K.k[r] = g.next();
    int b = 2;
    while ((int64_t(1) << b) < n) b += 2;
    hipLaunchKernelGGL(k_random_assign, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, n, p, b / 2, K, assign);
    check_launch(ctx, s, "random_assign");
    char* w = (char*)ws_get(ctx, "rand_perm", (size_t)n * 4 + (size_t)(p + 1) * 8 + 16);
    int32_t* perm = (int32_t*)w;
    int64_t* off = (int64_t*)(perm + n + (n & 1));
    group_by_key(ctx, s, assign, n, p, perm, off, nullptr, nullptr);
    means_t(ctx, s, X, d, perm, off, C, nullptr, p, nullptr, nullptr, nullptr);
  } else if (method == KRR_PART_GIVEN) {
    transpose_centroids(ctx, s, C, p, d, CT);
    assign_t(ctx, s, X, n, d, CT, p, assign, nullptr, nullptr, nullptr, nullptr, false);
  } else {
    // K-means: k-means++ seeding then Lloyd passes (Algorithm 2).
    kmeanspp_t(ctx, s, X, n, d, p, seed, C);
    char* w = (char*)ws_get(ctx, "lloyd", (size_t)n * 8 + (size_t)(p + 1) * 8 + (size_t)(2 * iters + 4) * 4 + 64);
    int32_t* perm = (int32_t*)w;
    int32_t* prev = perm + n;
    int64_t* off = (int64_t*)(prev + n + (n & 1));
    int32_t* deltas = (int32_t*)(off + p + 1);
    int32_t* done = deltas + iters + 1;   // done[it]: pass `it` is past the fixed point
    const int64_t nflags = 2 * (int64_t)iters + 3;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)ceil_div(nflags, 64)), dim3(64), 0, s, deltas, nflags, 0);
    check_launch(ctx, s, "fill");
    int32_t* cur = assign;
    int32_t* old = prev;
    // the mean step writes CT beside C, so only the seeds need a transpose
    transpose_centroids(ctx, s, C, p, d, CT);
    for (int it = 0; it < iters; ++it) {
      assign_t(ctx, s, X, n, d, CT, p, cur, nullptr, it == 0 ? nullptr : old, deltas + it, done + it, false);
      group_by_key(ctx, s, cur, n, p, perm, off, nullptr, done + it);
      means_t(ctx, s, X, d, perm, off, C, CT, p, done + it, deltas + it, done + it + 1);
      std::swap(cur, old);
    }
    assign_t(ctx, s, X, n, d, CT, p, assign, nullptr, nullptr, nullptr, nullptr, false);
    if (method == KRR_PART_KBALANCE || method == KRR_PART_KBALANCE_APPROX) {
      // Greedy capacity pass over the exact distances to the K-means centres,
      // then the centre recompute of Algorithm 4 (approximate parallel
      // variant: one independent pass per even segment of the samples).
      double* D = (double*)ws_get(ctx, "kbal_d", (size_t)n * p * 8);
      assign_t(ctx, s, X, n, d, CT, p, nullptr, D, nullptr, nullptr, nullptr, true);
      const int32_t* a0 = assign;  // unconstrained nearest centres
      int32_t* MB = prev;
      const int64_t cap = ceil_div(n, p);
      KernelTimer kt(ctx, s, "kbalance_greedy", 0.0, 0);
      if (method == KRR_PART_KBALANCE_APPROX) {
        hipLaunchKernelGGL(k_kbalance, dim3((unsigned)p), dim3(64), (size_t)p * 8, s, (const double*)D, a0, n, p, p,
                           (int64_t)0, MB);
        check_launch(ctx, s, "kbalance_segments");
      } else if (p <= KB_MAXP) {
        const int64_t nblk = ceil_div(n, KB_BLOCK);
        char* kw = (char*)ws_get(ctx, "kbal_ev", (size_t)nblk * p * 4 + (size_t)p * 8 + 64);
        int64_t* kst = (int64_t*)kw;
        int32_t* cs = (int32_t*)(kw + 16);
        int32_t* full = cs + p;
        int32_t* bc = full + p;
        hipLaunchKernelGGL(k_kbal_init, dim3((unsigned)ceil_div(p, 256)), dim3(256), 0, s, cs, full, p, kst);
        check_launch(ctx, s, "kbal_init");
        for (int round = 0; round <= p; ++round) {
          hipLaunchKernelGGL(k_kbal_choose, dim3((unsigned)nblk), dim3(KB_BLOCK), (size_t)p * 4, s, (const double*)D,
                             n, p, (const int32_t*)full, (const int64_t*)kst, MB, bc);
          check_launch(ctx, s, "kbal_choose");
          if (p <= KB_SMALLP)
            hipLaunchKernelGGL(k_kbal_event16, dim3(1), dim3(KB_BLOCK), 0, s, (const int32_t*)MB, (const int32_t*)bc,
                               nblk, n, p, cap, cs, full, kst);
          else
            hipLaunchKernelGGL(k_kbal_event, dim3(1), dim3(KB_MAXP), 0, s, (const int32_t*)MB, (const int32_t*)bc,
                               nblk, n, p, cap, cs, full, kst);
          check_launch(ctx, s, "kbal_event");
        }
      } else {
        hipLaunchKernelGGL(k_kbalance, dim3(1), dim3(64), (size_t)p * 8, s, (const double*)D, a0, n, p, 1, cap, MB);
        check_launch(ctx, s, "kbalance");
      }
      KRR_HIP(hipMemcpyAsync(assign, MB, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
      group_by_key(ctx, s, assign, n, p, perm, off, nullptr, nullptr);
      means_t(ctx, s, X, d, perm, off, C, nullptr, p, nullptr, nullptr, nullptr);
    }
  }
  // sizes: histogram of the final assignment
  int32_t* perm2 = (int32_t*)ws_get(ctx, "part_perm", (size_t)n * 4 + (size_t)(p + 1) * 8 + 16);
  int64_t* off2 = (int64_t*)(perm2 + n + (n & 1));
  group_by_key(ctx, s, assign, n, p, perm2, off2, sizes, nullptr);
}

void run_partition(krr_ctx ctx, hipStream_t s, const void* X, int dtype, int64_t n, int d, int p, int method,
                   int iters, uint64_t seed, double* C, int32_t* assign, int64_t* sizes) {
  if (dtype == KRR_F64)
    partition_t(ctx, s, (const double*)X, n, d, p, method, iters, seed, C, assign, sizes);
  else
    partition_t(ctx, s, (const float*)X, n, d, p, method, iters, seed, C, assign, sizes);
}

}  // namespace krr
