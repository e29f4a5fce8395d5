// Sparse input: the n x d training or test matrix given in CSR (compressed
// sparse row) form, as the paper's implementation holds its input matrix
// (Section 5.5; Section 6 on very sparse data), expanded once into the dense
// row-major matrix that every other kernel of the library reads.  The
// kernel matrix itself is dense whatever the input, and HBM holds the dense
// n x d input of the workloads many times over, so the hot path stays on
// dense, coalesced rows.
#include "common.hpp"

namespace krr {

namespace {

constexpr int CSR_ROWS = 4;   // rows per 256-thread workgroup, one wave each

__global__ void k_csr_clear(int32_t* bad) { bad[0] = 0; }

// Row i = 4 blockIdx.x + wave: the wave zeroes the row, then lane 0 adds the
// row's entries in storage order (repeated columns summed in that order, in
// T).  A malformed row (pointers outside [0, nnz] or decreasing, the first
// pointer not 0, the last not nnz) or column outside [0, d) writes nothing
// of that entry or row and sets bit 1 or 2 of *bad.
template <typename T>
__global__ __launch_bounds__(256) void k_csr_rows(const int64_t* __restrict__ indptr,
                                                  const int32_t* __restrict__ indices,
                                                  const T* __restrict__ values, int64_t n, int d, int64_t nnz,
                                                  T* __restrict__ X, int32_t* __restrict__ bad) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * CSR_ROWS + (threadIdx.x >> 6);
  const bool live = i < n;
  T* row = X + (live ? i : 0) * d;
  if (live)
    for (int c = lane; c < d; c += 64) row[c] = T(0);
  __syncthreads();   // the zeros are visible to lane 0 before it adds
  if (!live || lane != 0) return;
  const int64_t b = indptr[i], e = indptr[i + 1];
  const bool ok = b >= 0 && b <= e && e <= nnz && (i != 0 || b == 0) && (i != n - 1 || e == nnz);
  if (!ok) {
    atomicOr(bad, 1);
    return;
  }
  for (int64_t k = b; k < e; ++k) {
    const int32_t c = indices[k];
    if (c < 0 || c >= d) {
      atomicOr(bad, 2);
      continue;
    }
    row[c] = row[c] + values[k];
  }
}

}  // namespace

void run_csr_to_dense(krr_ctx ctx, hipStream_t s, const int64_t* indptr, const int32_t* indices, const void* values,
                      int dtype, int64_t n, int d, int64_t nnz, void* X) {
  int32_t* bad = (int32_t*)ws_get(ctx, "csr_bad", 256);
  hipLaunchKernelGGL(k_csr_clear, dim3(1), dim3(1), 0, s, bad);
  check_launch(ctx, s, "csr_clear");
  const dim3 grid((unsigned)ceil_div(n, CSR_ROWS));
  if (dtype == KRR_F64)
    hipLaunchKernelGGL(k_csr_rows<double>, grid, dim3(64 * CSR_ROWS), 0, s, indptr, indices, (const double*)values,
                       n, d, nnz, (double*)X, bad);
  else
    hipLaunchKernelGGL(k_csr_rows<float>, grid, dim3(64 * CSR_ROWS), 0, s, indptr, indices, (const float*)values,
                       n, d, nnz, (float*)X, bad);
  check_launch(ctx, s, "csr_rows");
  int32_t* h = (int32_t*)pinned_get(ctx, 64);
  KRR_HIP(hipMemcpyAsync(h, bad, 4, hipMemcpyDeviceToHost, s));
  KRR_HIP(hipStreamSynchronize(s));
  KRR_REQUIRE(!(h[0] & 1), "malformed CSR row pointers (indptr must rise from 0 to nnz)");
  KRR_REQUIRE(!(h[0] & 2), "CSR column index outside [0, d)");
}

}  // namespace krr
