// Tensors given by a formula of their indices (the streaming setting of
// Section 4.2, where each sub-tensor comes from a function of its indices and
// is never stored as a whole).  The Hilbert tensor of Section 4.3 / Table 1,
//     X(i_1, ..., i_d) = 1 / (1 - d + i_1 + ... + i_d),   1 <= i_q <= n_q,
// depends on the indices only through their sum.  On the split X_m (rows =
// modes 1..m, columns = modes m+1..d) that sum is a row part plus a column
// part, so X(row, col) = rec[row_t[row] + col_t[col]] with
//     row_t[row] = 1 + sum of the row's 0-based mode indices,
//     col_t[col] = sum of the column's 0-based mode indices,
//     rec[k]     = 1 / k (FP64, correctly rounded).
// The sketch and error kernels read these three small tables instead of X.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace pstt2 {

namespace {

// 0-based mode indices of a flat index over modes q0 .. q1-1 (first fastest), summed
__device__ __forceinline__ int32_t digit_sum(int64_t f, const int64_t* n, int q0, int q1) {
  int32_t s = 0;
  for (int q = q0; q < q1; ++q) {
    s += (int32_t)(f % n[q]);
    f /= n[q];
  }
  return s;
}

struct Modes {
  int64_t n[PSTT2_MAX_D];
};

__global__ void k_hilbert_tables(const Modes M, int d, int m, int64_t R, int64_t C, int64_t K,
                                 double* __restrict__ rec, int32_t* __restrict__ row_t,
                                 int32_t* __restrict__ col_t) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t i = t0; i < R; i += stride) row_t[i] = 1 + digit_sum(i, M.n, 0, m);
  for (int64_t i = t0; i < C; i += stride) col_t[i] = digit_sum(i, M.n, m, d);
  for (int64_t k = t0; k < K; k += stride) rec[k] = k == 0 ? 0.0 : 1.0 / (double)k;
}

}  // namespace

hipError_t hilbert_tables(const int64_t* n, int d, int m, int64_t R, int64_t C, double* rec, int32_t* row_t,
                          int32_t* col_t, hipStream_t s) {
  Modes M;
  for (int q = 0; q < PSTT2_MAX_D; ++q) M.n[q] = q < d ? n[q] : 1;
  const int64_t K = hilbert_rec_len(n, d);
  const int64_t work = std::max(std::max(R, C), K);
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 4096));
  hipLaunchKernelGGL(k_hilbert_tables, dim3(g), dim3(256), 0, s, M, d, m, R, C, K, rec, row_t, col_t);
  return hipGetLastError();
}

}  // namespace pstt2
