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
//
// The Gaussian-bump tensor of Section 4.4,
//     X(i) = sum_j exp(-gamma sum_q (x_q - c_{j,q})^2),   x_q = 2 i_q / n_q - 1,
// is a sum of products of one factor per mode, e_q(i_q, j) =
// exp(-gamma (x_q - c_{j,q})^2).  On X_m that is X(row, col) = sum_j
// a(row, j) b(col, j) with a = e_1(i_1, j) h(row / n_1, j), h the product of
// the factors of modes 2..m and b that of modes m+1..d.  The three tables are
// small (N (n_1 + R_m / n_1 + C_m) doubles); gauss_columns evaluates chunks of
// whole columns of X_m from them into a workspace that the memory kernels
// stream, at 2N FP64 flops per entry.
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

// out[j * cnt + f] = prod over modes q0..q1-1 of exp(-gamma (x_q - c_{j,q})^2), f a flat
// index over those modes (first fastest), x_q = 2 (i_q + 1) / n_q - 1 (0-based i_q)
__global__ void k_gauss_table(const Modes M, int q0, int q1, int64_t cnt, int64_t stride, const double* __restrict__ ctr,
                              int d, int nterms, double gamma, double* __restrict__ out) {
  const int64_t tot = cnt * nterms;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(t / cnt);
    int64_t f = t % cnt;
    double v = 1.0;
    for (int q = q0; q < q1; ++q) {
      const int64_t i = f % M.n[q];
      f /= M.n[q];
      const double x = 2.0 * (double)(i + 1) / (double)M.n[q] - 1.0;
      const double dl = x - ctr[(int64_t)j * d + q];
      v *= exp(-gamma * (dl * dl));
    }
    out[(int64_t)j * stride + t % cnt] = v;
  }
}

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) p[t] = v;
}

constexpr int kGaussBlock = 256;   // threads per workgroup of k_gauss_cols

// W(row, c) = sum_j a(row, j) b(c0 + c, j) for the columns [c0, c0 + nc) of X_m
// (W is R_m x nc, column-major).  A thread owns two rows (kGaussBlock apart)
// and kGaussCols columns: a row's a(row, j) is two lane-contiguous loads, the
// columns' b(col, j) are the same for the whole wave (uniform loads, each
// feeding both rows), and each j costs 2 kGaussCols FMAs.  The bumps are added
// in increasing j.
template <typename T>
__global__ __launch_bounds__(kGaussBlock) void k_gauss_cols(const GaussTabs g, int64_t c0, int64_t nc, T* __restrict__ W) {
  constexpr int CB = kGaussCols;
  const int64_t r0 = blockIdx.x * (int64_t)(2 * kGaussBlock) + threadIdx.x;
  const int64_t cb = c0 + (int64_t)blockIdx.y * CB;
  const int ncb = (int)std::min<int64_t>(CB, c0 + nc - cb);
  if (r0 >= g.R) return;
  // the second row is clamped into the matrix and dropped at the store
  const bool two = r0 + kGaussBlock < g.R;
  const int64_t r1 = two ? r0 + kGaussBlock : r0;
  const double* __restrict__ e1a = g.e1 + r0 % g.n1;
  const double* __restrict__ aha = g.ahi + r0 / g.n1;
  const double* __restrict__ e1b = g.e1 + r1 % g.n1;
  const double* __restrict__ ahb = g.ahi + r1 / g.n1;
  const double* __restrict__ bc = g.bc + cb;   // columns past C read the table's zero padding
  double acc0[CB], acc1[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) acc0[c] = acc1[c] = 0.0;
  for (int j = 0; j < g.nterms; ++j) {
    const double a0 = e1a[(int64_t)j * g.n1] * aha[(int64_t)j * g.rhi];
    const double a1 = e1b[(int64_t)j * g.n1] * ahb[(int64_t)j * g.rhi];
    const double* __restrict__ b = bc + (int64_t)j * g.bstride;
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      acc0[c] += a0 * b[c];
      acc1[c] += a1 * b[c];
    }
  }
  T* w0 = W + (cb - c0) * g.R + r0;
  T* w1 = W + (cb - c0) * g.R + r1;
#pragma unroll
  for (int c = 0; c < CB; ++c)
    if (c < ncb) {
      w0[(int64_t)c * g.R] = (T)acc0[c];
      if (two) w1[(int64_t)c * g.R] = (T)acc1[c];
    }
}

// W(row, c) = rec[row_t[row] + col_t[c0 + c]] for the columns [c0, c0 + nc) of X_m
template <typename T>
__global__ void k_hilbert_cols(const double* __restrict__ rec, const int32_t* __restrict__ row_t,
                               const int32_t* __restrict__ col_t, int64_t R, int64_t c0, int64_t nc,
                               T* __restrict__ W) {
  const int64_t tot = R * nc;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x)
    W[t] = (T)rec[row_t[t % R] + col_t[c0 + t / R]];
}

unsigned grid1(int64_t work) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 4096));
}

}  // namespace

int64_t gauss_table_doubles(const int64_t* n, int d, int m, int nterms) {
  int64_t R = 1, C = 1;
  for (int q = 0; q < m; ++q) R *= n[q];
  for (int q = m; q < d; ++q) C *= n[q];
  return (int64_t)nterms * (d + n[0] + R / n[0] + C + kGaussCols);
}

hipError_t gauss_tables(const int64_t* n, int d, int m, const double* centers_host, int nterms, double gamma,
                        double* buf, GaussTabs* out, hipStream_t s) {
  if (fault_take()) return hipErrorLaunchFailure;
  Modes M;
  for (int q = 0; q < PSTT2_MAX_D; ++q) M.n[q] = q < d ? n[q] : 1;
  int64_t R = 1, C = 1;
  for (int q = 0; q < m; ++q) R *= n[q];
  for (int q = m; q < d; ++q) C *= n[q];
  GaussTabs g;
  g.nterms = nterms;
  g.n1 = n[0];
  g.rhi = R / n[0];
  g.R = R;
  g.C = C;
  g.bstride = C + kGaussCols;
  double* ctr = buf;
  double* e1 = ctr + (int64_t)nterms * d;
  double* ahi = e1 + (int64_t)nterms * g.n1;
  double* bc = ahi + (int64_t)nterms * g.rhi;
  g.e1 = e1;
  g.ahi = ahi;
  g.bc = bc;
  // the centers are read by the kernels below only; copy them and wait, so the
  // caller's host array may go as soon as this returns
  hipError_t e = hipMemcpyAsync(ctr, centers_host, sizeof(double) * nterms * d, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gauss_table, dim3(grid1(g.n1 * nterms)), dim3(256), 0, s, M, 0, 1, g.n1, g.n1, ctr, d,
                     nterms, gamma, e1);
  hipLaunchKernelGGL(k_gauss_table, dim3(grid1(g.rhi * nterms)), dim3(256), 0, s, M, 1, m, g.rhi, g.rhi, ctr, d,
                     nterms, gamma, ahi);
  hipLaunchKernelGGL(k_fill, dim3(grid1(g.bstride * nterms)), dim3(256), 0, s, bc, g.bstride * nterms, 0.0);
  hipLaunchKernelGGL(k_gauss_table, dim3(grid1(C * nterms)), dim3(256), 0, s, M, m, d, C, g.bstride, ctr, d, nterms,
                     gamma, bc);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  *out = g;
  return hipStreamSynchronize(s);
}

int64_t gauss_chunk_cols(const GaussTabs& g, int elem_bytes) {
  int64_t by_bytes = std::max<int64_t>(1, PSTT2_GAUSS_CHUNK_BYTES / (g.R * elem_bytes));
  if (by_bytes > kGaussCols) by_bytes -= by_bytes % kGaussCols;   // whole column blocks
  const int64_t by_grid = (int64_t)65535 * kGaussCols;
  return std::min(std::min(by_bytes, by_grid), g.C);
}

hipError_t gauss_columns(const GaussTabs& g, int64_t c0, int64_t nc, int dtype, void* W, hipStream_t s) {
  if (nc <= 0) return hipSuccess;
  if (fault_take()) return hipErrorLaunchFailure;
  const dim3 grid((unsigned)((g.R + 2 * kGaussBlock - 1) / (2 * kGaussBlock)),
                  (unsigned)((nc + kGaussCols - 1) / kGaussCols));
  if (dtype == PSTT2_F64)
    hipLaunchKernelGGL(k_gauss_cols<double>, grid, dim3(kGaussBlock), 0, s, g, c0, nc, (double*)W);
  else
    hipLaunchKernelGGL(k_gauss_cols<float>, grid, dim3(kGaussBlock), 0, s, g, c0, nc, (float*)W);
  return hipGetLastError();
}

hipError_t hilbert_columns(const double* rec, const int32_t* row_t, const int32_t* col_t, int64_t R, int64_t c0,
                           int64_t nc, int dtype, void* W, hipStream_t s) {
  if (nc <= 0) return hipSuccess;
  if (fault_take()) return hipErrorLaunchFailure;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((R * nc + 255) / 256, 65536));
  if (dtype == PSTT2_F64)
    hipLaunchKernelGGL(k_hilbert_cols<double>, dim3(g), dim3(256), 0, s, rec, row_t, col_t, R, c0, nc, (double*)W);
  else
    hipLaunchKernelGGL(k_hilbert_cols<float>, dim3(g), dim3(256), 0, s, rec, row_t, col_t, R, c0, nc, (float*)W);
  return hipGetLastError();
}

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
