// Parallel-TTSVD (Section 3.1, Algorithm Parallel-TTSVD, Theorem perf_alg1):
// a truncated SVD of every unfolding X_k, then the cores from neighbouring
// left singular bases by equation "core".
//
// The SVD of an unfolding is taken by one-sided (Hestenes) Jacobi on its short
// side, directly on the data (no Gram matrix, so the singular values keep
// their relative accuracy): with s = min(R_k, C_k) and L = max(R_k, C_k), the
// work matrix W (L x s) is X_k^T when R_k <= C_k and X_k otherwise.  Pairs of
// columns are rotated until every pair is orthogonal to working precision; J
// (s x s) accumulates the rotations, so W J = W' has orthogonal columns whose
// norms are the singular values.  For W = X_k^T, J holds the left singular
// vectors of X_k; for W = X_k, they are the normalised columns of W'.
//
// Pairs follow the round-robin (circle) schedule: s - 1 rounds of s/2
// disjoint pairs (s padded to even with a zero column) meet every pair once
// per sweep; one launch per round, one workgroup per pair, sums in a fixed
// order, so results are bitwise repeatable.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace pstt2 {

namespace {
constexpr int kBS = 256;

// circle method: position 0 fixed, positions 1..s-1 rotate by one per round
__device__ __forceinline__ int rr_elem(int j, int k, int s) { return j == 0 ? 0 : 1 + (j - 1 + k) % (s - 1); }

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}
}  // namespace

// W (C x sp, column-major): W(c, r) = X_k(r, c) for r < R, zero columns r >= R.
// 32 x 32 tiles through LDS so both sides are read and written along rows.
__global__ void k_svd_transpose(const double* __restrict__ x, int64_t R, int64_t C, int sp, double* __restrict__ W) {
  __shared__ double t[32][33];
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
  for (int j = ty; j < 32; j += 8) {
    const int64_t r = r0 + tx, c = c0 + j;
    t[j][tx] = (r < R && c < C) ? x[r + R * c] : 0.0;
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int64_t c = c0 + tx, r = r0 + j;
    if (c < C && r < sp) W[c + C * r] = t[tx][j];
  }
}

// W (R x sp): a copy of X_k with zero columns past C.
__global__ void k_svd_copy(const double* __restrict__ x, int64_t R, int64_t C, int sp, double* __restrict__ W) {
  const int64_t tot = R * sp;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x)
    W[t] = t < R * C ? x[t] : 0.0;
}

// One round of the schedule: workgroup i rotates its pair (p, q) of W's and
// J's columns when they are not yet orthogonal (|w_p . w_q| > tol ||w_p|| ||w_q||).
__global__ __launch_bounds__(kBS) void k_jacobi_round(double* __restrict__ W, int64_t L, double* __restrict__ J,
                                                      int sp, int k, double tol, int* __restrict__ rotations) {
  __shared__ double red[kBS / 64];
  const int i = blockIdx.x;
  const int p = rr_elem(i, k, sp), q = rr_elem(sp - 1 - i, k, sp);
  double* wp = W + (int64_t)p * L;
  double* wq = W + (int64_t)q * L;
  double a = 0.0, b = 0.0, g = 0.0;
  for (int64_t t = threadIdx.x; t < L; t += kBS) {
    const double u = wp[t], v = wq[t];
    a += u * u;
    b += v * v;
    g += u * v;
  }
  a = block_sum(a, red);
  b = block_sum(b, red);
  g = block_sum(g, red);
  if (!(g != 0.0 && fabs(g) > tol * sqrt(a * b))) return;   // uniform across the workgroup
  // tan of the rotation angle that zeroes the off-diagonal entry of [[a, g], [g, b]]
  const double z = (b - a) / (2.0 * g);
  const double t = (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
  const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
  for (int64_t e = threadIdx.x; e < L; e += kBS) {
    const double u = wp[e], v = wq[e];
    wp[e] = c * u - s * v;
    wq[e] = s * u + c * v;
  }
  double* jp = J + (int64_t)p * sp;
  double* jq = J + (int64_t)q * sp;
  for (int e = threadIdx.x; e < sp; e += kBS) {
    const double u = jp[e], v = jq[e];
    jp[e] = c * u - s * v;
    jq[e] = s * u + c * v;
  }
  if (threadIdx.x == 0) atomicAdd(rotations, 1);
}

// sig[j] = ||W(:, j)||, one workgroup per column
__global__ __launch_bounds__(kBS) void k_svd_colnorm(const double* __restrict__ W, int64_t L,
                                                     double* __restrict__ sig) {
  __shared__ double red[kBS / 64];
  const double* w = W + (int64_t)blockIdx.x * L;
  double a = 0.0;
  for (int64_t t = threadIdx.x; t < L; t += kBS) a += w[t] * w[t];
  a = block_sum(a, red);
  if (threadIdx.x == 0) sig[blockIdx.x] = sqrt(a);
}

// dst (rows x r): dst(:, a) = src(:, idx[a]) / (sig ? sig[idx[a]] : 1), src with
// leading dimension ld.  A kept column with a zero singular value (X = 0) has no
// direction of its own: it becomes the unit vector e_a.
__global__ void k_svd_gather(const double* __restrict__ src, int64_t ld, int64_t rows, const int* __restrict__ idx,
                             const double* __restrict__ sig, int r, double* __restrict__ dst) {
  const int64_t tot = rows * r;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(t / rows);
    const int64_t row = t % rows;
    const int j = idx[a];
    if (!sig) dst[t] = src[(int64_t)j * ld + row];
    else dst[t] = sig[j] > 0.0 ? src[(int64_t)j * ld + row] / sig[j] : (row == a ? 1.0 : 0.0);
  }
}

// Last core G_d = Sigma_{d-1} V_{d-1}^T (r x n_d, column-major).  From J (the
// right singular vectors when W = X_{d-1}): G(a, i) = sig[idx a] J(i, idx a).
// From W' (when W = X_{d-1}^T, W' = X_{d-1}^T U): G(a, i) = W'(i, idx a).
__global__ void k_svd_last_core(const double* __restrict__ src, int64_t ld, const int* __restrict__ idx,
                                const double* __restrict__ sig, int r, int nd, double* __restrict__ G) {
  const int64_t tot = (int64_t)r * nd;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(t % r);
    const int i = (int)(t / r);
    const int j = idx[a];
    G[t] = src[(int64_t)j * ld + i] * (sig ? sig[j] : 1.0);
  }
}

__global__ void k_svd_eye(double* __restrict__ J, int sp, int* __restrict__ counter) {
  const int64_t tot = (int64_t)sp * sp;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x)
    J[t] = (t % sp) == (t / sp) ? 1.0 : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
}

__global__ void k_zero_int(int* p) { *p = 0; }

static unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

hipError_t svd_load(const double* x, int64_t R, int64_t C, int sp, double* W, hipStream_t s) {
  if (R <= C) {
    const dim3 g((unsigned)((C + 31) / 32), (unsigned)((sp + 31) / 32));
    hipLaunchKernelGGL(k_svd_transpose, g, dim3(256), 0, s, x, R, C, sp, W);
  } else {
    hipLaunchKernelGGL(k_svd_copy, dim3(grid_of(R * sp)), dim3(256), 0, s, x, R, C, sp, W);
  }
  return hipGetLastError();
}

hipError_t svd_init(double* J, int sp, int* counter, hipStream_t s) {
  hipLaunchKernelGGL(k_svd_eye, dim3(grid_of((int64_t)sp * sp)), dim3(256), 0, s, J, sp, counter);
  return hipGetLastError();
}

hipError_t svd_sweep(double* W, int64_t L, double* J, int sp, double tol, int* counter, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s, counter);
  for (int k = 0; k < sp - 1; ++k)
    hipLaunchKernelGGL(k_jacobi_round, dim3((unsigned)(sp / 2)), dim3(kBS), 0, s, W, L, J, sp, k, tol, counter);
  return hipGetLastError();
}

hipError_t svd_colnorms(const double* W, int64_t L, int scols, double* sig, hipStream_t s) {
  hipLaunchKernelGGL(k_svd_colnorm, dim3((unsigned)scols), dim3(kBS), 0, s, W, L, sig);
  return hipGetLastError();
}

hipError_t svd_gather(const double* src, int64_t ld, int64_t rows, const int* idx, const double* sig, int r,
                      double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_svd_gather, dim3(grid_of(rows * r)), dim3(256), 0, s, src, ld, rows, idx, sig, r, dst);
  return hipGetLastError();
}

hipError_t svd_last_core(const double* src, int64_t ld, const int* idx, const double* sig, int r, int nd, double* G,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_svd_last_core, dim3(grid_of((int64_t)r * nd)), dim3(256), 0, s, src, ld, idx, sig, r, nd, G);
  return hipGetLastError();
}

}  // namespace pstt2
