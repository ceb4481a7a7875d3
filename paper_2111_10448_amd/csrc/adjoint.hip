// Adjoint (vector-Jacobian product) of PSTT2-onepass: X -> sketches -> cores -> X~.
//
// The one-pass approximation depends on X only through the two sketches of the
// middle unfolding, Y_R = X_m Omega_m and T_m = Psi_m^T X_m (both linear in X),
// so for a cotangent gbar of X~
//     J^T gbar = Ybar Omega_m^T + Psi_m Tbar_m        (an X_m-shaped matrix).
// The pivots and ranks of the forward pass are held fixed (they are piecewise
// constant in X).  Three phases, all on the GPU in FP64:
//   B1  one stream over gbar: core cotangents through the interface matrices
//       L_m (products G_1..G_m per row of X_m) and Rt_{m+1} (G_{m+1}..G_d per
//       column): Lbar_m = gbar_m Rt^T and Rtbar = L_m^T gbar_m come from the
//       streaming dual-contraction kernel with dense tables in place of the
//       Khatri-Rao DRMs, then a backward sweep over the interface products.
//       For the Frobenius loss, gbar = -2 (X - L_m Rt) and the stream runs over
//       X itself; the rank-r_m part enters through L_m (Rt Rt^T) and
//       Rt^T (L_m^T L_m), so the cotangent is never formed;
//   B2  back through the recovery: middle least squares, outer cores, the
//       thin QR of the pivoted sketch columns, the mode-by-mode derived sketches
//       -> (Ybar, Tbar_m);
//   B3  one stream writing J^T gbar (plus 2 (X - X~) for the fused loss).
// Derivation of the middle least-squares adjoint: with W = (A A^T)^{-1} and
// G = Z A^T W,  Zbar = Gbar W A  and
//     Abar = W Gbar^T Z - G^T Gbar W A - W Gbar^T G A.
// Thin QR B = Q R (diag R > 0) with cotangent Qbar only:
//     Bbar = (Qbar + Q copyltu(M)) R^{-T},  M = -Qbar^T Q,
// where copyltu(M) mirrors the lower triangle of M onto the upper one.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace pstt2 {

static unsigned grid_for(int64_t n, int bs) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + bs - 1) / bs, 8192));
}

__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// ---- small dense FP64 products, column-major: C = alpha op(A) op(B) + beta C ----
__device__ __forceinline__ double at(const double* A, int64_t lda, bool t, int64_t i, int64_t k) {
  return t ? A[k + lda * i] : A[i + lda * k];
}

// one thread per entry of C (short contractions)
__global__ void k_gemm_t(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* __restrict__ A,
                         int64_t lda, const double* __restrict__ B, int64_t ldb, double beta, double* __restrict__ C,
                         int64_t ldc) {
  const int64_t tot = M * N;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t % M, j = t / M;
    double s = 0.0;
    for (int64_t k = 0; k < K; ++k) s += at(A, lda, ta, i, k) * at(B, ldb, !tb, j, k);
    double* c = C + i + ldc * j;
    *c = alpha * s + (beta == 0.0 ? 0.0 : beta * *c);
  }
}

// one wavefront per entry of C (long contractions)
__global__ __launch_bounds__(256) void k_gemm_w(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                                                const double* __restrict__ A, int64_t lda, const double* __restrict__ B,
                                                int64_t ldb, double beta, double* __restrict__ C, int64_t ldc) {
  const int lane = threadIdx.x & 63;
  const int64_t tot = M * N;
  for (int64_t t = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; t < tot;
       t += ((int64_t)gridDim.x * blockDim.x) >> 6) {
    const int64_t i = t % M, j = t / M;
    double s = 0.0;
    for (int64_t k = lane; k < K; k += 64) s += at(A, lda, ta, i, k) * at(B, ldb, !tb, j, k);
    s = wsum(s);
    if (lane == 0) {
      double* c = C + i + ldc * j;
      *c = alpha * s + (beta == 0.0 ? 0.0 : beta * *c);
    }
  }
}

// C = A^T B for tall, narrow A (K x M) and B (K x N), M, N <= 32, in two
// steps: workgroup g stages rows [g TN_ROWS, (g+1) TN_ROWS) of both operands in
// LDS, 64 rows at a time, and writes the partial product of its slice; a
// wavefront per entry of C then adds the slices' partials in slice order with a
// fixed butterfly (deterministic for any K).  A batch of products with the same
// A, C_i = A^T B_i (B_i = B + i sb, C_i = C + i sc), shares each launch: the
// batch index runs fastest over the workgroups, so the products of one row
// slice run together and read that slice of A once from HBM.
constexpr int TN_ROWS = 128;
constexpr int TN_SUB = 64;

__global__ __launch_bounds__(256) void k_gemm_tn_part(int M, int N, int64_t K, const double* __restrict__ A,
                                                      int64_t lda, const double* __restrict__ B, int64_t ldb,
                                                      double* __restrict__ part, int nbatch, int64_t sb, int nb) {
  __shared__ double As[TN_SUB][33];
  __shared__ double Bs[TN_SUB][33];
  const int t = threadIdx.x;
  const int nout = M * N;
  const int bi = (int)(blockIdx.x % nbatch);
  const int64_t g = blockIdx.x / nbatch;
  B += bi * sb;
  part += ((int64_t)bi * nb + g) * nout;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t r0 = g * TN_ROWS;
  const int64_t r1 = std::min<int64_t>(K, r0 + TN_ROWS);
  for (int64_t k0 = r0; k0 < r1; k0 += TN_SUB) {
    const int nr = (int)std::min<int64_t>(TN_SUB, r1 - k0);
    for (int e = t; e < TN_SUB * M; e += 256) {
      const int r = e % TN_SUB, c = e / TN_SUB;
      As[r][c] = r < nr ? A[k0 + r + lda * c] : 0.0;
    }
    for (int e = t; e < TN_SUB * N; e += 256) {
      const int r = e % TN_SUB, c = e / TN_SUB;
      Bs[r][c] = r < nr ? B[k0 + r + ldb * c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int o = t + 256 * q;
      if (o < nout) {
        const int i = o % M, j = o / M;
        double sacc = acc[q];
        for (int r = 0; r < TN_SUB; ++r) sacc += As[r][i] * Bs[r][j];
        acc[q] = sacc;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int o = t + 256 * q;
    if (o < nout) part[o] = acc[q];
  }
}

__global__ __launch_bounds__(256) void k_gemm_tn_sum(const double* __restrict__ part, int nb, int M, int N,
                                                     double alpha, double beta, double* __restrict__ C, int64_t ldc,
                                                     int nbatch, int64_t sc) {
  const int lane = threadIdx.x & 63;
  const int64_t ow = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int nout = M * N;
  if (ow >= (int64_t)nout * nbatch) return;
  const int bi = (int)(ow / nout), o = (int)(ow % nout);
  part += (int64_t)bi * nb * nout;
  C += bi * sc;
  double s = 0.0;
  for (int g = lane; g < nb; g += 64) s += part[(int64_t)g * nout + o];
  s = wsum(s);
  if (lane == 0) {
    double* c = C + (o % M) + ldc * (o / M);
    *c = alpha * s + (beta == 0.0 ? 0.0 : beta * *c);
  }
}

// op(B)(k, j): B is K x N (tb false) or N x K (tb true); at(B, ldb, !tb, j, k) reads it.
static hipError_t gemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                       const double* B, int64_t ldb, double beta, double* C, int64_t ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (ta && !tb && M <= 32 && N <= 32 && K >= 2 * TN_ROWS) {
    const int nb = (int)((K + TN_ROWS - 1) / TN_ROWS);
    double* part = nullptr;
    hipError_t e = ws_alloc((void**)&part, sizeof(double) * nb * M * N, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gemm_tn_part, dim3(nb), dim3(256), 0, s, (int)M, (int)N, K, A, lda, B, ldb, part, 1,
                       (int64_t)0, nb);
    hipLaunchKernelGGL(k_gemm_tn_sum, dim3((unsigned)((M * N + 3) / 4)), dim3(256), 0, s, part, nb, (int)M, (int)N,
                       alpha, beta, C, ldc, 1, (int64_t)0);
    e = hipGetLastError();
    ws_free(part, s);
    return e;
  }
  if (K >= 256)
    hipLaunchKernelGGL(k_gemm_w, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((M * N + 3) / 4, 16384))),
                       dim3(256), 0, s, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else
    hipLaunchKernelGGL(k_gemm_t, dim3(grid_for(M * N, 256)), dim3(256), 0, s, ta, tb, M, N, K, alpha, A, lda, B, ldb,
                       beta, C, ldc);
  return hipGetLastError();
}

// out[i * L4 + c] = in[i * si + c * sc] for c < cnt, 0 for cnt <= c < L4 (i < rows)
__global__ void k_table(const double* __restrict__ in, int64_t rows, int cnt, int64_t si, int64_t sc, int L4,
                        double* __restrict__ out) {
  const int64_t tot = rows * L4;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / L4;
    const int c = (int)(t % L4);
    out[t] = c < cnt ? in[i * si + c * sc] : 0.0;
  }
}

// B (rows x cols) = A^T for A cols x rows, both column-major
__global__ void k_transpose(const double* __restrict__ A, int64_t arows, int64_t acols, double* __restrict__ B) {
  const int64_t tot = arows * acols;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t % acols, i = t / acols;   // B(j, i) = A(i, j)
    B[j + acols * i] = A[i + arows * j];
  }
}

// Y += alpha X (n entries)
__global__ void k_axpy(int64_t n, double alpha, const double* __restrict__ X, double* __restrict__ Y) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    Y[t] += alpha * X[t];
}

// ---- middle least-squares adjoint (one workgroup; p = r_{m-1} n_m rows) ----
// G (p x r), Gbar (p x r), Z (p x ell), A (r x ell) -> Zbar (p x ell), Abar (r x ell).
__global__ __launch_bounds__(256) void k_ls_adjoint(const double* __restrict__ G, const double* __restrict__ Gb,
                                                    const double* __restrict__ Z, const double* __restrict__ A,
                                                    int64_t p, int r, int ell, double* __restrict__ Zb,
                                                    double* __restrict__ Ab) {
  constexpr int MX = PSTT2_MAX_ELL;
  __shared__ double Wm[MX][MX + 1];    // (A A^T)^{-1}, then scratch
  __shared__ double Aug[MX][2 * MX + 1];
  __shared__ double As[MX][MX + 1];    // A (r x ell)
  __shared__ double WA[MX][MX + 1];    // W A (r x ell)
  __shared__ double GbZ[MX][MX + 1];   // Gbar^T Z (r x ell)
  __shared__ double E[MX][MX + 1];     // G^T Gbar (r x r)
  const int t = threadIdx.x;
  for (int i = t; i < r * ell; i += blockDim.x) As[i % r][i / r] = A[i];
  __syncthreads();
  // A A^T and the augmented system [A A^T | I]
  for (int i = t; i < r * r; i += blockDim.x) {
    const int a = i % r, b = i / r;
    double s = 0.0;
    for (int c = 0; c < ell; ++c) s += As[a][c] * As[b][c];
    Aug[a][b] = s;
    Aug[a][r + b] = a == b ? 1.0 : 0.0;
  }
  // Gbar^T Z and G^T Gbar: one wavefront per entry
  const int lane = t & 63, wv = t >> 6;
  for (int i = wv; i < r * ell + r * r; i += 4) {
    double s = 0.0;
    if (i < r * ell) {
      const int a = i % r, c = i / r;
      for (int64_t q = lane; q < p; q += 64) s += Gb[(int64_t)a * p + q] * Z[(int64_t)c * p + q];
      s = wsum(s);
      if (lane == 0) GbZ[a][c] = s;
    } else {
      const int j = i - r * ell, a = j % r, b = j / r;
      for (int64_t q = lane; q < p; q += 64) s += G[(int64_t)a * p + q] * Gb[(int64_t)b * p + q];
      s = wsum(s);
      if (lane == 0) E[a][b] = s;
    }
  }
  __syncthreads();
  // Gauss-Jordan on the SPD system (no pivoting needed).  Thread t owns
  // column t; the multipliers of step k are staged first, since column k
  // itself is overwritten during the step.
  __shared__ double fcol[MX];
  for (int k = 0; k < r; ++k) {
    if (t < r) fcol[t] = Aug[t][k];
    __syncthreads();
    if (t < 2 * r) {
      const double pk = Aug[k][t] / fcol[k];
      Aug[k][t] = pk;
      for (int i = 0; i < r; ++i)
        if (i != k) Aug[i][t] -= fcol[i] * pk;
    }
    __syncthreads();
  }
  for (int i = t; i < r * r; i += blockDim.x) Wm[i % r][i / r] = Aug[i % r][r + i / r];
  __syncthreads();
  for (int i = t; i < r * ell; i += blockDim.x) {
    const int a = i % r, c = i / r;
    double s = 0.0;
    for (int b = 0; b < r; ++b) s += Wm[a][b] * As[b][c];
    WA[a][c] = s;
  }
  __syncthreads();
  // Zbar = Gbar (W A)
  for (int64_t i = t; i < p * ell; i += blockDim.x) {
    const int64_t q = i % p;
    const int c = (int)(i / p);
    double s = 0.0;
    for (int b = 0; b < r; ++b) s += Gb[(int64_t)b * p + q] * WA[b][c];
    Zb[i] = s;
  }
  // Abar = W (Gbar^T Z) - E (W A) - W E^T A
  for (int i = t; i < r * ell; i += blockDim.x) {
    const int a = i % r, c = i / r;
    double s = 0.0;
    for (int b = 0; b < r; ++b) {
      s += Wm[a][b] * GbZ[b][c] - E[a][b] * WA[b][c];
      double we = 0.0;   // (W E^T)(a, b)
      for (int k = 0; k < r; ++k) we += Wm[a][k] * E[b][k];
      s -= we * As[b][c];
    }
    Ab[i] = s;
  }
}

// ---- right outer cores: G_k(a, i, b) = sum_c Pp(i + nk c, a) Pk(c, b) ----
// Ppbar(i + nk c, a) += sum_b Gbar(a, i, b) Pk(c, b)
__global__ void k_core_right_adj_prev(const double* __restrict__ Gb, const double* __restrict__ Pk, int64_t Ck, int nk,
                                      int rp, int rk, double* __restrict__ Ppb) {
  const int64_t Cp = Ck * nk;
  const int64_t tot = Cp * rp;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t rowp = t % Cp;
    const int a = (int)(t / Cp);
    const int i = (int)(rowp % nk);
    const int64_t c = rowp / nk;
    double s = 0.0;
    for (int b = 0; b < rk; ++b) s += Gb[a + (int64_t)rp * (i + (int64_t)nk * b)] * Pk[(int64_t)b * Ck + c];
    Ppb[t] += s;
  }
}
// Pkbar(c, b) += sum_{a, i} Gbar(a, i, b) Pp(i + nk c, a)
__global__ void k_core_right_adj_next(const double* __restrict__ Gb, const double* __restrict__ Pp, int64_t Ck, int nk,
                                      int rp, int rk, double* __restrict__ Pkb) {
  const int64_t Cp = Ck * nk;
  const int64_t tot = Ck * rk;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = t % Ck;
    const int b = (int)(t / Ck);
    double s = 0.0;
    for (int a = 0; a < rp; ++a)
      for (int i = 0; i < nk; ++i)
        s += Gb[a + (int64_t)rp * (i + (int64_t)nk * b)] * Pp[(int64_t)a * Cp + i + (int64_t)nk * c];
    Pkb[t] += s;
  }
}

// effective DRM value as the sketch kernels used it (see recover.hip)
__device__ __forceinline__ double drm_eff(double v, int prec) {
  if (prec == PSTT2_P_F64) return v;
  const float f = (float)v;
  if (prec == PSTT2_P_F16) return (double)(float)(_Float16)f;
  if (prec != PSTT2_P_BF16) return (double)f;
  uint32_t u = __float_as_uint(f);
  const uint32_t h = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  return (double)__uint_as_float(h << 16);
}

// Pmbar(col, b) += sum_c Omega_m(col, c) Abar(b, c)
__global__ void k_pbar_from_abar(const double* __restrict__ om_tab, int L4, int64_t Cm, int rm, int ell, int prec,
                                 const double* __restrict__ Ab, double* __restrict__ Pb) {
  const int64_t tot = Cm * rm;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = t % Cm;
    const int b = (int)(t / Cm);
    double s = 0.0;
    for (int c = 0; c < ell; ++c) s += drm_eff(om_tab[col * L4 + c], prec) * Ab[b + (int64_t)rm * c];
    Pb[t] += s;
  }
}

// B (M x r) = the first r pivoted columns of S (M x ell)
__global__ void k_gather_cols(const double* __restrict__ S, int64_t M, const int* __restrict__ piv, int r,
                              double* __restrict__ B) {
  const int64_t tot = M * r;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t % M;
    const int j = (int)(t / M);
    B[t] = S[(int64_t)piv[j] * M + i];
  }
}

// Thin-QR adjoint, one thread per row i of B:
//   c = Qbar(i, :) + Q(i, :) copyltu(Mm);  Bbar(i, :) R^T = c;  Sbar(i, piv[j]) += Bbar(i, j).
// R and Mm are r x r column-major.
__global__ void k_qr_adj_rows(const double* __restrict__ Q, const double* __restrict__ Qb, int64_t M, int r,
                              const double* __restrict__ Rm, const double* __restrict__ Mm,
                              const int* __restrict__ piv, double* __restrict__ Sb) {
  constexpr int MX = PSTT2_MAX_ELL;
  __shared__ double Rs[MX][MX + 1], Cs[MX][MX + 1];
  for (int t = threadIdx.x; t < r * r; t += blockDim.x) {
    const int a = t % r, b = t / r;
    Rs[a][b] = Rm[t];
    // copyltu: lower triangle (a >= b) kept, upper mirrored from the lower
    Cs[a][b] = a >= b ? Mm[t] : Mm[b + (int64_t)r * a];
  }
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    double c[MX];
#pragma unroll
    for (int j = 0; j < MX; ++j) {
      if (j < r) {
        double s = Qb[(int64_t)j * M + i];
        for (int l = 0; l < r; ++l) s += Q[(int64_t)l * M + i] * Cs[l][j];
        c[j] = s;
      }
    }
    // sum_{l >= j} R(j, l) x(l) = c(j), from the last j down
#pragma unroll
    for (int j = MX - 1; j >= 0; --j) {
      if (j < r) {
        double s = c[j];
#pragma unroll
        for (int l = j + 1; l < MX; ++l)
          if (l < r) s -= Rs[j][l] * c[l];
        c[j] = s / Rs[j][j];
      }
    }
#pragma unroll
    for (int j = 0; j < MX; ++j)
      if (j < r) Sb[(int64_t)piv[j] * M + i] += c[j];
  }
}

// Sbar_{k+1}(row + Rk i, c) += Sbar_k(row, c) omega_{k+1}(i, c)   (adjoint of derive_left)
__global__ void k_derive_left_adj(const double* __restrict__ Sbk, double* __restrict__ Sbk1, int64_t Rk, int nk1,
                                  int ell, const double* __restrict__ om) {
  const int64_t Rk1 = Rk * nk1;
  const int64_t tot = Rk1 * ell;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t rr = t % Rk1;
    const int c = (int)(t / Rk1);
    const int64_t row = rr % Rk;
    const int i = (int)(rr / Rk);
    Sbk1[t] += Sbk[(int64_t)c * Rk + row] * om[i * ell + c];
  }
}

// Tbar_{k-1}(i + nk col, a) += psi_k(i, a) Tbar_k(col, a)   (adjoint of derive_right; C x ell layouts)
__global__ void k_derive_right_adj(const double* __restrict__ Tbk, double* __restrict__ Tbp, int64_t Ck, int nk,
                                   int ell, const double* __restrict__ ps) {
  const int64_t Cp = Ck * nk;
  const int64_t tot = Cp * ell;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cc = t % Cp;
    const int a = (int)(t / Cp);
    const int i = (int)(cc % nk);
    const int64_t col = cc / nk;
    Tbp[t] += ps[i * ell + a] * Tbk[(int64_t)a * Ck + col];
  }
}

// ---- B3: gx(row, col) = sum_c Ybar(row, c) Omega(col, c) + sum_a Psi(row, a) Tbar(col, a)
//                         [ + 2 (x - X~) for the fused loss ] [ + gx for ACC ] ----
// Block = 256 threads = 256 consecutive rows; columns in groups of 16 staged in LDS.
// A null Yb or Tbt drops that term (a pass group of the independent scheme
// with only one side); ACC adds into gx (the later groups).
struct AdjOutArgs {
  int64_t R, C;
  int ell, r, L4, prec, m;
  int32_t n[PSTT2_MAX_D];
  const double* fac;
  int64_t psi_off[PSTT2_MAX_D];
  const double* Yb;      // R x ell
  const double* Tbt;     // C x ell
  const double* om_tab;  // C x L4
  const double* L;       // R x r   (fused loss only)
  const double* Rt;      // r x C   (fused loss only)
  int gj;                // column groups
};

__device__ __forceinline__ double psi_prod(const AdjOutArgs& A, int64_t row, int a) {
  double v = 1.0;
  int64_t rr = row;
  for (int q = 1; q <= A.m; ++q) {
    const int64_t nq = A.n[q - 1];
    v *= A.fac[A.psi_off[q - 1] + (rr % nq) * A.ell + a];
    rr /= nq;
  }
  return v;
}

// MX: the sketch size and the rank rounded up to a multiple of 4 (the
// per-row operands live in registers, and their loops are unrolled to MX).
template <typename T, bool FUSED, bool ACC, int MX>
__global__ __launch_bounds__(256) void k_adj_out(const AdjOutArgs A, const T* __restrict__ x, T* __restrict__ gx) {
  constexpr int CB = 16;
  __shared__ double om[CB][MX], tb[CB][MX], rt[CB][FUSED ? MX : 1];
  const int64_t gi = blockIdx.x % ((A.R + 255) / 256);
  const int64_t gj = blockIdx.x / ((A.R + 255) / 256);
  const int64_t row = gi * 256 + threadIdx.x;
  const bool ok = row < A.R;
  const bool hy = A.Yb != nullptr, ht = A.Tbt != nullptr;
  double yb[MX], ps[MX], lr[FUSED ? MX : 1];
#pragma unroll
  for (int c = 0; c < MX; ++c) {
    yb[c] = (hy && ok && c < A.ell) ? A.Yb[(int64_t)c * A.R + row] : 0.0;
    ps[c] = (ht && ok && c < A.ell) ? drm_eff(psi_prod(A, row, c), A.prec) : 0.0;
    if constexpr (FUSED) lr[c] = (ok && c < A.r) ? A.L[(int64_t)c * A.R + row] : 0.0;
  }
  const int64_t cb = gj * A.C / A.gj, ce = (gj + 1) * A.C / A.gj;
  for (int64_t c0 = cb; c0 < ce; c0 += CB) {
    __syncthreads();
    for (int t = threadIdx.x; t < CB * MX; t += blockDim.x) {
      const int j = t / MX, c = t % MX;
      const int64_t col = c0 + j;
      const bool cok = col < ce;
      om[j][c] = (hy && cok && c < A.ell) ? drm_eff(A.om_tab[col * A.L4 + c], A.prec) : 0.0;
      tb[j][c] = (ht && cok && c < A.ell) ? A.Tbt[(int64_t)c * A.C + col] : 0.0;
      if constexpr (FUSED) rt[j][c] = (cok && c < A.r) ? A.Rt[c + (int64_t)A.r * col] : 0.0;
    }
    __syncthreads();
    if (!ok) continue;
    for (int j = 0; j < CB && c0 + j < ce; ++j) {
      double s = 0.0, xt = 0.0;
#pragma unroll
      for (int c = 0; c < MX; ++c) {
        s += yb[c] * om[j][c] + ps[c] * tb[j][c];
        if constexpr (FUSED) xt += lr[c] * rt[j][c];
      }
      const int64_t f = (c0 + j) * A.R + row;
      if (FUSED) s += 2.0 * ((double)x[f] - xt);
      if (ACC) s += (double)gx[f];
      gx[f] = (T)s;
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
hipError_t adj_gemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                    const double* B, int64_t ldb, double beta, double* C, int64_t ldc, hipStream_t s) {
  return gemm(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
}

hipError_t adj_gemm_tn_batch(int64_t M, int64_t N, int64_t K, int nbatch, const double* A, int64_t lda,
                             const double* B, int64_t ldb, int64_t sb, double* C, int64_t ldc, int64_t sc,
                             hipStream_t s) {
  if (M <= 0 || N <= 0 || nbatch <= 0) return hipSuccess;
  if (!(M <= 32 && N <= 32 && K >= 2 * TN_ROWS)) {
    hipError_t e = hipSuccess;
    for (int i = 0; i < nbatch && e == hipSuccess; ++i)
      e = gemm(true, false, M, N, K, 1.0, A, lda, B + i * sb, ldb, 0.0, C + i * sc, ldc, s);
    return e;
  }
  const int nb = (int)((K + TN_ROWS - 1) / TN_ROWS);
  const int64_t nout = M * N;
  double* part = nullptr;
  hipError_t e = ws_alloc((void**)&part, sizeof(double) * nb * nbatch * nout, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gemm_tn_part, dim3((unsigned)((int64_t)nb * nbatch)), dim3(256), 0, s, (int)M, (int)N, K, A,
                     lda, B, ldb, part, nbatch, sb, nb);
  hipLaunchKernelGGL(k_gemm_tn_sum, dim3((unsigned)((nout * nbatch + 3) / 4)), dim3(256), 0, s, part, nb, (int)M,
                     (int)N, 1.0, 0.0, C, ldc, nbatch, sc);
  e = hipGetLastError();
  ws_free(part, s);
  return e;
}

hipError_t adj_table(const double* in, int64_t rows, int cnt, int64_t si, int64_t sc, int L4, double* out,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_table, dim3(grid_for(rows * L4, 256)), dim3(256), 0, s, in, rows, cnt, si, sc, L4, out);
  return hipGetLastError();
}

hipError_t adj_transpose(const double* A, int64_t arows, int64_t acols, double* B, hipStream_t s) {
  hipLaunchKernelGGL(k_transpose, dim3(grid_for(arows * acols, 256)), dim3(256), 0, s, A, arows, acols, B);
  return hipGetLastError();
}

hipError_t adj_axpy(int64_t n, double alpha, const double* X, double* Y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(n, 256)), dim3(256), 0, s, n, alpha, X, Y);
  return hipGetLastError();
}

hipError_t adj_ls(const double* G, const double* Gb, const double* Z, const double* A, int64_t p, int r, int ell,
                  double* Zb, double* Ab, hipStream_t s) {
  hipLaunchKernelGGL(k_ls_adjoint, dim3(1), dim3(256), 0, s, G, Gb, Z, A, p, r, ell, Zb, Ab);
  return hipGetLastError();
}

hipError_t adj_core_right(const double* Gb, const double* Pp, const double* Pk, int64_t Ck, int nk, int rp, int rk,
                          double* Ppb, double* Pkb, hipStream_t s) {
  hipLaunchKernelGGL(k_core_right_adj_prev, dim3(grid_for(Ck * nk * rp, 256)), dim3(256), 0, s, Gb, Pk, Ck, nk, rp, rk,
                     Ppb);
  hipLaunchKernelGGL(k_core_right_adj_next, dim3(grid_for(Ck * rk, 256)), dim3(256), 0, s, Gb, Pp, Ck, nk, rp, rk,
                     Pkb);
  return hipGetLastError();
}

hipError_t adj_pbar(const double* om_tab, int L4, int64_t Cm, int rm, int ell, int prec, const double* Ab, double* Pb,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_pbar_from_abar, dim3(grid_for(Cm * rm, 256)), dim3(256), 0, s, om_tab, L4, Cm, rm, ell, prec,
                     Ab, Pb);
  return hipGetLastError();
}

// Sbar += thin-QR adjoint of the basis Q (M x r) of the pivoted columns of S (M x ell).
hipError_t adj_qr(const double* S, const double* Q, const double* Qb, int64_t M, int ell, int r, const int* piv,
                  double* Sb, hipStream_t s) {
  double *B = nullptr, *RM = nullptr;
  hipError_t e = ws_alloc((void**)&B, sizeof(double) * M * r, s);
  if (e == hipSuccess) e = ws_alloc((void**)&RM, sizeof(double) * 2 * r * r, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gather_cols, dim3(grid_for(M * r, 256)), dim3(256), 0, s, S, M, piv, r, B);
  e = gemm(true, false, r, r, M, 1.0, Q, M, B, M, 0.0, RM, r, s);                 // R = Q^T B
  if (e == hipSuccess) e = gemm(true, false, r, r, M, -1.0, Qb, M, Q, M, 0.0, RM + r * r, r, s);  // -Qbar^T Q
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_qr_adj_rows, dim3(grid_for(M, 256)), dim3(256), 0, s, Q, Qb, M, r, RM, RM + r * r, piv, Sb);
    e = hipGetLastError();
  }
  ws_free(B, s);
  ws_free(RM, s);
  return e;
}

hipError_t adj_derive_left(const double* Sbk, double* Sbk1, int64_t Rk, int nk1, int ell, const double* om,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_derive_left_adj, dim3(grid_for(Rk * nk1 * ell, 256)), dim3(256), 0, s, Sbk, Sbk1, Rk, nk1, ell,
                     om);
  return hipGetLastError();
}

hipError_t adj_derive_right(const double* Tbk, double* Tbp, int64_t Ck, int nk, int ell, const double* ps,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_derive_right_adj, dim3(grid_for(Ck * nk * ell, 256)), dim3(256), 0, s, Tbk, Tbp, Ck, nk, ell,
                     ps);
  return hipGetLastError();
}

template <int MX>
static void launch_adj_out(int dtype, bool fused, bool acc, dim3 grid, const AdjOutArgs& A, const void* x, void* gx,
                           hipStream_t s) {
  const dim3 block(256);
  if (dtype == PSTT2_F64) {
    if (fused)
      hipLaunchKernelGGL((k_adj_out<double, true, false, MX>), grid, block, 0, s, A, (const double*)x, (double*)gx);
    else if (acc)
      hipLaunchKernelGGL((k_adj_out<double, false, true, MX>), grid, block, 0, s, A, (const double*)x, (double*)gx);
    else
      hipLaunchKernelGGL((k_adj_out<double, false, false, MX>), grid, block, 0, s, A, (const double*)x, (double*)gx);
  } else {
    if (fused)
      hipLaunchKernelGGL((k_adj_out<float, true, false, MX>), grid, block, 0, s, A, (const float*)x, (float*)gx);
    else if (acc)
      hipLaunchKernelGGL((k_adj_out<float, false, true, MX>), grid, block, 0, s, A, (const float*)x, (float*)gx);
    else
      hipLaunchKernelGGL((k_adj_out<float, false, false, MX>), grid, block, 0, s, A, (const float*)x, (float*)gx);
  }
}

hipError_t adj_out(int dtype, const SketchArgs& g, int prec, const double* Yb, const double* Tbt, const double* L,
                   const double* Rt, int r, const void* x, void* gx, bool acc, hipStream_t s) {
  AdjOutArgs A;
  std::memset(&A, 0, sizeof(A));
  A.R = g.R;
  A.C = g.C;
  A.ell = g.ell;
  A.r = r;
  A.L4 = g.L4;
  A.prec = prec;
  A.m = g.m;
  for (int q = 0; q < PSTT2_MAX_D; ++q) {
    A.n[q] = g.n[q];
    A.psi_off[q] = g.psi_off[q];
  }
  A.fac = g.fac;
  A.Yb = Yb;
  A.Tbt = Tbt;
  A.om_tab = g.om_tab;
  A.L = L;
  A.Rt = Rt;
  const int64_t gi = (g.R + 255) / 256;
  // about four workgroups per CU: a thread's row operands (2 MX loads and the
  // Psi products) are set up once and then serve its share of the columns
  A.gj = (int)std::max<int64_t>(1, std::min<int64_t>(g.C, (1024 + gi - 1) / gi));
  const dim3 grid((unsigned)(gi * A.gj)), block(256);
  const bool fused = L != nullptr;
  if (fused && acc) return hipErrorInvalidValue;   // the loss term enters once, in the first group
  const int mx = (std::max(A.ell, fused ? r : 0) + 3) / 4 * 4;
  if (mx < 4 || mx > PSTT2_MAX_ELL) return hipErrorInvalidValue;
  switch (mx) {
    case 4: launch_adj_out<4>(dtype, fused, acc, grid, A, x, gx, s); break;
    case 8: launch_adj_out<8>(dtype, fused, acc, grid, A, x, gx, s); break;
    case 12: launch_adj_out<12>(dtype, fused, acc, grid, A, x, gx, s); break;
    case 16: launch_adj_out<16>(dtype, fused, acc, grid, A, x, gx, s); break;
    case 20: launch_adj_out<20>(dtype, fused, acc, grid, A, x, gx, s); break;
    case 24: launch_adj_out<24>(dtype, fused, acc, grid, A, x, gx, s); break;
    case 28: launch_adj_out<28>(dtype, fused, acc, grid, A, x, gx, s); break;
    default: launch_adj_out<32>(dtype, fused, acc, grid, A, x, gx, s); break;
  }
  return hipGetLastError();
}

}  // namespace pstt2
