// FP64 core recovery on the GPU (paper Section 3.2 and Section 4.2).
//
//  * derive_left / derive_right: the nested Khatri-Rao DRMs share one factor per
//    mode, so S_k = X_k Omega_k follows from S_{k+1} by contracting mode k+1
//    with omega_{k+1} (block form of equation "sketch_orig"), starting from
//    Y_R = S_m; T_k = Psi_k^T X_k follows from T_{k-1} by contracting mode k
//    with psi_k, starting from T_m.
//  * basis_factor / basis_form_q: an orthonormal basis of the sketch's range
//    by a column-pivoted QR (Algorithm PSTT, CPQR step).  Tall sketches are
//    first reduced by Householder TSQR (the skinny QR of Section 4.2), one
//    wavefront per 128-row block; the pivots of a matrix equal the pivots of
//    its R factor, so the pivoted QR runs on the final ell x ell R.  Signs are
//    fixed so that diag(R) >= 0.  Singular values (tolerance mode) come from a
//    one-sided Jacobi sweep on that R.
//  * core_left / core_right: equation "core" and its row-space mirror.
//  * middle_z / middle_a / middle_ls: the one-pass middle core, two products and
//    a least-squares solve (Section 4.2, "PSTT2-onepass").
//  * middle_twopass: equation "PSTT2_final_core" over a slab of X.
// All temporaries are stream-ordered (hipMallocAsync), so nothing here blocks
// the host.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace pstt2 {

constexpr int BRW = 128;  // rows per TSQR block: one wavefront, two rows per lane

static unsigned grid_for(int64_t n, int bs) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + bs - 1) / bs, 8192));
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// ---------------------------------------------------------------------------
// derived sketches
// ---------------------------------------------------------------------------
__global__ void k_derive_left(const double* __restrict__ Sin, double* __restrict__ Sout, int64_t Rk, int nk1,
                              int ell, const double* __restrict__ om) {
  const int64_t tot = Rk * ell;
  const int64_t Rk1 = Rk * nk1;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t / Rk);
    const int64_t row = t % Rk;
    double s = 0.0;
    for (int i = 0; i < nk1; ++i) s += Sin[(int64_t)c * Rk1 + row + Rk * i] * om[i * ell + c];
    Sout[(int64_t)c * Rk + row] = s;
  }
}

__global__ void k_derive_right(const double* __restrict__ Tin, double* __restrict__ Tout, int64_t Ck, int nk,
                               int ell, const double* __restrict__ ps) {
  const int64_t tot = Ck * ell;
  const int64_t Cprev = Ck * nk;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(t / Ck);
    const int64_t col = t % Ck;
    double s = 0.0;
    for (int i = 0; i < nk; ++i) s += ps[i * ell + a] * Tin[(int64_t)a * Cprev + i + (int64_t)nk * col];
    Tout[(int64_t)a * Ck + col] = s;
  }
}

hipError_t derive_left(const double* Sin, double* Sout, int64_t Rk, int nk1, int ell, const double* omega,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_derive_left, dim3(grid_for(Rk * ell, 256)), dim3(256), 0, s, Sin, Sout, Rk, nk1, ell, omega);
  return hipGetLastError();
}

hipError_t derive_right(const double* Tin, double* Tout, int64_t Ck, int nk, int ell, const double* psi,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_derive_right, dim3(grid_for(Ck * ell, 256)), dim3(256), 0, s, Tin, Tout, Ck, nk, ell, psi);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Householder QR of one 128 x ell block per wavefront (LAPACK dlarfg
// convention: H = I - tau v v^T, v(j) = 1, beta = -sign(alpha) ||x||, tau = 0
// when the column below the diagonal is already zero).  Lane t holds rows t
// and t + 64 of the block.  Rows past M are zero.
// ---------------------------------------------------------------------------
// Wave-local batched reduction: every lane holds p[c] for the columns c in
// (j, ell); returns, in every lane, the wave sums W[c] (read back from LDS).
// P is this wave's LDS scratch with row stride 65 (conflict-free transposes).
template <int LP>
__device__ __forceinline__ void wave_colsum(const double (&p)[LP], int j, int ell, double* P, double* W) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < LP; ++c)
    if (c > j && c < ell) P[c * 65 + lane] = p[c];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // lane (c, h): c = lane % 32 sums half h = lane / 32 of column c's 64 entries
  const int c = lane & 31, h = lane >> 5;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (c > j && c < ell) {
    const double* q = P + c * 65 + 32 * h;
#pragma unroll
    for (int i = 0; i < 32; i += 4) {
      s0 += q[i];
      s1 += q[i + 1];
      s2 += q[i + 2];
      s3 += q[i + 3];
    }
  }
  double s = (s0 + s1) + (s2 + s3);
  s += __shfl_xor(s, 32);
  if (h == 0 && c > j && c < ell) W[c] = s;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int LP>
__global__ __launch_bounds__(256) void k_hh_block(const double* __restrict__ A, int64_t M, int64_t lda, int ell,
                                                  int64_t nb, double* __restrict__ V, double* __restrict__ tau,
                                                  double* __restrict__ Rout, int64_t ldr) {
  __shared__ double Pbuf[4][LP * 65];
  __shared__ double Wbuf[4][LP];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t b = (int64_t)blockIdx.x * 4 + wv;
  if (b >= nb) return;
  double* P = Pbuf[wv];
  double* W = Wbuf[wv];
  const int64_t r0 = b * BRW + lane, r1 = r0 + 64;
  double a0[LP], a1[LP];
#pragma unroll
  for (int c = 0; c < LP; ++c) {
    a0[c] = (c < ell && r0 < M) ? A[(int64_t)c * lda + r0] : 0.0;
    a1[c] = (c < ell && r1 < M) ? A[(int64_t)c * lda + r1] : 0.0;
  }
  const int t0 = lane, t1 = lane + 64;   // row indices within the block
  for (int j = 0; j < ell; ++j) {
    // column j of the two rows (registers are indexed statically)
    double x0 = 0.0, x1 = 0.0;
#pragma unroll
    for (int c = 0; c < LP; ++c)
      if (c == j) {
        x0 = a0[c];
        x1 = a1[c];
      }
    const double sigma = wave_sum((t0 > j ? x0 * x0 : 0.0) + x1 * x1);
    const double alpha = __shfl(x0, j);   // row j (< 64) sits in lane j, first row
    double tj, beta, scal;
    if (sigma == 0.0) {
      tj = 0.0;
      beta = alpha;
      scal = 0.0;
    } else {
      beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
      tj = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    const double v0 = (t0 == j) ? 1.0 : (t0 > j ? x0 * scal : 0.0);
    const double v1 = x1 * scal;
    double p[LP];
#pragma unroll
    for (int c = 0; c < LP; ++c) p[c] = v0 * a0[c] + v1 * a1[c];
    wave_colsum<LP>(p, j, ell, P, W);
#pragma unroll
    for (int c = 0; c < LP; ++c) {
      if (c > j && c < ell) {
        const double wc = W[c] * tj;
        a0[c] -= wc * v0;
        a1[c] -= wc * v1;
      }
    }
#pragma unroll
    for (int c = 0; c < LP; ++c)
      if (c == j) {
        a0[c] = (t0 > j) ? v0 : (t0 == j ? beta : a0[c]);
        a1[c] = v1;
      }
    if (lane == 0) tau[b * ell + j] = tj;
  }
#pragma unroll
  for (int c = 0; c < LP; ++c) {
    if (c < ell) {
      V[(b * ell + c) * BRW + t0] = (t0 > c) ? a0[c] : (t0 == c ? 1.0 : 0.0);
      V[(b * ell + c) * BRW + t1] = a1[c];
      if (t0 < ell) Rout[(int64_t)c * ldr + b * ell + t0] = (t0 <= c) ? a0[c] : 0.0;
    }
  }
}

// Apply one block's Q (128 x ell reflectors) to [Zin(b*ell .. b*ell+ell-1, :); 0]
// and write rows [b*128, b*128 + 128) of Zout (masked to Mout rows).
template <int RP>
__global__ __launch_bounds__(256) void k_hh_apply(const double* __restrict__ V, const double* __restrict__ tau,
                                                  int ell, int64_t nb, const double* __restrict__ Zin, int64_t ldzi,
                                                  int r, double* __restrict__ Zout, int64_t ldzo, int64_t Mout) {
  __shared__ double Pbuf[4][RP * 65];
  __shared__ double Wbuf[4][RP];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t b = (int64_t)blockIdx.x * 4 + wv;
  if (b >= nb) return;
  double* P = Pbuf[wv];
  double* W = Wbuf[wv];
  double c0[RP], c1[RP];
#pragma unroll
  for (int c = 0; c < RP; ++c) {
    c0[c] = (c < r && lane < ell) ? Zin[(int64_t)c * ldzi + b * ell + lane] : 0.0;
    c1[c] = 0.0;
  }
  for (int j = ell - 1; j >= 0; --j) {
    const double tj = tau[b * ell + j];
    const double v0 = V[(b * ell + j) * BRW + lane];
    const double v1 = V[(b * ell + j) * BRW + lane + 64];
    double p[RP];
#pragma unroll
    for (int c = 0; c < RP; ++c) p[c] = v0 * c0[c] + v1 * c1[c];
    wave_colsum<RP>(p, -1, r, P, W);
#pragma unroll
    for (int c = 0; c < RP; ++c) {
      if (c < r) {
        const double wc = W[c] * tj;
        c0[c] -= wc * v0;
        c1[c] -= wc * v1;
      }
    }
  }
  const int64_t r0 = b * BRW + lane, r1 = r0 + 64;
#pragma unroll
  for (int c = 0; c < RP; ++c) {
    if (c < r) {
      if (r0 < Mout) Zout[(int64_t)c * ldzo + r0] = c0[c];
      if (r1 < Mout) Zout[(int64_t)c * ldzo + r1] = c1[c];
    }
  }
}

// Column-pivoted QR of the ell x ell matrix R, one wavefront.  Pivot: first
// column of largest remaining norm (norms recomputed exactly each step).
// Outputs: piv (ell) and Qc (ell x ell, columns sign-fixed so that diag >= 0).
__global__ __launch_bounds__(64) void k_cpqr(const double* __restrict__ R, int64_t ldr, int ell, int* __restrict__ piv,
                                             double* __restrict__ Qc) {
  __shared__ double As[PSTT2_MAX_ELL][PSTT2_MAX_ELL + 1];   // [col][row]
  __shared__ double Vs[PSTT2_MAX_ELL][PSTT2_MAX_ELL + 1];   // reflectors [j][row]
  __shared__ double taus[PSTT2_MAX_ELL], diag[PSTT2_MAX_ELL];
  __shared__ int pv[PSTT2_MAX_ELL];
  const int t = threadIdx.x;
  for (int c = 0; c < ell; ++c)
    if (t < ell) As[c][t] = R[(int64_t)c * ldr + t];
  if (t < ell) pv[t] = t;
  __syncthreads();
  for (int j = 0; j < ell; ++j) {
    // residual norms (lane = column), then first-index argmax across lanes
    double nrm = -1.0;
    if (t >= j && t < ell) {
      nrm = 0.0;
      for (int i = j; i < ell; ++i) nrm += As[t][i] * As[t][i];
    }
    int best = t;
    for (int o = 32; o > 0; o >>= 1) {
      const double on = __shfl_xor(nrm, o);
      const int ob = __shfl_xor(best, o);
      if (on > nrm || (on == nrm && ob < best)) {
        nrm = on;
        best = ob;
      }
    }
    best = __shfl(best, 0);
    if (best != j) {
      if (t < ell) {
        const double tmp = As[j][t];
        As[j][t] = As[best][t];
        As[best][t] = tmp;
      }
      if (t == 0) {
        const int tp = pv[j];
        pv[j] = pv[best];
        pv[best] = tp;
      }
    }
    __syncthreads();
    // Householder vector of column j (lane = row)
    const double x = (t < ell) ? As[j][t] : 0.0;
    const double sigma = wave_sum(t > j ? x * x : 0.0);
    const double alpha = __shfl(x, j);
    double tj, beta, scal;
    if (sigma == 0.0) {
      tj = 0.0;
      beta = alpha;
      scal = 0.0;
    } else {
      beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
      tj = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    if (t < ell) {
      Vs[j][t] = (t < j) ? 0.0 : (t == j ? 1.0 : x * scal);
      As[j][t] = (t < j) ? As[j][t] : (t == j ? beta : 0.0);
    }
    if (t == 0) {
      taus[j] = tj;
      diag[j] = beta;
    }
    __syncthreads();
    // apply to the remaining columns (lane = column)
    if (t > j && t < ell) {
      double p = 0.0;
      for (int i = j; i < ell; ++i) p += Vs[j][i] * As[t][i];
      p *= tj;
      for (int i = j; i < ell; ++i) As[t][i] -= p * Vs[j][i];
    }
    __syncthreads();
  }
  // Qc = H_0 ... H_{ell-1} I, column t by lane t (in LDS, reusing As), sign-fixed
  if (t < ell) {
    for (int i = 0; i < ell; ++i) As[t][i] = (i == t) ? 1.0 : 0.0;
    for (int j = ell - 1; j >= 0; --j) {
      double p = 0.0;
      for (int i = j; i < ell; ++i) p += Vs[j][i] * As[t][i];
      p *= taus[j];
      for (int i = j; i < ell; ++i) As[t][i] -= p * Vs[j][i];
    }
    const double sg = diag[t] < 0.0 ? -1.0 : 1.0;
    for (int i = 0; i < ell; ++i) Qc[(int64_t)t * ell + i] = sg * As[t][i];
    piv[t] = pv[t];
  }
}

// Singular values of an ell x ell matrix by one-sided (Hestenes) Jacobi.
// 16 wavefront halves; half h rotates pair h of the round-robin schedule, one
// row per lane.
__global__ __launch_bounds__(512) void k_jacobi_sv(const double* __restrict__ R, int64_t ldr, int ell,
                                                   double* __restrict__ sv) {
  __shared__ double U[PSTT2_MAX_ELL][PSTT2_MAX_ELL + 1];  // [col][row]
  __shared__ int rotated;
  const int t = threadIdx.x;
  const int half = t >> 5, li = t & 31;
  for (int i = t; i < ell * ell; i += blockDim.x) U[i / ell][i % ell] = R[(int64_t)(i / ell) * ldr + i % ell];
  const int E = (ell + 1) & ~1;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (t == 0) rotated = 0;
    __syncthreads();
    for (int rnd = 0; rnd < E - 1; ++rnd) {
      if (half < E / 2) {
        int p, q;
        if (half == 0) {
          p = E - 1;
          q = rnd;
        } else {
          p = (rnd + half) % (E - 1);
          q = (rnd - half + (E - 1)) % (E - 1);
        }
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        if (q < ell) {
          const double up = li < ell ? U[p][li] : 0.0, uq = li < ell ? U[q][li] : 0.0;
          double app = up * up, aqq = uq * uq, apq = up * uq;
          for (int o = 16; o > 0; o >>= 1) {
            app += __shfl_xor(app, o, 32);
            aqq += __shfl_xor(aqq, o, 32);
            apq += __shfl_xor(apq, o, 32);
          }
          if (fabs(apq) > 1e-15 * sqrt(app * aqq) && apq != 0.0) {
            const double zeta = (aqq - app) / (2.0 * apq);
            const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double cs = 1.0 / sqrt(1.0 + tt * tt);
            const double sn = cs * tt;
            if (li < ell) {
              U[p][li] = cs * up - sn * uq;
              U[q][li] = sn * up + cs * uq;
            }
            if (li == 0) rotated = 1;
          }
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  if (t == 0) {
    double s[PSTT2_MAX_ELL];
    for (int c = 0; c < ell; ++c) {
      double v = 0.0;
      for (int i = 0; i < ell; ++i) v += U[c][i] * U[c][i];
      s[c] = sqrt(v);
    }
    for (int i = 1; i < ell; ++i) {
      const double v = s[i];
      int j = i - 1;
      while (j >= 0 && s[j] < v) {
        s[j + 1] = s[j];
        --j;
      }
      s[j + 1] = v;
    }
    for (int c = 0; c < ell; ++c) sv[c] = s[c];
  }
}

struct Level {
  int64_t M;      // rows at this level
  int64_t nb;     // blocks
  double* V;      // nb * ell * BRW
  double* tau;    // nb * ell
  double* Rst;    // stacked R of this level (nb*ell x ell), input of the next level
};

struct BasisWork {
  int ell;
  hipStream_t s;
  std::vector<Level> lv;
  double* Qc = nullptr;  // ell x ell
  int* piv = nullptr;
  double* sv = nullptr;
  double* tmp = nullptr;  // scratch for Q formation
};

void basis_free(BasisWork* w) {
  if (!w) return;
  for (auto& l : w->lv) {
    hipFreeAsync(l.V, w->s);
    hipFreeAsync(l.tau, w->s);
    hipFreeAsync(l.Rst, w->s);
  }
  hipFreeAsync(w->Qc, w->s);
  hipFreeAsync(w->sv, w->s);
  hipFreeAsync(w->tmp, w->s);
  delete w;
}

#define HCK(x)                         \
  do {                                 \
    hipError_t e_ = (x);               \
    if (e_ != hipSuccess) return e_;   \
  } while (0)

template <int LP>
static void launch_hh(const double* A, int64_t M, int64_t lda, int ell, const Level& l, hipStream_t s) {
  hipLaunchKernelGGL((k_hh_block<LP>), dim3((unsigned)((l.nb + 3) / 4)), dim3(256), 0, s, A, M, lda, ell, l.nb, l.V,
                     l.tau, l.Rst, l.nb * ell);
}

hipError_t basis_factor(const double* A, int64_t M, int ell, int* piv_dev, bool want_sv, BasisWork** out,
                        hipStream_t s) {
  BasisWork* w = new BasisWork();
  w->ell = ell;
  w->s = s;
  w->piv = piv_dev;
  *out = w;
  const double* cur = A;
  int64_t curM = M, ld = M;
  for (;;) {
    Level l;
    l.M = curM;
    l.nb = (curM + BRW - 1) / BRW;
    HCK(hipMallocAsync((void**)&l.V, sizeof(double) * l.nb * ell * BRW, s));
    HCK(hipMallocAsync((void**)&l.tau, sizeof(double) * l.nb * ell, s));
    HCK(hipMallocAsync((void**)&l.Rst, sizeof(double) * l.nb * ell * ell, s));
    if (ell <= 8) launch_hh<8>(cur, curM, ld, ell, l, s);
    else if (ell <= 16) launch_hh<16>(cur, curM, ld, ell, l, s);
    else if (ell <= 24) launch_hh<24>(cur, curM, ld, ell, l, s);
    else launch_hh<32>(cur, curM, ld, ell, l, s);
    HCK(hipGetLastError());
    w->lv.push_back(l);
    if (l.nb == 1) break;
    cur = l.Rst;
    curM = l.nb * ell;
    ld = curM;
  }
  HCK(hipMallocAsync((void**)&w->Qc, sizeof(double) * ell * ell, s));
  const Level& top = w->lv.back();
  hipLaunchKernelGGL(k_cpqr, dim3(1), dim3(64), 0, s, top.Rst, (int64_t)ell, ell, w->piv, w->Qc);
  HCK(hipGetLastError());
  if (want_sv) {
    HCK(hipMallocAsync((void**)&w->sv, sizeof(double) * ell, s));
    hipLaunchKernelGGL(k_jacobi_sv, dim3(1), dim3(512), 0, s, top.Rst, (int64_t)ell, ell, w->sv);
    HCK(hipGetLastError());
  }
  return hipSuccess;
}

const double* basis_sv(BasisWork* w) { return w->sv; }

template <int RP>
static void launch_apply(const Level& l, int ell, const double* zin, int64_t ldzi, int r, double* zout,
                         hipStream_t s) {
  hipLaunchKernelGGL((k_hh_apply<RP>), dim3((unsigned)((l.nb + 3) / 4)), dim3(256), 0, s, l.V, l.tau, ell, l.nb, zin,
                     ldzi, r, zout, l.M, l.M);
}

hipError_t basis_form_q(BasisWork* w, int r, double* Q, hipStream_t s) {
  const int ell = w->ell;
  const int L = (int)w->lv.size();
  int64_t maxrows = 0;
  for (int i = 1; i < L; ++i) maxrows = std::max(maxrows, w->lv[i].M);
  if (!w->tmp && maxrows > 0) HCK(hipMallocAsync((void**)&w->tmp, sizeof(double) * 2 * maxrows * r, s));
  double* bufA = w->tmp;
  double* bufB = w->tmp ? w->tmp + maxrows * r : nullptr;
  const double* zin = w->Qc;   // ell x r (first r columns of Qc, ld ell)
  int64_t ldzi = ell;
  for (int i = L - 1; i >= 0; --i) {
    const Level& l = w->lv[i];
    double* zout = (i == 0) ? Q : ((L - 1 - i) % 2 == 0 ? bufA : bufB);
    if (r <= 8) launch_apply<8>(l, ell, zin, ldzi, r, zout, s);
    else if (r <= 16) launch_apply<16>(l, ell, zin, ldzi, r, zout, s);
    else if (r <= 24) launch_apply<24>(l, ell, zin, ldzi, r, zout, s);
    else launch_apply<32>(l, ell, zin, ldzi, r, zout, s);
    HCK(hipGetLastError());
    zin = zout;
    ldzi = l.M;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// cores: one wavefront per output entry, lanes split the contraction
// ---------------------------------------------------------------------------
// G(a, i, b) = sum_{row < Rprev} Qprev(row, a) Qk(row + Rprev i, b)
__global__ __launch_bounds__(256) void k_core_left(const double* __restrict__ Qp, int64_t Rp, int rp,
                                                   const double* __restrict__ Qk, int nk, int rk,
                                                   double* __restrict__ G) {
  const int64_t tot = (int64_t)rp * nk * rk;
  const int lane = threadIdx.x & 63;
  const int64_t Rk = Rp * nk;
  for (int64_t t = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; t < tot;
       t += ((int64_t)gridDim.x * blockDim.x) >> 6) {
    const int a = (int)(t % rp);
    const int i = (int)((t / rp) % nk);
    const int b = (int)(t / ((int64_t)rp * nk));
    double s = 0.0;
    for (int64_t row = lane; row < Rp; row += 64) s += Qp[(int64_t)a * Rp + row] * Qk[(int64_t)b * Rk + row + Rp * i];
    s = wave_sum(s);
    if (lane == 0) G[t] = s;
  }
}

// G(a, i, b) = sum_{c < Ck} Pprev(i + nk c, a) Pk(c, b)
__global__ __launch_bounds__(256) void k_core_right(const double* __restrict__ Pp, int64_t Cp, int rp,
                                                    const double* __restrict__ Pk, int64_t Ck, int nk, int rk,
                                                    double* __restrict__ G) {
  const int64_t tot = (int64_t)rp * nk * rk;
  const int lane = threadIdx.x & 63;
  for (int64_t t = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; t < tot;
       t += ((int64_t)gridDim.x * blockDim.x) >> 6) {
    const int a = (int)(t % rp);
    const int i = (int)((t / rp) % nk);
    const int b = (int)(t / ((int64_t)rp * nk));
    double s = 0.0;
    for (int64_t c = lane; c < Ck; c += 64) s += Pp[(int64_t)a * Cp + i + (int64_t)nk * c] * Pk[(int64_t)b * Ck + c];
    s = wave_sum(s);
    if (lane == 0) G[t] = s;
  }
}

static unsigned waves_grid(int64_t nout) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((nout + 3) / 4, 16384)); }

hipError_t core_left(const double* Qprev, int64_t Rprev, int rprev, const double* Qk, int nk, int rk, double* G,
                     hipStream_t s) {
  const int64_t tot = (int64_t)rprev * nk * rk;
  hipLaunchKernelGGL(k_core_left, dim3(waves_grid(tot)), dim3(256), 0, s, Qprev, Rprev, rprev, Qk, nk, rk, G);
  return hipGetLastError();
}

hipError_t core_right(const double* Pprev, int64_t Cprev, int rprev, const double* Pk, int64_t Ck, int nk, int rk,
                      double* G, hipStream_t s) {
  const int64_t tot = (int64_t)rprev * nk * rk;
  hipLaunchKernelGGL(k_core_right, dim3(waves_grid(tot)), dim3(256), 0, s, Pprev, Cprev, rprev, Pk, Ck, nk, rk, G);
  return hipGetLastError();
}

// Z(a + rp i, c) = sum_{row < Rp} Qprev(row, a) Y(row + Rp i, c);  Z is (rp nm) x ell.
__global__ __launch_bounds__(256) void k_middle_z(const double* __restrict__ Qp, int64_t Rp, int rp,
                                                  const double* __restrict__ Y, int64_t Rm, int nm, int ell,
                                                  double* __restrict__ Z) {
  const int64_t nz = (int64_t)rp * nm;
  const int64_t tot = nz * ell;
  const int lane = threadIdx.x & 63;
  for (int64_t t = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; t < tot;
       t += ((int64_t)gridDim.x * blockDim.x) >> 6) {
    const int64_t rho = t % nz;
    const int c = (int)(t / nz);
    const int a = (int)(rho % rp);
    const int i = (int)(rho / rp);
    double s = 0.0;
    for (int64_t row = lane; row < Rp; row += 64) s += Qp[(int64_t)a * Rp + row] * Y[(int64_t)c * Rm + row + Rp * i];
    s = wave_sum(s);
    if (lane == 0) Z[t] = s;
  }
}

hipError_t middle_z(const double* Qprev, int64_t Rprev, int rprev, const double* Y, int64_t Rm, int nm, int ell,
                    double* Z, hipStream_t s) {
  const int64_t tot = (int64_t)rprev * nm * ell;
  hipLaunchKernelGGL(k_middle_z, dim3(waves_grid(tot)), dim3(256), 0, s, Qprev, Rprev, rprev, Y, Rm, nm, ell, Z);
  return hipGetLastError();
}

// The value of a DRM entry as the sketch kernel used it: the FP64 product of
// factors rounded to the sketch arithmetic (FP32 for FP32 and split BF16, or
// BF16).  The
// one-pass middle core pairs Y_R with A = P_m^T Omega_m, so both must see the
// same Omega_m.
__device__ __forceinline__ double drm_effective(double v, int prec) {
  if (prec == PSTT2_P_F64) return v;
  const float f = (float)v;
  // split BF16 carries all 24 bits of the FP32 value in its three terms
  if (prec != PSTT2_P_BF16) return (double)f;
  uint32_t u = __float_as_uint(f);
  const uint32_t h = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  return (double)__uint_as_float(h << 16);
}

// A(b, c) = sum_col Pm(col, b) Omega_m(col, c).  Every block takes a contiguous
// range of columns in 64-column tiles staged through LDS (coalesced reads of
// Pm and of the Omega_m table) and writes its r_m x ell partial; a second
// kernel adds the partials in block order (deterministic).
constexpr int MA_TILE = 64;
constexpr int MA_BLOCKS = 256;

__global__ __launch_bounds__(256) void k_middle_a_part(const double* __restrict__ Pm, int64_t Cm, int rm,
                                                       const SketchArgs G, int prec, double* __restrict__ part) {
  __shared__ double Pl[MA_TILE][PSTT2_MAX_ELL + 1];
  __shared__ double Ol[MA_TILE][PSTT2_MAX_ELL + 1];
  const int ell = G.ell;
  const int nout = rm * ell;
  const int64_t c0 = (int64_t)blockIdx.x * Cm / gridDim.x, c1 = (int64_t)(blockIdx.x + 1) * Cm / gridDim.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};   // outputs t, t + 256, t + 512, t + 768
  for (int64_t base = c0; base < c1; base += MA_TILE) {
    const int nc = (int)std::min<int64_t>(MA_TILE, c1 - base);
    __syncthreads();
    for (int i = threadIdx.x; i < MA_TILE * rm; i += blockDim.x) {
      const int j = i % MA_TILE, b = i / MA_TILE;
      Pl[j][b] = j < nc ? Pm[(int64_t)b * Cm + base + j] : 0.0;
    }
    for (int i = threadIdx.x; i < MA_TILE * G.L4; i += blockDim.x) {
      const int j = i / G.L4, c = i % G.L4;
      if (c < ell) Ol[j][c] = j < nc ? drm_effective(G.om_tab[(base + j) * G.L4 + c], prec) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = threadIdx.x + 256 * q;
      if (t < nout) {
        const int b = t % rm, c = t / rm;
        double s = 0.0;
        for (int j = 0; j < nc; ++j) s += Pl[j][b] * Ol[j][c];
        acc[q] += s;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int t = threadIdx.x + 256 * q;
    if (t < nout) part[(int64_t)blockIdx.x * nout + t] = acc[q];
  }
}

__global__ void k_middle_a_sum(const double* __restrict__ part, int nb, int nout, double* __restrict__ A) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nout; t += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int g = 0; g < nb; ++g) s += part[(int64_t)g * nout + t];
    A[t] = s;   // t = b + rm * c
  }
}

hipError_t middle_a(const double* Pm, int64_t Cm, int rm, const SketchArgs& geo, int prec, double* A, hipStream_t s) {
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(MA_BLOCKS, (Cm + MA_TILE - 1) / MA_TILE));
  const int nout = rm * geo.ell;
  double* part = nullptr;
  hipError_t e = hipMallocAsync((void**)&part, sizeof(double) * nb * nout, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_middle_a_part, dim3(nb), dim3(256), 0, s, Pm, Cm, rm, geo, prec, part);
  hipLaunchKernelGGL(k_middle_a_sum, dim3((nout + 255) / 256), dim3(256), 0, s, part, nb, nout, A);
  e = hipGetLastError();
  (void)hipFreeAsync(part, s);
  return e;
}

// Least squares min ||G A - Z||_F for G (nz x rm), A (rm x ell), Z (nz x ell):
// A^T = Qa Ra by Householder QR (one wavefront, lane = row of A^T), then every
// row of G solves g Ra^T = z Qa.
__global__ __launch_bounds__(256) void k_middle_ls(const double* __restrict__ Z, int64_t nz,
                                                   const double* __restrict__ A, int rm, int ell,
                                                   double* __restrict__ G, int* flag) {
  __shared__ double At[PSTT2_MAX_ELL][PSTT2_MAX_ELL + 1];  // A^T: [col b][row c] (ell x rm)
  __shared__ double Vs[PSTT2_MAX_ELL][PSTT2_MAX_ELL + 1];
  __shared__ double taus[PSTT2_MAX_ELL];
  __shared__ double Qa[PSTT2_MAX_ELL][PSTT2_MAX_ELL + 1];  // [col b][row c]
  __shared__ double Ra[PSTT2_MAX_ELL][PSTT2_MAX_ELL + 1];  // [col][row]
  const int t = threadIdx.x;
  if (t < ell)
    for (int b = 0; b < rm; ++b) At[b][t] = A[(int64_t)t * rm + b];
  __syncthreads();
  if (t < 64) {   // first wavefront: Householder QR of A^T, lane = row
    for (int j = 0; j < rm; ++j) {
      const double x = (t < ell) ? At[j][t] : 0.0;
      const double sigma = wave_sum(t > j ? x * x : 0.0);
      const double alpha = __shfl(x, j);
      double tj, beta, scal;
      if (sigma == 0.0) {
        tj = 0.0;
        beta = alpha;
        scal = 0.0;
      } else {
        beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
        tj = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      const double v = (t < j || t >= ell) ? 0.0 : (t == j ? 1.0 : x * scal);
      if (t < ell) {
        Vs[j][t] = v;
        At[j][t] = (t < j) ? At[j][t] : (t == j ? beta : 0.0);
      }
      if (t == 0) taus[j] = tj;
      for (int c = j + 1; c < rm; ++c) {
        const double w = wave_sum(t < ell ? v * At[c][t] : 0.0) * tj;
        if (t < ell) At[c][t] -= w * v;
      }
    }
    // explicit Qa (ell x rm), lane = row
    for (int c = 0; c < rm; ++c) {
      double q = (t == c) ? 1.0 : 0.0;
      for (int j = rm - 1; j >= 0; --j) {
        const double v = (t < ell) ? Vs[j][t] : 0.0;
        const double w = wave_sum(v * q) * taus[j];
        q -= w * v;
      }
      if (t < ell) Qa[c][t] = q;
    }
    if (t < rm)
      for (int c = 0; c < rm; ++c) Ra[c][t] = At[c][t];
    if (t == 0) {
      double dmax = 0.0;
      for (int j = 0; j < rm; ++j) dmax = fmax(dmax, fabs(At[j][j]));
      for (int j = 0; j < rm; ++j)
        if (!(fabs(At[j][j]) > 1e-13 * dmax)) atomicOr(flag, 2);
    }
  }
  __syncthreads();
  for (int64_t rho = t; rho < nz; rho += blockDim.x) {
    double y[PSTT2_MAX_ELL];
    for (int b = 0; b < rm; ++b) {
      double s = 0.0;
      for (int c = 0; c < ell; ++c) s += Z[(int64_t)c * nz + rho] * Qa[b][c];
      y[b] = s;
    }
    // g Ra^T = y  <=>  sum_{b' >= b} g[b'] Ra(b, b') = y[b]
    for (int b = rm - 1; b >= 0; --b) {
      double s = y[b];
      for (int bp = b + 1; bp < rm; ++bp) s -= y[bp] * Ra[bp][b];
      y[b] = s / Ra[b][b];
    }
    for (int b = 0; b < rm; ++b) G[(int64_t)b * nz + rho] = y[b];
  }
}

hipError_t middle_ls(const double* Z, int64_t nz, const double* A, int rm, int ell, double* G, int* flag,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_middle_ls, dim3(1), dim3(256), 0, s, Z, nz, A, rm, ell, G, flag);
  return hipGetLastError();
}

// Two-pass middle core over a slab of X (flat entries [first, first+count)):
// G(a, i, b) += sum Qprev(row', a) X(row' + Rp i, col') Pm(col', b).
// One block per (i, col') fibre present in the slab; FP64.
template <typename T>
__global__ __launch_bounds__(256) void k_middle_twopass(const T* __restrict__ x, int64_t first, int64_t count,
                                                        int64_t Rp, int nm, int64_t Cm, const double* __restrict__ Qp,
                                                        int rp, const double* __restrict__ Pm, int rm,
                                                        double* __restrict__ G) {
  __shared__ double red[PSTT2_MAX_ELL][4];
  __shared__ double za[PSTT2_MAX_ELL];
  const int64_t fiber0 = first / Rp;
  const int64_t f = fiber0 + blockIdx.x;              // fibre index = i + nm col'
  const int i = (int)(f % nm);
  const int64_t col = f / nm;
  const int64_t lo = std::max<int64_t>(f * Rp, first);
  const int64_t hi = std::min<int64_t>((f + 1) * Rp, first + count);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double part[PSTT2_MAX_ELL];
  for (int a = 0; a < rp; ++a) part[a] = 0.0;
  for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
    const double xv = (double)x[e - first];
    const int64_t row = e - f * Rp;
    for (int a = 0; a < rp; ++a) part[a] += Qp[(int64_t)a * Rp + row] * xv;
  }
  for (int a = 0; a < rp; ++a) {
    double v = wave_sum(part[a]);
    if (lane == 0) red[a][w] = v;
  }
  __syncthreads();
  if (threadIdx.x < rp) za[threadIdx.x] = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
  __syncthreads();
  // every block with the same i adds into G(:, i, :): FP64 atomics
  for (int t = threadIdx.x; t < rp * rm; t += blockDim.x) {
    const int a = t % rp, b = t / rp;
    atomicAdd(&G[a + (int64_t)rp * (i + (int64_t)nm * b)], za[a] * Pm[(int64_t)b * Cm + col]);
  }
}

hipError_t middle_twopass(int dtype, const void* x, int64_t first, int64_t count, int64_t Rprev, int nm, int64_t Cm,
                          const double* Qprev, int rprev, const double* Pm, int rm, double* G, hipStream_t s) {
  const int64_t f0 = first / Rprev;
  const int64_t f1 = (first + count + Rprev - 1) / Rprev;
  const unsigned nb = (unsigned)(f1 - f0);
  if (nb == 0) return hipSuccess;
  if (dtype == PSTT2_F64)
    hipLaunchKernelGGL(k_middle_twopass<double>, dim3(nb), dim3(256), 0, s, (const double*)x, first, count, Rprev, nm,
                       Cm, Qprev, rprev, Pm, rm, G);
  else
    hipLaunchKernelGGL(k_middle_twopass<float>, dim3(nb), dim3(256), 0, s, (const float*)x, first, count, Rprev, nm,
                       Cm, Qprev, rprev, Pm, rm, G);
  return hipGetLastError();
}

}  // namespace pstt2
