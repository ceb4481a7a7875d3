// FP64 core recovery on the GPU (paper Section 3.2 and Section 4.2).
//
//  * derive_left / derive_right: the nested Khatri-Rao DRMs share one factor per
//    mode, so S_k = X_k Omega_k follows from S_{k+1} by contracting mode k+1
//    with omega_{k+1} (block form of equation "sketch_orig"), starting from
//    Y_R = S_m; T_k = Psi_k^T X_k follows from T_{k-1} by contracting mode k
//    with psi_k, starting from T_m.
//  * basis_factor_batch / basis_form_q_batch: orthonormal bases of the sketches' ranges
//    by a column-pivoted QR (Algorithm PSTT, CPQR step).  Tall sketches are
//    first reduced by Householder TSQR (the skinny QR of Section 4.2), one
//    workgroup per 512- or 1024-row block, all splits in one launch per tree
//    level; the pivots of a matrix equal the pivots of its R factor, so the
//    pivoted QR runs on the final ell x ell R.  Signs are fixed so that
//    diag(R) >= 0.  Singular values (tolerance mode) come from a one-sided
//    Jacobi sweep on that R.
//  * core_left / core_right: equation "core" and its row-space mirror.
//  * middle_z / middle_a / middle_ls: the one-pass middle core, two products and
//    a least-squares solve (Section 4.2, "PSTT2-onepass").
//  * middle_twopass: equation "PSTT2_final_core" over a slab of X.
// All temporaries are stream-ordered (hipMallocAsync), so nothing here blocks
// the host.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "internal.h"

namespace pstt2 {


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
    const double* sp = Sin + (int64_t)c * Rk1 + row;
    double s = 0.0;
    int i = 0;
    for (; i + 8 <= nk1; i += 8) {   // eight loads in flight, summed in order
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = sp[Rk * (i + u)];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u] * om[(i + u) * ell + c];
    }
    for (; i < nk1; ++i) s += sp[Rk * i] * om[i * ell + c];
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
    const double* tp = Tin + (int64_t)a * Cprev + (int64_t)nk * col;
    double s = 0.0;
    int i = 0;
    for (; i + 8 <= nk; i += 8) {   // eight loads in flight, summed in order
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = tp[i + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += ps[(i + u) * ell + a] * v[u];
    }
    for (; i < nk; ++i) s += ps[i * ell + a] * tp[i];
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
// TSQR leaves.  One workgroup (256 threads) factors a block of BR = 256 * RPT
// rows by Householder reflections (LAPACK dlarfg convention: H = I - tau v v^T,
// v(j) = 1, beta = -sign(alpha) ||x||, tau = 0 when the column below the
// diagonal is already zero).  Thread t holds block rows t + 256 k (k < RPT), so
// row j < ell sits in thread j.  Rows past M are zero.
//
// Step j needs sigma = sum_{i>j} a_ij^2 and p_c = sum_i v_i a_ic for c > j.
// With v_i = a_ij / (alpha - beta) below the diagonal and v_j = 1, both come
// from one reduction q_c = sum_{i>j} a_ij a_ic (c >= j; sigma = q_j) and the
// broadcast row j: p_c = q_c / (alpha - beta) + a_jc.
// ---------------------------------------------------------------------------
constexpr int RED_LD = 264;   // LDS row stride of the reduction buffer (bank spread)

// Value of v held by lane l of the wavefront (l wave-uniform), through the
// scalar unit rather than an LDS read.
__device__ __forceinline__ double lane_f64(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum Red[c][0..255] for c in [c0, n) into Out[c]; threads t < LP*8 take
// column t/8 and eight interleaved slices of it.  Caller synchronises.
template <int LP>
__device__ __forceinline__ void wg_colsum(double (*Red)[RED_LD], int c0, int n, double* Out) {
  const int t = threadIdx.x;
  if (t < LP * 8) {
    const int c = t >> 3, s8 = t & 7;
    double sum = 0.0;
    if (c >= c0 && c < n) {
#pragma unroll 8
      for (int i = 0; i < 32; ++i) sum += Red[c][s8 + 8 * i];
    }
    sum += __shfl_xor(sum, 1);
    sum += __shfl_xor(sum, 2);
    sum += __shfl_xor(sum, 4);
    if (s8 == 0 && c >= c0 && c < n) Out[c] = sum;
  }
}

// Independent problems (one per split) share each launch: workgroup g belongs
// to problem p with blk0[p] <= g < blk0[p + 1].
constexpr int MAXB = PSTT2_MAX_D;
struct LeafBatch {
  int n;
  const double* A[MAXB];
  int64_t M[MAXB], lda[MAXB];
  double* V[MAXB];
  double* tau[MAXB];
  double* Rst[MAXB];
  int64_t ldr[MAXB];
  int64_t blk0[MAXB + 1];
};

__device__ __forceinline__ int batch_find(const int64_t* blk0, int n, int64_t g) {
  int p = 0;
  while (p + 1 < n && blk0[p + 1] <= g) ++p;
  return p;
}

template <int LP, int RPT>
__global__ __launch_bounds__(256) void k_qr_leaf(const LeafBatch B, int ell) {
  constexpr int BR = 256 * RPT;
  __shared__ double Red[LP][RED_LD];
  __shared__ double Qs[LP];
  __shared__ double Rowj[2][LP];
  const int t = threadIdx.x;
  const int pb = batch_find(B.blk0, B.n, blockIdx.x);
  const double* __restrict__ A = B.A[pb];
  const int64_t M = B.M[pb], lda = B.lda[pb], ldr = B.ldr[pb];
  double* __restrict__ V = B.V[pb];
  double* __restrict__ tau = B.tau[pb];
  double* __restrict__ Rst = B.Rst[pb];
  const int64_t b = blockIdx.x - B.blk0[pb];
  const int64_t rb = b * BR;
  // columns ell..LP-1 are zero: their steps are exact no-ops (sigma = alpha = 0)
  double a[RPT][LP];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int64_t row = rb + t + 256 * k;
#pragma unroll
    for (int c = 0; c < LP; ++c) a[k][c] = (c < ell && row < M) ? A[(int64_t)c * lda + row] : 0.0;
  }
  // fully unrolled over the reflectors: every register index is a constant
#pragma unroll
  for (int j = 0; j < LP; ++j) {
    if (j < ell) {   // uniform: every thread takes the same branch
    // q_c partials over this thread's rows below j
#pragma unroll
    for (int c = j; c < LP; ++c) {
      double q = 0.0;
#pragma unroll
      for (int k = 0; k < RPT; ++k)
        if (t + 256 * k > j) q += a[k][j] * a[k][c];
      Red[c][t] = q;
    }
    if (t == j) {
#pragma unroll
      for (int c = j; c < LP; ++c) Rowj[j & 1][c] = a[0][c];
    }
    __syncthreads();
    wg_colsum<LP>(Red, j, LP, Qs);
    __syncthreads();
    const double sigma = Qs[j];
    const double alpha = Rowj[j & 1][j];
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
    double v[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int lr = t + 256 * k;
      v[k] = lr == j ? 1.0 : (lr > j ? a[k][j] * scal : 0.0);
    }
    // p_c is formed by lane c of every wave and broadcast from there (one LDS
    // read per lane instead of two per column)
    const int lane = t & 63;
    const double pl = lane < LP ? tj * (scal * Qs[lane] + Rowj[j & 1][lane]) : 0.0;
#pragma unroll
    for (int c = j + 1; c < LP; ++c) {
      const double pc = lane_f64(pl, c);
#pragma unroll
      for (int k = 0; k < RPT; ++k) a[k][c] -= pc * v[k];
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int lr = t + 256 * k;
      a[k][j] = lr > j ? v[k] : (lr == j ? beta : a[k][j]);
    }
    if (t == 0) tau[b * ell + j] = tj;
    }
  }
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int lr = t + 256 * k;
#pragma unroll
    for (int c = 0; c < LP; ++c) {
      if (c < ell) {
        V[(b * ell + c) * BR + lr] = lr > c ? a[k][c] : (lr == c ? 1.0 : 0.0);
        if (k == 0 && lr < ell) Rst[(int64_t)c * ldr + b * ell + lr] = lr <= c ? a[0][c] : 0.0;
      }
    }
  }
}

// Apply one block's Q (BR x ell reflectors) to [Zin(b*ell .. b*ell+ell-1, :); 0]
// and write rows [b*BR, b*BR + BR) of Zout (masked to Mout rows).
struct ApplyBatch {
  int n;
  const double* V[MAXB];
  const double* tau[MAXB];
  const double* Zin[MAXB];
  int64_t ldzi[MAXB];
  int r[MAXB];
  double* Zout[MAXB];
  int64_t ldzo[MAXB], Mout[MAXB];
  int64_t blk0[MAXB + 1];
};

template <int RP, int RPT>
__global__ __launch_bounds__(256) void k_qr_apply(const ApplyBatch B, int ell) {
  constexpr int BR = 256 * RPT;
  __shared__ double Red[RP][RED_LD];
  __shared__ double Ws[RP];
  const int t = threadIdx.x;
  const int pb = batch_find(B.blk0, B.n, blockIdx.x);
  const double* __restrict__ V = B.V[pb];
  const double* __restrict__ tau = B.tau[pb];
  const double* __restrict__ Zin = B.Zin[pb];
  const int64_t ldzi = B.ldzi[pb], ldzo = B.ldzo[pb], Mout = B.Mout[pb];
  const int r = B.r[pb];
  double* __restrict__ Zout = B.Zout[pb];
  const int64_t b = blockIdx.x - B.blk0[pb];
  double z[RPT][RP];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int lr = t + 256 * k;
#pragma unroll
    for (int c = 0; c < RP; ++c) z[k][c] = (c < r && lr < ell) ? Zin[(int64_t)c * ldzi + b * ell + lr] : 0.0;
  }
  // reflector j is loaded one step ahead of its use
  double vn[RPT];
  double tn = 0.0;
  if (ell > 0) {
    tn = tau[b * ell + ell - 1];
#pragma unroll
    for (int k = 0; k < RPT; ++k) vn[k] = V[(b * ell + ell - 1) * BR + t + 256 * k];
  }
  for (int j = ell - 1; j >= 0; --j) {
    const double tj = tn;
    double v[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) v[k] = vn[k];
    if (j > 0) {
      tn = tau[b * ell + j - 1];
#pragma unroll
      for (int k = 0; k < RPT; ++k) vn[k] = V[(b * ell + j - 1) * BR + t + 256 * k];
    }
#pragma unroll
    for (int c = 0; c < RP; ++c) {
      double q = 0.0;
#pragma unroll
      for (int k = 0; k < RPT; ++k) q += v[k] * z[k][c];
      if (c < r) Red[c][t] = q;
    }
    __syncthreads();
    wg_colsum<RP>(Red, 0, r, Ws);
    __syncthreads();
    const double wl = (t & 63) < r ? tj * Ws[t & 63] : 0.0;   // lane c holds w_c
#pragma unroll
    for (int c = 0; c < RP; ++c) {
      if (c < r) {
        const double wc = lane_f64(wl, c);
#pragma unroll
        for (int k = 0; k < RPT; ++k) z[k][c] -= wc * v[k];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int64_t row = b * BR + t + 256 * k;
#pragma unroll
    for (int c = 0; c < RP; ++c)
      if (c < r && row < Mout) Zout[(int64_t)c * ldzo + row] = z[k][c];
  }
}

// Column-pivoted QR of the ell x ell matrix R, one wavefront per problem.
// Lane t holds column t in registers; pivoting swaps positions, not data: pos
// is the lane's current column position.  Pivot: the column of largest
// remaining norm, first position on ties (norms recomputed exactly each
// step).  Outputs: piv (ell; piv[position] = original column) and Qc
// (ell x ell, columns sign-fixed so that diag(R) >= 0).
struct CpqrBatch {
  const double* R[MAXB];
  int64_t ldr[MAXB];
  int* piv[MAXB];
  double* Qc[MAXB];
};

template <int LP>
__global__ __launch_bounds__(64) void k_cpqr(const CpqrBatch B, int ell) {
  __shared__ double Vs[LP][LP + 1];
  __shared__ double taus[LP], diag[LP];
  const int pb = blockIdx.x;
  const double* __restrict__ R = B.R[pb];
  const int64_t ldr = B.ldr[pb];
  const int t = threadIdx.x;
  const bool act = t < ell;
  double a[LP];
#pragma unroll
  for (int i = 0; i < LP; ++i) a[i] = (act && i < ell) ? R[(int64_t)t * ldr + i] : 0.0;
  int pos = t;
#pragma clang loop unroll(full)
  for (int j = 0; j < LP; ++j) {
    if (j < ell) {   // uniform
      double nrm = 0.0;
#pragma unroll
      for (int i = j; i < LP; ++i) nrm += a[i] * a[i];
      double key = (act && pos >= j) ? nrm : -1.0;
      int kpos = pos, klane = t;
      for (int o = 32; o > 0; o >>= 1) {
        const double ok = __shfl_xor(key, o);
        const int op = __shfl_xor(kpos, o), ol = __shfl_xor(klane, o);
        if (ok > key || (ok == key && op < kpos)) {
          key = ok;
          kpos = op;
          klane = ol;
        }
      }
      const int w = __shfl(klane, 0);
      const int wpos = __shfl(pos, w);
      if (t == w) pos = j;
      else if (pos == j) pos = wpos;
      if (t == w) {
        double sigma = 0.0;
#pragma unroll
        for (int i = j + 1; i < LP; ++i) sigma += a[i] * a[i];
        const double alpha = a[j];
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
#pragma unroll
        for (int i = 0; i < LP; ++i) Vs[j][i] = i < j ? 0.0 : (i == j ? 1.0 : a[i] * scal);
        taus[j] = tj;
        diag[j] = beta;
        a[j] = beta;
#pragma unroll
        for (int i = j + 1; i < LP; ++i) a[i] = 0.0;
      }
      __syncthreads();
      if (act && pos > j) {
        double pd = 0.0;
#pragma unroll
        for (int i = j; i < LP; ++i) pd += Vs[j][i] * a[i];
        pd *= taus[j];
#pragma unroll
        for (int i = j; i < LP; ++i) a[i] -= pd * Vs[j][i];
      }
    }
  }
  // Qc = H_0 ... H_{ell-1} I: lane t forms column t (position t), sign-fixed
  if (act) {
    double q[LP];
#pragma unroll
    for (int i = 0; i < LP; ++i) q[i] = i == t ? 1.0 : 0.0;
#pragma clang loop unroll(full)
    for (int j = LP - 1; j >= 0; --j) {
      if (j < ell) {
        double pd = 0.0;
#pragma unroll
        for (int i = j; i < LP; ++i) pd += Vs[j][i] * q[i];
        pd *= taus[j];
#pragma unroll
        for (int i = j; i < LP; ++i) q[i] -= pd * Vs[j][i];
      }
    }
    const double sg = diag[t] < 0.0 ? -1.0 : 1.0;
    double* Qc = B.Qc[pb];
#pragma unroll
    for (int i = 0; i < LP; ++i)
      if (i < ell) Qc[(int64_t)t * ell + i] = sg * q[i];
    B.piv[pb][pos] = t;
  }
}

// Singular values of an ell x ell matrix by one-sided (Hestenes) Jacobi.
// 16 wavefront halves; half h rotates pair h of the round-robin schedule, one
// row per lane.
struct SvBatch {
  const double* R[MAXB];
  int64_t ldr[MAXB];
  double* sv[MAXB];
};

// One-sided (Hestenes) Jacobi on the ell x ell R factor, one wavefront per
// problem: a round rotates E/2 disjoint column pairs (round-robin ordering,
// E = ell rounded up to even), four lanes per pair with eight rows each, so a
// round is a few LDS accesses, two shuffle steps and one rotation per lane.
// Sweeps end when no pair needed a rotation (at most 40); the singular values
// are the final column norms, sorted in decreasing order.
__global__ __launch_bounds__(64) void k_jacobi_sv(const SvBatch B, int ell) {
  const double* __restrict__ R = B.R[blockIdx.x];
  const int64_t ldr = B.ldr[blockIdx.x];
  double* __restrict__ sv = B.sv[blockIdx.x];
  constexpr int MX = PSTT2_MAX_ELL;
  __shared__ double U[MX][MX + 1];  // [col][row], zero outside ell x ell
  const int t = threadIdx.x;
  for (int i = t; i < MX * MX; i += 64) {
    const int c = i / MX, r = i % MX;
    U[c][r] = (c < ell && r < ell) ? R[(int64_t)c * ldr + r] : 0.0;
  }
  __syncthreads();
  const int E = (ell + 1) & ~1;
  const int pr = t >> 2, r0 = (t & 3) * 8;
  // a pair counts as orthogonal once |u_p . u_q| <= ell eps |u_p| |u_q|, the
  // rounding level of the dot product itself (a tighter test keeps rotating on
  // rounding noise and never ends before the sweep cap)
  const double tol = ell * 2.220446049250313e-16;
  for (int sweep = 0; sweep < 40; ++sweep) {
    int rot = 0;
    for (int rnd = 0; rnd < E - 1; ++rnd) {
      int p = -1, q = -1;
      if (pr < E / 2) {
        if (pr == 0) {
          p = E - 1;
          q = rnd;
        } else {
          p = (rnd + pr) % (E - 1);
          q = (rnd - pr + (E - 1)) % (E - 1);
        }
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
      }
      const bool act = q >= 0 && q < ell;
      double up[8], uq[8];
      double app = 0.0, aqq = 0.0, apq = 0.0;
      if (act) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          up[i] = U[p][r0 + i];
          uq[i] = U[q][r0 + i];
          app += up[i] * up[i];
          aqq += uq[i] * uq[i];
          apq += up[i] * uq[i];
        }
      }
      // the four lanes of a pair are adjacent: two xor steps finish the sums
      for (int o = 1; o <= 2; o <<= 1) {
        app += __shfl_xor(app, o);
        aqq += __shfl_xor(aqq, o);
        apq += __shfl_xor(apq, o);
      }
      if (act && fabs(apq) > tol * sqrt(app * aqq) && apq != 0.0) {
        const double zeta = (aqq - app) / (2.0 * apq);
        const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + tt * tt);
        const double sn = cs * tt;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          U[p][r0 + i] = cs * up[i] - sn * uq[i];
          U[q][r0 + i] = sn * up[i] + cs * uq[i];
        }
        rot = 1;
      }
      __syncthreads();
    }
    if (!__any(rot)) break;
  }
  // lane c < ell holds column c's norm; its place in decreasing order (ties
  // by column index) is the number of columns ranked before it
  __shared__ double nrm[MX];
  if (t < ell) {
    double v = 0.0;
    for (int i = 0; i < ell; ++i) v += U[t][i] * U[t][i];
    nrm[t] = sqrt(v);
  }
  __syncthreads();
  if (t < ell) {
    const double v = nrm[t];
    int pos = 0;
    for (int c = 0; c < ell; ++c) pos += (nrm[c] > v || (nrm[c] == v && c < t)) ? 1 : 0;
    sv[pos] = v;
  }
}

struct Level {
  int64_t M;      // rows at this level
  int64_t nb;     // blocks
  double* V;      // nb * ell * br
  double* tau;    // nb * ell
  double* Rst;    // stacked R of this level (nb*ell x ell), input of the next level
};

struct BasisBatch {
  int n = 0, ell = 0, rpt = 2;
  hipStream_t s = nullptr;
  std::vector<std::vector<Level>> lv;   // per problem, leaves first
  double* ws = nullptr;                 // one stream-ordered workspace for everything
  std::vector<double*> Qc, sv;
  double* tmp = nullptr;                // Q formation ping-pong buffers
};

void basis_batch_free(BasisBatch* w) {
  if (!w) return;
  if (w->ws) ws_free(w->ws, w->s);
  if (w->tmp) ws_free(w->tmp, w->s);
  delete w;
}

#define HCK(x)                         \
  do {                                 \
    hipError_t e_ = (x);               \
    if (e_ != hipSuccess) return e_;   \
  } while (0)

// Sketches of up to 16 columns use 1024-row leaves (4 rows per thread); wider
// ones 512-row leaves, so the registers of a thread stay within 64 values.
static int leaf_rpt(int ell) { return ell <= 24 ? 4 : 2; }

static void launch_leaf(const LeafBatch& B, int64_t nblk, int ell, hipStream_t s) {
  const dim3 g((unsigned)nblk), b(256);
  if (ell <= 8) hipLaunchKernelGGL((k_qr_leaf<8, 4>), g, b, 0, s, B, ell);
  else if (ell <= 16) hipLaunchKernelGGL((k_qr_leaf<16, 4>), g, b, 0, s, B, ell);
  else if (ell <= 24) hipLaunchKernelGGL((k_qr_leaf<24, 4>), g, b, 0, s, B, ell);
  else hipLaunchKernelGGL((k_qr_leaf<32, 2>), g, b, 0, s, B, ell);
}

hipError_t basis_factor_batch(int n, const double* const* A, const int64_t* M, int ell, int* const* piv,
                              bool want_sv, BasisBatch** out, hipStream_t s) {
  BasisBatch* w = new BasisBatch();
  *out = w;
  w->n = n;
  w->ell = ell;
  w->rpt = leaf_rpt(ell);
  w->s = s;
  w->lv.resize(n);
  const int64_t br = 256 * (int64_t)w->rpt;
  // level shapes and one workspace
  int64_t tot = 0;
  int maxL = 0;
  for (int p = 0; p < n; ++p) {
    int64_t curM = M[p];
    for (;;) {
      Level l;
      l.M = curM;
      l.nb = (curM + br - 1) / br;
      tot += l.nb * ell * br + l.nb * ell + l.nb * ell * ell;
      w->lv[p].push_back(l);
      if (l.nb == 1) break;
      curM = l.nb * ell;
    }
    maxL = std::max(maxL, (int)w->lv[p].size());
    tot += ell * ell + (want_sv ? ell : 0);
  }
  HCK(ws_alloc((void**)&w->ws, sizeof(double) * tot, s));
  double* cur = w->ws;
  w->Qc.resize(n);
  w->sv.assign(n, nullptr);
  for (int p = 0; p < n; ++p) {
    for (Level& l : w->lv[p]) {
      l.V = cur;
      cur += l.nb * ell * br;
      l.tau = cur;
      cur += l.nb * ell;
      l.Rst = cur;
      cur += l.nb * ell * ell;
    }
    w->Qc[p] = cur;
    cur += ell * ell;
    if (want_sv) {
      w->sv[p] = cur;
      cur += ell;
    }
  }
  // one launch per tree level over every problem that still has it
  for (int L = 0; L < maxL; ++L) {
    LeafBatch B;
    std::memset(&B, 0, sizeof(B));
    int64_t nblk = 0;
    for (int p = 0; p < n; ++p) {
      if ((int)w->lv[p].size() <= L) continue;
      const Level& l = w->lv[p][L];
      const int i = B.n++;
      B.A[i] = L == 0 ? A[p] : w->lv[p][L - 1].Rst;
      B.M[i] = l.M;
      B.lda[i] = l.M;
      B.V[i] = l.V;
      B.tau[i] = l.tau;
      B.Rst[i] = l.Rst;
      B.ldr[i] = l.nb * ell;
      B.blk0[i] = nblk;
      nblk += l.nb;
    }
    B.blk0[B.n] = nblk;
    launch_leaf(B, nblk, ell, s);
    HCK(hipGetLastError());
  }
  CpqrBatch C;
  SvBatch S;
  std::memset(&C, 0, sizeof(C));
  std::memset(&S, 0, sizeof(S));
  for (int p = 0; p < n; ++p) {
    C.R[p] = S.R[p] = w->lv[p].back().Rst;
    C.ldr[p] = S.ldr[p] = ell;
    C.piv[p] = piv[p];
    C.Qc[p] = w->Qc[p];
    S.sv[p] = w->sv[p];
  }
  if (ell <= 8) hipLaunchKernelGGL((k_cpqr<8>), dim3(n), dim3(64), 0, s, C, ell);
  else if (ell <= 16) hipLaunchKernelGGL((k_cpqr<16>), dim3(n), dim3(64), 0, s, C, ell);
  else if (ell <= 24) hipLaunchKernelGGL((k_cpqr<24>), dim3(n), dim3(64), 0, s, C, ell);
  else hipLaunchKernelGGL((k_cpqr<32>), dim3(n), dim3(64), 0, s, C, ell);
  HCK(hipGetLastError());
  if (want_sv) {
    hipLaunchKernelGGL(k_jacobi_sv, dim3(n), dim3(64), 0, s, S, ell);
    HCK(hipGetLastError());
  }
  return hipSuccess;
}

const double* basis_batch_sv(BasisBatch* w, int p) { return w->sv[p]; }

static void launch_apply(const ApplyBatch& B, int64_t nblk, int rpt, int rmax, int ell, hipStream_t s) {
  const dim3 g((unsigned)nblk), b(256);
  if (rpt == 4) {
    if (rmax <= 8) hipLaunchKernelGGL((k_qr_apply<8, 4>), g, b, 0, s, B, ell);
    else if (rmax <= 16) hipLaunchKernelGGL((k_qr_apply<16, 4>), g, b, 0, s, B, ell);
    else hipLaunchKernelGGL((k_qr_apply<24, 4>), g, b, 0, s, B, ell);
  } else {
    if (rmax <= 8) hipLaunchKernelGGL((k_qr_apply<8, 2>), g, b, 0, s, B, ell);
    else if (rmax <= 16) hipLaunchKernelGGL((k_qr_apply<16, 2>), g, b, 0, s, B, ell);
    else if (rmax <= 24) hipLaunchKernelGGL((k_qr_apply<24, 2>), g, b, 0, s, B, ell);
    else hipLaunchKernelGGL((k_qr_apply<32, 2>), g, b, 0, s, B, ell);
  }
}

// Q_p (M_p x r_p) = first r_p columns of each problem's pivoted orthogonal
// factor: the reflector trees applied top-down, one launch per depth.
hipError_t basis_form_q_batch(BasisBatch* w, const int* r, double* const* Q, hipStream_t s) {
  const int n = w->n, ell = w->ell;
  int maxL = 0, rmax = 1;
  int64_t tmpsz = 0;
  std::vector<int64_t> off(n, 0);
  for (int p = 0; p < n; ++p) {
    const int L = (int)w->lv[p].size();
    maxL = std::max(maxL, L);
    rmax = std::max(rmax, r[p]);
    int64_t maxrows = 0;
    for (int i = 1; i < L; ++i) maxrows = std::max(maxrows, w->lv[p][i].M);
    off[p] = tmpsz;
    tmpsz += 2 * maxrows * r[p];
  }
  if (tmpsz > 0) HCK(ws_alloc((void**)&w->tmp, sizeof(double) * tmpsz, s));
  std::vector<const double*> zin(n);
  std::vector<int64_t> ldzi(n, ell);
  for (int p = 0; p < n; ++p) zin[p] = w->Qc[p];   // ell x r (first r columns of Qc, ld ell)
  for (int step = 0; step < maxL; ++step) {
    ApplyBatch B;
    std::memset(&B, 0, sizeof(B));
    int64_t nblk = 0;
    std::vector<std::pair<int, double*>> outs;
    for (int p = 0; p < n; ++p) {
      const int L = (int)w->lv[p].size();
      const int i_l = L - 1 - step;   // this problem's level at this depth
      if (i_l < 0) continue;
      const Level& l = w->lv[p][i_l];
      double* zout;
      if (i_l == 0) {
        zout = Q[p];
      } else {
        int64_t mr = 0;
        for (int i = 1; i < L; ++i) mr = std::max(mr, w->lv[p][i].M);
        zout = w->tmp + off[p] + (step % 2) * mr * r[p];
      }
      const int i = B.n++;
      B.V[i] = l.V;
      B.tau[i] = l.tau;
      B.Zin[i] = zin[p];
      B.ldzi[i] = ldzi[p];
      B.r[i] = r[p];
      B.Zout[i] = zout;
      B.ldzo[i] = l.M;
      B.Mout[i] = l.M;
      B.blk0[i] = nblk;
      nblk += l.nb;
      outs.push_back({p, zout});
    }
    B.blk0[B.n] = nblk;
    launch_apply(B, nblk, w->rpt, rmax, ell, s);
    HCK(hipGetLastError());
    for (auto& o : outs) {
      const int L = (int)w->lv[o.first].size();
      zin[o.first] = o.second;
      ldzi[o.first] = w->lv[o.first][L - 1 - step].M;
    }
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
  if (Rprev >= 4096) {
    // tall Q_{k-1}: one wave per entry would read Q_{k-1} r_{k-1} n_k r_k / R... times
    // over; per i, G(:, i, :) = Q_{k-1}^T Q_k(rows R_{k-1} i ..) is a tall-skinny
    // product with fixed-order partial sums, writing G with leading dimension r_{k-1} n_k;
    // the n_k products share one launch (and each row slice of Q_{k-1})
    const int64_t Rk = Rprev * nk;
    return adj_gemm_tn_batch(rprev, rk, Rprev, nk, Qprev, Rprev, Qk, Rk, Rprev, G, (int64_t)rprev * nk, rprev, s);
  }
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
// Z(a + rp i, c) = sum_row Qp(row, a) Y(row + Rp i, c): for each i a small
// (rp x Rp)(Rp x ell) product.  A workgroup owns one i and a contiguous share
// of the rows, stages 64-row tiles of Qp and of Y's slice in LDS and keeps up to
// four of the rp x ell outputs per thread in registers across the tiles; with
// nsplit > 1 shares it writes partials that k_sum_splits adds in a fixed order.
__global__ __launch_bounds__(256) void k_middle_z(const double* __restrict__ Qp, int64_t Rp, int rp,
                                                  const double* __restrict__ Y, int64_t Rm, int nm, int ell,
                                                  int nsplit, double* __restrict__ out) {
  constexpr int MX = PSTT2_MAX_ELL, TR = 64;
  __shared__ double Qs[TR][MX + 1], Ys[TR][MX + 1];
  const int i = (int)(blockIdx.x % nm);
  const int sp = (int)(blockIdx.x / nm);
  const int64_t r0 = sp * Rp / nsplit, r1 = (sp + 1) * Rp / nsplit;
  const int nout = rp * ell;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t base = r0; base < r1; base += TR) {
    const int nr = (int)(r1 - base < TR ? r1 - base : TR);
    __syncthreads();
    for (int e = threadIdx.x; e < TR * MX; e += blockDim.x) {
      const int r = e % TR, j = e / TR;
      Qs[r][j] = (r < nr && j < rp) ? Qp[(int64_t)j * Rp + base + r] : 0.0;
      Ys[r][j] = (r < nr && j < ell) ? Y[(int64_t)j * Rm + base + r + Rp * i] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int o = threadIdx.x + 256 * k;
      if (o < nout) {
        const int a = o % rp, c = o / rp;
        double sum = acc[k];
        for (int r = 0; r < nr; ++r) sum += Qs[r][a] * Ys[r][c];
        acc[k] = sum;
      }
    }
  }
  const int64_t nz = (int64_t)rp * nm;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int o = threadIdx.x + 256 * k;
    if (o < nout) {
      const int a = o % rp, c = o / rp;
      out[sp * nz * ell + a + (int64_t)rp * i + nz * c] = acc[k];
    }
  }
}

__global__ void k_sum_splits(const double* __restrict__ part, int nsplit, int64_t n, double* __restrict__ out) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double sum = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) sum += part[sp * n + t];
    out[t] = sum;
  }
}

hipError_t middle_z(const double* Qprev, int64_t Rprev, int rprev, const double* Y, int64_t Rm, int nm, int ell,
                    double* Z, hipStream_t s) {
  if (rprev * ell > 1024 || rprev > PSTT2_MAX_ELL || ell > PSTT2_MAX_ELL) return hipErrorInvalidValue;
  // enough workgroups to spread over the chip: split the rows when n_m is small
  const int64_t want = (256 + nm - 1) / nm;
  const int nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(want, (Rprev + 255) / 256));
  const int64_t n = (int64_t)rprev * nm * ell;
  double* part = Z;
  if (nsplit > 1) {
    hipError_t e = ws_alloc((void**)&part, sizeof(double) * n * nsplit, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_middle_z, dim3((unsigned)(nm * nsplit)), dim3(256), 0, s, Qprev, Rprev, rprev, Y, Rm, nm, ell,
                     nsplit, part);
  hipError_t e = hipGetLastError();
  if (nsplit > 1) {
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_sum_splits, dim3(grid_for(n, 256)), dim3(256), 0, s, part, nsplit, n, Z);
      e = hipGetLastError();
    }
    ws_free(part, s);
  }
  return e;
}

__global__ void k_kr_table(const double* __restrict__ fac, const KRChain ch, int64_t rows, int ell,
                           double* __restrict__ out) {
  const int64_t tot = rows * ell;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int u = (int)(t / rows);
    int64_t row = t % rows;
    double f = 1.0;
    for (int q = 0; q < ch.cnt; ++q) {
      const int64_t i = row % ch.n[q];
      row /= ch.n[q];
      f *= fac[ch.off[q] + i * ell + u];
    }
    out[t] = f;
  }
}

hipError_t kr_table(const double* fac, const KRChain& ch, int64_t rows, int ell, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_kr_table, dim3(grid_for(rows * ell, 256)), dim3(256), 0, s, fac, ch, rows, ell, out);
  return hipGetLastError();
}

__global__ void k_eye(int k, double* __restrict__ out) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < k * k; t += gridDim.x * blockDim.x)
    out[t] = (t % k == t / k) ? 1.0 : 0.0;
}

hipError_t eye(int k, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_eye, dim3(1), dim3(256), 0, s, k, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Two-sided sketches of every split in two launches.  B_k = Psi_k^T S_k
// (k < m, operand S_k = X_k Omega_k, R_k rows) or B_k = T_k Omega_k (k >= m,
// operand T_k^T, C_k rows).  A workgroup takes B.steps[p] slices of TS_ROWS
// rows of one split's operand (up to TS_STEPS, when the operand is tall
// enough to keep the CUs busy with fewer workgroups).  Per slice it stages the operand rows and the
// matching Khatri-Rao DRM rows in LDS and adds their ell x ell product into
// registers (slices in order); it writes one partial, and a wavefront per
// entry then adds a split's partials in workgroup order (deterministic).
// A DRM row is the product of the chain's factor rows; with row = i + n_0 h
// (n_0 the chain's first mode) it is psi_0(i, u) * H(h, u), where H is the
// product of the other modes' rows: a slice spans at most TS_HMAX values of
// h when n_0 >= 4, so H is formed once per h into LDS (the divisions it needs
// are per h, not per entry); smaller n_0 takes the per-entry product.
// ---------------------------------------------------------------------------
constexpr int TS_ROWS = 128;
constexpr int TS_STEPS = 8;   // slices per workgroup at most
constexpr int TS_HMAX = TS_ROWS / 4 + 2;

__device__ __forceinline__ double chain_product(const TwoSidedBatch& B, const int64_t* off, const int64_t* nmode,
                                                int q0, int j0, int cnt, int64_t rest, int u) {
  double fv = 1.0;
  if (rest <= 0xffffffffLL) {   // 32-bit index arithmetic (far fewer instructions per division)
    uint32_t r = (uint32_t)rest;
    for (int j = j0; j < cnt; ++j) {
      const uint32_t nq = (uint32_t)nmode[q0 + j];
      const uint32_t i = r % nq;
      r /= nq;
      fv *= B.fac[off[j] + (int64_t)i * B.ell + u];
    }
  } else {
    int64_t r = rest;
    for (int j = j0; j < cnt; ++j) {
      const int64_t nq = nmode[q0 + j];
      const int64_t i = r % nq;
      r /= nq;
      fv *= B.fac[off[j] + i * B.ell + u];
    }
  }
  return fv;
}

typedef double ts_d4 __attribute__((ext_vector_type(4)));

// The product on FP64 matrix cores: each wave takes 32 rows of a slice in
// 16x16x4 steps (K = 4 rows) over the output padded to 32 x 32 (four tiles).
// Lane (g, l): A operand row 4 kk + g of the first factor at column 16 a + l,
// B operand the same row of the second at column 16 b + l; tile element e
// lands at output (16 a + 4 e + g, 16 b + l).  The waves' tiles are added in
// wave order at the end.
__global__ __launch_bounds__(256) void k_two_sided_part(const TwoSidedBatch B, double* __restrict__ part) {
  __shared__ double Ss[PSTT2_MAX_ELL][TS_ROWS + 1];   // operand slice, [column][row]; reused for the wave sums
  __shared__ double Fs[PSTT2_MAX_ELL][TS_ROWS + 1];   // the slice's Khatri-Rao rows, [column][row]
  __shared__ double Hs[TS_HMAX][PSTT2_MAX_ELL + 1];
  __shared__ int32_t ri[TS_ROWS], rh[TS_ROWS];   // a slice row as i + n_0 (h0 + rh)
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6, g = lane >> 4, l = lane & 15;
  const int ell = B.ell, d = B.d;
  const int p = batch_find(B.blk0, B.n, blockIdx.x);
  const int64_t K = B.K[p];
  const int nsteps = B.steps[p];
  const int64_t r0 = (blockIdx.x - B.blk0[p]) * (int64_t)TS_ROWS * nsteps;
  const int k = B.split[p], right = B.right[p];
  const int q0 = right ? k : 0, cnt = right ? d - k : k;
  const int64_t* off = B.chain + ((int64_t)k * 2 + right) * d;
  const int64_t* nmode = B.chain + (int64_t)(d + 1) * 2 * d;
  const double* __restrict__ S = B.S[p];
  const int sc = B.scols[p] > 0 ? B.scols[p] : ell;
  const int64_t n0 = nmode[q0];
  const bool htab = n0 >= 4;
  const int nout = ell * ell;
  ts_d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = ts_d4{0.0, 0.0, 0.0, 0.0};
  // the operand slice is loaded one slice ahead into registers: thread t
  // holds rows t % TS_ROWS of columns t / TS_ROWS + 2 j (coalesced down the rows)
  constexpr int NPRE = PSTT2_MAX_ELL * TS_ROWS / 256;
  static_assert(256 % TS_ROWS == 0 && NPRE * 256 == PSTT2_MAX_ELL * TS_ROWS, "staging layout");
  double pre[NPRE];
  auto load_slice = [&](int64_t rb) {
    const int64_t row = rb + t % TS_ROWS;
#pragma unroll
    for (int j = 0; j < NPRE; ++j) {
      const int u = t / TS_ROWS + (256 / TS_ROWS) * j;
      pre[j] = (row < K && u < sc) ? S[(int64_t)u * K + row] : 0.0;
    }
  };
  if (r0 < K) load_slice(r0);
  for (int st = 0; st < nsteps; ++st) {
    const int64_t rb = r0 + (int64_t)st * TS_ROWS;
    if (rb >= K) break;
    const int64_t h0 = rb / n0;
    __syncthreads();   // the last slice's LDS reads are done
#pragma unroll
    for (int j = 0; j < NPRE; ++j) Ss[t / TS_ROWS + (256 / TS_ROWS) * j][t % TS_ROWS] = pre[j];
    if (htab) {
      const int64_t rl = std::min<int64_t>(rb + TS_ROWS, K) - 1;
      const int nh = (int)(rl / n0 - h0 + 1);   // <= TS_ROWS / n_0 + 2 <= TS_HMAX
      for (int e = t; e < nh * ell; e += 256) {
        const int hh = e % nh, u = e / nh;
        Hs[hh][u] = chain_product(B, off, nmode, q0, 1, cnt, (h0 + hh), u);
      }
      if (t < TS_ROWS) {
        const int64_t row = rb + t, h = row / n0;
        ri[t] = (int32_t)(row - h * n0);
        rh[t] = (int32_t)(h - h0);
      }
    }
    __syncthreads();
    // the Khatri-Rao rows of the slice, all independent loads in one phase
    for (int e = t; e < PSTT2_MAX_ELL * TS_ROWS; e += 256) {
      const int r = e % TS_ROWS, u = e / TS_ROWS;
      const int64_t row = rb + r;
      double f = 0.0;
      if (row < K && u < ell)
        f = htab ? B.fac[off[0] + (int64_t)ri[r] * ell + u] * Hs[rh[r]][u]
                 : chain_product(B, off, nmode, q0, 0, cnt, row, u);
      Fs[u][r] = f;
    }
    __syncthreads();
    if (st + 1 < nsteps && rb + TS_ROWS < K) load_slice(rb + TS_ROWS);   // lands during this slice's products
#pragma unroll 2
    for (int kk = 0; kk < 8; ++kk) {
      const int r = 32 * w + 4 * kk + g;
      double f[2], sv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        sv[a] = Ss[16 * a + l][r];
        f[a] = Fs[16 * a + l][r];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          // left: Psi_k(row, u) S_k(row, v); right: T_k(u, col) Omega_k(col, v)
          const double x = right ? sv[a] : f[a], y = right ? f[c] : sv[c];
          acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc[a][c], 0, 0, 0);
        }
    }
  }
  // the four waves' tiles through LDS (Ss as scratch), added in wave order
  __syncthreads();
  double* red = &Ss[0][0];   // 4 waves x 32 x 32 doubles fit in Ss (32 x 129)
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) red[w * 1024 + (16 * a + 4 * e + g) * 32 + 16 * c + l] = acc[a][c][e];
  __syncthreads();
  for (int o = t; o < nout; o += 256) {
    const int u = o % ell, v = o / ell;
    double sum = red[u * 32 + v];
#pragma unroll
    for (int ww = 1; ww < 4; ++ww) sum += red[ww * 1024 + u * 32 + v];
    part[(int64_t)blockIdx.x * nout + o] = sum;
  }
}

// H(h, u) of one problem for every h, row-major (ell per row): the product of
// the factor rows of the chain's modes after the first, taken in the order
// chain_product takes them, so the values equal the per-slice table's.
// One launch for the whole batch: blockIdx.y is the problem.
__global__ void k_two_sided_htab(const TwoSidedBatch B) {
  const int p = blockIdx.y;
  const int ell = B.ell, d = B.d;
  const int k = B.split[p], right = B.right[p];
  const int q0 = right ? k : 0, cnt = right ? d - k : k;
  const int64_t* off = B.chain + ((int64_t)k * 2 + right) * d;
  const int64_t* nmode = B.chain + (int64_t)(d + 1) * 2 * d;
  const int64_t n0 = nmode[q0];
  const int64_t tot = (B.K[p] + n0 - 1) / n0 * ell;
  double* __restrict__ H = const_cast<double*>(B.H[p]);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x)
    H[e] = chain_product(B, off, nmode, q0, 1, cnt, e / ell, (int)(e % ell));
}

// The same product when every problem of the batch has n_0 >= 4 and a whole H
// table (k_two_sided_htab): the next slice's operand rows, its H rows (one
// contiguous run) and each lane's first-mode factor entries are loaded into
// registers while the current slice runs on the matrix cores, and each lane
// forms its Khatri-Rao operand (first-mode factor times H) as it feeds it, so a
// slice costs two barriers and no dependent cache round trip.  Values and the
// order of every sum are those of k_two_sided_part.  FTAB: the first mode's
// factor rows (n_0 ell <= TS_FTAB entries for every problem) sit in LDS, so a
// lane keeps only their row indices, and three workgroups fit on a compute unit.
constexpr int TS_FTAB = 1024;

template <bool FTAB>
__global__ __launch_bounds__(256, FTAB ? 3 : 2) void k_two_sided_part_h(const TwoSidedBatch B,
                                                                        double* __restrict__ part) {
  __shared__ double Ss[PSTT2_MAX_ELL][TS_ROWS + 1];   // operand slice, [column][row]; reused for the wave sums
  __shared__ double Hs[TS_HMAX][PSTT2_MAX_ELL + 1];
  __shared__ double F1[FTAB ? TS_FTAB : 1];
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6, g = lane >> 4, l = lane & 15;
  const int ell = B.ell, d = B.d;
  const int p = batch_find(B.blk0, B.n, blockIdx.x);
  const int64_t K = B.K[p];
  const int nsteps = B.steps[p];
  const int64_t r0 = (blockIdx.x - B.blk0[p]) * (int64_t)TS_ROWS * nsteps;
  const int k = B.split[p], right = B.right[p];
  const int q0 = right ? k : 0;
  const int64_t* off = B.chain + ((int64_t)k * 2 + right) * d;
  const int64_t* nmode = B.chain + (int64_t)(d + 1) * 2 * d;
  const double* __restrict__ S = B.S[p];
  const double* __restrict__ H = B.H[p];
  const int sc = B.scols[p] > 0 ? B.scols[p] : ell;
  const int64_t n0 = nmode[q0];
  const int64_t off0 = off[0];
  const int nout = ell * ell;
  if constexpr (FTAB) {
    for (int e = t; e < n0 * ell; e += 256) F1[e] = B.fac[off0 + e];   // visible after the first barrier
  }
  ts_d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = ts_d4{0.0, 0.0, 0.0, 0.0};
  constexpr int NPRE = PSTT2_MAX_ELL * TS_ROWS / 256;
  constexpr int NHP = (TS_HMAX * PSTT2_MAX_ELL + 255) / 256;
  double pre[NPRE], hpre[NHP];
  // lane operands: rows 32 w + 4 kk + g of the slice, columns 16 a + l
  double fv[FTAB ? 1 : 2][8][2];
  int fi[FTAB ? 2 : 1][8];   // FTAB: first-mode index of each of the lane's rows
  int rh[2][8];
  uint32_t rok[2];
  // the register buffer is a template argument, so every index stays static
  auto load_slice = [&](int64_t rb, auto bsel) {
    constexpr int b = decltype(bsel)::value;
    const int64_t row = rb + t % TS_ROWS;
#pragma unroll
    for (int j = 0; j < NPRE; ++j) {
      const int u = t / TS_ROWS + (256 / TS_ROWS) * j;
      pre[j] = (row < K && u < sc) ? S[(int64_t)u * K + row] : 0.0;
    }
    const int64_t h0 = rb / n0;
    const int64_t rl = std::min<int64_t>(rb + TS_ROWS, K) - 1;
    const int64_t nhe = (rl / n0 - h0 + 1) * ell;   // <= TS_HMAX ell
#pragma unroll
    for (int m = 0; m < NHP; ++m) {
      const int e = t + 256 * m;
      hpre[m] = e < nhe ? H[h0 * ell + e] : 0.0;
    }
    // first-mode index and H row of each of the lane's rows (n_0 >= 4: a step
    // of four rows wraps the first mode at most once)
    const int64_t base = rb + 32 * w + g;
    int64_t i = base % n0, hq = base / n0;
    uint32_t ok = 0;
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      if (kk > 0) {
        i += 4;
        if (i >= n0) {
          i -= n0;
          ++hq;
        }
      }
      const bool in = base + 4 * kk < K;
      ok |= (in ? 1u : 0u) << kk;
      rh[b][kk] = (int)(hq - h0);
      if constexpr (FTAB) {
        fi[b][kk] = (int)i;
      } else {
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const int u = 16 * a + l;
          fv[b][kk][a] = (in && u < ell) ? B.fac[off0 + i * ell + u] : 0.0;
        }
      }
    }
    rok[b] = ok;
  };
  auto slice = [&](int64_t rb, auto bsel) {
    constexpr int b = decltype(bsel)::value;
    const int64_t h0 = rb / n0;
    __syncthreads();   // the last slice's LDS reads are done
#pragma unroll
    for (int j = 0; j < NPRE; ++j) Ss[t / TS_ROWS + (256 / TS_ROWS) * j][t % TS_ROWS] = pre[j];
    {
      const int64_t rl = std::min<int64_t>(rb + TS_ROWS, K) - 1;
      const int nhe = (int)((rl / n0 - h0 + 1) * ell);
#pragma unroll
      for (int m = 0; m < NHP; ++m) {
        const int e = t + 256 * m;
        if (e < nhe) Hs[e / ell][e % ell] = hpre[m];
      }
    }
    __syncthreads();
    if (rb + TS_ROWS < std::min<int64_t>(K, r0 + (int64_t)TS_ROWS * nsteps)) load_slice(rb + TS_ROWS, std::integral_constant<int, b ^ 1>{});
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int r = 32 * w + 4 * kk + g;
      const bool in = (rok[b] >> kk) & 1u;
      double f[2], sv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int u = 16 * a + l;
        sv[a] = Ss[u][r];
        if constexpr (FTAB) f[a] = (in && u < ell) ? F1[fi[b][kk] * ell + u] * Hs[rh[b][kk]][u] : 0.0;
        else f[a] = (in && u < ell) ? fv[b][kk][a] * Hs[rh[b][kk]][u] : 0.0;
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const double x = right ? sv[a] : f[a], y = right ? f[c] : sv[c];
          acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc[a][c], 0, 0, 0);
        }
    }
  };
  const std::integral_constant<int, 0> b0{};
  const std::integral_constant<int, 1> b1{};
  if (r0 < K) load_slice(r0, b0);
  int st = 0;
  for (; st + 1 < nsteps; st += 2) {
    const int64_t rb = r0 + (int64_t)st * TS_ROWS;
    if (rb >= K) break;
    slice(rb, b0);
    if (rb + TS_ROWS >= K) break;
    slice(rb + TS_ROWS, b1);
  }
  if (st + 1 == nsteps) {
    const int64_t rb = r0 + (int64_t)st * TS_ROWS;
    if (rb < K) slice(rb, b0);
  }
  __syncthreads();
  double* red = &Ss[0][0];   // 4 waves x 32 x 32 doubles fit in Ss (32 x 129)
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) red[w * 1024 + (16 * a + 4 * e + g) * 32 + 16 * c + l] = acc[a][c][e];
  __syncthreads();
  for (int o = t; o < nout; o += 256) {
    const int u = o % ell, v = o / ell;
    double sum = red[u * 32 + v];
#pragma unroll
    for (int ww = 1; ww < 4; ++ww) sum += red[ww * 1024 + u * 32 + v];
    part[(int64_t)blockIdx.x * nout + o] = sum;
  }
}

__global__ __launch_bounds__(256) void k_two_sided_sum(const TwoSidedBatch B, const double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int nout = B.ell * B.ell;
  const int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  if (w >= (int64_t)B.n * nout) return;
  const int p = (int)(w / nout), o = (int)(w % nout);
  double s = 0.0;
  for (int64_t g = B.blk0[p] + lane; g < B.blk0[p + 1]; g += 64) s += part[g * nout + o];
  s = wave_sum(s);
  if (lane == 0) B.out[p][o] = s;
}

// Two-level sum for problems with many slice partials: workgroup (x, p) adds,
// for every output, the partials of its contiguous run of problem p's slices in
// slice order (threads over outputs, so the reads are coalesced), then
// k_two_sided_sum2 adds the runs in run order with the fixed butterfly.
constexpr int TS_SPLIT = 256;   // runs per problem

__global__ __launch_bounds__(256) void k_two_sided_split(const TwoSidedBatch B, const double* __restrict__ part,
                                                         double* __restrict__ runs) {
  const int p = blockIdx.y;
  const int nout = B.ell * B.ell;
  const int64_t b0 = B.blk0[p], nb = B.blk0[p + 1] - b0;
  const int64_t g0 = b0 + blockIdx.x * nb / TS_SPLIT, g1 = b0 + (blockIdx.x + 1) * nb / TS_SPLIT;
  for (int o = threadIdx.x; o < nout; o += 256) {
    double s = 0.0;
    for (int64_t g = g0; g < g1; ++g) s += part[g * nout + o];
    runs[((int64_t)p * TS_SPLIT + blockIdx.x) * nout + o] = s;
  }
}

__global__ __launch_bounds__(256) void k_two_sided_sum2(const TwoSidedBatch B, const double* __restrict__ runs) {
  const int lane = threadIdx.x & 63;
  const int nout = B.ell * B.ell;
  const int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  if (w >= (int64_t)B.n * nout) return;
  const int p = (int)(w / nout), o = (int)(w % nout);
  double s = 0.0;
  for (int g = lane; g < TS_SPLIT; g += 64) s += runs[((int64_t)p * TS_SPLIT + g) * nout + o];
  s = wave_sum(s);
  if (lane == 0) B.out[p][o] = s;
}

hipError_t two_sided_batch(TwoSidedBatch& B, hipStream_t s) {
  int64_t nblk = 0;
  for (int p = 0; p < B.n; ++p) {
    B.blk0[p] = nblk;
    // several slices per workgroup only while at least 512 workgroups remain
    B.steps[p] = (int)std::max<int64_t>(1, std::min<int64_t>(TS_STEPS, B.K[p] / ((int64_t)TS_ROWS * 512)));
    const int64_t rows = (int64_t)TS_ROWS * B.steps[p];
    nblk += std::max<int64_t>(1, (B.K[p] + rows - 1) / rows);
  }
  B.blk0[B.n] = nblk;
  if (B.n == 0) return hipSuccess;
  // whole H tables when every problem's first chain mode has n_0 >= 4 (mode
  // sizes known to the caller)
  bool tab = true;
  int64_t hrows[PSTT2_MAX_D] = {};
  int64_t htot = 0;
  for (int p = 0; p < B.n && tab; ++p) {
    const int64_t n0 = B.nmode[B.right[p] ? B.split[p] : 0];
    tab = n0 >= 4;
    hrows[p] = tab ? (B.K[p] + n0 - 1) / n0 : 0;
    htot += hrows[p] * B.ell;
  }
  double* part = nullptr;
  double* htab = nullptr;
  hipError_t e = ws_alloc((void**)&part, sizeof(double) * nblk * B.ell * B.ell, s);
  if (e != hipSuccess) return e;
  if (tab) {
    e = ws_alloc((void**)&htab, sizeof(double) * std::max<int64_t>(htot, 1), s);
    if (e != hipSuccess) {
      ws_free(part, s);
      return e;
    }
    int64_t o = 0, most = 0;
    for (int p = 0; p < B.n; ++p) {
      B.H[p] = htab + o;
      o += hrows[p] * B.ell;
      most = std::max<int64_t>(most, hrows[p] * B.ell);
    }
    const unsigned gh = (unsigned)std::max<int64_t>(1, std::min<int64_t>((most + 255) / 256, 16384));
    hipLaunchKernelGGL(k_two_sided_htab, dim3(gh, (unsigned)B.n), dim3(256), 0, s, B);
    bool ftab = true;
    for (int p = 0; p < B.n; ++p) ftab = ftab && B.nmode[B.right[p] ? B.split[p] : 0] * B.ell <= TS_FTAB;
    if (ftab) hipLaunchKernelGGL(k_two_sided_part_h<true>, dim3((unsigned)nblk), dim3(256), 0, s, B, part);
    else hipLaunchKernelGGL(k_two_sided_part_h<false>, dim3((unsigned)nblk), dim3(256), 0, s, B, part);
  } else {
    hipLaunchKernelGGL(k_two_sided_part, dim3((unsigned)nblk), dim3(256), 0, s, B, part);
  }
  const int64_t waves = (int64_t)B.n * B.ell * B.ell;
  int64_t most = 0;
  for (int p = 0; p < B.n; ++p) most = std::max<int64_t>(most, B.blk0[p + 1] - B.blk0[p]);
  double* runs = nullptr;
  if (most >= 16 * TS_SPLIT) {
    // many slices: two levels (a wave striding over tens of thousands of
    // partials 8 ell^2 bytes apart reads one double per cache line)
    e = hipGetLastError();
    if (e == hipSuccess) e = ws_alloc((void**)&runs, sizeof(double) * B.n * TS_SPLIT * B.ell * B.ell, s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_two_sided_split, dim3(TS_SPLIT, (unsigned)B.n), dim3(256), 0, s, B, part, runs);
      hipLaunchKernelGGL(k_two_sided_sum2, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, B, runs);
    }
  } else {
    hipLaunchKernelGGL(k_two_sided_sum, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, B, part);
  }
  if (e == hipSuccess) e = hipGetLastError();
  if (runs) ws_free(runs, s);
  if (htab) ws_free(htab, s);
  ws_free(part, s);
  return e;
}

// The value of a DRM entry as the sketch kernel used it: the FP64 product of
// factors rounded to the sketch arithmetic (FP32 for FP32 and split BF16, or
// BF16, or FP16).  The
// one-pass middle core pairs Y_R with A = P_m^T Omega_m, so both must see the
// same Omega_m.
__device__ __forceinline__ double drm_effective(double v, int prec) {
  if (prec == PSTT2_P_F64) return v;
  const float f = (float)v;
  if (prec == PSTT2_P_F16) return (double)(float)(_Float16)f;
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

// one wavefront per entry of A; lanes take partials g = lane, lane + 64, ...
// and a fixed butterfly adds them (deterministic)
__global__ __launch_bounds__(256) void k_middle_a_sum(const double* __restrict__ part, int nb, int nout,
                                                      double* __restrict__ A) {
  const int lane = threadIdx.x & 63;
  const int t = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (t >= nout) return;
  double s = 0.0;
  for (int g = lane; g < nb; g += 64) s += part[(int64_t)g * nout + t];
  s = wave_sum(s);
  if (lane == 0) A[t] = s;   // t = b + rm * c
}

hipError_t middle_a(const double* Pm, int64_t Cm, int rm, const SketchArgs& geo, int prec, double* A, hipStream_t s) {
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(MA_BLOCKS, (Cm + MA_TILE - 1) / MA_TILE));
  const int nout = rm * geo.ell;
  double* part = nullptr;
  hipError_t e = ws_alloc((void**)&part, sizeof(double) * nb * nout, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_middle_a_part, dim3(nb), dim3(256), 0, s, Pm, Cm, rm, geo, prec, part);
  hipLaunchKernelGGL(k_middle_a_sum, dim3((nout + 3) / 4), dim3(256), 0, s, part, nb, nout, A);
  e = hipGetLastError();
  ws_free(part, s);
  return e;
}

// Least squares min ||G A - Z||_F for G (nz x rm), A (rm x ell), Z (nz x ell),
// A of full row rank: G = Z A^+ with A^+ = A^T W, W = (A A^T)^{-1}.  W comes
// from Gauss-Jordan elimination on the rm x rm SPD matrix A A^T (one thread per
// column); then Bm = A^T W (ell x rm) and every row of G is z Bm.  A is a
// Gaussian-like rm x ell matrix (rm < ell), so cond(A A^T) = cond(A)^2 stays
// small.  A pivot below 1e-26 of the largest diagonal (A numerically
// rank-deficient) sets flag bit 2.
__global__ __launch_bounds__(256) void k_middle_ls(const double* __restrict__ Z, int64_t nz,
                                                   const double* __restrict__ A, int rm, int ell,
                                                   double* __restrict__ G, int* flag) {
  constexpr int MX = PSTT2_MAX_ELL;
  __shared__ double As[MX][MX + 1];        // A (rm x ell)
  __shared__ double Aug[MX][2 * MX + 1];   // [A A^T | I] -> [I | W]
  __shared__ double Bm[MX][MX + 1];        // A^T W: [c][b]
  __shared__ double fcol[MX];
  __shared__ double dmax;
  const int t = threadIdx.x;
  for (int i = t; i < rm * ell; i += blockDim.x) As[i % rm][i / rm] = A[i];
  __syncthreads();
  for (int i = t; i < rm * rm; i += blockDim.x) {
    const int a = i % rm, b = i / rm;
    double sum = 0.0;
    for (int c = 0; c < ell; ++c) sum += As[a][c] * As[b][c];
    Aug[a][b] = sum;
    Aug[a][rm + b] = a == b ? 1.0 : 0.0;
  }
  __syncthreads();
  if (t == 0) {
    double mx = 0.0;
    for (int a = 0; a < rm; ++a) mx = fmax(mx, Aug[a][a]);
    dmax = mx;
  }
  for (int k = 0; k < rm; ++k) {
    if (t < rm) fcol[t] = Aug[t][k];
    __syncthreads();
    if (t == 0 && blockIdx.x == 0 && !(fcol[k] > 1e-26 * dmax)) atomicOr(flag, 2);
    if (t < 2 * rm) {
      const double pk = Aug[k][t] / fcol[k];
      Aug[k][t] = pk;
      for (int i = 0; i < rm; ++i)
        if (i != k) Aug[i][t] -= fcol[i] * pk;
    }
    __syncthreads();
  }
  for (int i = t; i < ell * rm; i += blockDim.x) {
    const int c = i % ell, b = i / ell;
    double sum = 0.0;
    for (int a = 0; a < rm; ++a) sum += As[a][c] * Aug[a][rm + b];
    Bm[c][b] = sum;
  }
  __syncthreads();
  // G(rho, b) = sum_c Z(rho, c) Bm(c, b): every workgroup forms the same small
  // Bm (identical arithmetic) and applies it to its own rows of Z, one row per
  // thread (its ell entries read once, consecutive threads on consecutive rows)
  for (int64_t rho = blockIdx.x * (int64_t)blockDim.x + t; rho < nz; rho += (int64_t)gridDim.x * blockDim.x) {
    double z[MX];
#pragma unroll
    for (int c = 0; c < MX; ++c) z[c] = c < ell ? Z[(int64_t)c * nz + rho] : 0.0;
    for (int b = 0; b < rm; ++b) {
      double sum = 0.0;
#pragma unroll
      for (int c = 0; c < MX; ++c)
        if (c < ell) sum += z[c] * Bm[c][b];
      G[rho + nz * b] = sum;
    }
  }
}

hipError_t middle_ls(const double* Z, int64_t nz, const double* A, int rm, int ell, double* G, int* flag,
                     hipStream_t s) {
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((nz + 255) / 256, 1024));
  hipLaunchKernelGGL(k_middle_ls, dim3(nb), dim3(256), 0, s, Z, nz, A, rm, ell, G, flag);
  return hipGetLastError();
}

// Two-pass middle core over a slab of X (flat entries [first, first+count)):
// G(a, i, b) += sum Qprev(row', a) X(row' + Rp i, col') Pm(col', b).
// One block per (i, col') fibre present in the slab; FP64.  Used when X_m has a
// single column (the one-sided algorithm's last core, Pm = 1), where col' = 0
// and each block owns its own i: a block adds its fibre's share into G with a
// plain read-modify-write (slabs are applied in stream order), so the result
// is bitwise repeatable.  Otherwise the two fixed-order kernels below.
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
  for (int t = threadIdx.x; t < rp * rm; t += blockDim.x) {
    const int a = t % rp, b = t / rp;
    G[a + (int64_t)rp * (i + (int64_t)nm * b)] += za[a] * Pm[(int64_t)b * Cm + col];
  }
}

// Two steps in a fixed order (no atomics) when X_m has more than one column:
// (1) Z = X_m(:, slab) P_m(slab, :), R_m x r_m: a thread owns one row of X_m
//     and walks its share of the slab's columns; P_m is staged row-major with
//     its rows padded to RK (Pt, zero past r_m), so a column's weights are one
//     contiguous wave-uniform read; column shares go to gj partials.
// (2) G(a, i, b) += sum_{row'} Qprev(row', a) Z(row' + R_{m-1} i, b): one block
//     per (i, b), the partials added in increasing share order.
template <typename T, int RK>
__global__ __launch_bounds__(256) void k_twopass_z(const T* __restrict__ x, int64_t first, int64_t count, int64_t R,
                                                   const double* __restrict__ Pt, int rm, int gi_count, int gj_count,
                                                   double* __restrict__ Zp) {
  const int gi = blockIdx.x % gi_count, g = blockIdx.x / gi_count;
  const int64_t row = (int64_t)gi * 256 + threadIdx.x;
  if (row >= R) return;
  const int64_t c0 = first / R, c1 = (first + count + R - 1) / R;
  const int64_t cb = c0 + g * (c1 - c0) / gj_count, ce = c0 + (g + 1) * (c1 - c0) / gj_count;
  double acc[RK];
#pragma unroll
  for (int b = 0; b < RK; ++b) acc[b] = 0.0;
  // eight columns' loads in flight; an entry outside the slab (rows of a partial
  // first or last column) reads the slab's first entry and is given weight 0
  constexpr int U = 8;
  auto load = [&](int64_t col) -> double {
    const int64_t e = col * R + row;
    const bool ok = e >= first && e < first + count;
    const double v = (double)x[ok ? e - first : 0];
    return ok ? v : 0.0;
  };
  int64_t col = cb;
  for (; col + U <= ce; col += U) {
    double xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = load(col + u);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double* p = Pt + (col + u) * RK;
#pragma unroll
      for (int b = 0; b < RK; ++b) acc[b] += xv[u] * p[b];
    }
  }
  for (; col < ce; ++col) {
    const double xv = load(col);
    const double* p = Pt + col * RK;
#pragma unroll
    for (int b = 0; b < RK; ++b) acc[b] += xv * p[b];
  }
#pragma unroll
  for (int b = 0; b < RK; ++b)
    if (b < rm) Zp[((int64_t)g * rm + b) * R + row] = acc[b];
}

// The same for FP64 slabs of whole columns with R even: a lane owns rows
// (2t, 2t + 1) and reads both with one 16-byte load per column.  cols are
// local to the slab (column c0 + col of X_m is x + col R).
template <int RK>
__global__ __launch_bounds__(256) void k_twopass_z2(const double* __restrict__ x, int64_t R, int64_t c0, int64_t ncol,
                                                    const double* __restrict__ Pt, int rm, int gi_count, int gj_count,
                                                    double* __restrict__ Zp) {
  const int gi = blockIdx.x % gi_count, g = blockIdx.x / gi_count;
  const int64_t row = ((int64_t)gi * 256 + threadIdx.x) * 2;
  if (row >= R) return;
  const int64_t cb = g * ncol / gj_count, ce = (g + 1) * ncol / gj_count;
  double acc0[RK], acc1[RK];
#pragma unroll
  for (int b = 0; b < RK; ++b) acc0[b] = acc1[b] = 0.0;
  constexpr int U = 8;
  int64_t col = cb;
  for (; col + U <= ce; col += U) {
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = *(const double2*)(x + (col + u) * R + row);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double* p = Pt + (c0 + col + u) * RK;
#pragma unroll
      for (int b = 0; b < RK; ++b) {
        acc0[b] += v[u].x * p[b];
        acc1[b] += v[u].y * p[b];
      }
    }
  }
  for (; col < ce; ++col) {
    const double2 v = *(const double2*)(x + col * R + row);
    const double* p = Pt + (c0 + col) * RK;
#pragma unroll
    for (int b = 0; b < RK; ++b) {
      acc0[b] += v.x * p[b];
      acc1[b] += v.y * p[b];
    }
  }
#pragma unroll
  for (int b = 0; b < RK; ++b)
    if (b < rm) {
      Zp[((int64_t)g * rm + b) * R + row] = acc0[b];
      Zp[((int64_t)g * rm + b) * R + row + 1] = acc1[b];
    }
}

__global__ __launch_bounds__(256) void k_twopass_g(const double* __restrict__ Zp, int gj_count, int64_t Rp, int nm,
                                                   const double* __restrict__ Qp, int rp, int rm,
                                                   double* __restrict__ G) {
  constexpr int MX = PSTT2_MAX_ELL;
  __shared__ double red[MX][4];
  const int i = (int)(blockIdx.x % nm), b = (int)(blockIdx.x / nm);
  const int64_t R = Rp * nm;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double part[MX];
#pragma unroll
  for (int a = 0; a < MX; ++a) part[a] = 0.0;
  for (int64_t rr = threadIdx.x; rr < Rp; rr += blockDim.x) {
    const int64_t row = rr + Rp * i;
    double z = 0.0;
    for (int g = 0; g < gj_count; ++g) z += Zp[((int64_t)g * rm + b) * R + row];
#pragma unroll
    for (int a = 0; a < MX; ++a)
      if (a < rp) part[a] += Qp[(int64_t)a * Rp + rr] * z;
  }
#pragma unroll
  for (int a = 0; a < MX; ++a) {
    if (a < rp) {
      const double v = wave_sum(part[a]);
      if (lane == 0) red[a][w] = v;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < rp) {
    const int a = threadIdx.x;
    G[a + (int64_t)rp * (i + (int64_t)nm * b)] += red[a][0] + red[a][1] + red[a][2] + red[a][3];
  }
}

// Pt(col, b) = Pm(col, b) for b < rm, 0 for rm <= b < RK (Pt row-major, RK per row)
__global__ void k_twopass_pt(const double* __restrict__ Pm, int64_t Cm, int rm, int RK, double* __restrict__ Pt) {
  const int64_t tot = Cm * RK;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(t % RK);
    Pt[t] = b < rm ? Pm[(int64_t)b * Cm + t / RK] : 0.0;
  }
}

static int twopass_rk(int rm) { return rm <= 8 ? 8 : rm <= 16 ? 16 : rm <= 24 ? 24 : 32; }

template <typename T>
static void launch_twopass_z(const T* x, int64_t first, int64_t count, int64_t R, const double* Pt, int rm, int gi,
                             int gj, double* Zp, hipStream_t s) {
  const dim3 g((unsigned)(gi * gj)), bl(256);
  switch (twopass_rk(rm)) {
    case 8: hipLaunchKernelGGL((k_twopass_z<T, 8>), g, bl, 0, s, x, first, count, R, Pt, rm, gi, gj, Zp); break;
    case 16: hipLaunchKernelGGL((k_twopass_z<T, 16>), g, bl, 0, s, x, first, count, R, Pt, rm, gi, gj, Zp); break;
    case 24: hipLaunchKernelGGL((k_twopass_z<T, 24>), g, bl, 0, s, x, first, count, R, Pt, rm, gi, gj, Zp); break;
    default: hipLaunchKernelGGL((k_twopass_z<T, 32>), g, bl, 0, s, x, first, count, R, Pt, rm, gi, gj, Zp); break;
  }
}

hipError_t middle_twopass(int dtype, const void* x, int64_t first, int64_t count, int64_t Rprev, int nm, int64_t Cm,
                          const double* Qprev, int rprev, const double* Pm, int rm, double* G, hipStream_t s) {
  const int64_t f0 = first / Rprev;
  const int64_t f1 = (first + count + Rprev - 1) / Rprev;
  const unsigned nb = (unsigned)(f1 - f0);
  if (nb == 0) return hipSuccess;
  if (fault_take()) return hipErrorLaunchFailure;
  if (Cm > 1) {
    const int64_t R = Rprev * nm;
    const int64_t ncol = (first + count + R - 1) / R - first / R;
    // pair loads: FP64 slab of whole columns, R even, 16-byte aligned base
    const bool pair = dtype == PSTT2_F64 && R % 2 == 0 && first % R == 0 && count % R == 0 &&
                      ((uintptr_t)x % 16) == 0;
    const int gi = (int)(pair ? (R + 511) / 512 : (R + 255) / 256);
    const int gj = (int)std::max<int64_t>(1, std::min<int64_t>(ncol, 2048 / gi));
    const int RK = twopass_rk(rm);
    double *Zp = nullptr, *Pt = nullptr;
    hipError_t e = ws_alloc((void**)&Zp, sizeof(double) * gj * rm * R, s);
    if (e == hipSuccess) e = ws_alloc((void**)&Pt, sizeof(double) * Cm * RK, s);
    if (e != hipSuccess) {
      if (Zp) ws_free(Zp, s);
      return e;
    }
    hipLaunchKernelGGL(k_twopass_pt, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((Cm * RK + 255) / 256, 4096))),
                       dim3(256), 0, s, Pm, Cm, rm, RK, Pt);
    if (pair) {
      const dim3 g((unsigned)(gi * gj)), bl(256);
      const double* xd = (const double*)x;
      const int64_t c0 = first / R;
      switch (RK) {
        case 8: hipLaunchKernelGGL((k_twopass_z2<8>), g, bl, 0, s, xd, R, c0, ncol, Pt, rm, gi, gj, Zp); break;
        case 16: hipLaunchKernelGGL((k_twopass_z2<16>), g, bl, 0, s, xd, R, c0, ncol, Pt, rm, gi, gj, Zp); break;
        case 24: hipLaunchKernelGGL((k_twopass_z2<24>), g, bl, 0, s, xd, R, c0, ncol, Pt, rm, gi, gj, Zp); break;
        default: hipLaunchKernelGGL((k_twopass_z2<32>), g, bl, 0, s, xd, R, c0, ncol, Pt, rm, gi, gj, Zp); break;
      }
    } else if (dtype == PSTT2_F64) {
      launch_twopass_z((const double*)x, first, count, R, Pt, rm, gi, gj, Zp, s);
    } else {
      launch_twopass_z((const float*)x, first, count, R, Pt, rm, gi, gj, Zp, s);
    }
    hipLaunchKernelGGL(k_twopass_g, dim3((unsigned)(nm * rm)), dim3(256), 0, s, Zp, gj, Rprev, nm, Qprev, rprev, rm, G);
    e = hipGetLastError();
    ws_free(Pt, s);
    ws_free(Zp, s);
    return e;
  }
  // a single column: one fibre per i (see k_middle_twopass)
  if (nb > (unsigned)nm) return hipErrorInvalidValue;
  if (dtype == PSTT2_F64)
    hipLaunchKernelGGL(k_middle_twopass<double>, dim3(nb), dim3(256), 0, s, (const double*)x, first, count, Rprev, nm,
                       Cm, Qprev, rprev, Pm, rm, G);
  else
    hipLaunchKernelGGL(k_middle_twopass<float>, dim3(nb), dim3(256), 0, s, (const float*)x, first, count, Rprev, nm,
                       Cm, Qprev, rprev, Pm, rm, G);
  return hipGetLastError();
}

}  // namespace pstt2
