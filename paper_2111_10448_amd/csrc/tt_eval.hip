// Evaluation of a tensor train against a dense tensor (Section 2.2 entry
// formula; relative Frobenius error of equation "FrobeniusNorm").
//
// The train is split at mode m: the left interface L (R_m x r_m) holds the
// products G_1(i_1) ... G_m(i_m) for every row of X_m and the right interface
// Rt (r_m x C_m) the products G_{m+1}(i_{m+1}) ... G_d(i_d) for every column, so
// that X~_m = L Rt.  tt_error streams X once: lanes run along rows with 8- or
// 16-byte loads (each column of X_m is contiguous), every lane keeps its rows
// of L in registers, and the column's Rt(:, col) is wave-uniform (scalar
// loads).  Squared differences are summed in FP64, never through
// ||X||^2 - 2<X, X~> + ||X~||^2, which cancels.
#include <algorithm>

#include "internal.h"

namespace pstt2 {

static unsigned grid_for(int64_t n, int bs) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + bs - 1) / bs, 8192));
}

// L_k(row + R_{k-1} i, b) = sum_a L_{k-1}(row, a) G_k(a, i, b)
// One thread per row of L_k: its rp entries of L_{k-1} are read once and kept
// in registers for all rk outputs (consecutive threads on consecutive rows).
__global__ void k_left_iface(const double* __restrict__ Lp, int64_t Rp, int rp, const double* __restrict__ G, int nk,
                             int rk, double* __restrict__ L) {
  constexpr int MX = PSTT2_MAX_ELL;
  const int64_t Rk = Rp * nk;
  for (int64_t rr = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; rr < Rk; rr += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = rr % Rp;
    const int i = (int)(rr / Rp);
    double lp[MX];
#pragma unroll
    for (int a = 0; a < MX; ++a) lp[a] = a < rp ? Lp[(int64_t)a * Rp + row] : 0.0;
    for (int b = 0; b < rk; ++b) {
      const double* g = G + (int64_t)rp * (i + (int64_t)nk * b);
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < MX; ++a)
        if (a < rp) s += lp[a] * g[a];
      L[rr + Rk * b] = s;
    }
  }
}

// Rt_k(a, i + n_k col) = sum_b G_k(a, i, b) Rt_{k+1}(b, col); Rt_{k+1} is r_k x C_k.
__global__ void k_right_iface(const double* __restrict__ G, int rp, int nk, int rk, const double* __restrict__ Rn,
                              int64_t Ck, double* __restrict__ Rt) {
  const int64_t Cp = Ck * nk;
  const int64_t tot = (int64_t)rp * Cp;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(t % rp);
    const int64_t cc = t / rp;
    const int i = (int)(cc % nk);
    const int64_t col = cc / nk;
    double s = 0.0;
    for (int b = 0; b < rk; ++b) s += G[a + (int64_t)rp * (i + (int64_t)nk * b)] * Rn[b + (int64_t)rk * col];
    Rt[t] = s;
  }
}

// Interfaces in one stream-ordered allocation: *base is returned for a single
// hipFreeAsync on the same stream; *Lout (R_split x r_split) and *Rout
// (r_split x C_split) point into it.
hipError_t tt_interfaces(const tt_cores* c, int split, double** Lout, double** Rout, double** base, hipStream_t s) {
  const int d = c->d;
  // sizes of every intermediate level
  int64_t tot = 0, Rp = c->n[0];
  tot += Rp * c->r[1];
  for (int k = 1; k < split; ++k) {
    Rp *= c->n[k];
    tot += Rp * c->r[k + 1];
  }
  int64_t Ck = c->n[d - 1];
  tot += Ck * c->r[d - 1];
  for (int k = d - 2; k >= split; --k) {
    Ck *= c->n[k];
    tot += Ck * c->r[k];
  }
  double* ws = nullptr;
  hipError_t e = ws_alloc((void**)&ws, sizeof(double) * tot, s);
  if (e != hipSuccess) return e;
  *base = ws;
  double* cur = ws;
  Rp = c->n[0];
  double* L = c->core[0];   // L_1 = G_1 (read only)
  for (int k = 1; k < split; ++k) {
    const int nk = (int)c->n[k];
    double* Ln = cur;
    cur += Rp * nk * c->r[k + 1];
    hipLaunchKernelGGL(k_left_iface, dim3(grid_for(Rp * nk, 256)), dim3(256), 0, s, L, Rp, c->r[k], c->core[k], nk,
                       c->r[k + 1], Ln);
    L = Ln;
    Rp *= nk;
  }
  Ck = c->n[d - 1];
  double* R = c->core[d - 1];   // Rt_d = G_d (read only)
  for (int k = d - 2; k >= split; --k) {
    const int nk = (int)c->n[k];
    double* Rn = cur;
    cur += Ck * nk * c->r[k];
    hipLaunchKernelGGL(k_right_iface, dim3(grid_for(Ck * nk * c->r[k], 256)), dim3(256), 0, s, c->core[k], c->r[k],
                       nk, c->r[k + 1], R, Ck, Rn);
    R = Rn;
    Ck *= nk;
  }
  *Lout = L;
  *Rout = R;
  return hipGetLastError();
}

// ---- tt_error: one streaming pass over X ----
// Block = 4 waves; a wave owns 128 consecutive rows (2 per lane) of X_m and
// walks the block's column range.  PAIR (R even): a lane's two rows are one
// aligned 2-element load.  The loop body has no branches: lanes past the last
// row read a valid row and drop it (their L rows are zero).  Rt comes padded
// to RK rows with zeros, so a column's RK entries are one contiguous run (wide
// scalar loads).  Eight columns per step keep
// eight loads in flight; every lane still adds its columns in increasing order.
// FN: X is the Hilbert tensor, X(row, col) = fn_rec[fn_row[row] + fn_col[col]],
// evaluated in place of the loads.
struct FnTabs {
  const double* rec;
  const int32_t* row;
  const int32_t* col;
};

template <typename T, int RK, bool PAIR, bool FN>
__global__ __launch_bounds__(256) void k_tt_error(const T* __restrict__ x, int64_t R, int64_t C, int r,
                                                  const double* __restrict__ L, const double* __restrict__ Rt,
                                                  int gi_count, int gj_count, double* __restrict__ part,
                                                  const FnTabs fn) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int gi = blockIdx.x % gi_count, gj = blockIdx.x / gi_count;
  const int64_t row = (int64_t)gi * 512 + w * 128 + 2 * lane;
  const int64_t cb = gj * C / gj_count, ce = (gj + 1) * C / gj_count;
  const bool ok0 = row < R, ok1 = row + 1 < R;
  double l0[RK], l1[RK];
#pragma unroll
  for (int k = 0; k < RK; ++k) {
    l0[k] = (ok0 && k < r) ? L[(int64_t)k * R + row] : 0.0;
    l1[k] = (ok1 && k < r) ? L[(int64_t)k * R + row + 1] : 0.0;
  }
  // rows read by this lane (clamped into the matrix; dropped via w0, w1)
  const int64_t r0c = ok0 ? row : 0, r1c = ok1 ? row + 1 : 0;
  const double w0 = ok0 ? 1.0 : 0.0, w1 = ok1 ? 1.0 : 0.0;
  int fr0 = 0, fr1 = 0;
  if constexpr (FN) {
    fr0 = fn.row[r0c];
    fr1 = fn.row[r1c];
  }
  auto load2 = [&](int64_t col, double& x0, double& x1) {
    if constexpr (FN) {
      const int fc = fn.col[col];
      x0 = fn.rec[fr0 + fc];
      x1 = fn.rec[fr1 + fc];
    } else if constexpr (PAIR) {
      const T* p = x + col * R + r0c;
      if constexpr (sizeof(T) == 8) {
        const double2 v = *(const double2*)p;
        x0 = v.x;
        x1 = v.y;
      } else {
        const float2 v = *(const float2*)p;
        x0 = v.x;
        x1 = v.y;
      }
    } else {
      x0 = (double)x[col * R + r0c];
      x1 = (double)x[col * R + r1c];
    }
    x0 *= w0;
    x1 *= w1;
  };
  double e2 = 0.0, x2 = 0.0;
  auto accum = [&](int64_t col, double x0, double x1) {
    const double* rc = Rt + (int64_t)RK * col;
    double t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int k = 0; k < RK; ++k) {
      const double rv = rc[k];
      t0 += l0[k] * rv;
      t1 += l1[k] * rv;
    }
    const double d0 = x0 - t0, d1 = x1 - t1;
    e2 += d0 * d0 + d1 * d1;
    x2 += x0 * x0 + x1 * x1;
  };
  constexpr int U = 8;
  int64_t col = cb;
  for (; col + U <= ce; col += U) {
    double xa[U], xb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) load2(col + u, xa[u], xb[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) accum(col + u, xa[u], xb[u]);
  }
  for (; col < ce; ++col) {
    double a0, a1;
    load2(col, a0, a1);
    accum(col, a0, a1);
  }
  __shared__ double red[2][4];
  for (int o = 32; o > 0; o >>= 1) {
    e2 += __shfl_xor(e2, o);
    x2 += __shfl_xor(x2, o);
  }
  if (lane == 0) {
    red[0][w] = e2;
    red[1][w] = x2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    part[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

// Fixed-order sum of nb (e2, x2) pairs: strided per thread, then a tree.
__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double sa[256], sb[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sa[threadIdx.x] += sa[threadIdx.x + o];
      sb[threadIdx.x] += sb[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sa[0];
    out[1] = sb[0];
  }
}

// Rt (r x C, column-major) -> Rp (RK x C) with zero rows r..RK-1
__global__ void k_pad_rt(const double* __restrict__ Rt, int r, int RK, int64_t C, double* __restrict__ Rp) {
  const int64_t tot = (int64_t)RK * C;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(t % RK);
    Rp[t] = k < r ? Rt[(t / RK) * r + k] : 0.0;
  }
}

static int rk_slot(int r) { return r <= 4 ? 4 : r <= 8 ? 8 : r <= 12 ? 12 : r <= 16 ? 16 : r <= 24 ? 24 : 32; }

template <typename T, bool PAIR, bool FN>
static hipError_t launch_err_p(const T* x, int64_t R, int64_t C, int r, const double* L, const double* Rt, int gi,
                               int gj, double* part, const FnTabs& fn, hipStream_t s) {
  dim3 g((unsigned)(gi * gj)), b(256);
  if (r <= 4) hipLaunchKernelGGL((k_tt_error<T, 4, PAIR, FN>), g, b, 0, s, x, R, C, r, L, Rt, gi, gj, part, fn);
  else if (r <= 8) hipLaunchKernelGGL((k_tt_error<T, 8, PAIR, FN>), g, b, 0, s, x, R, C, r, L, Rt, gi, gj, part, fn);
  else if (r <= 12)
    hipLaunchKernelGGL((k_tt_error<T, 12, PAIR, FN>), g, b, 0, s, x, R, C, r, L, Rt, gi, gj, part, fn);
  else if (r <= 16)
    hipLaunchKernelGGL((k_tt_error<T, 16, PAIR, FN>), g, b, 0, s, x, R, C, r, L, Rt, gi, gj, part, fn);
  else if (r <= 24)
    hipLaunchKernelGGL((k_tt_error<T, 24, PAIR, FN>), g, b, 0, s, x, R, C, r, L, Rt, gi, gj, part, fn);
  else hipLaunchKernelGGL((k_tt_error<T, 32, PAIR, FN>), g, b, 0, s, x, R, C, r, L, Rt, gi, gj, part, fn);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_err(const T* x, int64_t R, int64_t C, int r, const double* L, const double* Rt, int gi,
                             int gj, double* part, hipStream_t s) {
  // aligned pair loads need an even column length (and an aligned base)
  const bool pair = (R % 2) == 0 && ((uintptr_t)x % (2 * sizeof(T))) == 0;
  const FnTabs none{nullptr, nullptr, nullptr};
  return pair ? launch_err_p<T, true, false>(x, R, C, r, L, Rt, gi, gj, part, none, s)
              : launch_err_p<T, false, false>(x, R, C, r, L, Rt, gi, gj, part, none, s);
}

// x == nullptr: the Hilbert tensor (fn != 0), evaluated from its index tables
hipError_t tt_error_run(const tt_cores* c, const void* x, int dtype, double* e2x2, hipStream_t s, int fn) {
  const int d = c->d;
  const int split = (d + 1) / 2;
  double *L = nullptr, *Rt = nullptr, *ifb = nullptr;
  hipError_t e = tt_interfaces(c, split, &L, &Rt, &ifb, s);
  if (e != hipSuccess) return e;
  int64_t R = 1, C = 1;
  for (int k = 0; k < split; ++k) R *= c->n[k];
  for (int k = split; k < d; ++k) C *= c->n[k];
  const int r = c->r[split];
  const int gi = (int)((R + 511) / 512);
  const int gj = (int)std::max<int64_t>(1, std::min<int64_t>(C, (4096 + gi - 1) / gi));
  double *part = nullptr, *Rp = nullptr, *rec = nullptr;
  int32_t *row_t = nullptr, *col_t = nullptr;
  const int RK = rk_slot(r);
  e = ws_alloc((void**)&part, sizeof(double) * 2 * ((int64_t)gi * gj + 1), s);
  if (e == hipSuccess) e = ws_alloc((void**)&Rp, sizeof(double) * RK * C, s);
  if (fn) {
    if (e == hipSuccess) e = ws_alloc((void**)&rec, sizeof(double) * hilbert_rec_len(c->n, d), s);
    if (e == hipSuccess) e = ws_alloc((void**)&row_t, sizeof(int32_t) * R, s);
    if (e == hipSuccess) e = ws_alloc((void**)&col_t, sizeof(int32_t) * C, s);
    if (e == hipSuccess) e = hilbert_tables(c->n, d, split, R, C, rec, row_t, col_t, s);
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pad_rt, dim3(grid_for(RK * C, 256)), dim3(256), 0, s, Rt, r, RK, C, Rp);
  if (fn) e = launch_err_p<double, false, true>(nullptr, R, C, r, L, Rp, gi, gj, part, FnTabs{rec, row_t, col_t}, s);
  else if (dtype == PSTT2_F64) e = launch_err((const double*)x, R, C, r, L, Rp, gi, gj, part, s);
  else e = launch_err((const float*)x, R, C, r, L, Rp, gi, gj, part, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, part, gi * gj, part + 2 * (int64_t)gi * gj);
    e = hipMemcpyAsync(e2x2, part + 2 * (int64_t)gi * gj, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
  }
  ws_free(part, s);
  ws_free(Rp, s);
  if (rec) ws_free(rec, s);
  if (row_t) ws_free(row_t, s);
  if (col_t) ws_free(col_t, s);
  ws_free(ifb, s);
  hipError_t e2 = hipStreamSynchronize(s);
  return e != hipSuccess ? e : e2;
}

// The Gaussian-bump tensor: chunks of whole columns of X_m are evaluated into a
// workspace (gauss_columns) and run through the memory kernel against the
// matching columns of Rt; every chunk's workgroup partials are kept and summed
// in one fixed-order pass at the end.
hipError_t tt_error_run_gauss(const tt_cores* c, const double* centers_host, int nterms, double gamma,
                              double* e2x2, hipStream_t s) {
  const int d = c->d;
  const int split = (d + 1) / 2;
  int64_t R = 1, C = 1;
  for (int k = 0; k < split; ++k) R *= c->n[k];
  for (int k = split; k < d; ++k) C *= c->n[k];
  double* tabs = nullptr;
  hipError_t e = ws_alloc((void**)&tabs, sizeof(double) * gauss_table_doubles(c->n, d, split, nterms), s);
  if (e != hipSuccess) return e;
  GaussTabs g;
  e = gauss_tables(c->n, d, split, centers_host, nterms, gamma, tabs, &g, s);
  double *L = nullptr, *Rt = nullptr, *ifb = nullptr;
  if (e == hipSuccess) e = tt_interfaces(c, split, &L, &Rt, &ifb, s);
  if (e != hipSuccess) {
    ws_free(tabs, s);
    return e;
  }
  const int r = c->r[split];
  const int RK = rk_slot(r);
  const int64_t ncmax = gauss_chunk_cols(g, sizeof(double));
  const int64_t nchunk = (C + ncmax - 1) / ncmax;
  const int gi = (int)((R + 511) / 512);
  const int gjmax = (int)std::max<int64_t>(1, std::min<int64_t>(ncmax, (4096 + gi - 1) / gi));
  double *part = nullptr, *Rp = nullptr, *W = nullptr;
  e = ws_alloc((void**)&part, sizeof(double) * 2 * ((int64_t)gi * gjmax * nchunk + 1), s);
  if (e == hipSuccess) e = ws_alloc((void**)&Rp, sizeof(double) * RK * C, s);
  if (e == hipSuccess) e = ws_alloc((void**)&W, sizeof(double) * R * ncmax, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_pad_rt, dim3(grid_for(RK * C, 256)), dim3(256), 0, s, Rt, r, RK, C, Rp);
    const bool pair = (R % 2) == 0;
    const FnTabs none{nullptr, nullptr, nullptr};
    int64_t np = 0;   // partial pairs written so far
    for (int64_t c0 = 0; c0 < C && e == hipSuccess; c0 += ncmax) {
      const int64_t nc = std::min(ncmax, C - c0);
      const int gj = (int)std::max<int64_t>(1, std::min<int64_t>(nc, (4096 + gi - 1) / gi));
      e = gauss_columns(g, c0, nc, PSTT2_F64, W, s);
      if (e != hipSuccess) break;
      e = pair ? launch_err_p<double, true, false>(W, R, nc, r, L, Rp + RK * c0, gi, gj, part + 2 * np, none, s)
               : launch_err_p<double, false, false>(W, R, nc, r, L, Rp + RK * c0, gi, gj, part + 2 * np, none, s);
      np += (int64_t)gi * gj;
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, part, (int)np, part + 2 * np);
      e = hipMemcpyAsync(e2x2, part + 2 * np, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
    }
  }
  if (part) ws_free(part, s);
  if (Rp) ws_free(Rp, s);
  if (W) ws_free(W, s);
  ws_free(ifb, s);
  ws_free(tabs, s);
  hipError_t e2 = hipStreamSynchronize(s);
  return e != hipSuccess ? e : e2;
}

template <typename T>
__global__ void k_reconstruct(T* __restrict__ out, int64_t first, int64_t count, int64_t R, int r,
                              const double* __restrict__ L, const double* __restrict__ Rt) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t f = first + t;
    const int64_t row = f % R, col = f / R;
    double s = 0.0;
    for (int b = 0; b < r; ++b) s += L[(int64_t)b * R + row] * Rt[b + (int64_t)r * col];
    out[t] = (T)s;
  }
}

hipError_t tt_reconstruct_run(const tt_cores* c, void* out, int dtype, int64_t first, int64_t count, hipStream_t s) {
  const int d = c->d;
  const int split = (d + 1) / 2;
  double *L = nullptr, *Rt = nullptr, *ifb = nullptr;
  hipError_t e = tt_interfaces(c, split, &L, &Rt, &ifb, s);
  if (e != hipSuccess) return e;
  int64_t R = 1;
  for (int k = 0; k < split; ++k) R *= c->n[k];
  const int r = c->r[split];
  if (count > 0) {
    if (dtype == PSTT2_F64)
      hipLaunchKernelGGL(k_reconstruct<double>, dim3(grid_for(count, 256)), dim3(256), 0, s, (double*)out, first,
                         count, R, r, L, Rt);
    else
      hipLaunchKernelGGL(k_reconstruct<float>, dim3(grid_for(count, 256)), dim3(256), 0, s, (float*)out, first,
                         count, R, r, L, Rt);
    e = hipGetLastError();
  }
  ws_free(ifb, s);
  hipError_t e2 = hipStreamSynchronize(s);
  return e != hipSuccess ? e : e2;
}

}  // namespace pstt2
