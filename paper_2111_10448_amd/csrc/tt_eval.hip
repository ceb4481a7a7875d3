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
#include <mutex>

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

// Doubles of every intermediate interface level at this split.
static int64_t tt_interfaces_doubles(const tt_cores* c, int split) {
  const int d = c->d;
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
  return tot;
}

// The interface levels built into ws (tt_interfaces_doubles of them); *Lout
// (R_split x r_split) and *Rout (r_split x C_split) point into ws or at a core.
static hipError_t tt_interfaces_in(const tt_cores* c, int split, double* ws, double** Lout, double** Rout,
                                   hipStream_t s) {
  const int d = c->d;
  double* cur = ws;
  int64_t Rp = c->n[0];
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
  int64_t Ck = c->n[d - 1];
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

// Interfaces in one stream-ordered workspace allocation: *base is returned for
// a single ws_free on the same stream.
hipError_t tt_interfaces(const tt_cores* c, int split, double** Lout, double** Rout, double** base, hipStream_t s) {
  double* ws = nullptr;
  hipError_t e = ws_alloc((void**)&ws, sizeof(double) * tt_interfaces_doubles(c, split), s);
  if (e != hipSuccess) return e;
  *base = ws;
  return tt_interfaces_in(c, split, ws, Lout, Rout, s);
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
// out[0..1] = (e2, x2); with rel, out[0..2] = (relative error, e2, x2), the
// relative error by the host rule (sqrt(e2 / x2); for x2 = 0: 0 if e2 = 0,
// else +inf).
__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ part, int nb, double* __restrict__ out,
                                                   bool rel) {
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
    const int o = rel ? 1 : 0;
    out[o] = sa[0];
    out[o + 1] = sb[0];
    if (rel) out[0] = sb[0] > 0.0 ? sqrt(sa[0] / sb[0]) : (sa[0] > 0.0 ? INFINITY : 0.0);
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

// Geometry and scratch of one error pass over X_m at the middle split.
struct ErrPlan {
  int split, r, RK, gi, gj;
  int64_t R, C;
  int64_t n_iface, n_part, n_rp;   // doubles of the interfaces, the partials (+ the 3 results), padded Rt
};

static ErrPlan err_plan(const tt_cores* c) {
  ErrPlan p;
  const int d = c->d;
  p.split = (d + 1) / 2;
  p.R = p.C = 1;
  for (int k = 0; k < p.split; ++k) p.R *= c->n[k];
  for (int k = p.split; k < d; ++k) p.C *= c->n[k];
  p.r = c->r[p.split];
  p.RK = rk_slot(p.r);
  p.gi = (int)((p.R + 511) / 512);
  p.gj = (int)std::max<int64_t>(1, std::min<int64_t>(p.C, (4096 + p.gi - 1) / p.gi));
  p.n_iface = tt_interfaces_doubles(c, p.split);
  p.n_part = 2 * (int64_t)p.gi * p.gj + 3;
  p.n_rp = (int64_t)p.RK * p.C;
  return p;
}

// The pass itself into caller-provided scratch: interfaces, padded Rt, the
// workgroup partials and their fixed-order sum at out: (e2, x2), or with rel
// (relative error, e2, x2).
// Every scratch entry is written before it is read: nothing needs clearing.
static hipError_t err_launch(const tt_cores* c, const ErrPlan& p, const void* x, int dtype, const FnTabs& fn,
                             double* iface, double* part, double* Rp, double* out, bool rel, hipStream_t s) {
  double *L = nullptr, *Rt = nullptr;
  hipError_t e = tt_interfaces_in(c, p.split, iface, &L, &Rt, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pad_rt, dim3(grid_for(p.n_rp, 256)), dim3(256), 0, s, Rt, p.r, p.RK, p.C, Rp);
  if (fn.rec) e = launch_err_p<double, false, true>(nullptr, p.R, p.C, p.r, L, Rp, p.gi, p.gj, part, fn, s);
  else if (dtype == PSTT2_F64) e = launch_err((const double*)x, p.R, p.C, p.r, L, Rp, p.gi, p.gj, part, s);
  else e = launch_err((const float*)x, p.R, p.C, p.r, L, Rp, p.gi, p.gj, part, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, part, p.gi * p.gj, out, rel);
  return hipGetLastError();
}

// x == nullptr: the Hilbert tensor (fn != 0), evaluated from its index tables
hipError_t tt_error_run(const tt_cores* c, const void* x, int dtype, double* e2x2, hipStream_t s, int fn) {
  const ErrPlan p = err_plan(c);
  double *iface = nullptr, *part = nullptr, *Rp = nullptr, *rec = nullptr;
  int32_t *row_t = nullptr, *col_t = nullptr;
  hipError_t e = ws_alloc((void**)&iface, sizeof(double) * std::max<int64_t>(p.n_iface, 1), s);
  if (e == hipSuccess) e = ws_alloc((void**)&part, sizeof(double) * p.n_part, s);
  if (e == hipSuccess) e = ws_alloc((void**)&Rp, sizeof(double) * p.n_rp, s);
  if (fn) {
    if (e == hipSuccess) e = ws_alloc((void**)&rec, sizeof(double) * hilbert_rec_len(c->n, c->d), s);
    if (e == hipSuccess) e = ws_alloc((void**)&row_t, sizeof(int32_t) * p.R, s);
    if (e == hipSuccess) e = ws_alloc((void**)&col_t, sizeof(int32_t) * p.C, s);
    if (e == hipSuccess) e = hilbert_tables(c->n, c->d, p.split, p.R, p.C, rec, row_t, col_t, s);
  }
  double* out = part ? part + 2 * (int64_t)p.gi * p.gj : nullptr;
  if (e == hipSuccess) e = err_launch(c, p, x, dtype, FnTabs{rec, row_t, col_t}, iface, part, Rp, out, false, s);
  if (e == hipSuccess) e = hipMemcpyAsync(e2x2, out, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (part) ws_free(part, s);
  if (Rp) ws_free(Rp, s);
  if (rec) ws_free(rec, s);
  if (row_t) ws_free(row_t, s);
  if (col_t) ws_free(col_t, s);
  if (iface) ws_free(iface, s);
  hipError_t e2 = hipStreamSynchronize(s);
  return e != hipSuccess ? e : e2;
}

// ---- the same pass with no allocation (tt_error_noalloc) ----
// The scratch is one file-scope device array.  Host code never uses its name as
// an address: the device address comes from hipGetSymbolAddress, once per
// device (each device holds its own copy), and only that pointer reaches the
// kernels.  Calls that overlap on one device share the array and race.
static __device__ __align__(256) unsigned char scratch[PSTT2_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

hipError_t scratch_base(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

int64_t align_doubles(int64_t n) { return (n + 31) / 32 * 32; }   // 256-byte steps
}  // namespace

// Bytes of static scratch an error pass of these cores needs.
int64_t tt_error_scratch_bytes(const tt_cores* c) {
  const ErrPlan p = err_plan(c);
  return 8 * (align_doubles(std::max<int64_t>(p.n_iface, 1)) + align_doubles(p.n_part) + align_doubles(p.n_rp));
}

hipError_t tt_error_noalloc_run(const tt_cores* c, const void* x, int dtype, double* err_dev, hipStream_t s) {
  const ErrPlan p = err_plan(c);
  void* base = nullptr;
  hipError_t e = scratch_base(&base);
  if (e != hipSuccess) return e;
  double* iface = (double*)base;
  double* part = iface + align_doubles(std::max<int64_t>(p.n_iface, 1));
  double* Rp = part + align_doubles(p.n_part);
  // the three results go straight to the caller's buffer
  return err_launch(c, p, x, dtype, FnTabs{nullptr, nullptr, nullptr}, iface, part, Rp, err_dev, true, s);
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
      hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, part, (int)np, part + 2 * np, false);
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
