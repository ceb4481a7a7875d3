// Fixed-order reduction of the sketch kernels' workgroup partials into the
// FP64 sketches Y_R and T_m of the middle unfolding (PSTT2-onepass, Section
// 3.2): every entry adds its partials in increasing partial index, so the
// sketches are bitwise reproducible for a given launch sequence.
#include "internal.h"

namespace pstt2 {

// ---- fixed-order reduction of the tile partials into the FP64 sketches ----
template <typename P>
__global__ void k_reduce_y(const P* __restrict__ yp, int gj_count, int64_t R, int ell, double* __restrict__ Y,
                           int* flag) {
  const int64_t tot = R * ell;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    double s = Y[i];
    for (int g = 0; g < gj_count; ++g) s += (double)yp[(int64_t)g * tot + i];
    Y[i] = s;
    if (!isfinite(s)) atomicOr(flag, 1);
  }
}

// Tt is C x ell column-major (the transposed left sketch); tpart is [gi][a][gcol].
// One launch covers every segment of a sketch launch (blockIdx.y = segment).
// Each thread adds the gi partials of one entry in increasing g, sixteen loads
// in flight: the order, and so the result, does not depend on the launch shape.
// Offset of entry (a, col) in one row block's T partial and the stride between
// row blocks, for both partial layouts (SketchArgs::tlp).
__device__ __forceinline__ int64_t tpart_at(const SketchArgs& A, int a, int64_t col) {
  return A.tlp ? col * A.tlp + a : (int64_t)a * A.C + col;
}
__device__ __forceinline__ int64_t tpart_stride(const SketchArgs& A) {
  return A.tlp ? A.C * A.tlp : (int64_t)A.ell * A.C;
}

template <typename P>
__global__ void k_reduce_t(const P* __restrict__ tp, const SketchArgs A, double* __restrict__ Tt, int* flag) {
  constexpr int U = 16;
  const int64_t gc0 = A.seg[blockIdx.y].gcol0, ncols = A.seg[blockIdx.y].ncols;
  const int ell = A.ell, gi = A.gi_count;
  const int64_t C = A.C, st = tpart_stride(A);
  const int64_t tot = ncols * ell;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    // sketch index fastest for the contiguous layout, column fastest otherwise (coalesced reads)
    const int a = (int)(A.tlp ? i % ell : i / ncols);
    const int64_t col = gc0 + (A.tlp ? i / ell : i % ncols);
    const P* p = tp + tpart_at(A, a, col);
    double s = Tt[(int64_t)a * C + col];
    int g = 0;
    for (; g + U <= gi; g += U) {
      P v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = p[(int64_t)(g + u) * st];
#pragma unroll
      for (int u = 0; u < U; ++u) s += (double)v[u];
    }
    for (; g < gi; ++g) s += (double)p[(int64_t)g * st];
    Tt[(int64_t)a * C + col] = s;
    if (!isfinite(s)) atomicOr(flag, 1);
  }
}

// Few T entries and many row blocks (a very tall X_m with few columns, as in
// the one-sided algorithm's pass at split d-1): one thread per entry would add
// ~1e5 partials serially.  Then the row blocks are cut into nsplit contiguous
// groups, each group summed in increasing g into its own partial, and the
// group partials added in increasing group order (deterministic, as the split
// depends only on the shapes).
template <typename P>
__global__ void k_reduce_t_split(const P* __restrict__ tp, const SketchArgs A, int seg, int nsplit,
                                 double* __restrict__ out) {
  const int64_t gc0 = A.seg[seg].gcol0, ncols = A.seg[seg].ncols;
  const int ell = A.ell, gi = A.gi_count;
  const int64_t C = A.C, st = tpart_stride(A);
  const int64_t tot = ncols * ell;
  const int sp = blockIdx.y;
  const int g0 = (int)((int64_t)sp * gi / nsplit), g1 = (int)((int64_t)(sp + 1) * gi / nsplit);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(i / ncols);
    const int64_t col = gc0 + i % ncols;
    const P* p = tp + tpart_at(A, a, col);
    double sum = 0.0;
    for (int g = g0; g < g1; ++g) sum += (double)p[(int64_t)g * st];
    out[(int64_t)sp * tot + i] = sum;
  }
}

__global__ void k_reduce_t_join(const double* __restrict__ part, const SketchArgs A, int seg, int nsplit,
                                double* __restrict__ Tt, int* flag) {
  const int64_t gc0 = A.seg[seg].gcol0, ncols = A.seg[seg].ncols;
  const int64_t C = A.C, tot = ncols * A.ell;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(i / ncols);
    const int64_t col = gc0 + i % ncols;
    double sum = Tt[(int64_t)a * C + col];
    for (int sp = 0; sp < nsplit; ++sp) sum += part[(int64_t)sp * tot + i];
    Tt[(int64_t)a * C + col] = sum;
    if (!isfinite(sum)) atomicOr(flag, 1);
  }
}

hipError_t launch_reduce(int prec, const SketchArgs& a, double* Y, double* Tt, int* flag, hipStream_t s) {
  if (fault_take()) return hipErrorLaunchFailure;
  const int bs = 256;
  const int64_t ny = a.R * a.ell;
  const unsigned gy = (unsigned)std::min<int64_t>((ny + bs - 1) / bs, 4096);
  // With ydirect the sketch kernel has already added its one Y partial into Y.
  if (!a.ydirect && prec == PSTT2_P_F64)
    hipLaunchKernelGGL(k_reduce_y<double>, dim3(gy), dim3(bs), 0, s, (const double*)a.ypart, a.gj_count, a.R,
                       a.ell, Y, flag);
  else if (!a.ydirect)
    hipLaunchKernelGGL(k_reduce_y<float>, dim3(gy), dim3(bs), 0, s, (const float*)a.ypart, a.gj_count, a.R,
                       a.ell, Y, flag);
  int64_t nt = 0;
  for (int i = 0; i < a.nseg; ++i) nt = std::max<int64_t>(nt, a.seg[i].ncols * a.ell);
  if (a.nseg > 0 && nt < 16384 && a.gi_count >= 4096) {
    // two-level sum (see k_reduce_t_split), one segment at a time
    const int nsplit = (int)std::min<int64_t>(a.gi_count / 256, std::max<int64_t>(1, 65536 / std::max<int64_t>(nt, 1)));
    double* part = nullptr;
    hipError_t e = ws_alloc((void**)&part, sizeof(double) * nsplit * nt, s);
    if (e != hipSuccess) return e;
    for (int sg = 0; sg < a.nseg && e == hipSuccess; ++sg) {
      const int64_t tot = a.seg[sg].ncols * a.ell;
      const unsigned gx = (unsigned)std::max<int64_t>(1, (tot + bs - 1) / bs);
      if (prec == PSTT2_P_F64)
        hipLaunchKernelGGL(k_reduce_t_split<double>, dim3(gx, (unsigned)nsplit), dim3(bs), 0, s,
                           (const double*)a.tpart, a, sg, nsplit, part);
      else
        hipLaunchKernelGGL(k_reduce_t_split<float>, dim3(gx, (unsigned)nsplit), dim3(bs), 0, s,
                           (const float*)a.tpart, a, sg, nsplit, part);
      hipLaunchKernelGGL(k_reduce_t_join, dim3(gx), dim3(bs), 0, s, part, a, sg, nsplit, Tt, flag);
      e = hipGetLastError();
    }
    ws_free(part, s);
    if (e != hipSuccess) return e;
  } else if (a.nseg > 0) {
    const unsigned gt = (unsigned)std::max<int64_t>(1, std::min<int64_t>((nt + bs - 1) / bs, 4096));
    if (prec == PSTT2_P_F64)
      hipLaunchKernelGGL(k_reduce_t<double>, dim3(gt, (unsigned)a.nseg), dim3(bs), 0, s, (const double*)a.tpart, a,
                         Tt, flag);
    else
      hipLaunchKernelGGL(k_reduce_t<float>, dim3(gt, (unsigned)a.nseg), dim3(bs), 0, s, (const float*)a.tpart, a,
                         Tt, flag);
  }
  return hipGetLastError();
}

}  // namespace pstt2
