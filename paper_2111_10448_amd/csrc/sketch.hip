// Streaming dual sketch of the middle unfolding (PSTT2-onepass, Section 3.2;
// Algorithm "parsketch": every sketch from a single read of each sub-tensor).
//
// For a tile X(I, J) of the middle unfolding X_m (column-major, leading
// dimension R = n_1...n_m) the kernel adds
//     Y_R(I, :) += X(I, J) Omega_m(J, :)        (right sketch, ell columns)
//     T_m(:, J) += Psi_m(I, :)^T X(I, J)         (left sketch, ell rows)
// where the Khatri-Rao DRM rows are products of per-mode Gaussian factors
// (equation "sketch_orig"): Omega_m(j, c) = prod_{q>m} omega_q(j_q, c),
// Psi_m(i, a) = prod_{q<=m} psi_q(i_q, a).
//
// Work decomposition (one workgroup = 4 waves of 64 lanes, two workgroups per
// compute unit):
//   * a workgroup owns a block of 4*RW consecutive rows and a contiguous share of
//     the launch's 16-column chunks; each wave owns RW of the rows;
//   * per chunk a wave loads its RW x 16 tile with 16-byte coalesced loads,
//     stages it in a wave-private LDS tile, and runs matrix-core (MFMA) tiles
//       right sketch: Y(rows, ell) += X(rows, 16 cols) * Omega(16 cols, ell)
//       left sketch : T(ell, 16 cols) = Psi(rows, ell)^T * X(rows, 16 cols);
//   * Y accumulates in registers over the workgroup's whole column share and is
//     written once as a partial; T of the 4 waves is summed through LDS and
//     written per chunk as a partial (one per row block);
//   * Psi rows are stationary (computed once per workgroup from the factors);
//     Omega rows of a chunk are built cooperatively into LDS two chunks ahead.
// A separate kernel sums the partials in a fixed order into the FP64 sketches,
// so results are bitwise reproducible.
#include "internal.h"

namespace pstt2 {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));

// Two 4-element bf16 operands as one 8-element operand of the 16x16x32 bf16
// matrix instruction.  Both operands of a product are joined the same way, so
// element v of lane l pairs the same K index in A and B whatever order the
// hardware assigns to the 32 K slots.
__device__ __forceinline__ b8 join8(s4 lo, s4 hi) {
  const s8 v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_bit_cast(b8, v);
}

enum { P_F64 = 0, P_F32 = 1, P_BF16 = 2, P_BF16X3 = 3, P_F16 = 4 };

constexpr int KC = 16;  // columns per chunk

// Round-to-nearest-even FP32 -> BF16 (bit pattern in the low 16 bits).
__device__ __forceinline__ uint32_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
// x = t0 + t1 + t2 with t0 = bf16(x), t1 = bf16(x - t0), t2 = bf16(x - t0 - t1).
// Each subtraction is exact in FP32 and the three terms hold the whole 24-bit
// significand, so the split of an FP32 value is exact (barring underflow).
struct Split3 {
  short t0, t1, t2;
};
__device__ __forceinline__ Split3 split3(float f) {
  const uint32_t h = bf16_rne(f);
  const float r1 = f - __uint_as_float(h << 16);
  const uint32_t m = bf16_rne(r1);
  const float r2 = r1 - __uint_as_float(m << 16);
  const uint32_t l = bf16_rne(r2);
  return Split3{(short)h, (short)m, (short)l};
}
// Three-term splits of four FP32 values (one MFMA operand per term).
__device__ __forceinline__ void split3x4(float a, float b, float c, float d, s4& t0, s4& t1, s4& t2) {
  const Split3 sa = split3(a), sb = split3(b), sc = split3(c), sd = split3(d);
  t0 = s4{sa.t0, sb.t0, sc.t0, sd.t0};
  t1 = s4{sa.t1, sb.t1, sc.t1, sd.t1};
  t2 = s4{sa.t2, sb.t2, sc.t2, sd.t2};
}

template <int PREC>
struct Eng;
template <>
struct Eng<P_F64> {
  using elem = double;   // X in HBM
  using lds_t = double;  // X and Omega in LDS
  using acc = double;
  using accv = d4;
  using part = double;   // partial sums written to HBM
  static constexpr int KPL = 1, KSTEP = 4, RW = 64, VEC = 2, PAD = 2, NPL = 1;
};
template <>
struct Eng<P_F32> {
  using elem = float;
  using lds_t = float;
  using acc = float;
  using accv = f4;
  using part = float;
  static constexpr int KPL = 1, KSTEP = 4, RW = 128, VEC = 4, PAD = 4, NPL = 1;
};
// Split BF16: X and the DRM are split into three bf16 terms once, when they
// are staged in LDS (three planes); the six products of order <= 2 are summed.
template <>
struct Eng<P_BF16X3> {
  using elem = float;
  using lds_t = uint16_t;
  using acc = float;
  using accv = f4;
  using part = float;
  static constexpr int KPL = 4, KSTEP = 16, RW = 64, VEC = 4, PAD = 4, NPL = 3;
};

// Hardware round-to-nearest-even FP32 -> BF16 of two values (packed, first in
// the low half), and the exact three-term split of two FP32 values into packed
// bf16 planes: t0 = bf16(x), t1 = bf16(x - t0), t2 = bf16(x - t0 - t1).
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t cvt2(float a, float b) {
  const f2v v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf2v));
}
__device__ __forceinline__ float lo_f(uint32_t p) { return __uint_as_float(p << 16); }
__device__ __forceinline__ float hi_f(uint32_t p) { return __uint_as_float(p & 0xffff0000u); }
__device__ __forceinline__ void split3_pk(float a, float b, uint32_t& t0, uint32_t& t1, uint32_t& t2) {
  t0 = cvt2(a, b);
  const float ra = a - lo_f(t0), rb = b - hi_f(t0);
  t1 = cvt2(ra, rb);
  t2 = cvt2(ra - lo_f(t1), rb - hi_f(t1));
}
// four bf16 of one plane at stride st (elements) as an MFMA operand
__device__ __forceinline__ s4 gather4(const uint16_t* p, int st) {
  return s4{(short)p[0], (short)p[st], (short)p[2 * st], (short)p[3 * st]};
}
// eight of them (the 32-deep and 32x32x16 instruction operands)
__device__ __forceinline__ b8 gather8(const uint16_t* p, int st) {
  const s8 v = {(short)p[0],      (short)p[st],     (short)p[2 * st], (short)p[3 * st],
                (short)p[4 * st], (short)p[5 * st], (short)p[6 * st], (short)p[7 * st]};
  return __builtin_bit_cast(b8, v);
}

template <int PREC>
__device__ __forceinline__ typename Eng<PREC>::lds_t to_lds(typename Eng<PREC>::elem v);
template <>
__device__ __forceinline__ double to_lds<P_F64>(double v) { return v; }
template <>
__device__ __forceinline__ float to_lds<P_F32>(float v) { return v; }

// DRM value (FP64 product of factors) converted to the LDS representation.
template <int PREC>
__device__ __forceinline__ typename Eng<PREC>::lds_t drm_to_lds(double v) {
  if constexpr (PREC == P_F64) return v;
  else return (float)v;
}

// Row of element v of a lane's 16x16 MFMA accumulator tile (column = lane % 16).
// FP64 16x16x4 places element v at row 4*v + lane/16; the FP32-accumulating
// 16x16 instructions at row 4*(lane/16) + v.
template <int PREC>
__device__ __forceinline__ int acc_row(int g4, int v) {
  return PREC == P_F64 ? 4 * v + g4 : 4 * g4 + v;
}

// Psi_m(row, a) = psi_1(i_1, a) * psi_hi(h, a) for the row i_1 + n_1 h of X_m:
// psi_hi is the product of the factor entries of modes 2..m (the mixed-radix
// digits of h), multiplied in increasing mode order.
__device__ __forceinline__ double psi_hi(const SketchArgs& A, int64_t h, int a) {
  double v = 1.0;
  if (h <= 0xffffffffLL) {
    // 32-bit index arithmetic: a few instructions per division instead of the 64-bit sequence
    uint32_t r = (uint32_t)h;
    for (int q = 2; q <= A.m; ++q) {
      const uint32_t nq = (uint32_t)A.n[q - 1];
      const uint32_t iq = r % nq;
      r /= nq;
      v *= A.fac[A.psi_off[q - 1] + (int64_t)iq * A.ell + a];
    }
    return v;
  }
  int64_t r = h;
  for (int q = 2; q <= A.m; ++q) {
    const int64_t nq = A.n[q - 1];
    const int64_t iq = r % nq;
    r /= nq;
    v *= A.fac[A.psi_off[q - 1] + iq * A.ell + a];
  }
  return v;
}

// Psi_m(row, a) for a global row of X_m (0 outside the matrix / sketch).
__device__ __forceinline__ double psi_row(const SketchArgs& A, int64_t row, int a) {
  if (row >= A.R || a >= A.ell) return 0.0;
  if (A.psi_tab) return A.psi_tab[row * A.L4 + a];
  const int64_t h = row / A.n[0];
  const int64_t i1 = row - h * A.n[0];
  return A.fac[A.psi_off[0] + i1 * A.ell + a] * psi_hi(A, h, a);
}

// A lane's rows of Psi_m, visited in increasing order by the workgroup
// prologues: (i_1, h) with row = i_1 + n_1 h is advanced without division, and
// the caller forms psi_hi again only when h changes (and only inside the
// matrix, where h's top digit is a valid index).  Values equal psi_row's.
struct PsiCursor {
  int64_t row = 0, h = 0, hc = -1;
  int64_t i1 = 0;
  __device__ __forceinline__ void init(const SketchArgs& A, int64_t r) {
    row = r;
    h = r / A.n[0];
    i1 = r - h * A.n[0];
  }
  __device__ __forceinline__ void advance(const SketchArgs& A, int by) {
    row += by;
    i1 += by;
    while (i1 >= A.n[0]) {
      i1 -= A.n[0];
      ++h;
    }
  }
  // true when the caller must recompute its psi_hi values for this row
  __device__ __forceinline__ bool refresh(const SketchArgs& A) {
    if (row >= A.R || A.psi_tab || h == hc) return false;
    hc = h;
    return true;
  }
  __device__ __forceinline__ double at(const SketchArgs& A, int a, double hi) const {
    if (row >= A.R || a >= A.ell) return 0.0;
    if (A.psi_tab) return A.psi_tab[row * A.L4 + a];
    return A.fac[A.psi_off[0] + i1 * A.ell + a] * hi;
  }
};

// Omega_m(gcol, c) for a global column of X_m.
__device__ __forceinline__ double omega_col(const SketchArgs& A, int64_t gcol, int c) {
  double v = 1.0;
  int64_t r = gcol;
  for (int q = A.m + 1; q <= A.d; ++q) {
    int64_t nq = A.n[q - 1];
    int64_t iq = r % nq;
    r /= nq;
    v *= A.fac[A.omega_off[q - 1] + iq * A.ell + c];
  }
  return v;
}

struct ChunkInfo {
  const char* ptr;   // column 0 of the chunk's segment
  int64_t lcol0;     // first column of the chunk within its segment
  int64_t gcol0;     // global column of the chunk's first column
  int ncols;         // valid columns (<= KC)
};

__device__ __forceinline__ ChunkInfo chunk_info(const SketchArgs& A, int64_t ci) {
  int s = 0;
  while (s + 1 < A.nseg && A.seg[s + 1].chunk0 <= ci) ++s;
  ChunkInfo c;
  c.ptr = (const char*)A.seg[s].ptr;
  c.lcol0 = (ci - A.seg[s].chunk0) * KC;
  c.gcol0 = A.seg[s].gcol0 + c.lcol0;
  int64_t left = A.seg[s].ncols - c.lcol0;
  c.ncols = (int)(left < KC ? left : KC);
  return c;
}

// Chunk geometry for a workgroup that visits its chunks in increasing order:
// the segment index only moves forward, so each lookup costs O(1) amortised
// instead of a search over all segments.
struct SegCursor {
  int s = 0;
  __device__ __forceinline__ ChunkInfo at(const SketchArgs& A, int64_t ci) {
    while (s + 1 < A.nseg && A.seg[s + 1].chunk0 <= ci) ++s;
    ChunkInfo c;
    c.ptr = (const char*)A.seg[s].ptr;
    c.lcol0 = (ci - A.seg[s].chunk0) * KC;
    c.gcol0 = A.seg[s].gcol0 + c.lcol0;
    const int64_t left = A.seg[s].ncols - c.lcol0;
    c.ncols = (int)(left < KC ? left : KC);
    return c;
  }
};

// Chunk geometry when the launch holds one segment (the whole-tensor case):
// closed form, no search over segments.
__device__ __forceinline__ ChunkInfo chunk_info1(const SketchArgs& A, int64_t ci) {
  ChunkInfo c;
  c.ptr = (const char*)A.seg[0].ptr;
  c.lcol0 = ci * KC;
  c.gcol0 = A.seg[0].gcol0 + c.lcol0;
  const int64_t left = A.seg[0].ncols - c.lcol0;
  c.ncols = (int)(left < KC ? left : KC);
  return c;
}

// Workgroups of 4 waves, two per CU (as the FP64 kernel).
constexpr int NWS = 4;

template <int PREC, int LP, bool ALIGNED, bool SEG1>
__global__ __launch_bounds__(NWS * 64, 2) void k_sketch(const SketchArgs A) {
  using E = Eng<PREC>;
  using elem = typename E::elem;
  using lds_t = typename E::lds_t;
  using acc = typename E::acc;
  using accv = typename E::accv;
  using part = typename E::part;
  constexpr int RW = E::RW;
  constexpr int ST = RW + E::PAD;   // LDS column stride of the X tile (elements)
  constexpr int MT = RW / 16;       // row tiles per wave (right sketch)
  constexpr int NT = LP / 16;       // ell tiles
  constexpr int KT = RW / E::KSTEP; // K steps over rows (left sketch)
  constexpr int VEC = E::VEC;       // elements per 16-byte load
  constexpr int NLD = KC * RW / (64 * VEC);  // 16-byte loads per lane per chunk

  constexpr int NTH = NWS * 64;          // threads
  constexpr int NRT = (LP * KC + NTH - 1) / NTH;   // T outputs per thread in the reduction
  static_assert(KC * LP / 2 <= NTH, "one Omega pair per thread");
  static_assert(sizeof(elem) == 4 && VEC == 4, "FP32 tensors, 16-byte loads of four entries");
  constexpr int NPL = E::NPL;                // bf16 planes of X and Omega in LDS (1 otherwise)
  __shared__ __align__(16) lds_t Xl[NWS][NPL * KC * ST];
  __shared__ acc Tred[2][NWS][LP * KC];
  __shared__ __align__(16) lds_t Om[4][NPL * KC * LP];   // 4 buffers: each write is a barrier past the last read

  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int gi = blockIdx.x % A.gi_count;
  const int gj = blockIdx.x / A.gi_count;
  const int64_t row0w = (int64_t)gi * (NWS * RW) + (int64_t)w * RW;
  const int64_t cb = (int64_t)gj * A.nchunks / A.gj_count;
  const int64_t ce = (int64_t)(gj + 1) * A.nchunks / A.gj_count;
  const int l16 = lane & 15, g4 = lane >> 4;

  // ---- stationary left-DRM operand (A operand of the left-sketch MFMA) ----
  // element [a][row] with a = 16*mt + l16 and row = K index
  // (BF16X3: psiA, psiM, psiL are the three split terms)
  constexpr bool X3 = PREC == P_BF16X3;
  typename std::conditional<E::KPL == 1, lds_t, s4>::type psiA[KT][NT];
  s4 psiM[X3 ? KT : 1][X3 ? NT : 1];
  s4 psiL[X3 ? KT : 1][X3 ? NT : 1];
  (void)psiM;
  (void)psiL;
  {
    PsiCursor pc;
    double hv[NT];
    if constexpr (E::KPL == 1) {   // rows row0w + KSTEP ks + g4
      pc.init(A, row0w + g4);
#pragma unroll
      for (int ks = 0; ks < KT; ++ks) {
        if (ks > 0) pc.advance(A, E::KSTEP);
        if (pc.refresh(A)) {
#pragma unroll
          for (int mt = 0; mt < NT; ++mt) hv[mt] = psi_hi(A, pc.h, 16 * mt + l16);
        }
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) psiA[ks][mt] = drm_to_lds<PREC>(pc.at(A, 16 * mt + l16, hv[mt]));
      }
    } else {   // rows row0w + 16 ks + 4 g4 + v, v = 0..3
      pc.init(A, row0w + 4 * g4);
#pragma unroll
      for (int ks = 0; ks < KT; ++ks) {
        float p[4][NT];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (ks > 0 || v > 0) pc.advance(A, v > 0 ? 1 : 13);
          if (pc.refresh(A)) {
#pragma unroll
            for (int mt = 0; mt < NT; ++mt) hv[mt] = psi_hi(A, pc.h, 16 * mt + l16);
          }
#pragma unroll
          for (int mt = 0; mt < NT; ++mt) p[v][mt] = (float)pc.at(A, 16 * mt + l16, hv[mt]);
        }
#pragma unroll
        for (int mt = 0; mt < NT; ++mt)
          split3x4(p[0][mt], p[1][mt], p[2][mt], p[3][mt], psiA[ks][mt], psiM[ks][mt], psiL[ks][mt]);
      }
    }
  }

  // one cursor per stream of lookups (X loads, Omega loads, T partials), each
  // visiting chunks in increasing order
  SegCursor cx, co, ct;
  auto info = [&](SegCursor& cu, int64_t ci) -> ChunkInfo { return SEG1 ? chunk_info1(A, ci) : cu.at(A, ci); };

  // Omega_m rows of a chunk: thread t < KC*LP/2 holds entries e = 2t, 2t + 1 of
  // row e / LP (LP is even; the table's columns ell..L4-1 are zero and the
  // ones past L4 are skipped).  Loaded one iteration before they are written
  // to LDS, so waiting for them never waits for the X prefetch (loads retire
  // in order).
  // NB register slots: with NB = 2 (sketch size <= 16, where registers allow)
  // two chunks of X are in flight while one is computed.  UNC: every memory
  // operation of the chunk loop is issued by every lane (addresses clamped
  // into the data, values zeroed when staged, idle lanes storing to spare
  // entries), so no branch separates one step's loads and stores from the
  // next and the loop waits only for the loads it needs.  Measured: a gain
  // with two chunks in flight, a small loss with one.
  constexpr int NB = LP == 16 ? 2 : 1;
  constexpr bool UNC = NB == 2;
  double2 omv;
  bool omok = true;
  auto load_omega = [&](int64_t ci) {
    const int e = 2 * threadIdx.x;
    if constexpr (UNC) {
      ChunkInfo ch = info(co, ci < ce ? ci : ce - 1);
      const int col = e / LP, c = e % LP;
      omok = e < KC * LP && ci < ce && col < ch.ncols && c < A.L4;
      omv = *(const double2*)&A.om_tab[(ch.gcol0 + (omok ? col : 0)) * A.L4 + (omok ? c : 0)];
    } else {
      omv = double2{0.0, 0.0};
      if (e < KC * LP && ci < ce) {
        ChunkInfo ch = info(co, ci);
        const int col = e / LP, c = e % LP;
        if (col < ch.ncols && c < A.L4) omv = *(const double2*)&A.om_tab[(ch.gcol0 + col) * A.L4 + c];
      }
    }
  };
  auto store_omega = [&](int buf) {
    const int e = 2 * threadIdx.x;
    if (UNC && !omok) omv = double2{0.0, 0.0};
    if (e < KC * LP) {
      if constexpr (X3) {
        uint32_t t0, t1, t2;
        split3_pk((float)omv.x, (float)omv.y, t0, t1, t2);
        *(uint32_t*)&Om[buf][e] = t0;
        *(uint32_t*)&Om[buf][KC * LP + e] = t1;
        *(uint32_t*)&Om[buf][2 * KC * LP + e] = t2;
      } else {
        Om[buf][e] = drm_to_lds<PREC>(omv.x);
        Om[buf][e + 1] = drm_to_lds<PREC>(omv.y);
      }
    }
  };

  // ---- global loads of one chunk (16-byte, coalesced along rows) ----
  elem xr[NB][NLD][VEC];
  bool xok[NB][NLD][ALIGNED ? 1 : VEC];   // loaded entry lies in the matrix
  auto load_chunk = [&](int64_t ci, int slot) {
    ChunkInfo ch = info(cx, ci);
    const elem* base = (const elem*)ch.ptr;
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      const int cc = i * (64 * VEC / RW) + lane / (RW / VEC);
      const int r = (lane % (RW / VEC)) * VEC;
      const int64_t row = row0w + r;
      const bool colok = cc < ch.ncols;
      const elem* col = base + (ch.lcol0 + (colok ? cc : 0)) * A.R;
      if constexpr (!UNC) {
        if constexpr (ALIGNED) {
          float4 v = float4{0.0f, 0.0f, 0.0f, 0.0f};
          if (colok && row < A.R) v = *(const float4*)(col + row);
          xr[slot][i][0] = v.x;
          xr[slot][i][1] = v.y;
          xr[slot][i][2] = v.z;
          xr[slot][i][3] = v.w;
        } else {
#pragma unroll
          for (int v = 0; v < VEC; ++v) xr[slot][i][v] = (colok && row + v < A.R) ? col[row + v] : (elem)0;
        }
      } else if constexpr (ALIGNED) {
        const bool ok = colok && row < A.R;
        const float4 v = *(const float4*)(col + (ok ? row : 0));
        xr[slot][i][0] = v.x;
        xr[slot][i][1] = v.y;
        xr[slot][i][2] = v.z;
        xr[slot][i][3] = v.w;
        xok[slot][i][0] = ok;
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const bool ok = colok && row + v < A.R;
          xr[slot][i][v] = col[ok ? row + v : 0];
          xok[slot][i][v] = ok;
        }
      }
    }
  };
  auto store_chunk = [&](int slot) {
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      if constexpr (UNC) {
#pragma unroll
        for (int v = 0; v < VEC; ++v)
          if (!xok[slot][i][ALIGNED ? 0 : v]) xr[slot][i][v] = (elem)0;
      }
      const int cc = i * (64 * VEC / RW) + lane / (RW / VEC);
      const int r = (lane % (RW / VEC)) * VEC;
      if constexpr (X3) {
        uint32_t a0, a1, a2, b0, b1, b2;
        split3_pk(xr[slot][i][0], xr[slot][i][1], a0, a1, a2);
        split3_pk(xr[slot][i][2], xr[slot][i][3], b0, b1, b2);
        *(uint2*)&Xl[w][cc * ST + r] = uint2{a0, b0};
        *(uint2*)&Xl[w][KC * ST + cc * ST + r] = uint2{a1, b1};
        *(uint2*)&Xl[w][2 * KC * ST + cc * ST + r] = uint2{a2, b2};
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) Xl[w][cc * ST + r + v] = to_lds<PREC>(xr[slot][i][v]);
      }
    }
  };

  // live = false (before the first chunk) sends every store to the spare entries
  auto reduce_t = [&](int buf, int64_t ci, bool live) {
    ChunkInfo ch = info(ct, ci);
    part* tp = (part*)A.tpart;
    const int64_t spare = (int64_t)A.gi_count * A.ell * A.C;
#pragma unroll
    for (int q = 0; q < NRT; ++q) {
      const int t = threadIdx.x + NTH * q;
      const int tc = t < LP * KC ? t : 0;
      const int a = tc / KC, col = tc % KC;
      acc s = 0;
#pragma unroll
      for (int ww = 0; ww < NWS; ++ww) s += Tred[buf][ww][a * KC + col];
      const bool ok = live && t < LP * KC && a < A.ell && col < ch.ncols;
      if constexpr (UNC)
        tp[ok ? ((int64_t)gi * A.ell + a) * A.C + ch.gcol0 + col : spare + t] = (part)s;
      else if (ok)
        tp[((int64_t)gi * A.ell + a) * A.C + ch.gcol0 + col] = (part)s;
    }
  };

  // Split BF16 at sketch size 32: the right sketch runs on 32x32x16 bf16 tiles
  // (32 rows x all 32 sketch columns x the chunk's 16 columns per
  // instruction).  Accumulator element v of lane l sits at row
  // 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32 of the tile.
  constexpr bool W32 = X3 && LP == 32 && MT % 2 == 0;
  accv yacc[W32 ? 1 : MT][NT];
  f16v y32[W32 ? MT / 2 : 1];
#pragma unroll
  for (int mt = 0; mt < (W32 ? 1 : MT); ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) yacc[mt][nt] = accv{0, 0, 0, 0};
#pragma unroll
  for (int h = 0; h < (W32 ? MT / 2 : 1); ++h)
#pragma unroll
    for (int v = 0; v < 16; ++v) y32[h][v] = 0.0f;

  if (cb < ce) {
    load_omega(cb);
    store_omega(0);
    load_omega(cb + 1);
    store_omega(1);
    load_chunk(cb, 0);
    load_omega(cb + 2);
    if (NB == 2) load_chunk(cb + 1 < ce ? cb + 1 : ce - 1, 1);
  }

  // one chunk: slot is a constant at every call (the loop below is unrolled by NB)
  auto chunk_step = [&](int64_t ci, int it, int slot) {
    // (a) stage this chunk in the wave's LDS tile and the Omega rows of chunk
    //     ci + 2 (both loaded earlier); one barrier per chunk
    store_chunk(slot);
    store_omega((it + 2) % 4);
    __syncthreads();
    // (b) prefetch: Omega three chunks ahead, then the chunk NB ahead into the
    //     slot just staged (loads retire in order, so the Omega rows the next
    //     step stages never wait for the newest X chunk)
    if constexpr (NB == 1) {
      if (ci + 1 < ce) load_chunk(ci + 1, 0);
      load_omega(ci + 3);
    } else {   // the last chunk again at the end: the loads stay unconditional
      load_omega(ci + 3);
      load_chunk(ci + 2 < ce ? ci + 2 : ce - 1, slot);
    }
    // (c) finish the previous chunk's left sketch
    if (UNC || it >= 1) reduce_t((it - 1) & 1, it >= 1 ? ci - 1 : ci, it >= 1);
    // (d) matrix-core tiles, at raised wave priority: the two workgroups on a
    //     compute unit then drift out of step, so one's matrix-core phase
    //     covers the other's load and barrier phase (measured: split BF16
    //     -6% and FP32 -2% per launch; no gain for the FP64 kernel)
    __builtin_amdgcn_s_setprio(1);
    const lds_t* xw = Xl[w];
    const lds_t* om = Om[it % 4];
    // right sketch: Y(rows, ell) += X(rows, cols) Omega(cols, ell)
    if constexpr (E::KPL == 1) {
#pragma unroll
      for (int ks = 0; ks < KC / 4; ++ks) {
        lds_t b[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) b[nt] = om[(4 * ks + g4) * LP + 16 * nt + l16];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const lds_t a = xw[(4 * ks + g4) * ST + 16 * mt + l16];
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            if constexpr (PREC == P_F64)
              yacc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[nt], yacc[mt][nt], 0, 0, 0);
            else
              yacc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[nt], yacc[mt][nt], 0, 0, 0);
          }
        }
      }
    } else if constexpr (W32) {
      // six products t_i * t_j with i + j <= 2, smallest first; K index
      // 8 (l / 32) + j of both operands is chunk column 8 (l / 32) + j
      const int ob = 8 * (lane >> 5) * LP + (lane & 31);
      const b8 w0 = gather8(om + ob, LP), w1 = gather8(om + KC * LP + ob, LP), w2 = gather8(om + 2 * KC * LP + ob, LP);
#pragma unroll
      for (int h = 0; h < MT / 2; ++h) {
        const int o = 8 * (lane >> 5) * ST + 32 * h + (lane & 31);
        const b8 a0 = gather8(xw + o, ST), a1 = gather8(xw + KC * ST + o, ST), a2 = gather8(xw + 2 * KC * ST + o, ST);
        f16v y = y32[h];
        y = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, w0, y, 0, 0, 0);
        y = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, w1, y, 0, 0, 0);
        y = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, w2, y, 0, 0, 0);
        y = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, w0, y, 0, 0, 0);
        y = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, w1, y, 0, 0, 0);
        y32[h] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, w0, y, 0, 0, 0);
      }
    } else {
      // six products t_i * t_j with i + j <= 2, smallest first
      s4 b0[NT], b1[NT], b2[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int o = 4 * g4 * LP + 16 * nt + l16;
        b0[nt] = gather4(om + o, LP);
        b1[nt] = gather4(om + KC * LP + o, LP);
        b2[nt] = gather4(om + 2 * KC * LP + o, LP);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int o = 4 * g4 * ST + 16 * mt + l16;
        const s4 a0 = gather4(xw + o, ST), a1 = gather4(xw + KC * ST + o, ST), a2 = gather4(xw + 2 * KC * ST + o, ST);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          accv y = yacc[mt][nt];
          y = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2, b0[nt], y, 0, 0, 0);
          y = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b1[nt], y, 0, 0, 0);
          y = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b2[nt], y, 0, 0, 0);
          y = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b0[nt], y, 0, 0, 0);
          y = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b1[nt], y, 0, 0, 0);
          yacc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b0[nt], y, 0, 0, 0);
        }
      }
    }
    // left sketch: T(ell, cols) = Psi(rows, ell)^T X(rows, cols)
    accv tacc[NT];
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) tacc[mt] = accv{0, 0, 0, 0};
    if constexpr (X3) {
      // split BF16: two 16-row K steps per 16x16x32 instruction (rows
      // 32j + 4 g4 + v and 32j + 16 + 4 g4 + v in the two halves of an
      // operand), half the instructions of the 16x16x16 form
      static_assert(KT % 2 == 0, "pairs of 16-row K steps");
#pragma unroll
      for (int j = 0; j < KT / 2; ++j) {
        const int ka = 2 * j, kb = 2 * j + 1;
        {
          const int oa = l16 * ST + 16 * ka + 4 * g4, ob = l16 * ST + 16 * kb + 4 * g4;
          const b8 b0 = join8(*(const s4*)&xw[oa], *(const s4*)&xw[ob]);
          const b8 b1 = join8(*(const s4*)&xw[KC * ST + oa], *(const s4*)&xw[KC * ST + ob]);
          const b8 b2 = join8(*(const s4*)&xw[2 * KC * ST + oa], *(const s4*)&xw[2 * KC * ST + ob]);
#pragma unroll
          for (int mt = 0; mt < NT; ++mt) {
            const b8 pA = join8(psiA[ka][mt], psiA[kb][mt]);
            const b8 pM = join8(psiM[ka][mt], psiM[kb][mt]);
            const b8 pL = join8(psiL[ka][mt], psiL[kb][mt]);
            accv t = tacc[mt];
            t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pL, b0, t, 0, 0, 0);
            t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pM, b1, t, 0, 0, 0);
            t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pA, b2, t, 0, 0, 0);
            t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pM, b0, t, 0, 0, 0);
            t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pA, b1, t, 0, 0, 0);
            tacc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pA, b0, t, 0, 0, 0);
          }
        }
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < KT; ++ks) {
        const lds_t b = xw[l16 * ST + 4 * ks + g4];
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) {
          if constexpr (PREC == P_F64)
            tacc[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(psiA[ks][mt], b, tacc[mt], 0, 0, 0);
          else
            tacc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(psiA[ks][mt], b, tacc[mt], 0, 0, 0);
        }
      }
    }
    __builtin_amdgcn_s_setprio(0);
    acc* tr = Tred[it & 1][w];
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) tr[(16 * mt + acc_row<PREC>(g4, v)) * KC + l16] = tacc[mt][v];
  };

  int it = 0;
  int64_t ci = cb;
  if constexpr (NB == 2) {
    for (; ci + 1 < ce; ci += 2, it += 2) {
      chunk_step(ci, it, 0);
      chunk_step(ci + 1, it + 1, 1);
    }
  }
  for (; ci < ce; ++ci, ++it) chunk_step(ci, it, 0);
  __syncthreads();
  if (it >= 1) reduce_t((it - 1) & 1, ce - 1, true);

  // ---- right-sketch partial of this workgroup ----
  part* yp = (part*)A.ypart;
  if constexpr (W32) {
#pragma unroll
    for (int h = 0; h < MT / 2; ++h)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = row0w + 32 * h + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
        const int c = lane & 31;
        if (row < A.R && c < A.ell) yp[((int64_t)gj * A.ell + c) * A.R + row] = (part)y32[h][v];
      }
  } else {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = row0w + 16 * mt + acc_row<PREC>(g4, v);
          const int c = 16 * nt + l16;
          if (row < A.R && c < A.ell) yp[((int64_t)gj * A.ell + c) * A.R + row] = (part)yacc[mt][nt][v];
        }
  }
}

// ---------------------------------------------------------------------------
// 16-bit sketch kernels for FP32 tensors: plain BF16, FP16 and split BF16
// (three bf16 planes).  Workgroup = NW waves; a wave owns 64 rows of X_m and
// the workgroup a contiguous share of 32-column chunks.  Per chunk a lane
// loads eight 16-byte fragments: rows 16 rt + 4 (l / 16) .. + 3 of column
// 16 ct + l % 16 (rt < 4, ct < 2), which is exactly the B operand of the
// 16 x 16 x 16 product for the left sketch T = Psi^T X (K = rows).  So:
//   * the left sketch runs straight from the converted load registers (two
//     16-row fragments joined into one 32-deep operand, Psi joined the same
//     way, so element v of every lane pairs the same row in both operands);
//   * the right sketch Y = X Omega needs K = columns: the converted fragments
//     are written to a wave-private column-major LDS tile (one 8-byte store
//     each) and read back with the transposing 16-bit LDS read, which hands
//     each lane one row and four consecutive columns (lane i of a 16-lane
//     group receives element e from the address of lane 4 e + i / 4 at
//     half-word i % 4);
//   * the Omega operands come pre-rounded (per plane) from a 16-bit table
//     (L2-resident), loaded into registers one chunk ahead by every wave;
//   * FP32 -> 16-bit conversion is the hardware packed conversion (round to
//     nearest even), two values per instruction; split BF16 takes the exact
//     three-term split of each value (t0 + t1 + t2).
// Raw X of two chunks is in flight per wave (register double buffer, every
// load unconditional: out-of-range entries read a valid address and are
// zeroed when converted).  There is no workgroup barrier in the chunk loop:
// the waves' T tiles of a chunk go to one of NS LDS slots, each wave then
// counts itself in with an LDS atomic, and the last wave to arrive adds the
// NW tiles in increasing wave order (the same order whichever wave it is, so
// the result is deterministic), writes the T partial and releases the slot
// (a generation count the waves check before reusing it).  Waves therefore
// drift freely, up to NS chunks apart.
// ---------------------------------------------------------------------------
constexpr int KC16 = 32;   // columns per chunk

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h2v __attribute__((ext_vector_type(2)));

template <int PREC>
__device__ __forceinline__ uint32_t cvt_pk16(float a, float b) {
  const f2v v = {a, b};
  if constexpr (PREC == P_F16) return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, h2v));
  else return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf2v));
}

// 32-deep product of two joined operands with FP32 accumulation
template <int PREC>
__device__ __forceinline__ f4 mfma32(s4 alo, s4 ahi, s4 blo, s4 bhi, f4 c) {
  const s8 a = __builtin_shufflevector(alo, ahi, 0, 1, 2, 3, 4, 5, 6, 7);
  const s8 b = __builtin_shufflevector(blo, bhi, 0, 1, 2, 3, 4, 5, 6, 7);
  if constexpr (PREC == P_F16)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0, 0, 0);
  else return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, a), __builtin_bit_cast(b8, b), c, 0, 0, 0);
}

// Four FP32 values (zeroed where bit v of ok is clear) -> four 16-bit values.
template <int PREC>
__device__ __forceinline__ s4 cvt4(float4 x, uint32_t ok) {
  const float a = (ok & 1) ? x.x : 0.0f, b = (ok & 2) ? x.y : 0.0f, c = (ok & 4) ? x.z : 0.0f,
              d = (ok & 8) ? x.w : 0.0f;
  return __builtin_bit_cast(s4, uint2{cvt_pk16<PREC>(a, b), cvt_pk16<PREC>(c, d)});
}

typedef __attribute__((address_space(3))) s4 lds_s4;

// Chunk geometry for 32-column chunks, visited in increasing order (segments
// hold chunk0 counted in 32-column chunks): forward-only segment cursor.
struct Cursor16 {
  int sg = 0;
  template <bool SEG1>
  __device__ __forceinline__ ChunkInfo at(const SketchArgs& A, int64_t ci) {
    if constexpr (!SEG1) {
      while (sg + 1 < A.nseg && A.seg[sg + 1].chunk0 <= ci) ++sg;
    }
    ChunkInfo c;
    c.ptr = (const char*)A.seg[sg].ptr;
    c.lcol0 = (ci - A.seg[sg].chunk0) * KC16;
    c.gcol0 = A.seg[sg].gcol0 + c.lcol0;
    const int64_t left = A.seg[sg].ncols - c.lcol0;
    c.ncols = (int)(left < KC16 ? left : KC16);
    return c;
  }
};

template <int PREC, int LP, int NW, int NS, bool ALIGNED, bool SEG1>
__global__ __launch_bounds__(NW * 64, NW == 4 ? 2 : 1) void k_sketch16(const SketchArgs A) {
  constexpr int RT = 4;                 // 16-row tiles per wave (64 rows)
  constexpr int CT = KC16 / 16;         // 16-column tiles per chunk
  constexpr int NT = LP / 16;           // sketch-column tiles
  constexpr int XS = 64 + 8;            // column stride of the LDS X tile (16-bit words)
  constexpr int TS = LP + 4;            // column stride of the T tiles (floats; sketch index contiguous)
  __shared__ __align__(16) uint16_t Xl[NW][KC16 * XS];
  // stationary Psi operands, in LDS (each lane reads back its own), sparing the
  // registers for two chunks of X in flight
  __shared__ __align__(16) s4 Pl[NW][RT][NT][64];
  __shared__ __align__(16) float Tred[NS][NW][KC16 * TS];
  __shared__ int arrived[NS];   // waves that have written their tile of the slot's chunk
  __shared__ int released[NS];  // times the slot has been summed and freed

  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int gi = blockIdx.x % A.gi_count;
  const int gj = blockIdx.x / A.gi_count;
  const int64_t row0w = (int64_t)gi * (NW * 64) + (int64_t)w * 64;
  const int64_t cb = (int64_t)gj * A.nchunks / A.gj_count;
  const int64_t ce = (int64_t)(gj + 1) * A.nchunks / A.gj_count;
  const int l16 = lane & 15, g4 = lane >> 4;
  if (threadIdx.x < NS) {
    arrived[threadIdx.x] = 0;
    released[threadIdx.x] = 0;
  }

  // ---- stationary left-DRM operands Psi(row0w + 16 rt + 4 g4 + v, 16 mt + l16) ----
  {
    PsiCursor pc;
    pc.init(A, row0w + 4 * g4);
    double hv[NT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      float p[4][NT];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (rt > 0 || v > 0) pc.advance(A, v > 0 ? 1 : 13);
        if (pc.refresh(A)) {
#pragma unroll
          for (int mt = 0; mt < NT; ++mt) hv[mt] = psi_hi(A, pc.h, 16 * mt + l16);
        }
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) p[v][mt] = (float)pc.at(A, 16 * mt + l16, hv[mt]);
      }
#pragma unroll
      for (int mt = 0; mt < NT; ++mt)
        Pl[w][rt][mt][lane] = cvt4<PREC>(float4{p[0][mt], p[1][mt], p[2][mt], p[3][mt]}, 0xfu);
    }
  }
  __syncthreads();   // the slot counters are zero

  Cursor16 cx, co, ct_;   // X loads (two ahead), Omega loads (one ahead), T partial stores

  // ---- raw X of a chunk (two register slots) and its validity bits ----
  float4 xr[2][RT][CT];
  uint32_t xok[2];
  auto load_chunk = [&](int64_t ci, int slot) {
    const ChunkInfo ch = cx.at<SEG1>(A, ci < ce ? ci : ce - 1);
    const float* base = (const float*)ch.ptr;
    uint32_t ok = 0;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int cc = 16 * ct + l16;
        const int64_t row = row0w + 16 * rt + 4 * g4;
        const bool colok = cc < ch.ncols;
        const float* col = base + (ch.lcol0 + (colok ? cc : 0)) * A.R;
        const int bit = 4 * (rt * CT + ct);
        if constexpr (ALIGNED) {   // R % 4 == 0: the four rows are in or out together
          const bool in = colok && row < A.R;
          xr[slot][rt][ct] = *(const float4*)(col + (in ? row : 0));
          ok |= (in ? 0xfu : 0u) << bit;
        } else {
          float v4[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const bool in = colok && row + v < A.R;
            v4[v] = col[in ? row + v : 0];
            ok |= (in ? 1u : 0u) << (bit + v);
          }
          xr[slot][rt][ct] = float4{v4[0], v4[1], v4[2], v4[3]};
        }
      }
    xok[slot] = ok;
  };

  // ---- Omega operands of a chunk: lane (g4, l16), tile nt, K step ks holds
  //      Omega(columns 16 ks + 4 g4 .. + 3, sketch column 16 nt + l16).  Two
  //      register sets: the next chunk's are requested before the X loads of
  //      the chunk after it, so that waiting for them (loads complete in
  //      order) never waits for X that is still in flight. ----
  //      The loads are unconditional: the table rows have a stride that is a
  //      multiple of four and slack after the last row, so the aligned 8-byte
  //      word holding a lane's first column and the word after it are always
  //      in the table; the four columns are shifted out of the pair only when
  //      the operand is used (a use right after the load would wait for it).
  //      Columns past the chunk read whatever the table holds there, a finite
  //      value that meets a zeroed X column. ----
  uint2 wo[2][NT][2][2];
  int osh[2];
  auto load_omega = [&](int64_t ci, int b) {
    const ChunkInfo ch = co.at<SEG1>(A, ci < ce ? ci : ce - 1);
    const int64_t cs = omega16_stride(A.C);
    const int sh = (int)(ch.gcol0 & 3);
    osh[b] = sh;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const uint16_t* src = A.om16 + (int64_t)(16 * nt + l16) * cs + (ch.gcol0 - sh) + 16 * ks + 4 * g4;
        wo[b][nt][ks][0] = *(const uint2*)src;
        wo[b][nt][ks][1] = sh ? *(const uint2*)(src + 4) : uint2{0u, 0u};
      }
  };
  auto omega_op = [&](int b, int nt, int ks) -> s4 {
    const uint64_t lo = __builtin_bit_cast(uint64_t, wo[b][nt][ks][0]);
    const uint64_t hi = __builtin_bit_cast(uint64_t, wo[b][nt][ks][1]);
    const int sh = osh[b];
    return __builtin_bit_cast(s4, sh ? (lo >> (16 * sh)) | (hi << (64 - 16 * sh)) : lo);
  };

  f4 yacc[RT][NT];
#pragma unroll
  for (int mt = 0; mt < RT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) yacc[mt][nt] = f4{0, 0, 0, 0};

  if (cb < ce) {
    load_chunk(cb, 0);
    load_omega(cb, 0);
    load_chunk(cb + 1, 1);
  }

  auto chunk_step = [&](int64_t ci, int it, int slot) {
    // (a) convert this chunk's fragments; write them to the wave's LDS tile
    s4 fx[RT][CT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        fx[rt][ct] = cvt4<PREC>(xr[slot][rt][ct], xok[slot] >> (4 * (rt * CT + ct)));
        *(s4*)&Xl[w][(16 * ct + l16) * XS + 16 * rt + 4 * g4] = fx[rt][ct];
      }
    // (b) Omega operands of the next chunk, then chunk ci + 2 into the X slot
    //     just converted
    load_omega(ci + 1, slot ^ 1);
    load_chunk(ci + 2, slot);
    // (c) left sketch from the registers: T(16 mt + .., 16 ct + l16), K = the wave's 64 rows
    f4 tacc[CT][NT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) {
        f4 t = f4{0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < RT / 2; ++j) {
          const int ka = 2 * j, kb = 2 * j + 1;
          t = mfma32<PREC>(Pl[w][ka][mt][lane], Pl[w][kb][mt][lane], fx[ka][ct], fx[kb][ct], t);
        }
        tacc[ct][mt] = t;
      }
    // (d) right sketch: X rows from the LDS tile (transposing reads)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int mt = 0; mt < RT; ++mt) {
      s4 xa[2];
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
        xa[ks] = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
            (lds_s4*)&Xl[w][(16 * ks + 4 * g4 + (l16 >> 2)) * XS + 16 * mt + 4 * (l16 & 3)]);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        yacc[mt][nt] = mfma32<PREC>(xa[0], xa[1], omega_op(slot, nt, 0), omega_op(slot, nt, 1), yacc[mt][nt]);
    }
    // (e) this wave's T tile into slot it % NS once the slot's previous chunk
    //     has been summed (bounded wait: see the kernel comment)
    const int sl = it % NS;
    const int gen = it / NS;
    while (__hip_atomic_load(&released[sl], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < gen)
      __builtin_amdgcn_s_sleep(1);
    // element v of tacc[ct][mt] is T(16 mt + 4 g4 + v, 16 ct + l16): four consecutive
    // sketch rows of one column, one 16-byte store
    float* tr = Tred[sl][w];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) *(f4*)&tr[(16 * ct + l16) * TS + 16 * mt + 4 * g4] = tacc[ct][mt];
    int before = 0;
    if (lane == 0)
      before = __hip_atomic_fetch_add(&arrived[sl], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
    before = __builtin_amdgcn_readfirstlane(before);
    if (before == NW - 1) {
      // last to arrive: every wave's tile is in the slot
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      // four consecutive sketch rows of one column per item, 16-byte LDS reads and
      // stores into the T partial [row block][column][LP] (sketch index contiguous)
      const ChunkInfo ch = ct_.at<SEG1>(A, ci);
      float* tp = (float*)A.tpart;
      const int64_t spare = (int64_t)A.gi_count * A.C * LP;
      constexpr int NA = LP / 4;   // four-row groups per column
#pragma unroll 2
      for (int q = 0; q < KC16 * NA / 64; ++q) {
        const int item = lane + 64 * q;
        const int col = item / NA, a4 = 4 * (item % NA);
        f4 sum = *(const f4*)&Tred[sl][0][col * TS + a4];
#pragma unroll
        for (int ww = 1; ww < NW; ++ww) sum += *(const f4*)&Tred[sl][ww][col * TS + a4];
        const bool ok = col < ch.ncols;
        *(f4*)&tp[ok ? ((int64_t)gi * A.C + ch.gcol0 + col) * LP + a4 : spare + 4 * item] = sum;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      if (lane == 0) {
        __hip_atomic_store(&arrived[sl], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(&released[sl], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    } else {
      (void)ct_.at<SEG1>(A, ci);   // keep the cursor in step
    }
  };

  int it = 0;
  int64_t ci = cb;
  for (; ci + 1 < ce; ci += 2, it += 2) {
    chunk_step(ci, it, 0);
    chunk_step(ci + 1, it + 1, 1);
  }
  if (ci < ce) chunk_step(ci, it, 0);

  // ---- right-sketch partial of this workgroup: element v of yacc[mt][nt] at
  //      (row 16 mt + 4 g4 + v, sketch column 16 nt + l16) ----
  float* yp = (float*)A.ypart;
#pragma unroll
  for (int mt = 0; mt < RT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = row0w + 16 * mt + 4 * g4 + v;
        const int c = 16 * nt + l16;
        if (row < A.R && c < A.ell) yp[((int64_t)gj * A.ell + c) * A.R + row] = yacc[mt][nt][v];
      }
}

// Omega_m rounded to the 16-bit arithmetic: om16[c cs + col] = Omega_m(col, c)
// with row stride cs = C rounded up to a multiple of four (zero for c >= ell,
// for the padding columns and for the slack after the last row).  Same
// rounding (FP64 -> FP32 -> 16 bits, nearest even) as the effective DRM the
// middle core uses.
__global__ void k_omega16_table(const double* __restrict__ om_tab, int64_t C, int L4, int ell, int LP, int prec,
                                uint16_t* __restrict__ om16) {
  const int64_t cs = omega16_stride(C);
  const int64_t tot = omega16_entries(C, LP);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = t / cs;
    const int64_t col = t % cs;
    const float f = c < ell && col < C ? (float)om_tab[col * L4 + c] : 0.0f;
    om16[t] = (uint16_t)(prec == P_F16 ? cvt_pk16<P_F16>(f, 0.0f) : cvt_pk16<P_BF16>(f, 0.0f));
  }
}

hipError_t build_omega16_table(const double* om_tab, int64_t C, int L4, int ell, int LP, int prec, uint16_t* om16,
                               hipStream_t s) {
  const int64_t tot = omega16_entries(C, LP);
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((tot + 255) / 256, 16384));
  hipLaunchKernelGGL(k_omega16_table, dim3(g), dim3(256), 0, s, om_tab, C, L4, ell, LP, prec, om16);
  return hipGetLastError();
}

// The one-term 16-bit formats run on k_sketch16.  Split BF16 stays on k_sketch:
// its six products per element keep the matrix cores busy enough that the
// barrier-per-chunk kernel with two workgroups per compute unit measured
// faster (1.3 against 1.7 ms at d = 5, n = 64) than k_sketch16 at the one
// workgroup per compute unit its register and LDS use allow.
int omega16_planes(int prec) { return (prec == P_BF16 || prec == P_F16) ? 1 : 0; }

constexpr int kNW16 = 4;   // waves per 16-bit sketch workgroup
constexpr int kNS16 = 2;   // T-tile slots in flight per workgroup

template <int PREC, int LP>
static hipError_t launch_16(const SketchArgs& a, bool aligned, hipStream_t s) {
  dim3 grid((unsigned)(a.gi_count * a.gj_count)), block(kNW16 * 64);
  const bool seg1 = a.nseg == 1 && a.seg[0].chunk0 == 0;
  if (!a.om16) return hipErrorInvalidValue;
  if (aligned) {
    if (seg1) hipLaunchKernelGGL((k_sketch16<PREC, LP, kNW16, kNS16, true, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_sketch16<PREC, LP, kNW16, kNS16, true, false>), grid, block, 0, s, a);
  } else {
    if (seg1) hipLaunchKernelGGL((k_sketch16<PREC, LP, kNW16, kNS16, false, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_sketch16<PREC, LP, kNW16, kNS16, false, false>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 kernel with the sketch size covered exactly: ell (rounded up to a
// multiple of 4) = 16*NQ + 4*NS.  The 16-wide part of each side runs on
// 16x16x4 FP64 MFMA tiles, the remaining 4-wide groups on the 4-block 4x4x4
// FP64 MFMA, whose X operands have the same lane layout (A: row lane%16,
// k lane/16; B: k lane/16, column lane%16), so one LDS read feeds both.
// Output layouts: 16x16x4 element v of lane l at (4v + l/16, l%16); 4x4x4
// block b = (l/4)%4 at (l/16, l%4) of that block.
// ---------------------------------------------------------------------------
// FP64 workgroups: for ell (rounded to 4) <= 28, 4 waves (256 rows) and two
// workgroups per CU, so one workgroup's matrix-core work overlaps the other's
// barrier and load phases (measured 8% faster at ell = 20 than one 8-wave
// workgroup).  For ell = 32 two such workgroups no longer fit in LDS, and one
// 8-wave workgroup (two waves per SIMD) beats one 4-wave workgroup by 7%.
constexpr int nwf_for(int L4) { return L4 > 28 ? 8 : 4; }
constexpr int f64_wg_per_cu(int L4) { return L4 > 28 ? 1 : 2; }

// FN: the tensor is the Hilbert tensor, evaluated from the index tables in
// place of the loads of X (one launch segment, no memory behind it).
// X32: X holds FP32 entries, widened to FP64 as they are loaded (FP64
// arithmetic on FP32 data); the rest of the kernel is the same.
template <int L4, bool ALIGNED, bool SEG1, bool FN, bool X32 = false>
__global__ __launch_bounds__(nwf_for(L4) * 64, f64_wg_per_cu(L4)) void k_sketch_f64(const SketchArgs A) {
  constexpr int NWF = nwf_for(L4);
  constexpr int RW = 64;
  constexpr int ST = RW + 2;
  constexpr int NQ = L4 / 16;          // 16-wide tiles
  constexpr int NS = (L4 % 16) / 4;    // 4-wide groups
  constexpr int KT = RW / 4;           // K steps over rows (left sketch)
  constexpr int NLD = KC * RW / (64 * 2);
  constexpr int NT = NWF * 64;         // threads
  constexpr int NOM = (KC * L4 + NT - 1) / NT;   // staged Omega / T entries per thread
  static_assert(L4 % 4 == 0 && L4 >= 4, "ell padded to a multiple of 4");

  __shared__ double Xl[NWF][KC * ST];
  __shared__ double Tred[2][NWF][L4 * KC];
  __shared__ __align__(16) double Om[4][KC * L4];  // 4 buffers: each write is a barrier past the last read

  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int gi = blockIdx.x % A.gi_count;
  const int gj = blockIdx.x / A.gi_count;
  const int64_t row0w = (int64_t)gi * (NWF * RW) + (int64_t)w * RW;
  const int64_t cb = (int64_t)gj * A.nchunks / A.gj_count;
  const int64_t ce = (int64_t)(gj + 1) * A.nchunks / A.gj_count;
  const int l16 = lane & 15, g4 = lane >> 4, l4 = lane & 3, blk = (lane >> 2) & 3;
  SegCursor cx, co, ct;   // X loads, Omega loads, T partials: each in increasing chunk order
  auto info = [&](SegCursor& cu, int64_t ci) -> ChunkInfo { return SEG1 ? chunk_info1(A, ci) : cu.at(A, ci); };

  // stationary left-DRM operands: Psi(row0w + 4 ks + g4, a)
  double psiq[KT][NQ > 0 ? NQ : 1];
  double psis[KT][NS > 0 ? NS : 1];
  {
    PsiCursor pc;
    pc.init(A, row0w + g4);
    double hq[NQ > 0 ? NQ : 1], hs[NS > 0 ? NS : 1];
#pragma unroll
    for (int ks = 0; ks < KT; ++ks) {
      if (ks > 0) pc.advance(A, 4);
      if (pc.refresh(A)) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) hq[q] = psi_hi(A, pc.h, 16 * q + l16);
#pragma unroll
        for (int s = 0; s < NS; ++s) hs[s] = psi_hi(A, pc.h, 16 * NQ + 4 * s + l4);
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) psiq[ks][q] = pc.at(A, 16 * q + l16, hq[q]);
#pragma unroll
      for (int s = 0; s < NS; ++s) psis[ks][s] = pc.at(A, 16 * NQ + 4 * s + l4, hs[s]);
    }
  }

  // Omega_m rows of a chunk: thread t < KC*L4/2 holds entries (e, e + 1),
  // e = 2t, of row e / L4 (L4 is even, so both sit in one row; the table's
  // padding columns ell..L4-1 are zero).  The loads are issued one iteration
  // before their values are written to LDS, so waiting for them never waits
  // for the X prefetch (loads retire in order).
  static_assert(KC * L4 / 2 <= NT, "one Omega pair per thread");
  double2 omv;
  auto load_omega = [&](int64_t ci) {
    const int e = 2 * threadIdx.x;
    omv = double2{0.0, 0.0};
    if (e < KC * L4 && ci < ce) {
      ChunkInfo ch = info(co, ci);
      const int col = e / L4, c = e % L4;
      if (col < ch.ncols) omv = *(const double2*)&A.om_tab[(ch.gcol0 + col) * A.L4 + c];
    }
  };
  auto store_omega = [&](int buf) {
    const int e = 2 * threadIdx.x;
    if (e < KC * L4) *(double2*)&Om[buf][e] = omv;
  };

  // X32: the prefetched pairs stay FP32 in registers and are widened when the
  // chunk is staged (widening at the load would wait for every load in turn)
  typename std::conditional<X32, float, double>::type xr[NLD][2];
  // FN: index-table entries of this lane's two rows (fixed for the launch)
  int fr0 = 0, fr1 = 0;
  if constexpr (FN) {
    const int64_t row = row0w + (lane & 31) * 2;
    fr0 = row < A.R ? A.fn_row[row] : 0;
    fr1 = row + 1 < A.R ? A.fn_row[row + 1] : 0;
  }
  auto load_chunk = [&](int64_t ci) {
    ChunkInfo ch = info(cx, ci);
    const double* base = (const double*)ch.ptr;
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      const int cc = 2 * i + (lane >> 5);
      const int r = (lane & 31) * 2;
      const int64_t row = row0w + r;
      const bool colok = cc < ch.ncols;
      const double* p = base + (ch.lcol0 + cc) * A.R + row;
      if constexpr (FN) {
        const int fc = colok ? A.fn_col[ch.gcol0 + cc] : 0;
        xr[i][0] = (colok && row < A.R) ? A.fn_rec[fr0 + fc] : 0.0;
        xr[i][1] = (colok && row + 1 < A.R) ? A.fn_rec[fr1 + fc] : 0.0;
      } else if constexpr (X32) {
        const float* pf = (const float*)ch.ptr + (ch.lcol0 + cc) * A.R + row;
        if constexpr (ALIGNED) {   // R even, 8-byte pairs
          if (colok && row < A.R) {
            const float2 v = *(const float2*)pf;
            xr[i][0] = v.x;
            xr[i][1] = v.y;
          } else {
            xr[i][0] = xr[i][1] = 0.0f;
          }
        } else {
          xr[i][0] = (colok && row < A.R) ? pf[0] : 0.0f;
          xr[i][1] = (colok && row + 1 < A.R) ? pf[1] : 0.0f;
        }
      } else if constexpr (ALIGNED) {
        if (colok && row < A.R) {
          const double2 v = *(const double2*)p;
          xr[i][0] = v.x;
          xr[i][1] = v.y;
        } else {
          xr[i][0] = xr[i][1] = 0.0;
        }
      } else {
        xr[i][0] = (colok && row < A.R) ? p[0] : 0.0;
        xr[i][1] = (colok && row + 1 < A.R) ? p[1] : 0.0;
      }
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      const int cc = 2 * i + (lane >> 5);
      const int r = (lane & 31) * 2;
      Xl[w][cc * ST + r] = (double)xr[i][0];
      Xl[w][cc * ST + r + 1] = (double)xr[i][1];
    }
  };
  auto reduce_t = [&](int buf, int64_t ci) {
    ChunkInfo ch = info(ct, ci);
#pragma unroll
    for (int k = 0; k < NOM; ++k) {
      const int e = threadIdx.x + NT * k;
      if (e < L4 * KC) {
        const int a = e / KC, col = e % KC;
        double s = 0.0;
#pragma unroll
        for (int ww = 0; ww < NWF; ++ww) s += Tred[buf][ww][a * KC + col];
        if (a < A.ell && col < ch.ncols)
          ((double*)A.tpart)[((int64_t)gi * A.ell + a) * A.C + ch.gcol0 + col] = s;
      }
    }
  };

  d4 yq[4][NQ > 0 ? NQ : 1];
  double ys[4][NS > 0 ? NS : 1];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) yq[mt][q] = d4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < NS; ++s) ys[mt][s] = 0.0;
  }

  if (cb < ce) {
    load_omega(cb);
    store_omega(0);
    load_omega(cb + 1);
    store_omega(1);
    load_chunk(cb);
    load_omega(cb + 2);
  }
  int it = 0;
  for (int64_t ci = cb; ci < ce; ++ci, ++it) {
    // (a) stage this chunk's X tile and the Omega rows of chunk ci + 2 (both
    //     loaded one iteration ago) in LDS
    store_chunk();
    store_omega((it + 2) % 4);
    __syncthreads();
    // (b) prefetch the next chunk; Omega three chunks ahead
    if (ci + 1 < ce) load_chunk(ci + 1);
    load_omega(ci + 3);
    // (c) finish the previous chunk's left sketch
    if (it >= 1) reduce_t((it - 1) & 1, ci - 1);
    const double* xw = Xl[w];
    const double* om = Om[it % 4];
    // (d) matrix-core tiles; the left sketch uses two accumulator chains
    //     (even / odd K steps) interleaved with the right sketch
    d4 tq[2][NQ > 0 ? NQ : 1];
    double ts[2][NS > 0 ? NS : 1];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) tq[h][q] = d4{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < NS; ++s) ts[h][s] = 0.0;
    }
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int col = 4 * ks + g4;
      double bq[NQ > 0 ? NQ : 1], bs[NS > 0 ? NS : 1];
#pragma unroll
      for (int q = 0; q < NQ; ++q) bq[q] = om[col * L4 + 16 * q + l16];
#pragma unroll
      for (int s = 0; s < NS; ++s) bs[s] = om[col * L4 + 16 * NQ + 4 * s + l4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        const double a = xw[col * ST + 16 * mt + l16];
#pragma unroll
        for (int q = 0; q < NQ; ++q) yq[mt][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bq[q], yq[mt][q], 0, 0, 0);
#pragma unroll
        for (int s = 0; s < NS; ++s) ys[mt][s] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, bs[s], ys[mt][s], 0, 0, 0);
      }
      // left sketch, K steps 4*ks .. 4*ks + 3
#pragma unroll
      for (int kk = 0; kk < KT / (KC / 4); ++kk) {
        const int k2 = ks * (KT / (KC / 4)) + kk;
        const double b = xw[l16 * ST + 4 * k2 + g4];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          tq[kk & 1][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(psiq[k2][q], b, tq[kk & 1][q], 0, 0, 0);
#pragma unroll
        for (int s = 0; s < NS; ++s)
          ts[kk & 1][s] = __builtin_amdgcn_mfma_f64_4x4x4f64(psis[k2][s], b, ts[kk & 1][s], 0, 0, 0);
      }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) tq[0][q] += tq[1][q];
#pragma unroll
    for (int s = 0; s < NS; ++s) ts[0][s] += ts[1][s];
    double* tr = Tred[it & 1][w];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) tr[(16 * q + 4 * v + g4) * KC + l16] = tq[0][q][v];
    // 4x4x4: block blk holds columns 4*blk + l4, rows (a) 16*NQ + 4s + g4
#pragma unroll
    for (int s = 0; s < NS; ++s) tr[(16 * NQ + 4 * s + g4) * KC + 4 * blk + l4] = ts[0][s];
  }
  __syncthreads();
  if (it >= 1) reduce_t((it - 1) & 1, ce - 1);

  // One column group: each entry of Y_R has this workgroup as its only
  // writer, so the tile is added into Y_R here (the same single addition the
  // reduction would make) instead of going through the partial buffer.  The
  // first launch after a reset that left Y_R unwritten stores 0 + tile.
  double* yp = (double*)A.ypart;
  double* yd = A.ydirect;
  bool bad = false;
  auto put = [&](int64_t row, int c, double v) {
    if (yd) {
      const int64_t i = (int64_t)c * A.R + row;
      const double s = (A.ystore ? 0.0 : yd[i]) + v;
      yd[i] = s;
      bad = bad || !isfinite(s);
    } else {
      yp[((int64_t)gj * A.ell + c) * A.R + row] = v;
    }
  };
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = row0w + 16 * mt + 4 * v + g4;
        const int c = 16 * q + l16;
        if (row < A.R && c < A.ell) put(row, c, yq[mt][q][v]);
      }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int64_t row = row0w + 16 * mt + 4 * blk + g4;
      const int c = 16 * NQ + 4 * s + l4;
      if (row < A.R && c < A.ell) put(row, c, ys[mt][s]);
    }
  }
  if (bad) atomicOr(A.yflag, 1);
}

template <int L4>
static hipError_t launch_f64(const SketchArgs& a, bool aligned, hipStream_t s) {
  dim3 grid((unsigned)(a.gi_count * a.gj_count)), block(nwf_for(L4) * 64);
  if (a.ydirect && (a.gj_count != 1 || !a.yflag)) return hipErrorInvalidValue;
  if (a.ystore && !a.ydirect) return hipErrorInvalidValue;
  const bool seg1 = a.nseg == 1 && a.seg[0].chunk0 == 0;
  if (a.fn) {
    if (!seg1 || a.fn != 1 || !a.fn_rec || !a.fn_row || !a.fn_col || a.x32) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_sketch_f64<L4, true, true, true>), grid, block, 0, s, a);
  } else if (a.x32) {
    if (aligned) {
      if (seg1) hipLaunchKernelGGL((k_sketch_f64<L4, true, true, false, true>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_sketch_f64<L4, true, false, false, true>), grid, block, 0, s, a);
    } else {
      if (seg1) hipLaunchKernelGGL((k_sketch_f64<L4, false, true, false, true>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_sketch_f64<L4, false, false, false, true>), grid, block, 0, s, a);
    }
  } else if (aligned) {
    if (seg1) hipLaunchKernelGGL((k_sketch_f64<L4, true, true, false>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_sketch_f64<L4, true, false, false>), grid, block, 0, s, a);
  } else {
    if (seg1) hipLaunchKernelGGL((k_sketch_f64<L4, false, true, false>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_sketch_f64<L4, false, false, false>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

// Table of the right DRM of the middle unfolding, Omega_m(col, c), FP64, C x L4
// (columns c >= ell are zero).  Built once per context; the sketch kernels
// stream 16-row blocks of it per chunk instead of re-forming the products.
__global__ void k_omega_table(const SketchArgs A, int L4, double* __restrict__ tab) {
  const int64_t tot = A.C * L4;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = t / L4;
    const int c = (int)(t % L4);
    tab[t] = c < A.ell ? omega_col(A, col, c) : 0.0;
  }
}

hipError_t build_omega_table(const SketchArgs& a, int L4, double* tab, hipStream_t s) {
  const int64_t tot = a.C * L4;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((tot + 255) / 256, 16384));
  hipLaunchKernelGGL(k_omega_table, dim3(g), dim3(256), 0, s, a, L4, tab);
  return hipGetLastError();
}

int sketch_chunk_cols(int prec) { return omega16_planes(prec) ? KC16 : KC; }

void sketch_geometry(int prec, int ell, int* rows_per_block, int* threads, int* wg_per_cu) {
  const int L4 = (ell + 3) / 4 * 4;
  if (omega16_planes(prec)) {
    *rows_per_block = kNW16 * 64;
    *threads = kNW16 * 64;
    *wg_per_cu = 2;
    return;
  }
  *threads = prec == P_F64 ? nwf_for(L4) * 64 : NWS * 64;
  // FP64: see nwf_for; the FP32-family kernels always fit two workgroups
  *wg_per_cu = prec == P_F64 ? f64_wg_per_cu(L4) : 2;
  switch (prec) {
    case P_F64: *rows_per_block = nwf_for(L4) * Eng<P_F64>::RW; break;
    case P_F32: *rows_per_block = NWS * Eng<P_F32>::RW; break;
    default: *rows_per_block = NWS * Eng<P_BF16X3>::RW; break;
  }
}

template <int PREC, int LP>
static hipError_t launch_t(const SketchArgs& a, bool aligned, hipStream_t s) {
  dim3 grid((unsigned)(a.gi_count * a.gj_count)), block(NWS * 64);
  const bool seg1 = a.nseg == 1 && a.seg[0].chunk0 == 0;
  if (aligned) {
    if (seg1) hipLaunchKernelGGL((k_sketch<PREC, LP, true, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_sketch<PREC, LP, true, false>), grid, block, 0, s, a);
  } else {
    if (seg1) hipLaunchKernelGGL((k_sketch<PREC, LP, false, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_sketch<PREC, LP, false, false>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_sketch(int prec, int lp, const SketchArgs& a, hipStream_t s) {
  if (fault_take()) return hipErrorLaunchFailure;
  if ((a.fn || a.ydirect || a.ystore) && prec != P_F64) return hipErrorInvalidValue;
  // 16-byte loads need every column (and segment start) 16-byte aligned.
  const int esz = prec == P_F64 && !a.x32 ? 8 : 4;
  bool aligned = ((a.R * esz) % 16) == 0;
  for (int i = 0; i < a.nseg; ++i) aligned = aligned && (((uintptr_t)a.seg[i].ptr) % 16 == 0);
  if (prec == P_F64) {
    switch ((a.ell + 3) / 4 * 4) {
      case 4: return launch_f64<4>(a, aligned, s);
      case 8: return launch_f64<8>(a, aligned, s);
      case 12: return launch_f64<12>(a, aligned, s);
      case 16: return launch_f64<16>(a, aligned, s);
      case 20: return launch_f64<20>(a, aligned, s);
      case 24: return launch_f64<24>(a, aligned, s);
      case 28: return launch_f64<28>(a, aligned, s);
      case 32: return launch_f64<32>(a, aligned, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (prec * 100 + lp) {
    case P_F32 * 100 + 16: return launch_t<P_F32, 16>(a, aligned, s);
    case P_F32 * 100 + 32: return launch_t<P_F32, 32>(a, aligned, s);
    case P_BF16 * 100 + 16: return launch_16<P_BF16, 16>(a, aligned, s);
    case P_BF16 * 100 + 32: return launch_16<P_BF16, 32>(a, aligned, s);
    case P_F16 * 100 + 16: return launch_16<P_F16, 16>(a, aligned, s);
    case P_F16 * 100 + 32: return launch_16<P_F16, 32>(a, aligned, s);
    case P_BF16X3 * 100 + 16: return launch_t<P_BF16X3, 16>(a, aligned, s);
    case P_BF16X3 * 100 + 32: return launch_t<P_BF16X3, 32>(a, aligned, s);
    default: return hipErrorInvalidValue;
  }
}

// ---- one partial column (slab edges that cut a column of X_m), FP64 ----
template <typename T>
__global__ void k_partial_col(const T* __restrict__ x, int64_t r0, int64_t r1, int64_t gcol, const SketchArgs A,
                              double* __restrict__ Y, double* __restrict__ Tt) {
  __shared__ double red[PSTT2_MAX_ELL][8];
  double om[PSTT2_MAX_ELL];
  for (int c = 0; c < A.ell; ++c) om[c] = omega_col(A, gcol, c);
  double t[PSTT2_MAX_ELL];
  for (int a = 0; a < A.ell; ++a) t[a] = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    const double xv = (double)x[r - r0];
    for (int c = 0; c < A.ell; ++c) Y[(int64_t)c * A.R + r] += xv * om[c];
    for (int a = 0; a < A.ell; ++a) t[a] += psi_row(A, r, a) * xv;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int a = 0; a < A.ell; ++a) {
    double v = t[a];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[a][w] = v;
  }
  __syncthreads();
  if (threadIdx.x < A.ell) {
    double s = 0.0;
    for (int ww = 0; ww < (int)(blockDim.x >> 6); ++ww) s += red[threadIdx.x][ww];
    Tt[(int64_t)threadIdx.x * A.C + gcol] += s;
  }
}

hipError_t launch_partial_col(int dtype, const void* x, int64_t r0, int64_t r1, int64_t gcol, const SketchArgs& a,
                              double* Y, double* Tt, hipStream_t s) {
  if (fault_take()) return hipErrorLaunchFailure;
  if (dtype == PSTT2_F64)
    hipLaunchKernelGGL(k_partial_col<double>, dim3(1), dim3(512), 0, s, (const double*)x, r0, r1, gcol, a, Y, Tt);
  else
    hipLaunchKernelGGL(k_partial_col<float>, dim3(1), dim3(512), 0, s, (const float*)x, r0, r1, gcol, a, Y, Tt);
  return hipGetLastError();
}

}  // namespace pstt2
