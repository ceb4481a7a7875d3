// C ABI of libpstt2 (declared in include/pstt2.h): context lifecycle, slab
// bookkeeping and the host orchestration of the PSTT2-onepass pipeline.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "internal.h"

using namespace pstt2;

static thread_local std::string g_tls_err;
void pstt2_set_tls_error(const std::string& msg) { g_tls_err = msg; }

namespace pstt2 {
hipError_t tt_error_run(const tt_cores* c, const void* x, int dtype, double* e2x2, hipStream_t s, int fn);
hipError_t tt_error_run_gauss(const tt_cores* c, const double* centers_host, int nterms, double gamma,
                              double* e2x2, hipStream_t s);
hipError_t tt_reconstruct_run(const tt_cores* c, void* out, int dtype, int64_t first, int64_t count, hipStream_t s);
}

struct pstt2_ctx {
  pstt2_desc desc;
  hipStream_t stream = nullptr;
  int d = 0, m = 0, ell = 0, lp = 0, prec = 0, dtype = 0, ncu = 256;
  int64_t n[PSTT2_MAX_D] = {};
  int64_t Rk[PSTT2_MAX_D + 1] = {};  // Rk[k] = n_1 ... n_k
  int64_t N = 0, R = 0, C = 0;       // entries; rows / columns of X_m
  double* fac = nullptr;
  int64_t psi_off[PSTT2_MAX_D] = {}, omega_off[PSTT2_MAX_D] = {};
  double* Y = nullptr;   // R x ell column-major
  double* Tt = nullptr;  // C x ell column-major (T_m transposed)
  void* ypart = nullptr;
  void* tpart = nullptr;
  int gi = 1, gj_max = 1;
  int* flag = nullptr;     // device: bit 0 non-finite sketch, bit 1 singular LS
  int* piv_dev = nullptr;  // (d + 1) x ell pivots of every split
  std::map<int64_t, int64_t> cover;  // first -> end of streamed ranges
  int64_t covered = 0;
  // recovery products kept for queries and the two-pass middle core
  std::vector<double*> S;      // S[k], k = 1..m-1, R_k x ell (S[m] aliases Y)
  std::vector<double*> Tk;     // Tk[k], k = m+1..d-1, C_k x ell (Tk[m] aliases Tt)
  std::vector<double*> basis;  // Q_k (k < m) or P_k (k >= m)
  Arena arena;                 // recovery workspace: sketches, bases, temporaries
  Arena varena;                // workspace of pstt2_vjp (rewound at every call)
  double* Bk = nullptr;        // two-sided sketches, split k at Bk + k ell^2 (ell x ell)
  int64_t* chain_dev = nullptr;  // per split: factor offsets of its left / right DRM chains, then n
  double* H = nullptr;         // two-sided middle sketch, (ell n_m) x ell (TWOSIDED only)
  int ranks[PSTT2_MAX_D + 1] = {};
  bool recovered = false;
  double* one = nullptr;       // device scalar 1.0 (Q_0 when m == 1)
  double* om_tab = nullptr;    // Omega_m table, C x L4 (independent scheme: split m's)
  uint16_t* om16 = nullptr;    // 16-bit precisions: the same rounded per plane (see build_omega16_table)
  std::vector<uint16_t*> iom16;   // independent scheme: 16-bit tables of the right splits k < m
  int L4 = 4;
  // independent DRM scheme: per-split factor offsets, Omega_m tables of the
  // right splits k < m, the extra sketches of X_m, and sinks for pass groups
  // with only one side
  bool indep = false;
  bool pstt = false;   // one-sided Algorithm PSTT: the pass sketches split d-1
  int64_t ipsi_off[PSTT2_MAX_D + 1][PSTT2_MAX_D] = {};  // [split k][mode q-1]
  int64_t iom_off[PSTT2_MAX_D + 1][PSTT2_MAX_D] = {};
  std::vector<double*> iom_tab;   // [k], k < m
  std::vector<double*> iY;        // [k], k < m: X_m Omega_m^(k), R x ell
  std::vector<double*> iT;        // [k], m < k < d: (Psi_m^(k)T X_m)^T, C x ell
  double* sinkY = nullptr;
  double* sinkT = nullptr;
  bool profile = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used, ev_pool;
  // tolerance mode: factor applied to eps by the rank rule (pstt2_recover_certified)
  // and the singular values of the last recovery's R factors, [k * ell + i]
  double eps_scale = 1.0;
  std::vector<double> sv_last;
  // index tables of the Hilbert tensor (pstt2_sketch_fn), built on first use
  double* fn_rec = nullptr;
  int32_t* fn_row = nullptr;
  int32_t* fn_col = nullptr;
  // launches that added into the sketches; a call that fails after one of them
  // leaves the sketches partly accumulated, which poisons the context until
  // pstt2_reset
  int64_t accum = 0;
  bool poisoned = false;
  // Y has not been written since pstt2_reset and stands for zero: reset skips
  // zeroing it when every sketch launch has one column group (the FP64
  // kernel's direct Y tile), the first such launch stores its tile instead of
  // adding it, and any other writer or reader zeroes Y first (y_settle)
  bool y_unset = false;
  std::string err;
};

namespace {

// Small pinned host buffer for device-to-host results (flags, singular values,
// error sums): copies into pageable memory take a slow staged path.  One per
// host thread, allocated on first use, held until the process ends.
double* pinned_scratch() {
  thread_local double* buf = nullptr;
  if (!buf && hipHostMalloc((void**)&buf, sizeof(double) * (PSTT2_MAX_D + 1) * PSTT2_MAX_ELL, 0) != hipSuccess)
    buf = nullptr;
  return buf;
}

// Workspace arena of tt_error for the current device on this host thread;
// held until the process ends.
Arena* error_arena() {
  thread_local std::map<int, Arena*> by_dev;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  Arena*& a = by_dev[dev];
  if (!a) a = new Arena();
  return a;
}

pstt2_status fail(pstt2_ctx* c, pstt2_status st, const std::string& msg) {
  if (c) c->err = msg;
  pstt2_set_tls_error(msg);
  return st;
}

pstt2_status hfail(pstt2_ctx* c, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(c, e == hipErrorOutOfMemory ? PSTT2_ENOMEM : PSTT2_EDEVICE, m);
}

#define HIPCK(ctx, call)                                      \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return hfail((ctx), e_, #call);     \
  } while (0)

// The recovery products live in the context's arena until the next recovery;
// forgetting them is enough.
void free_recovery(pstt2_ctx* c) {
  c->H = nullptr;
  c->S.assign(c->d + 1, nullptr);
  c->Tk.assign(c->d + 1, nullptr);
  c->basis.assign(c->d + 1, nullptr);
  c->recovered = false;
}

// Split k's left DRM Psi_k (modes 1..k) and right DRM Omega_k (modes k+1..d)
// as chains of factors in the context's factor buffer
KRChain left_chain(const pstt2_ctx* c, int k) {
  KRChain ch;
  std::memset(&ch, 0, sizeof(ch));
  for (int q = 1; q <= k; ++q) {
    ch.n[ch.cnt] = (int32_t)c->n[q - 1];
    ch.off[ch.cnt++] = c->indep ? c->ipsi_off[k][q - 1] : c->psi_off[q - 1];
  }
  return ch;
}

KRChain right_chain(const pstt2_ctx* c, int k) {
  KRChain ch;
  std::memset(&ch, 0, sizeof(ch));
  for (int q = k + 1; q <= c->d; ++q) {
    ch.n[ch.cnt] = (int32_t)c->n[q - 1];
    ch.off[ch.cnt++] = c->indep ? c->iom_off[k][q - 1] : c->omega_off[q - 1];
  }
  return ch;
}

SketchArgs base_args(const pstt2_ctx* c) {
  SketchArgs a;
  std::memset(&a, 0, sizeof(a));
  a.R = c->R;
  a.C = c->C;
  a.ell = c->ell;
  a.d = c->d;
  a.m = c->m;
  for (int q = 0; q < c->d; ++q) a.n[q] = (int32_t)c->n[q];
  a.fac = c->fac;
  for (int q = 0; q < PSTT2_MAX_D; ++q) {
    a.psi_off[q] = c->indep ? c->ipsi_off[c->m][q] : c->psi_off[q];
    a.omega_off[q] = c->indep ? c->iom_off[c->m][q] : c->omega_off[q];
  }
  a.ypart = c->ypart;
  a.tpart = c->tpart;
  a.gi_count = c->gi;
  a.om_tab = c->om_tab;
  a.om16 = c->om16;
  a.tlp = omega16_planes(c->prec) ? c->lp : 0;
  a.x32 = c->dtype == PSTT2_F32 && c->prec == PSTT2_P_F64;
  a.L4 = c->L4;
  return a;
}

pstt2_status check_range(pstt2_ctx* c, int64_t first, int64_t count) {
  if (first < 0 || count < 0 || first + count > c->N)
    return fail(c, PSTT2_EINVAL, "slab range outside the tensor");
  if (first % c->n[0] != 0 || count % c->n[0] != 0)
    return fail(c, PSTT2_EINVAL, "slab first/count must be multiples of n_1 (whole mode-1 fibres)");
  if (count == 0) return PSTT2_OK;
  auto it = c->cover.upper_bound(first);
  if (it != c->cover.end() && it->first < first + count)
    return fail(c, PSTT2_ESTATE, "slab overlaps an earlier slab");
  if (it != c->cover.begin()) {
    auto pv = std::prev(it);
    if (pv->second > first) return fail(c, PSTT2_ESTATE, "slab overlaps an earlier slab");
  }
  return PSTT2_OK;
}

constexpr const char* kPoisoned =
    "an earlier call failed after adding part of its data to the sketches: call pstt2_reset";

// A failed accumulating call that had already added into the sketches
// (c->accum moved since `before`) poisons the context.
pstt2_status settle(pstt2_ctx* c, pstt2_status st, int64_t before) {
  if (st != PSTT2_OK && c->accum != before) c->poisoned = true;
  return st;
}

void add_cover(pstt2_ctx* c, int64_t first, int64_t count) {
  if (count == 0) return;
  c->cover[first] = first + count;
  c->covered += count;
}

struct Piece {
  const void* x;   // slab pointer
  int64_t first;   // flat index of x[0]
  int64_t count;
};

// Stream a list of slabs: partial columns one by one, whole columns batched.
// Pass groups.  Nested scheme: one group (Y_R and T_m).  Independent scheme:
// group g forms the right sketch of split g + 1 (if g + 1 <= m) and the left
// sketch of split m + g (if m + g <= d - 1), each with its own factors; the
// absent side of a group goes to a sink.
int pass_groups(const pstt2_ctx* c) { return c->indep ? std::max(c->m, c->d - c->m) : 1; }

SketchArgs group_args(const pstt2_ctx* c, int g, double** Ydst, double** Tdst) {
  SketchArgs a = base_args(c);
  if (!c->indep) {
    *Ydst = c->Y;
    *Tdst = c->Tt;
    return a;
  }
  const int m = c->m, d = c->d;
  const int kr = g + 1, kl = m + g;
  if (kr <= m) {
    for (int q = 0; q < PSTT2_MAX_D; ++q) a.omega_off[q] = c->iom_off[kr][q];
    a.om_tab = kr == m ? c->om_tab : c->iom_tab[kr];
    a.om16 = kr == m ? c->om16 : c->iom16[kr];
    *Ydst = kr == m ? c->Y : c->iY[kr];
  } else {
    *Ydst = c->sinkY;
  }
  if (kl <= d - 1) {
    for (int q = 0; q < PSTT2_MAX_D; ++q) a.psi_off[q] = c->ipsi_off[kl][q];
    *Tdst = kl == m ? c->Tt : c->iT[kl];
  } else {
    *Tdst = c->sinkT;
  }
  return a;
}

pstt2_status launch_segs(pstt2_ctx* c, const SketchArgs& ga, const std::vector<Seg>& segs, double* Yd, double* Td);
hipError_t y_settle(pstt2_ctx* c);

pstt2_status run_slabs(pstt2_ctx* c, const std::vector<Piece>& ps) {
  const int esz = c->dtype == PSTT2_F64 ? 8 : 4;
  const int64_t R = c->R;
  std::vector<Seg> segs;
  struct Edge {
    const char* x;
    int64_t r0, r1, col;
  };
  std::vector<Edge> edges;
  for (const Piece& p : ps) {
    if (p.count == 0) continue;
    const int64_t lo = p.first, hi = p.first + p.count;
    const int64_t c0 = (lo + R - 1) / R, c1 = hi / R;   // whole columns [c0, c1)
    const char* base = (const char*)p.x;
    if (lo % R != 0) {   // head piece of column lo / R
      const int64_t col = lo / R;
      const int64_t r0 = lo % R, r1 = std::min<int64_t>(R, r0 + p.count);
      edges.push_back(Edge{base, r0, r1, col});
    }
    if (c1 > c0) segs.push_back(Seg{base + (c0 * R - lo) * esz, c0, c1 - c0, 0});
    if (hi % R != 0 && hi / R >= c0 && (lo / R != hi / R || lo % R == 0)) {   // tail piece
      const int64_t col = hi / R;
      edges.push_back(Edge{base + (col * R - lo) * esz, 0, hi % R, col});
    }
  }
  if (!edges.empty()) HIPCK(c, y_settle(c));   // partial columns add into Y
  for (int g = 0; g < pass_groups(c); ++g) {
    double *Yd = nullptr, *Td = nullptr;
    const SketchArgs ga = group_args(c, g, &Yd, &Td);
    for (const Edge& ed : edges) {
      HIPCK(c, launch_partial_col(c->dtype, ed.x, ed.r0, ed.r1, ed.col, ga, Yd, Td, c->stream));
      ++c->accum;
    }
    const pstt2_status st = launch_segs(c, ga, segs, Yd, Td);
    if (st != PSTT2_OK) return st;
  }
  return PSTT2_OK;
}

// One pass group over runs of whole columns: up to kMaxSeg runs per launch of
// the streaming kernel, then the fixed-order reduction of its partials.
pstt2_status launch_segs(pstt2_ctx* c, const SketchArgs& ga, const std::vector<Seg>& segs, double* Yd, double* Td) {
  {
    for (size_t s0 = 0; s0 < segs.size(); s0 += kMaxSeg) {
      SketchArgs a = ga;
      const size_t s1 = std::min(segs.size(), s0 + kMaxSeg);
      int64_t nch = 0;
      a.nseg = (int32_t)(s1 - s0);
      const int kc = sketch_chunk_cols(c->prec);
      for (size_t i = s0; i < s1; ++i) {
        Seg sg = segs[i];
        sg.chunk0 = nch;
        nch += (sg.ncols + kc - 1) / kc;
        a.seg[i - s0] = sg;
      }
      a.nchunks = nch;
      a.gj_count = (int32_t)std::max<int64_t>(1, std::min<int64_t>(nch, c->gj_max));
      if (c->prec == PSTT2_P_F64 && a.gj_count == 1) {
        a.ydirect = Yd;
        a.yflag = c->flag;
        a.ystore = Yd == c->Y && c->y_unset;   // Y still stands for zero: store the tile
      }
      if (Yd == c->Y && c->y_unset && !a.ystore) HIPCK(c, y_settle(c));
      std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
      if (c->profile) {
        if (c->ev_pool.empty()) {
          HIPCK(c, hipEventCreate(&ev.first));
          HIPCK(c, hipEventCreate(&ev.second));
        } else {
          ev = c->ev_pool.back();
          c->ev_pool.pop_back();
        }
        HIPCK(c, hipEventRecord(ev.first, c->stream));
      }
      HIPCK(c, launch_sketch(c->prec, c->lp, a, c->stream));
      if (a.ystore) c->y_unset = false;
      if (a.ydirect) ++c->accum;   // Y_R already holds this launch's data
      if (c->profile) {
        HIPCK(c, hipEventRecord(ev.second, c->stream));
        c->ev_used.push_back(ev);
      }
      HIPCK(c, launch_reduce(c->prec, a, Yd, Td, c->flag, c->stream));
      if (!a.ydirect) ++c->accum;
    }
  }
  return PSTT2_OK;
}

__global__ void k_zero_sketches(double* __restrict__ Y, int64_t ny, double* __restrict__ T, int64_t nt, int* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t i = t0; i < ny; i += stride) Y[i] = 0.0;
  for (int64_t i = t0; i < nt; i += stride) T[i] = 0.0;
  if (t0 == 0 && flag) *flag = 0;
}

// Zero Y if it still stands for zero (see pstt2_ctx::y_unset).
hipError_t y_settle(pstt2_ctx* c) {
  if (!c->y_unset) return hipSuccess;
  hipLaunchKernelGGL(k_zero_sketches, dim3(1024), dim3(256), 0, c->stream, c->Y, c->R * c->ell, nullptr, 0,
                     nullptr);
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) c->y_unset = false;
  return e;
}

__global__ void k_transpose_last(const double* P, int64_t rows, int r, double* G) {
  // G_d(a, i) = P(i, a): P is rows x r column-major, G is r x rows column-major
  const int64_t tot = rows * r;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(t % r);
    const int64_t i = t / r;
    G[t] = P[(int64_t)a * rows + i];
  }
}

// smallest r with sum_{i>r} sigma_i^2 <= eps^2/(d-1) * sum sigma_i^2, at least 1
int tolerance_rank(const double* s, int ell, double eps, int d);

// Rank of split k in tolerance mode: the eps rule on its singular values,
// capped at rmax, at ell - 2 and at the unfolding's size.
int rank_from_rule(const pstt2_ctx* c, int k, const double* sv, double eps) {
  const int ell = c->ell;
  const int64_t cap = std::min<int64_t>({c->Rk[k], c->N / c->Rk[k], (int64_t)ell});
  int rmax = c->desc.rmax > 0 ? c->desc.rmax : ell;
  rmax = std::min(rmax, std::max(1, ell - 2));
  const int rr = tolerance_rank(sv + (size_t)k * ell, ell, eps, c->d);
  return (int)std::min<int64_t>({(int64_t)rr, (int64_t)rmax, cap});
}

int tolerance_rank(const double* s, int ell, double eps, int d) {
  double tot = 0.0;
  for (int i = 0; i < ell; ++i) tot += s[i] * s[i];
  const double thr = eps * eps / (d - 1) * tot;
  int rr = ell;
  double tail = 0.0;
  for (int i = ell - 1; i >= 0; --i) {
    if (tail + s[i] * s[i] <= thr) {
      tail += s[i] * s[i];
      rr = i;
    } else {
      break;
    }
  }
  return std::max(rr, 1);
}

// Doubles of the packed factor buffer and, when c is given, every factor's
// offset: nested psi_1..psi_{d-1}, omega_2..omega_d; independent: per split
// k, psi^(k)_1..psi^(k)_k then omega^(k)_{k+1}..omega^(k)_d.
int64_t factor_layout(const pstt2_desc* desc, pstt2_ctx* c) {
  const int d = desc->d;
  const int64_t ell = desc->ell;
  int64_t off = 0;
  if (desc->drm != PSTT2_DRM_INDEPENDENT) {
    for (int q = 1; q <= d - 1; ++q) {
      if (c) c->psi_off[q - 1] = off;
      off += desc->n[q - 1] * ell;
    }
    for (int q = 2; q <= d; ++q) {
      if (c) c->omega_off[q - 1] = off;
      off += desc->n[q - 1] * ell;
    }
  } else {
    for (int k = 1; k <= d - 1; ++k) {
      for (int q = 1; q <= k; ++q) {
        if (c) c->ipsi_off[k][q - 1] = off;
        off += desc->n[q - 1] * ell;
      }
      for (int q = k + 1; q <= d; ++q) {
        if (c) c->iom_off[k][q - 1] = off;
        off += desc->n[q - 1] * ell;
      }
    }
  }
  return off;
}

}  // namespace

extern "C" {

const char* pstt2_version(void) { return "pstt2-mi355x 0.2 (gfx950)"; }

const char* pstt2_last_error(const pstt2_ctx* ctx) { return ctx ? ctx->err.c_str() : g_tls_err.c_str(); }

pstt2_status pstt2_create(const pstt2_desc* desc, void* hip_stream, pstt2_ctx** out) {
  if (!desc || !out) return fail(nullptr, PSTT2_EINVAL, "null descriptor or output");
  *out = nullptr;
  const int d = desc->d;
  if (d < 2 || d > PSTT2_MAX_D) return fail(nullptr, PSTT2_EINVAL, "d must be in [2, 32]");
  if (desc->ell < 1 || desc->ell > PSTT2_MAX_ELL) return fail(nullptr, PSTT2_EINVAL, "ell must be in [1, 32]");
  if (desc->dtype != PSTT2_F64 && desc->dtype != PSTT2_F32) return fail(nullptr, PSTT2_EINVAL, "bad dtype");
  if (desc->prec < PSTT2_P_F64 || desc->prec > PSTT2_P_F16) return fail(nullptr, PSTT2_EINVAL, "bad prec");
  if (desc->dtype == PSTT2_F64 && desc->prec != PSTT2_P_F64)
    return fail(nullptr, PSTT2_EINVAL, "FP64 tensors use PSTT2_P_F64 arithmetic");
  if (desc->mid != PSTT2_MID_ONEPASS && desc->mid != PSTT2_MID_TWOPASS && desc->mid != PSTT2_MID_TWOSIDED)
    return fail(nullptr, PSTT2_EINVAL, "bad mid");
  if (desc->drm != PSTT2_DRM_NESTED && desc->drm != PSTT2_DRM_INDEPENDENT) return fail(nullptr, PSTT2_EINVAL, "bad drm");
  if (desc->algo != PSTT2_ALGO_PSTT2 && desc->algo != PSTT2_ALGO_PSTT) return fail(nullptr, PSTT2_EINVAL, "bad algo");
  if (desc->algo == PSTT2_ALGO_PSTT && desc->mid == PSTT2_MID_TWOSIDED)
    return fail(nullptr, PSTT2_EINVAL, "the one-sided algorithm has no two-sided middle core");
  const bool tol = desc->ranks[0] <= 0;
  if (tol && !(desc->eps > 0.0 && desc->eps < 1.0)) return fail(nullptr, PSTT2_EINVAL, "tolerance mode needs 0 < eps < 1");
  int64_t N = 1;
  for (int q = 0; q < d; ++q) {
    if (desc->n[q] < 1) return fail(nullptr, PSTT2_EINVAL, "mode sizes must be >= 1");
    if (desc->n[q] > (1 << 30)) return fail(nullptr, PSTT2_EINVAL, "mode size too large");
    N *= desc->n[q];
    if (N > (int64_t(1) << 46)) return fail(nullptr, PSTT2_EINVAL, "tensor too large");
  }
  if (!tol)
    for (int k = 0; k < d - 1; ++k)
      if (desc->ranks[k] < 1) return fail(nullptr, PSTT2_EINVAL, "ranks must be >= 1");

  pstt2_ctx* c = new pstt2_ctx();
  c->desc = *desc;
  c->stream = (hipStream_t)hip_stream;
  c->d = d;
  // the pass sketches the middle split (PSTT2) or the last split (PSTT)
  c->m = desc->algo == PSTT2_ALGO_PSTT ? d - 1 : (d + 1) / 2;
  c->pstt = desc->algo == PSTT2_ALGO_PSTT;
  c->ell = desc->ell;
  c->lp = desc->ell <= 16 ? 16 : 32;
  c->prec = desc->prec;
  c->dtype = desc->dtype;
  c->Rk[0] = 1;
  for (int q = 0; q < d; ++q) {
    c->n[q] = desc->n[q];
    c->Rk[q + 1] = c->Rk[q] * desc->n[q];
  }
  c->N = N;
  c->R = c->Rk[c->m];
  c->C = N / c->R;
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (c->ncu <= 0) c->ncu = 256;

  // factors: given by the caller, or drawn from the seed (rng.hip)
  c->indep = desc->drm == PSTT2_DRM_INDEPENDENT;
  const int64_t off = factor_layout(desc, c);
  std::vector<double> drawn;
  const double* fac_host = desc->drm_factors;
  if (!fac_host) {
    drawn.resize((size_t)off);
    gaussian_fill(desc->seed, 0, off, drawn.data());
    fac_host = drawn.data();
  }
  auto bail = [&](hipError_t e, const char* w) {
    pstt2_status st = hfail(c, e, w);
    pstt2_destroy(c);
    return st;
  };
  hipError_t e;
  if ((e = dev_malloc(&c->fac, sizeof(double) * off)) != hipSuccess) return bail(e, "hipMalloc(factors)");
  if ((e = hipMemcpy(c->fac, fac_host, sizeof(double) * off, hipMemcpyHostToDevice)) != hipSuccess)
    return bail(e, "hipMemcpy(factors)");
  if ((e = dev_malloc(&c->Y, sizeof(double) * c->R * c->ell)) != hipSuccess) return bail(e, "hipMalloc(Y)");
  if ((e = dev_malloc(&c->Tt, sizeof(double) * c->C * c->ell)) != hipSuccess) return bail(e, "hipMalloc(T)");
  if ((e = dev_malloc(&c->flag, sizeof(int))) != hipSuccess) return bail(e, "hipMalloc(flag)");
  if ((e = dev_malloc(&c->piv_dev, sizeof(int) * (d + 1) * c->ell)) != hipSuccess) return bail(e, "hipMalloc(piv)");
  {
    // keep stream-ordered workspace in the device's default pool between
    // synchronisations (the recovery and the error pass allocate and free
    // small buffers every call; returning them to the HIP runtime costs ~0.3 ms)
    hipMemPool_t pool = nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess && pool) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
  }
  if ((e = dev_malloc(&c->one, sizeof(double))) != hipSuccess) return bail(e, "hipMalloc(one)");
  if ((e = dev_malloc(&c->Bk, sizeof(double) * (d + 1) * c->ell * c->ell)) != hipSuccess) return bail(e, "hipMalloc(Bk)");
  {
    std::vector<int64_t> ch((size_t)(d + 1) * 2 * d + d, 0);
    for (int k = 1; k <= d - 1; ++k) {
      const KRChain l = left_chain(c, k), r = right_chain(c, k);
      for (int j = 0; j < l.cnt; ++j) ch[((size_t)k * 2 + 0) * d + j] = l.off[j];
      for (int j = 0; j < r.cnt; ++j) ch[((size_t)k * 2 + 1) * d + j] = r.off[j];
    }
    for (int q = 0; q < d; ++q) ch[(size_t)(d + 1) * 2 * d + q] = c->n[q];
    if ((e = dev_malloc(&c->chain_dev, sizeof(int64_t) * ch.size())) != hipSuccess) return bail(e, "hipMalloc(chain)");
    if ((e = hipMemcpy(c->chain_dev, ch.data(), sizeof(int64_t) * ch.size(), hipMemcpyHostToDevice)) != hipSuccess)
      return bail(e, "hipMemcpy(chain)");
  }
  const double one = 1.0;
  if ((e = hipMemcpy(c->one, &one, sizeof(double), hipMemcpyHostToDevice)) != hipSuccess) return bail(e, "hipMemcpy");
  int rows_per_block = 0, threads = 0, wg_per_cu = 1;
  sketch_geometry(c->prec, c->ell, &rows_per_block, &threads, &wg_per_cu);
  c->gi = (int)((c->R + rows_per_block - 1) / rows_per_block);
  c->gj_max = std::max(1, c->ncu * wg_per_cu / c->gi);
  const size_t psz = c->prec == PSTT2_P_F64 ? 8 : 4;
  if ((e = dev_malloc(&c->ypart, psz * c->gj_max * c->ell * c->R)) != hipSuccess) return bail(e, "hipMalloc(ypart)");
  const int64_t trows = omega16_planes(c->prec) ? c->lp : c->ell;   // see SketchArgs::tlp
  if ((e = dev_malloc(&c->tpart, psz * (c->gi * trows * c->C + kTPartPad))) != hipSuccess)
    return bail(e, "hipMalloc(tpart)");
  c->L4 = (c->ell + 3) / 4 * 4;
  if ((e = dev_malloc(&c->om_tab, sizeof(double) * c->C * c->L4)) != hipSuccess) return bail(e, "hipMalloc(omega)");
  if ((e = build_omega_table(base_args(c), c->L4, c->om_tab, c->stream)) != hipSuccess)
    return bail(e, "omega table");
  const int npl16 = omega16_planes(c->prec);
  if (npl16) {
    const size_t b16 = sizeof(uint16_t) * npl16 * omega16_entries(c->C, c->lp);
    if ((e = dev_malloc(&c->om16, b16)) != hipSuccess) return bail(e, "hipMalloc(omega16)");
    if ((e = build_omega16_table(c->om_tab, c->C, c->L4, c->ell, c->lp, c->prec, c->om16, c->stream)) != hipSuccess)
      return bail(e, "omega16 table");
  }
  if (c->indep) {
    c->iom_tab.assign(d + 1, nullptr);
    c->iom16.assign(d + 1, nullptr);
    c->iY.assign(d + 1, nullptr);
    c->iT.assign(d + 1, nullptr);
    for (int k = 1; k < c->m; ++k) {
      if ((e = dev_malloc(&c->iom_tab[k], sizeof(double) * c->C * c->L4)) != hipSuccess) return bail(e, "hipMalloc(omega)");
      if ((e = dev_malloc(&c->iY[k], sizeof(double) * c->R * c->ell)) != hipSuccess) return bail(e, "hipMalloc(Y)");
      SketchArgs a = base_args(c);
      for (int q = 0; q < PSTT2_MAX_D; ++q) a.omega_off[q] = c->iom_off[k][q];
      if ((e = build_omega_table(a, c->L4, c->iom_tab[k], c->stream)) != hipSuccess) return bail(e, "omega table");
      if (npl16) {
        const size_t b16 = sizeof(uint16_t) * npl16 * omega16_entries(c->C, c->lp);
        if ((e = dev_malloc(&c->iom16[k], b16)) != hipSuccess) return bail(e, "hipMalloc(omega16)");
        if ((e = build_omega16_table(c->iom_tab[k], c->C, c->L4, c->ell, c->lp, c->prec, c->iom16[k], c->stream)) !=
            hipSuccess)
          return bail(e, "omega16 table");
      }
    }
    for (int k = c->m + 1; k <= d - 1; ++k)
      if ((e = dev_malloc(&c->iT[k], sizeof(double) * c->C * c->ell)) != hipSuccess) return bail(e, "hipMalloc(T)");
    if ((e = dev_malloc(&c->sinkY, sizeof(double) * c->R * c->ell)) != hipSuccess) return bail(e, "hipMalloc(sink)");
    if ((e = dev_malloc(&c->sinkT, sizeof(double) * c->C * c->ell)) != hipSuccess) return bail(e, "hipMalloc(sink)");
  }
  c->S.assign(d + 1, nullptr);
  c->Tk.assign(d + 1, nullptr);
  c->basis.assign(d + 1, nullptr);
  pstt2_status st = pstt2_reset(c);
  if (st != PSTT2_OK) {
    pstt2_destroy(c);
    return st;
  }
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return bail(e, "create");
  *out = c;
  return PSTT2_OK;
}

pstt2_status pstt2_reset(pstt2_ctx* c) {
  if (!c) return fail(nullptr, PSTT2_EINVAL, "null context");
  free_recovery(c);
  // one fill launch for both middle sketches and the flag word; Y is left to
  // the first sketch launch when every launch has one column group (FP64)
  c->y_unset = false;
  const bool lazy_y = !c->indep && c->prec == PSTT2_P_F64 && c->gj_max == 1;
  hipLaunchKernelGGL(k_zero_sketches, dim3(1024), dim3(256), 0, c->stream, c->Y, lazy_y ? 0 : c->R * c->ell, c->Tt,
                     c->C * c->ell, c->flag);
  HIPCK(c, hipGetLastError());
  c->y_unset = lazy_y;
  for (double* y : c->iY)
    if (y) HIPCK(c, hipMemsetAsync(y, 0, sizeof(double) * c->R * c->ell, c->stream));
  for (double* t : c->iT)
    if (t) HIPCK(c, hipMemsetAsync(t, 0, sizeof(double) * c->C * c->ell, c->stream));
  c->cover.clear();
  c->covered = 0;
  c->poisoned = false;
  return PSTT2_OK;
}

pstt2_status pstt2_profile(pstt2_ctx* c, int32_t enable) {
  if (!c) return fail(nullptr, PSTT2_EINVAL, "null context");
  c->profile = enable != 0;
  if (!c->profile) {
    for (auto& e : c->ev_used) c->ev_pool.push_back(e);
    c->ev_used.clear();
  }
  return PSTT2_OK;
}

pstt2_status pstt2_profile_read(pstt2_ctx* c, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches) return fail(c, PSTT2_EINVAL, "null argument");
  HIPCK(c, hipStreamSynchronize(c->stream));
  double tot = 0.0;
  for (auto& e : c->ev_used) {
    float ms = 0.0f;
    HIPCK(c, hipEventElapsedTime(&ms, e.first, e.second));
    tot += ms;
    c->ev_pool.push_back(e);
  }
  *total_ms = tot;
  *launches = (int64_t)c->ev_used.size();
  c->ev_used.clear();
  return PSTT2_OK;
}

void pstt2_destroy(pstt2_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto& e : c->ev_used) c->ev_pool.push_back(e);
  for (auto& e : c->ev_pool) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  free_recovery(c);
  arena_release(&c->arena, c->stream);
  arena_release(&c->varena, c->stream);
  (void)hipStreamSynchronize(c->stream);
  dev_free(c->fac);
  dev_free(c->Y);
  dev_free(c->Tt);
  dev_free(c->ypart);
  dev_free(c->tpart);
  dev_free(c->flag);
  dev_free(c->piv_dev);
  dev_free(c->one);
  dev_free(c->Bk);
  dev_free(c->chain_dev);
  dev_free(c->om_tab);
  dev_free(c->om16);
  for (uint16_t* p : c->iom16) dev_free(p);
  for (double* p : c->iom_tab) dev_free(p);
  for (double* p : c->iY) dev_free(p);
  for (double* p : c->iT) dev_free(p);
  dev_free(c->sinkY);
  dev_free(c->sinkT);
  dev_free(c->fn_rec);
  dev_free(c->fn_row);
  dev_free(c->fn_col);
  delete c;
}

pstt2_status pstt2_sketch(pstt2_ctx* c, const void* x_dev, int64_t first, int64_t count) {
  if (!c) return fail(nullptr, PSTT2_EINVAL, "null context");
  if (!x_dev && count > 0) return fail(c, PSTT2_EINVAL, "null slab pointer");
  if (c->poisoned) return fail(c, PSTT2_ESTATE, kPoisoned);
  if (c->recovered) return fail(c, PSTT2_ESTATE, "sketch after recover: call pstt2_reset first");
  pstt2_status st = check_range(c, first, count);
  if (st != PSTT2_OK) return st;
  const int64_t before = c->accum;
  st = settle(c, run_slabs(c, {Piece{x_dev, first, count}}), before);
  if (st != PSTT2_OK) return st;
  add_cover(c, first, count);
  return PSTT2_OK;
}

// fields of a tensor function (kind, and for GAUSS the bump parameters)
static const char* fn_invalid(const pstt2_fn* fn) {
  if (fn->kind == PSTT2_FN_HILBERT) return nullptr;
  if (fn->kind != PSTT2_FN_GAUSS) return "unknown tensor function";
  if (fn->n_terms < 1 || fn->n_terms > PSTT2_GAUSS_MAX_TERMS) return "n_terms must be in [1, PSTT2_GAUSS_MAX_TERMS]";
  if (!(fn->gamma > 0.0) || !std::isfinite(fn->gamma)) return "gamma must be positive and finite";
  if (!fn->centers) return "null centers";
  return nullptr;
}

// Gaussian bumps: chunks of whole columns of X_m evaluated into a workspace in
// the context's dtype, each streamed by the memory path like a slab.
static pstt2_status sketch_gauss(pstt2_ctx* c, const pstt2_fn* fn, int64_t first, int64_t count) {
  hipStream_t s = c->stream;
  double* tabs = nullptr;
  hipError_t e = ws_alloc((void**)&tabs, sizeof(double) * gauss_table_doubles(c->n, c->d, c->m, fn->n_terms), s);
  if (e != hipSuccess) return hfail(c, e, "Gaussian-bump tables");
  GaussTabs g;
  e = gauss_tables(c->n, c->d, c->m, fn->centers, fn->n_terms, fn->gamma, tabs, &g, s);
  const int esz = c->dtype == PSTT2_F64 ? 8 : 4;
  const int64_t ncmax = e == hipSuccess ? gauss_chunk_cols(g, esz) : 1;   // g is set only on success
  void* W = nullptr;
  if (e == hipSuccess) e = ws_alloc(&W, (size_t)esz * c->R * std::min(ncmax, count / c->R), s);
  pstt2_status st = PSTT2_OK;
  if (e != hipSuccess) st = hfail(c, e, "Gaussian-bump workspace");
  for (int64_t c0 = first / c->R; st == PSTT2_OK && c0 < (first + count) / c->R; c0 += ncmax) {
    const int64_t nc = std::min(ncmax, (first + count) / c->R - c0);
    e = gauss_columns(g, c0, nc, c->dtype, W, s);
    if (e != hipSuccess) st = hfail(c, e, "Gaussian-bump columns");
    else st = run_slabs(c, {Piece{W, c0 * c->R, nc * c->R}});
  }
  if (W) ws_free(W, s);
  ws_free(tabs, s);
  return st;
}

pstt2_status pstt2_sketch_fn(pstt2_ctx* c, const pstt2_fn* fn, int64_t first, int64_t count) {
  if (!c) return fail(nullptr, PSTT2_EINVAL, "null context");
  if (!fn) return fail(c, PSTT2_EINVAL, "null function");
  if (const char* why = fn_invalid(fn)) return fail(c, PSTT2_EINVAL, why);
  if (fn->kind == PSTT2_FN_HILBERT && (c->dtype != PSTT2_F64 || c->prec != PSTT2_P_F64))
    return fail(c, PSTT2_EINVAL, "the Hilbert function needs an FP64 context with FP64 sketches");
  if (c->poisoned) return fail(c, PSTT2_ESTATE, kPoisoned);
  if (c->recovered) return fail(c, PSTT2_ESTATE, "sketch after recover: call pstt2_reset first");
  if (first % c->R != 0 || count % c->R != 0)
    return fail(c, PSTT2_EINVAL, "first/count must be multiples of n_1...n_m (whole columns of X_m)");
  pstt2_status st = check_range(c, first, count);
  if (st != PSTT2_OK) return st;
  if (count == 0) return PSTT2_OK;
  const int64_t before = c->accum;
  if (fn->kind == PSTT2_FN_GAUSS) {
    st = settle(c, sketch_gauss(c, fn, first, count), before);
    if (st == PSTT2_OK) add_cover(c, first, count);
    return st;
  }
  hipError_t e = hipSuccess;
  if (!c->fn_rec) {
    double* rec = nullptr;
    int32_t *row_t = nullptr, *col_t = nullptr;
    e = dev_malloc(&rec, sizeof(double) * hilbert_rec_len(c->n, c->d));
    if (e == hipSuccess) e = dev_malloc(&row_t, sizeof(int32_t) * c->R);
    if (e == hipSuccess) e = dev_malloc(&col_t, sizeof(int32_t) * c->C);
    if (e == hipSuccess) e = hilbert_tables(c->n, c->d, c->m, c->R, c->C, rec, row_t, col_t, c->stream);
    if (e != hipSuccess) {
      dev_free(rec);
      dev_free(row_t);
      dev_free(col_t);
      return hfail(c, e, "Hilbert tables");
    }
    c->fn_rec = rec;
    c->fn_row = row_t;
    c->fn_col = col_t;
  }
  const std::vector<Seg> segs{Seg{nullptr, first / c->R, count / c->R, 0}};
  for (int g = 0; g < pass_groups(c); ++g) {
    double *Yd = nullptr, *Td = nullptr;
    SketchArgs ga = group_args(c, g, &Yd, &Td);
    ga.fn = 1;
    ga.fn_rec = c->fn_rec;
    ga.fn_row = c->fn_row;
    ga.fn_col = c->fn_col;
    st = settle(c, launch_segs(c, ga, segs, Yd, Td), before);
    if (st != PSTT2_OK) return st;
  }
  add_cover(c, first, count);
  return PSTT2_OK;
}

pstt2_status pstt2_sketch_slabs(pstt2_ctx* c, int32_t nslabs, const void* const* xs, const int64_t* firsts,
                                const int64_t* counts) {
  if (!c) return fail(nullptr, PSTT2_EINVAL, "null context");
  if (nslabs < 0 || (nslabs > 0 && (!xs || !firsts || !counts))) return fail(c, PSTT2_EINVAL, "bad slab arrays");
  if (c->poisoned) return fail(c, PSTT2_ESTATE, kPoisoned);
  if (c->recovered) return fail(c, PSTT2_ESTATE, "sketch after recover: call pstt2_reset first");
  // validate every slab (including overlaps among themselves) before launching
  std::map<int64_t, int64_t> saved = c->cover;
  int64_t saved_cov = c->covered;
  std::vector<Piece> ps;
  for (int s = 0; s < nslabs; ++s) {
    pstt2_status st = (!xs[s] && counts[s] > 0) ? fail(c, PSTT2_EINVAL, "null slab pointer")
                                                : check_range(c, firsts[s], counts[s]);
    if (st != PSTT2_OK) {
      c->cover = saved;
      c->covered = saved_cov;
      return st;
    }
    add_cover(c, firsts[s], counts[s]);
    ps.push_back(Piece{xs[s], firsts[s], counts[s]});
  }
  const int64_t before = c->accum;
  pstt2_status st = settle(c, run_slabs(c, ps), before);
  if (st != PSTT2_OK) {
    c->cover = saved;
    c->covered = saved_cov;
  }
  return st;
}

pstt2_status pstt2_recover(pstt2_ctx* c, tt_cores* out) {
  if (!c || !out) return fail(c, PSTT2_EINVAL, "null argument");
  if (c->poisoned) return fail(c, PSTT2_ESTATE, kPoisoned);
  if (c->covered != c->N) return fail(c, PSTT2_ESTATE, "not every entry of X was streamed exactly once");
  free_recovery(c);
  HIPCK(c, y_settle(c));
  const int d = c->d, m = c->m, ell = c->ell;
  hipStream_t s = c->stream;
  HIPCK(c, arena_begin(&c->arena, s));
  ArenaScope arena_scope(&c->arena);
  // (1) every split's sketch
  c->S[m] = c->Y;
  c->Tk[m] = c->Tt;
  if (!c->indep) {
    for (int k = m - 1; k >= 1; --k) {
      HIPCK(c, ws_alloc((void**)&c->S[k], sizeof(double) * c->Rk[k] * ell, s));
      HIPCK(c, derive_left(c->S[k + 1], c->S[k], c->Rk[k], (int)c->n[k], ell, c->fac + c->omega_off[k], s));
    }
    for (int k = m + 1; k <= d - 1; ++k) {
      const int64_t Ck = c->N / c->Rk[k];
      HIPCK(c, ws_alloc((void**)&c->Tk[k], sizeof(double) * Ck * ell, s));
      HIPCK(c, derive_right(c->Tk[k - 1], c->Tk[k], Ck, (int)c->n[k - 1], ell, c->fac + c->psi_off[k - 1], s));
    }
  } else {
    // split k's own sketch of X_m, contracted down mode by mode with split k's factors
    for (int k = 1; k < m; ++k) {
      const double* cur = c->iY[k];
      for (int q = m; q >= k + 1; --q) {   // contract mode q: R_q -> R_{q-1} rows
        double* nxt = nullptr;
        HIPCK(c, ws_alloc((void**)&nxt, sizeof(double) * c->Rk[q - 1] * ell, s));
        HIPCK(c, derive_left(cur, nxt, c->Rk[q - 1], (int)c->n[q - 1], ell, c->fac + c->iom_off[k][q - 1], s));
        if (cur != c->iY[k]) ws_free((void*)cur, s);
        cur = nxt;
      }
      c->S[k] = (double*)cur;
    }
    for (int k = m + 1; k <= d - 1; ++k) {
      const double* cur = c->iT[k];
      for (int q = m + 1; q <= k; ++q) {   // contract mode q: C_{q-1} -> C_q columns
        const int64_t Cq = c->N / c->Rk[q];
        double* nxt = nullptr;
        HIPCK(c, ws_alloc((void**)&nxt, sizeof(double) * Cq * ell, s));
        HIPCK(c, derive_right(cur, nxt, Cq, (int)c->n[q - 1], ell, c->fac + c->ipsi_off[k][q - 1], s));
        if (cur != c->iT[k]) ws_free((void*)cur, s);
        cur = nxt;
      }
      c->Tk[k] = (double*)cur;
    }
  }
  // two-sided sketches: B_k = Psi_k^T S_k (k < m), B_k = T_k Omega_k (k >= m)
  {
    TwoSidedBatch tb;
    std::memset(&tb, 0, sizeof(tb));
    tb.d = d;
    tb.ell = ell;
    tb.fac = c->fac;
    tb.chain = c->chain_dev;
    for (int q = 0; q < d; ++q) tb.nmode[q] = c->n[q];
    for (int k = 1; k <= d - 1; ++k) {
      const int p = tb.n++;
      const bool col = k < m || c->pstt;   // operand S_k (PSTT: S_{d-1} = Y)
      tb.split[p] = k;
      tb.right[p] = !col;
      tb.S[p] = col ? c->S[k] : c->Tk[k];
      tb.K[p] = col ? c->Rk[k] : c->N / c->Rk[k];
      tb.out[p] = c->Bk + (int64_t)k * ell * ell;
    }
    HIPCK(c, two_sided_batch(tb, s));
  }
  // (2) factor every sketch (one batched TSQR over all splits); the ranks come
  // from the descriptor or, in tolerance mode, from the singular values (one
  // host synchronisation)
  const bool tol = c->desc.ranks[0] <= 0;
  std::vector<const double*> Ap(d - 1);
  std::vector<int64_t> Mp(d - 1);
  std::vector<int*> pivp(d - 1);
  for (int k = 1; k <= d - 1; ++k) {
    const bool col = k < m || c->pstt;   // column basis Q_k from S_k, else row basis P_k from T_k
    Ap[k - 1] = col ? c->S[k] : c->Tk[k];
    Mp[k - 1] = col ? c->Rk[k] : c->N / c->Rk[k];
    pivp[k - 1] = c->piv_dev + (int64_t)k * ell;
  }
  BasisBatch* bw = nullptr;
  {
    hipError_t e = basis_factor_batch(d - 1, Ap.data(), Mp.data(), ell, pivp.data(), tol, &bw, s);
    if (e != hipSuccess) {
      basis_batch_free(bw);
      return hfail(c, e, "basis_factor_batch");
    }
  }
  int r[PSTT2_MAX_D + 1];
  r[0] = r[d] = 1;
  std::vector<double> sv((size_t)(d + 1) * ell, 0.0);
  if (tol) {
    double* pin = pinned_scratch();
    for (int k = 1; k <= d - 1; ++k) {
      hipError_t e = hipMemcpyAsync(pin ? pin + (size_t)k * ell : sv.data() + (size_t)k * ell,
                                    basis_batch_sv(bw, k - 1), sizeof(double) * ell, hipMemcpyDeviceToHost, s);
      if (e != hipSuccess) {
        basis_batch_free(bw);
        return hfail(c, e, "hipMemcpyAsync(sv)");
      }
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      basis_batch_free(bw);
      return hfail(c, e, "recover");
    }
    if (pin)
      for (int k = 1; k <= d - 1; ++k)
        for (int i = 0; i < ell; ++i) sv[(size_t)k * ell + i] = pin[(size_t)k * ell + i];
  }
  for (int k = 1; k <= d - 1; ++k) {
    const int64_t cap = std::min<int64_t>({c->Rk[k], c->N / c->Rk[k], (int64_t)ell});
    r[k] = tol ? rank_from_rule(c, k, sv.data(), c->desc.eps * c->eps_scale)
               : (int)std::min<int64_t>(c->desc.ranks[k - 1], cap);
  }
  if (tol) c->sv_last = sv;
  // (3) bases
  {
    std::vector<double*> Qp(d - 1);
    hipError_t e = hipSuccess;
    for (int k = 1; k <= d - 1 && e == hipSuccess; ++k) {
      e = ws_alloc((void**)&c->basis[k], sizeof(double) * Mp[k - 1] * r[k], s);
      Qp[k - 1] = c->basis[k];
    }
    if (e == hipSuccess) e = basis_form_q_batch(bw, r + 1, Qp.data(), s);
    basis_batch_free(bw);
    if (e != hipSuccess) return hfail(c, e, "basis_form_q_batch");
  }
  for (int k = 0; k <= d; ++k) c->ranks[k] = r[k];
  // (4) cores, one allocation based at core[0]
  tt_cores tc;
  std::memset(&tc, 0, sizeof(tc));
  tc.d = d;
  tc.owned = 1;
  int64_t tot = 0;
  for (int k = 0; k < d; ++k) {
    tc.n[k] = c->n[k];
    tot += (int64_t)r[k] * c->n[k] * r[k + 1];
  }
  for (int k = 0; k <= d; ++k) tc.r[k] = r[k];
  double* base = nullptr;
  HIPCK(c, dev_malloc_async((void**)&base, sizeof(double) * tot, s));
  tc.stream = (void*)s;
  int64_t o = 0;
  for (int k = 0; k < d; ++k) {
    tc.core[k] = base + o;
    o += (int64_t)r[k] * c->n[k] * r[k + 1];
  }
  auto cfail = [&](hipError_t e, const char* w) {
    tt_cores_free(&tc);
    return hfail(c, e, w);
  };
  hipError_t e = hipSuccess;
  // column-basis cores G_1 .. G_{m-1} (PSTT: G_1 .. G_{d-1})
  const int kl_end = c->pstt ? d - 1 : m - 1;
  for (int k = 1; k <= kl_end && e == hipSuccess; ++k) {
    if (k == 1)
      e = hipMemcpyAsync(tc.core[0], c->basis[1], sizeof(double) * c->n[0] * r[1], hipMemcpyDeviceToDevice, s);
    else
      e = core_left(c->basis[k - 1], c->Rk[k - 1], r[k - 1], c->basis[k], (int)c->n[k - 1], r[k], tc.core[k - 1], s);
  }
  if (c->pstt) {
    if (e != hipSuccess) return cfail(e, "cores");
    // last core G_d (r_{d-1} x n_d).  One pass: G_d = (Psi^T Q)^+ T with
    // Psi = Psi_{d-1}, Q = Q_{d-1} and T = T_{d-1} = Psi^T X_{d-1} (kept
    // transposed, n_d x ell): G_d^T = T^T A (A^T A)^{-1} with A = Psi^T Q
    // (ell x r), i.e. the least-squares kernel with right-hand side T^T and
    // system matrix A^T.  Two pass: zero here, pstt2_middle_pass adds Q^T X_{d-1}.
    const int rl = r[d - 1];
    const int64_t nd = c->n[d - 1];
    if (c->desc.mid == PSTT2_MID_TWOPASS) {
      e = hipMemsetAsync(tc.core[d - 1], 0, sizeof(double) * rl * nd, s);
    } else {
      double *A = nullptr, *At = nullptr, *Gt = nullptr;
      e = ws_alloc((void**)&A, sizeof(double) * ell * ell, s);
      if (e == hipSuccess) e = ws_alloc((void**)&At, sizeof(double) * rl * ell, s);
      if (e == hipSuccess) e = ws_alloc((void**)&Gt, sizeof(double) * nd * rl, s);
      if (e == hipSuccess) {
        TwoSidedBatch tb;
        std::memset(&tb, 0, sizeof(tb));
        tb.d = d;
        tb.ell = ell;
        tb.fac = c->fac;
        tb.chain = c->chain_dev;
        for (int q = 0; q < d; ++q) tb.nmode[q] = c->n[q];
        tb.n = 1;
        tb.split[0] = d - 1;
        tb.right[0] = 0;
        tb.S[0] = c->basis[d - 1];
        tb.scols[0] = rl;
        tb.K[0] = c->Rk[d - 1];
        tb.out[0] = A;   // ell x ell, columns >= r zero
        e = two_sided_batch(tb, s);
      }
      if (e == hipSuccess) e = adj_transpose(A, ell, rl, At, s);
      if (e == hipSuccess) e = middle_ls(c->Tt, nd, At, rl, ell, Gt, c->flag, s);
      if (e == hipSuccess) e = adj_transpose(Gt, nd, rl, tc.core[d - 1], s);
      ws_free(A, s);
      ws_free(At, s);
      ws_free(Gt, s);
    }
    if (e != hipSuccess) return cfail(e, "last core");
  }
  for (int k = m + 1; k <= d && e == hipSuccess && !c->pstt; ++k) {
    if (k == d) {
      const int64_t rows = c->n[d - 1];
      hipLaunchKernelGGL(k_transpose_last, dim3(64), dim3(256), 0, s, c->basis[d - 1], rows, r[d - 1], tc.core[d - 1]);
      e = hipGetLastError();
    } else {
      const int64_t Cp = c->N / c->Rk[k - 1], Ck = c->N / c->Rk[k];
      e = core_right(c->basis[k - 1], Cp, r[k - 1], c->basis[k], Ck, (int)c->n[k - 1], r[k], tc.core[k - 1], s);
    }
  }
  if (e != hipSuccess) return cfail(e, "cores");
  const double* Qprev = m >= 2 ? c->basis[m - 1] : c->one;
  const int64_t Rprev = c->Rk[m - 1];
  const int64_t nz = (int64_t)r[m - 1] * c->n[m - 1];
  if (c->pstt) {
    // every core is formed above
  } else if (c->desc.mid == PSTT2_MID_ONEPASS || c->desc.mid == PSTT2_MID_TWOSIDED) {
    double *Z = nullptr, *A = nullptr;
    const int nm = (int)c->n[m - 1];
    e = ws_alloc((void**)&Z, sizeof(double) * nz * ell, s);
    if (e == hipSuccess) e = ws_alloc((void**)&A, sizeof(double) * r[m] * ell, s);
    if (c->desc.mid == PSTT2_MID_ONEPASS || m == 1) {
      // Z = (I (x) Q_{m-1})^T Y_R
      if (e == hipSuccess) e = middle_z(Qprev, Rprev, r[m - 1], c->Y, c->R, nm, ell, Z, s);
    } else {
      // H = (I (x) Psi')^T Y_R with Psi' split (m-1)'s left DRM; then
      // Z = (I (x) M1) H with M1 = (Psi'^T Q_{m-1})^+ = (A1^T A1)^{-1} A1^T,
      // A1 = Psi'^T Q_{m-1} (ell x r_{m-1}).  The least-squares kernel with
      // right-hand side I_ell and system matrix A1^T returns M1^T.
      const int rp = r[m - 1];
      double *ptab = nullptr, *a1t = nullptr, *id = nullptr, *m1t = nullptr;
      if (e == hipSuccess) e = ws_alloc((void**)&c->H, sizeof(double) * ell * nm * ell, s);
      if (e == hipSuccess) e = ws_alloc((void**)&ptab, sizeof(double) * Rprev * ell, s);
      if (e == hipSuccess) e = ws_alloc((void**)&a1t, sizeof(double) * rp * ell, s);
      if (e == hipSuccess) e = ws_alloc((void**)&id, sizeof(double) * ell * ell, s);
      if (e == hipSuccess) e = ws_alloc((void**)&m1t, sizeof(double) * ell * rp, s);
      if (e == hipSuccess) e = kr_table(c->fac, left_chain(c, m - 1), Rprev, ell, ptab, s);
      if (e == hipSuccess) e = middle_z(ptab, Rprev, ell, c->Y, c->R, nm, ell, c->H, s);
      if (e == hipSuccess) e = adj_gemm(true, false, rp, ell, Rprev, 1.0, Qprev, Rprev, ptab, Rprev, 0.0, a1t, rp, s);
      if (e == hipSuccess) e = eye(ell, id, s);
      if (e == hipSuccess) e = middle_ls(id, ell, a1t, rp, ell, m1t, c->flag, s);
      if (e == hipSuccess) e = middle_z(m1t, ell, rp, c->H, (int64_t)ell * nm, nm, ell, Z, s);
      ws_free(ptab, s);
      ws_free(a1t, s);
      ws_free(id, s);
      ws_free(m1t, s);
    }
    SketchArgs geo = base_args(c);
    if (e == hipSuccess) e = middle_a(c->basis[m], c->C, r[m], geo, c->prec, A, s);
    if (e == hipSuccess) e = middle_ls(Z, nz, A, r[m], ell, tc.core[m - 1], c->flag, s);
    ws_free(Z, s);
    ws_free(A, s);
  } else {
    e = hipMemsetAsync(tc.core[m - 1], 0, sizeof(double) * nz * r[m], s);
  }
  if (e != hipSuccess) return cfail(e, "middle core");
  // (5) the single completion point: non-finite sketches, singular LS
  int hflag = 0;
  int* pin = (int*)pinned_scratch();
  e = hipMemcpyAsync(pin ? pin : &hflag, c->flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (pin) hflag = *pin;
  if (e != hipSuccess) return cfail(e, "recover");
  if (hflag & 1) {
    tt_cores_free(&tc);
    return fail(c, PSTT2_ENUMERIC, "non-finite values in the sketches (NaN/Inf in X)");
  }
  if (hflag & 2) {
    tt_cores_free(&tc);
    return fail(c, PSTT2_ENUMERIC, "rank-deficient least-squares system for the middle core");
  }
  *out = tc;
  c->recovered = true;
  return PSTT2_OK;
}

pstt2_status pstt2_recover_certified(pstt2_ctx* c, const void* x_dev, const pstt2_fn* fn, int32_t max_tries,
                                     tt_cores* out, double* rel_err) {
  if (!c || !out || !rel_err) return fail(c, PSTT2_EINVAL, "null argument");
  if ((x_dev == nullptr) == (fn == nullptr)) return fail(c, PSTT2_EINVAL, "give exactly one of x_dev and fn");
  if (fn && fn_invalid(fn)) return fail(c, PSTT2_EINVAL, fn_invalid(fn));
  if (c->desc.ranks[0] > 0) return fail(c, PSTT2_ESTATE, "certified recovery needs a tolerance-mode context");
  if (c->desc.mid == PSTT2_MID_TWOPASS) return fail(c, PSTT2_ESTATE, "certified recovery covers the one-pass cores");
  if (max_tries < 1) return fail(c, PSTT2_EINVAL, "max_tries must be >= 1");
  const int d = c->d;
  double scale = 1.0, err = INFINITY;
  tt_cores best;
  std::memset(&best, 0, sizeof(best));
  bool have = false;
  pstt2_status st = PSTT2_OK;
  for (int t = 0; t < max_tries; ++t) {
    c->eps_scale = scale;
    tt_cores tc;
    std::memset(&tc, 0, sizeof(tc));
    st = pstt2_recover(c, &tc);
    if (st != PSTT2_OK) break;
    double e = 0.0;
    st = x_dev ? tt_error(&tc, x_dev, (pstt2_dtype)c->dtype, &e, c->stream) : tt_error_fn(&tc, fn, &e, c->stream);
    if (st != PSTT2_OK) {
      c->err = g_tls_err;
      tt_cores_free(&tc);
      break;
    }
    if (have) tt_cores_free(&best);
    best = tc;
    have = true;
    err = e;
    if (e <= c->desc.eps) break;
    // tighten the rule until some rank grows (the singular values do not depend
    // on eps, so the next recovery takes exactly these ranks); stop when every
    // rank sits at its cap: then only a larger sketch size helps
    bool grew = false;
    for (int j = 0; j < 64 && !grew; ++j) {
      scale *= 0.5;
      for (int k = 1; k <= d - 1 && !grew; ++k)
        grew = rank_from_rule(c, k, c->sv_last.data(), c->desc.eps * scale) > c->ranks[k];
    }
    if (!grew) break;
  }
  c->eps_scale = 1.0;
  if (st != PSTT2_OK) {
    if (have) tt_cores_free(&best);
    return st;
  }
  *out = best;
  *rel_err = err;
  return PSTT2_OK;
}

pstt2_status pstt2_middle_pass(pstt2_ctx* c, tt_cores* cores, const void* x_dev, int64_t first, int64_t count) {
  if (!c || !cores) return fail(c, PSTT2_EINVAL, "null argument");
  if (c->poisoned) return fail(c, PSTT2_ESTATE, kPoisoned);
  if (c->desc.mid != PSTT2_MID_TWOPASS || !c->recovered)
    return fail(c, PSTT2_ESTATE, "middle pass needs a two-pass context after pstt2_recover");
  if (first < 0 || count < 0 || first + count > c->N) return fail(c, PSTT2_EINVAL, "slab range outside the tensor");
  if (first % c->n[0] != 0 || count % c->n[0] != 0) return fail(c, PSTT2_EINVAL, "slab must hold whole mode-1 fibres");
  const int m = c->m;
  if (c->pstt) {
    // last core of the one-sided algorithm: G_d(a, i) += sum_row Q_{d-1}(row, a) X(row + R_{d-1} i)
    const int d = c->d;
    HIPCK(c, middle_twopass(c->dtype, x_dev, first, count, c->Rk[d - 1], (int)c->n[d - 1], 1, c->basis[d - 1],
                            c->ranks[d - 1], c->one, 1, cores->core[d - 1], c->stream));
    return PSTT2_OK;
  }
  const double* Qprev = m >= 2 ? c->basis[m - 1] : c->one;
  HIPCK(c, middle_twopass(c->dtype, x_dev, first, count, c->Rk[m - 1], (int)c->n[m - 1], c->C, Qprev,
                          c->ranks[m - 1], c->basis[m], c->ranks[m], cores->core[m - 1], c->stream));
  return PSTT2_OK;
}

pstt2_status pstt2_middle_pass_fn(pstt2_ctx* c, tt_cores* cores, const pstt2_fn* fn, int64_t first,
                                  int64_t count) {
  if (!c || !cores || !fn) return fail(c, PSTT2_EINVAL, "null argument");
  if (const char* why = fn_invalid(fn)) return fail(c, PSTT2_EINVAL, why);
  if (c->poisoned) return fail(c, PSTT2_ESTATE, kPoisoned);
  if (c->desc.mid != PSTT2_MID_TWOPASS || !c->recovered)
    return fail(c, PSTT2_ESTATE, "middle pass needs a two-pass context after pstt2_recover");
  if (first < 0 || count < 0 || first + count > c->N) return fail(c, PSTT2_EINVAL, "slab range outside the tensor");
  if (first % c->R != 0 || count % c->R != 0)
    return fail(c, PSTT2_EINVAL, "first/count must be whole columns of the pass's unfolding");
  if (count == 0) return PSTT2_OK;
  hipStream_t s = c->stream;
  const int esz = c->dtype == PSTT2_F64 ? 8 : 4;
  // tables of the split the pass runs at (m, or d - 1 for the one-sided algorithm)
  GaussTabs g;
  double* tabs = nullptr;
  int32_t *row_t = nullptr, *col_t = nullptr;
  hipError_t e = hipSuccess;
  int64_t ncmax = 1;   // set from the tables once they exist
  if (fn->kind == PSTT2_FN_GAUSS) {
    e = ws_alloc((void**)&tabs, sizeof(double) * gauss_table_doubles(c->n, c->d, c->m, fn->n_terms), s);
    if (e == hipSuccess) e = gauss_tables(c->n, c->d, c->m, fn->centers, fn->n_terms, fn->gamma, tabs, &g, s);
    if (e == hipSuccess) ncmax = gauss_chunk_cols(g, esz);
  } else {
    e = ws_alloc((void**)&tabs, sizeof(double) * hilbert_rec_len(c->n, c->d), s);
    if (e == hipSuccess) e = ws_alloc((void**)&row_t, sizeof(int32_t) * c->R, s);
    if (e == hipSuccess) e = ws_alloc((void**)&col_t, sizeof(int32_t) * c->C, s);
    if (e == hipSuccess) e = hilbert_tables(c->n, c->d, c->m, c->R, c->C, tabs, row_t, col_t, s);
    ncmax = std::min(c->C, std::max<int64_t>(1, PSTT2_GAUSS_CHUNK_BYTES / (c->R * esz)));
  }
  void* W = nullptr;
  if (e == hipSuccess) e = ws_alloc(&W, (size_t)esz * c->R * std::min(ncmax, count / c->R), s);
  pstt2_status st = e == hipSuccess ? PSTT2_OK : hfail(c, e, "tensor-function workspace");
  bool added = false;   // a chunk already added into the middle core
  for (int64_t c0 = first / c->R; st == PSTT2_OK && c0 < (first + count) / c->R; c0 += ncmax) {
    const int64_t nc = std::min(ncmax, (first + count) / c->R - c0);
    e = fn->kind == PSTT2_FN_GAUSS ? gauss_columns(g, c0, nc, c->dtype, W, s)
                                   : hilbert_columns(tabs, row_t, col_t, c->R, c0, nc, c->dtype, W, s);
    st = e == hipSuccess ? pstt2_middle_pass(c, cores, W, c0 * c->R, nc * c->R) : hfail(c, e, "tensor-function columns");
    if (st == PSTT2_OK) added = true;
  }
  if (st != PSTT2_OK && added) c->poisoned = true;
  if (W) ws_free(W, s);
  if (col_t) ws_free(col_t, s);
  if (row_t) ws_free(row_t, s);
  if (tabs) ws_free(tabs, s);
  return st;
}

pstt2_status pstt2_vjp(pstt2_ctx* c, const tt_cores* cores, const void* x_dev, const void* gbar_dev,
                       void* gx_dev) {
  if (!c || !cores || !gx_dev) return fail(c, PSTT2_EINVAL, "null argument");
  if (!gbar_dev && !x_dev) return fail(c, PSTT2_EINVAL, "x_dev is needed for the fused loss (gbar_dev == NULL)");
  if (c->poisoned) return fail(c, PSTT2_ESTATE, kPoisoned);
  if (!c->recovered) return fail(c, PSTT2_ESTATE, "pstt2_vjp needs a successful pstt2_recover first");
  if (c->desc.mid == PSTT2_MID_TWOPASS) return fail(c, PSTT2_ESTATE, "pstt2_vjp covers the one-pass middle cores only");
  if (c->pstt) return fail(c, PSTT2_ESTATE, "pstt2_vjp covers the two-sided algorithm only");
  const int d = c->d, m = c->m, ell = c->ell;
  if (cores->d != d) return fail(c, PSTT2_EINVAL, "cores do not match the context");
  for (int k = 0; k < d; ++k)
    if (cores->n[k] != c->n[k] || !cores->core[k]) return fail(c, PSTT2_EINVAL, "cores do not match the context");
  for (int k = 0; k <= d; ++k)
    if (cores->r[k] != c->ranks[k]) return fail(c, PSTT2_EINVAL, "core ranks differ from the last recovery");
  hipStream_t s = c->stream;
  const int* r = c->ranks;
  const int64_t* Rk = c->Rk;
  auto Ck = [&](int k) { return c->N / Rk[k]; };
  // every temporary comes from the context's adjoint arena (pstt2_vjp returns
  // only after its stream is idle, so the next call may rewind it)
  hipError_t e = arena_begin(&c->varena, s);
  ArenaScope arena_scope(&c->varena);
  auto take = [&](int64_t count, bool zero) -> double* {
    void* p = nullptr;
    if (e != hipSuccess) return nullptr;
    e = ws_alloc(&p, sizeof(double) * std::max<int64_t>(count, 1), s);
    if (e != hipSuccess) return nullptr;
    if (zero) e = hipMemsetAsync(p, 0, sizeof(double) * std::max<int64_t>(count, 1), s);
    return (double*)p;
  };
  auto release = [&]() {};
#define VJPCK(call)                        \
  do {                                     \
    if (e == hipSuccess) e = (call);       \
  } while (0)
  // ---- interfaces L_k (R_k x r_k), k = 1..m, and Rt_k (r_{k-1} x C_{k-1}), k = m+1..d ----
  std::vector<const double*> Lv(d + 2, nullptr), Rv(d + 2, nullptr);
  Lv[1] = cores->core[0];
  for (int k = 2; k <= m; ++k) {
    double* L = take(Rk[k] * r[k], false);
    VJPCK(adj_gemm(false, false, Rk[k - 1], c->n[k - 1] * r[k], r[k - 1], 1.0, Lv[k - 1], Rk[k - 1],
                   cores->core[k - 1], r[k - 1], 0.0, L, Rk[k - 1], s));
    Lv[k] = L;
  }
  Rv[d] = cores->core[d - 1];
  for (int k = d - 1; k >= m + 1; --k) {
    double* Rt = take((int64_t)r[k - 1] * Ck(k - 1), false);
    VJPCK(adj_gemm(false, false, (int64_t)r[k - 1] * c->n[k - 1], Ck(k), r[k], 1.0, cores->core[k - 1],
                   (int64_t)r[k - 1] * c->n[k - 1], Rv[k + 1], r[k], 0.0, Rt, (int64_t)r[k - 1] * c->n[k - 1], s));
    Rv[k] = Rt;
  }
  const int rm = r[m];
  const double* Lm = Lv[m];
  const double* Rtm = Rv[m + 1];
  // ---- B1: U = gbar_m Rt^T (R x r_m) and Vt = gbar_m^T L (C x r_m), the cotangent's
  //      contraction with the interfaces, by the FP64 dual-sketch kernel with L and
  //      Rt^T as its DRM tables.  A given gbar is streamed as it is.  For the
  //      Frobenius loss, gbar = -2 (X - L Rt) and the second term has rank r_m, so
  //      U = -2 (X_m Rt^T - L (Rt Rt^T)) and Vt = -2 (X_m^T L - Rt^T (L^T L)): the
  //      kernel streams X itself and two r_m x r_m Gram matrices supply the rest,
  //      so no tensor-sized cotangent is ever formed. ----
  const void* src = gbar_dev ? gbar_dev : x_dev;
  const int L4r = (rm + 3) / 4 * 4;
  double* psiT = take(c->R * L4r, false);
  double* omT = take(c->C * L4r, false);
  VJPCK(adj_table(Lm, c->R, rm, 1, c->R, L4r, psiT, s));
  VJPCK(adj_table(Rtm, c->C, rm, rm, 1, L4r, omT, s));
  SketchArgs a = base_args(c);
  a.ell = rm;
  a.L4 = L4r;
  a.om_tab = omT;
  a.psi_tab = psiT;
  int rpb = 0, thr = 0, wpc = 1;
  sketch_geometry(PSTT2_P_F64, rm, &rpb, &thr, &wpc);
  a.gi_count = (int)((c->R + rpb - 1) / rpb);
  a.nchunks = (c->C + 15) / 16;
  a.gj_count = (int)std::max<int64_t>(1, std::min<int64_t>(a.nchunks, std::max(1, c->ncu * wpc / a.gi_count)));
  a.nseg = 1;
  a.seg[0].ptr = src;
  a.seg[0].gcol0 = 0;
  a.seg[0].ncols = c->C;
  a.seg[0].chunk0 = 0;
  a.ypart = take((int64_t)a.gj_count * rm * c->R, false);
  a.tpart = take((int64_t)a.gi_count * rm * c->C + kTPartPad, false);
  a.tlp = 0;   // the FP64 kernel's partial layout
  a.om16 = nullptr;
  a.x32 = c->dtype == PSTT2_F32;   // FP32 entries are widened as they are loaded
  double* U = take(c->R * rm, true);    // Lbar_m = gbar_m Rt^T        (R x r_m)
  double* Vt = take(c->C * rm, true);   // (L_m^T gbar_m)^T           (C x r_m)
  if (e == hipSuccess) e = launch_sketch(PSTT2_P_F64, 0, a, s);
  if (e == hipSuccess) e = launch_reduce(PSTT2_P_F64, a, U, Vt, c->flag, s);
  if (!gbar_dev) {
    double* Gr = take((int64_t)rm * rm, false);   // Rt Rt^T
    double* Gl = take((int64_t)rm * rm, false);   // L^T L
    VJPCK(adj_gemm(false, true, rm, rm, c->C, 1.0, Rtm, rm, Rtm, rm, 0.0, Gr, rm, s));
    VJPCK(adj_gemm(true, false, rm, rm, c->R, 1.0, Lm, c->R, Lm, c->R, 0.0, Gl, rm, s));
    VJPCK(adj_gemm(false, false, c->R, rm, rm, 2.0, Lm, c->R, Gr, rm, -2.0, U, c->R, s));
    VJPCK(adj_gemm(true, false, c->C, rm, rm, 2.0, Rtm, rm, Gl, rm, -2.0, Vt, c->C, s));
  }
  // core cotangents, laid out like the cores
  std::vector<double*> Gb(d, nullptr);
  for (int k = 0; k < d; ++k) Gb[k] = take((int64_t)r[k] * c->n[k] * r[k + 1], true);
  const double* Lb = U;
  for (int k = m; k >= 2; --k) {
    const int64_t nr = c->n[k - 1] * r[k];
    VJPCK(adj_gemm(true, false, r[k - 1], nr, Rk[k - 1], 1.0, Lv[k - 1], Rk[k - 1], Lb, Rk[k - 1], 0.0, Gb[k - 1],
                   r[k - 1], s));
    double* Lbp = take(Rk[k - 1] * r[k - 1], false);
    VJPCK(adj_gemm(false, true, Rk[k - 1], r[k - 1], nr, 1.0, Lb, Rk[k - 1], cores->core[k - 1], r[k - 1], 0.0, Lbp,
                   Rk[k - 1], s));
    Lb = Lbp;
  }
  VJPCK(adj_axpy(c->n[0] * r[1], 1.0, Lb, Gb[0], s));
  double* Rb = take((int64_t)rm * c->C, false);
  VJPCK(adj_transpose(Vt, c->C, rm, Rb, s));
  for (int k = m + 1; k <= d - 1; ++k) {
    const int64_t rn = (int64_t)r[k - 1] * c->n[k - 1];
    VJPCK(adj_gemm(false, true, rn, r[k], Ck(k), 1.0, Rb, rn, Rv[k + 1], r[k], 0.0, Gb[k - 1], rn, s));
    double* Rbn = take((int64_t)r[k] * Ck(k), false);
    VJPCK(adj_gemm(true, false, r[k], Ck(k), rn, 1.0, cores->core[k - 1], rn, Rb, rn, 0.0, Rbn, r[k], s));
    Rb = Rbn;
  }
  VJPCK(adj_axpy((int64_t)r[d - 1] * c->n[d - 1], 1.0, Rb, Gb[d - 1], s));
  // ---- B2: back through the recovery ----
  std::vector<double*> Qb(d + 1, nullptr);
  for (int k = 1; k <= d - 1; ++k) Qb[k] = take((k < m ? Rk[k] : Ck(k)) * r[k], true);
  const double* Qprev = m >= 2 ? c->basis[m - 1] : c->one;
  const int64_t Rprev = Rk[m - 1];
  const int rprev = r[m - 1];
  const int nm = (int)c->n[m - 1];
  const int64_t p = (int64_t)rprev * nm;
  double* Z = take(p * ell, false);
  double* A = take((int64_t)rm * ell, false);
  double* Zb = take(p * ell, false);
  double* Ab = take((int64_t)rm * ell, false);
  // two-sided rule (d >= 3): Z = (I (x) M1) H with H = (I (x) Psi')^T Y_R and
  // M1 = (Psi'^T Q_{m-1})^+; rebuilt here as the recovery built it
  const bool two = c->desc.mid == PSTT2_MID_TWOSIDED && m >= 2;
  double *ptab = nullptr, *a1t = nullptr, *m1t = nullptr;
  if (!two) {
    VJPCK(middle_z(Qprev, Rprev, rprev, c->Y, c->R, nm, ell, Z, s));
  } else {
    ptab = take(Rprev * ell, false);
    a1t = take((int64_t)rprev * ell, false);
    m1t = take((int64_t)ell * rprev, false);
    double* id = take((int64_t)ell * ell, false);
    VJPCK(kr_table(c->fac, left_chain(c, m - 1), Rprev, ell, ptab, s));
    VJPCK(adj_gemm(true, false, rprev, ell, Rprev, 1.0, Qprev, Rprev, ptab, Rprev, 0.0, a1t, rprev, s));
    VJPCK(eye(ell, id, s));
    VJPCK(middle_ls(id, ell, a1t, rprev, ell, m1t, c->flag, s));
    VJPCK(middle_z(m1t, ell, rprev, c->H, (int64_t)ell * nm, nm, ell, Z, s));
  }
  SketchArgs geo = base_args(c);
  VJPCK(middle_a(c->basis[m], c->C, rm, geo, c->prec, A, s));
  VJPCK(adj_ls(cores->core[m - 1], Gb[m - 1], Z, A, p, rm, ell, Zb, Ab, s));
  double* Yb = take(c->R * ell, true);
  if (!two) {
    if (m >= 2)
      VJPCK(adj_gemm(false, true, Rprev, rprev, (int64_t)nm * ell, 1.0, c->Y, Rprev, Zb, rprev, 1.0, Qb[m - 1],
                     Rprev, s));
    VJPCK(adj_gemm(false, false, Rprev, (int64_t)nm * ell, rprev, 1.0, Qprev, Rprev, Zb, rprev, 1.0, Yb, Rprev, s));
  } else {
    // Z3(p, j, c) = sum_a M1^T(a, p) H3(a, j, c):
    //   Hbar = M1^T Zbar and M1^T-bar = H Zbar^T, with H as ell x (n_m ell), Zbar as r_{m-1} x (n_m ell)
    const int64_t w = (int64_t)nm * ell;
    double* Hb = take((int64_t)ell * w, false);
    double* M1b = take((int64_t)ell * rprev, false);   // cotangent of M1^T
    VJPCK(adj_gemm(false, false, ell, w, rprev, 1.0, m1t, ell, Zb, rprev, 0.0, Hb, ell, s));
    VJPCK(adj_gemm(false, true, ell, rprev, w, 1.0, c->H, ell, Zb, rprev, 0.0, M1b, ell, s));
    // pseudo-inverse of the full-column-rank A1 = Psi'^T Q (ell x r), W = A1^+ = (A1^T A1)^{-1} A1^T:
    //   dW = -W dA1 W + (A1^T A1)^{-1} dA1^T (I - A1 W), so with (A1^T A1)^{-1} = W W^T
    //   A1bar = -W^T Wbar W^T + (I - A1 W) Wbar^T W W^T.
    // In M1^T = W^T and its cotangent Mb = Wbar^T:  T1 = Mb^T M1^T, T2 = M1 M1^T,
    //   A1bar = -M1^T T1 + Mb T2 - A1 (T1^T T2).
    const int rp = rprev;
    double* T1 = take((int64_t)rp * rp, false);
    double* T2 = take((int64_t)rp * rp, false);
    double* T4 = take((int64_t)rp * rp, false);
    double* A1b = take((int64_t)ell * rp, false);
    VJPCK(adj_gemm(true, false, rp, rp, ell, 1.0, M1b, ell, m1t, ell, 0.0, T1, rp, s));
    VJPCK(adj_gemm(true, false, rp, rp, ell, 1.0, m1t, ell, m1t, ell, 0.0, T2, rp, s));
    VJPCK(adj_gemm(true, false, rp, rp, rp, 1.0, T1, rp, T2, rp, 0.0, T4, rp, s));
    VJPCK(adj_gemm(false, false, ell, rp, rp, -1.0, m1t, ell, T1, rp, 0.0, A1b, ell, s));
    VJPCK(adj_gemm(false, false, ell, rp, rp, 1.0, M1b, ell, T2, rp, 1.0, A1b, ell, s));
    VJPCK(adj_gemm(true, false, ell, rp, rp, -1.0, a1t, rp, T4, rp, 1.0, A1b, ell, s));
    // A1 = Psi'^T Q_{m-1}: Qbar_{m-1} += Psi' A1bar;  H = (I (x) Psi')^T Y_R: Ybar += (I (x) Psi') Hbar
    VJPCK(adj_gemm(false, false, Rprev, rp, ell, 1.0, ptab, Rprev, A1b, ell, 1.0, Qb[m - 1], Rprev, s));
    VJPCK(adj_gemm(false, false, Rprev, w, ell, 1.0, ptab, Rprev, Hb, ell, 1.0, Yb, Rprev, s));
  }
  VJPCK(adj_pbar(c->om_tab, c->L4, c->C, rm, ell, c->prec, Ab, Qb[m], s));
  for (int k = m - 1; k >= 2; --k) {
    const int64_t nr = c->n[k - 1] * r[k];
    VJPCK(adj_gemm(false, true, Rk[k - 1], r[k - 1], nr, 1.0, c->basis[k], Rk[k - 1], Gb[k - 1], r[k - 1], 1.0,
                   Qb[k - 1], Rk[k - 1], s));
    VJPCK(adj_gemm(false, false, Rk[k - 1], nr, r[k - 1], 1.0, c->basis[k - 1], Rk[k - 1], Gb[k - 1], r[k - 1], 1.0,
                   Qb[k], Rk[k - 1], s));
  }
  if (m >= 2) VJPCK(adj_axpy(c->n[0] * r[1], 1.0, Gb[0], Qb[1], s));
  for (int k = m + 1; k <= d - 1; ++k)
    VJPCK(adj_core_right(Gb[k - 1], c->basis[k - 1], c->basis[k], Ck(k), (int)c->n[k - 1], r[k - 1], r[k], Qb[k - 1],
                         Qb[k], s));
  {
    // G_d = P_{d-1}^T: Pbar_{d-1} += Gbar_d^T
    double* tmp = take((int64_t)r[d - 1] * c->n[d - 1], false);
    VJPCK(adj_transpose(Gb[d - 1], r[d - 1], c->n[d - 1], tmp, s));
    VJPCK(adj_axpy((int64_t)r[d - 1] * c->n[d - 1], 1.0, tmp, Qb[d - 1], s));
  }
  // sketch cotangents: Sbar_k (k < m), Ybar (= Sbar_m), Tbar_k (k >= m, transposed layout)
  std::vector<double*> Sb(d + 1, nullptr);
  for (int k = 1; k < m; ++k) Sb[k] = take(Rk[k] * ell, true);
  Sb[m] = Yb;
  std::vector<double*> Tb(d + 1, nullptr);
  for (int k = m; k <= d - 1; ++k) Tb[k] = take(Ck(k) * ell, true);
  for (int k = 1; k <= d - 1; ++k) {
    const bool left = k < m;
    const int64_t Mk = left ? Rk[k] : Ck(k);
    VJPCK(adj_qr(left ? c->S[k] : c->Tk[k], c->basis[k], Qb[k], Mk, ell, r[k], c->piv_dev + (int64_t)k * ell,
                 left ? Sb[k] : Tb[k], s));
  }
  const bool fused = gbar_dev == nullptr;
  if (!c->indep) {
    for (int k = 1; k <= m - 1; ++k)
      VJPCK(adj_derive_left(Sb[k], Sb[k + 1], Rk[k], (int)c->n[k], ell, c->fac + c->omega_off[k], s));
    for (int k = d - 1; k >= m + 1; --k)
      VJPCK(adj_derive_right(Tb[k], Tb[k - 1], Ck(k), (int)c->n[k - 1], ell, c->fac + c->psi_off[k - 1], s));
    // ---- B3: gx = Ybar Omega_m^T + Psi_m Tbar_m  (+ 2 (X - X~)) ----
    VJPCK(adj_out(c->dtype, geo, c->prec, Yb, Tb[m], fused ? Lm : nullptr, fused ? Rtm : nullptr, rm, x_dev, gx_dev,
                  false, s));
  } else {
    // independent scheme: split k's sketch was contracted from its own sketch
    // of X_m with its own factors, so its cotangent runs back up that chain
    // alone, to the cotangent of X_m Omega_m^(k) (k < m) or of
    // (Psi_m^(k)T X_m)^T (k > m)
    std::vector<double*> iYb(d + 1, nullptr), iTb(d + 1, nullptr);
    for (int k = 1; k < m; ++k) {
      const double* cur = Sb[k];
      for (int q = k + 1; q <= m; ++q) {   // undo the contraction of mode q: R_{q-1} -> R_q rows
        double* nxt = take(Rk[q] * ell, true);
        VJPCK(adj_derive_left(cur, nxt, Rk[q - 1], (int)c->n[q - 1], ell, c->fac + c->iom_off[k][q - 1], s));
        cur = nxt;
      }
      iYb[k] = (double*)cur;
    }
    for (int k = m + 1; k <= d - 1; ++k) {
      const double* cur = Tb[k];
      for (int q = k; q >= m + 1; --q) {   // undo the contraction of mode q: C_q -> C_{q-1} columns
        double* nxt = take(Ck(q - 1) * ell, true);
        VJPCK(adj_derive_right(cur, nxt, Ck(q), (int)c->n[q - 1], ell, c->fac + c->ipsi_off[k][q - 1], s));
        cur = nxt;
      }
      iTb[k] = (double*)cur;
    }
    // ---- B3, one launch per pass group (the factor sets the sketch pass
    //      paired): gx = sum_g Ybar_g Omega_m^(g)T + Psi_m^(g) Tbar_g (+ 2 (X - X~)) ----
    for (int g = 0; g < pass_groups(c); ++g) {
      double *yd = nullptr, *td = nullptr;
      const SketchArgs ga = group_args(c, g, &yd, &td);
      const int kr = g + 1, kl = m + g;
      const double* yg = kr < m ? iYb[kr] : (kr == m ? Yb : nullptr);
      const double* tg = kl == m ? Tb[m] : (kl <= d - 1 ? iTb[kl] : nullptr);
      const bool first = g == 0;
      VJPCK(adj_out(c->dtype, ga, c->prec, yg, tg, fused && first ? Lm : nullptr, fused && first ? Rtm : nullptr,
                    rm, x_dev, gx_dev, !first, s));
    }
  }
#undef VJPCK
  release();
  int hflag = 0;
  int* pin = (int*)pinned_scratch();
  if (e == hipSuccess) e = hipMemcpyAsync(pin ? pin : &hflag, c->flag, sizeof(int), hipMemcpyDeviceToHost, s);
  hipError_t e2 = hipStreamSynchronize(s);
  if (pin) hflag = *pin;
  if (e != hipSuccess) return hfail(c, e, "pstt2_vjp");
  if (e2 != hipSuccess) return hfail(c, e2, "pstt2_vjp");
  if (hflag & 1) return fail(c, PSTT2_ENUMERIC, "non-finite values in the cotangent");
  return PSTT2_OK;
}

pstt2_status pstt2_get_sketch(pstt2_ctx* c, int32_t which, int32_t k, double* host_out, int64_t* rows,
                              int64_t* cols) {
  if (!c || !rows || !cols) return fail(c, PSTT2_EINVAL, "null argument");
  if (!c->recovered) return fail(c, PSTT2_ESTATE, "sketches are available after pstt2_recover");
  const double* p = nullptr;
  if (which == 0 && k >= 1 && k <= c->m) {
    p = c->S[k];
    *rows = c->Rk[k];
  } else if (which == 1 && k >= c->m && k <= c->d - 1) {
    p = c->Tk[k];
    *rows = c->N / c->Rk[k];
  } else if (which == 2 && k >= 1 && k <= c->d - 1) {
    p = c->Bk + (int64_t)k * c->ell * c->ell;
    *rows = c->ell;
  } else if (which == 3 && c->H) {
    p = c->H;
    *rows = (int64_t)c->ell * c->n[c->m - 1];
  } else {
    return fail(c, PSTT2_EINVAL, "no such sketch");
  }
  *cols = c->ell;
  if (host_out) {
    HIPCK(c, hipMemcpyAsync(host_out, p, sizeof(double) * (*rows) * c->ell, hipMemcpyDeviceToHost, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
  }
  return PSTT2_OK;
}

pstt2_status pstt2_get_pivots(pstt2_ctx* c, int32_t k, int32_t* host_piv) {
  if (!c || !host_piv) return fail(c, PSTT2_EINVAL, "null argument");
  if (!c->recovered || k < 1 || k > c->d - 1) return fail(c, PSTT2_ESTATE, "no pivots for this split");
  HIPCK(c, hipMemcpyAsync(host_piv, c->piv_dev + (int64_t)k * c->ell, sizeof(int) * c->ell, hipMemcpyDeviceToHost,
                          c->stream));
  HIPCK(c, hipStreamSynchronize(c->stream));
  return PSTT2_OK;
}

pstt2_status tt_cores_copy(const tt_cores* src, tt_cores* dst, void* hip_stream) {
  if (!src || !dst || src->d != dst->d || src->d < 2 || src->d > PSTT2_MAX_D)
    return fail(nullptr, PSTT2_EINVAL, "bad cores");
  for (int k = 0; k < src->d; ++k)
    if (src->n[k] != dst->n[k] || src->r[k] != dst->r[k] || src->r[k + 1] != dst->r[k + 1] || !src->core[k] ||
        !dst->core[k])
      return fail(nullptr, PSTT2_EINVAL, "core shapes differ");
  hipStream_t s = (hipStream_t)hip_stream;
  for (int k = 0; k < src->d; ++k) {
    hipError_t e = hipMemcpyAsync(dst->core[k], src->core[k], sizeof(double) * src->r[k] * src->n[k] * src->r[k + 1],
                                  hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hfail(nullptr, e, "tt_cores_copy");
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hfail(nullptr, e, "tt_cores_copy");
  return PSTT2_OK;
}

pstt2_status pstt2_parallel_ttsvd(int32_t d, const int64_t* n, const double* x_dev, double eps, int32_t rmax,
                                  void* hip_stream, tt_cores* out) {
  if (!n || !x_dev || !out) return fail(nullptr, PSTT2_EINVAL, "null argument");
  if (d < 2 || d > PSTT2_MAX_D) return fail(nullptr, PSTT2_EINVAL, "d must be in [2, 32]");
  if (!(eps > 0.0 && eps < 1.0)) return fail(nullptr, PSTT2_EINVAL, "eps must be in (0, 1)");
  int64_t Rk[PSTT2_MAX_D + 1];
  Rk[0] = 1;
  for (int q = 0; q < d; ++q) {
    if (n[q] < 1 || n[q] > (1 << 30)) return fail(nullptr, PSTT2_EINVAL, "mode sizes must be in [1, 2^30]");
    Rk[q + 1] = Rk[q] * n[q];
    if (Rk[q + 1] > (int64_t(1) << 36)) return fail(nullptr, PSTT2_EINVAL, "tensor too large for the Jacobi SVDs");
  }
  const int64_t N = Rk[d];
  int64_t wmax = 0;
  int spmax = 2;
  for (int k = 1; k <= d - 1; ++k) {
    const int64_t R = Rk[k], C = N / R, sh = std::min(R, C);
    if (sh > PSTT2_TTSVD_MAX_SIDE)
      return fail(nullptr, PSTT2_EINVAL, "an unfolding's short side exceeds PSTT2_TTSVD_MAX_SIDE");
    const int sp = (int)(sh + (sh & 1));
    spmax = std::max(spmax, sp);
    wmax = std::max(wmax, std::max(R, C) * sp);
  }
  hipStream_t s = (hipStream_t)hip_stream;
  double *W = nullptr, *J = nullptr, *sig = nullptr;
  int *idx = nullptr, *cnt = nullptr;
  std::vector<double*> U(d + 1, nullptr);
  int r[PSTT2_MAX_D + 1];
  r[0] = r[d] = 1;
  tt_cores tc;
  std::memset(&tc, 0, sizeof(tc));
  double* base = nullptr;
  auto cleanup = [&]() {
    for (double* u : U) dev_free_async(u, s);
    dev_free_async(W, s);
    dev_free_async(J, s);
    dev_free_async(sig, s);
    dev_free_async(idx, s);
    dev_free_async(cnt, s);
  };
  auto bail = [&](pstt2_status st) {
    if (base) dev_free_async(base, s);
    cleanup();
    (void)hipStreamSynchronize(s);
    return st;
  };
#define SVDCK(call)                                                \
  do {                                                             \
    hipError_t e_ = (call);                                        \
    if (e_ != hipSuccess) return bail(hfail(nullptr, e_, #call)); \
  } while (0)
  SVDCK(dev_malloc_async((void**)&W, sizeof(double) * wmax, s));
  SVDCK(dev_malloc_async((void**)&J, sizeof(double) * spmax * spmax, s));
  SVDCK(dev_malloc_async((void**)&sig, sizeof(double) * spmax, s));
  SVDCK(dev_malloc_async((void**)&idx, sizeof(int) * spmax, s));
  SVDCK(dev_malloc_async((void**)&cnt, sizeof(int), s));
  // the last core is formed with its split's SVD; the others from U by equation "core"
  const int nd = (int)n[d - 1];
  std::vector<double> g_last;
  double* glast = nullptr;
  for (int k = 1; k <= d - 1; ++k) {
    const int64_t R = Rk[k], C = N / R, L = std::max(R, C);
    const int sh = (int)std::min(R, C), sp = sh + (sh & 1);
    const double tol = std::sqrt((double)L) * 2.220446049250313e-16;
    SVDCK(svd_load(x_dev, R, C, sp, W, s));
    SVDCK(svd_init(J, sp, cnt, s));
    bool converged = false;
    for (int sweep = 0; sweep < 40 && !converged; ++sweep) {
      int rot = 0;
      SVDCK(svd_sweep(W, L, J, sp, tol, cnt, s));
      SVDCK(hipMemcpyAsync(&rot, cnt, sizeof(int), hipMemcpyDeviceToHost, s));
      SVDCK(hipStreamSynchronize(s));
      converged = rot == 0;
    }
    if (!converged) return bail(fail(nullptr, PSTT2_ENUMERIC, "Jacobi SVD did not converge in 40 sweeps"));
    std::vector<double> sv(sh);
    SVDCK(svd_colnorms(W, L, sh, sig, s));
    SVDCK(hipMemcpyAsync(sv.data(), sig, sizeof(double) * sh, hipMemcpyDeviceToHost, s));
    SVDCK(hipStreamSynchronize(s));
    double tot = 0.0;
    for (double v : sv) {
      if (!std::isfinite(v)) return bail(fail(nullptr, PSTT2_ENUMERIC, "non-finite values in X"));
      tot += v * v;
    }
    // singular values in decreasing order (ties keep column order)
    std::vector<int> order(sh);
    for (int i = 0; i < sh; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sv[a] > sv[b]; });
    // Section 2.2's truncation with the per-unfolding share of Algorithm
    // Parallel-TTSVD: smallest r with sum_{i > r} sigma_i^2 <= eps^2 ||X||_F^2 / (d - 1)
    const double thr = eps * eps * tot / (d - 1);
    int rk = sh;
    double tail = 0.0;
    for (int i = sh - 1; i >= 1; --i) {
      if (tail + sv[order[i]] * sv[order[i]] <= thr) {
        tail += sv[order[i]] * sv[order[i]];
        rk = i;
      } else {
        break;
      }
    }
    if (rmax > 0) rk = std::min(rk, (int)rmax);
    rk = std::min(rk, PSTT2_MAX_ELL);
    r[k] = rk;
    SVDCK(hipMemcpyAsync(idx, order.data(), sizeof(int) * rk, hipMemcpyHostToDevice, s));
    SVDCK(dev_malloc_async((void**)&U[k], sizeof(double) * R * rk, s));
    if (R <= C) SVDCK(svd_gather(J, sp, R, idx, nullptr, rk, U[k], s));   // U = J
    else SVDCK(svd_gather(W, R, R, idx, sig, rk, U[k], s));              // U = W' / sigma
    if (k == d - 1) {
      SVDCK(dev_malloc_async((void**)&glast, sizeof(double) * rk * nd, s));
      U[0] = glast;   // released with the rest
      if (R > C) SVDCK(svd_last_core(J, sp, idx, sig, rk, nd, glast, s));   // Sigma V^T from J
      else SVDCK(svd_last_core(W, C, idx, nullptr, rk, nd, glast, s));      // U^T X = W'^T
    }
    // the sizes were read back above: idx may be refilled by the next split
    SVDCK(hipStreamSynchronize(s));
  }
  int64_t tot = 0;
  for (int k = 0; k < d; ++k) tot += (int64_t)r[k] * n[k] * r[k + 1];
  SVDCK(dev_malloc_async((void**)&base, sizeof(double) * tot, s));
  tc.d = d;
  tc.owned = 1;
  tc.stream = (void*)s;
  int64_t o = 0;
  for (int k = 0; k < d; ++k) {
    tc.n[k] = n[k];
    tc.core[k] = base + o;
    o += (int64_t)r[k] * n[k] * r[k + 1];
  }
  for (int k = 0; k <= d; ++k) tc.r[k] = r[k];
  // G_1 = U_1; G_k = U_{k-1}^T reshape(U_k, R_{k-1}, n_k r_k) (equation "core"); G_d = Sigma V^T
  SVDCK(hipMemcpyAsync(tc.core[0], U[1], sizeof(double) * n[0] * r[1], hipMemcpyDeviceToDevice, s));
  for (int k = 2; k <= d - 1; ++k)
    SVDCK(core_left(U[k - 1], Rk[k - 1], r[k - 1], U[k], (int)n[k - 1], r[k], tc.core[k - 1], s));
  SVDCK(hipMemcpyAsync(tc.core[d - 1], glast, sizeof(double) * r[d - 1] * nd, hipMemcpyDeviceToDevice, s));
#undef SVDCK
  cleanup();
  const hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    tt_cores_free(&tc);
    return hfail(nullptr, e, "pstt2_parallel_ttsvd");
  }
  *out = tc;
  return PSTT2_OK;
}

pstt2_status pstt2_drm_factors(const pstt2_desc* desc, double* host_out, int64_t* count) {
  if (!desc || !count) return fail(nullptr, PSTT2_EINVAL, "null argument");
  if (desc->d < 2 || desc->d > PSTT2_MAX_D) return fail(nullptr, PSTT2_EINVAL, "d must be in [2, 32]");
  if (desc->ell < 1 || desc->ell > PSTT2_MAX_ELL) return fail(nullptr, PSTT2_EINVAL, "ell must be in [1, 32]");
  if (desc->drm != PSTT2_DRM_NESTED && desc->drm != PSTT2_DRM_INDEPENDENT) return fail(nullptr, PSTT2_EINVAL, "bad drm");
  for (int q = 0; q < desc->d; ++q)
    if (desc->n[q] < 1 || desc->n[q] > (1 << 30)) return fail(nullptr, PSTT2_EINVAL, "bad mode size");
  const int64_t off = factor_layout(desc, nullptr);
  if (host_out) {
    if (*count < off) return fail(nullptr, PSTT2_EINVAL, "host_out holds fewer than the factor count");
    gaussian_fill(desc->seed, 0, off, host_out);
  }
  *count = off;
  return PSTT2_OK;
}

pstt2_status pstt2_set_memory_limit(int64_t bytes) {
  mem_limit_set(bytes);
  return PSTT2_OK;
}

pstt2_status pstt2_memory_stats(int64_t* live_bytes, int64_t* peak_bytes, int64_t* limit_bytes) {
  mem_stats(live_bytes, peak_bytes, limit_bytes);
  return PSTT2_OK;
}

pstt2_status pstt2_inject_launch_failure(int64_t count) {
  fault_arm(count);
  return PSTT2_OK;
}

void tt_cores_free(tt_cores* t) {
  if (!t) return;
  // one stream-ordered allocation, based at core[0]
  if (t->owned && t->d >= 1) dev_free_async(t->core[0], (hipStream_t)t->stream);
  std::memset(t, 0, sizeof(*t));
}

static pstt2_status check_cores(const tt_cores* t) {
  if (!t || t->d < 2 || t->d > PSTT2_MAX_D) return fail(nullptr, PSTT2_EINVAL, "bad cores");
  if (t->r[0] != 1 || t->r[t->d] != 1) return fail(nullptr, PSTT2_EINVAL, "boundary ranks must be 1");
  for (int k = 0; k < t->d; ++k) {
    if (!t->core[k] || t->n[k] < 1 || t->r[k + 1] < 1) return fail(nullptr, PSTT2_EINVAL, "bad core");
    if (t->r[k + 1] > PSTT2_MAX_ELL) return fail(nullptr, PSTT2_EINVAL, "rank above 32 not supported");
  }
  return PSTT2_OK;
}

static pstt2_status error_common(const tt_cores* cores, const void* x_dev, pstt2_dtype dtype, const pstt2_fn* fn,
                                 double* rel_err, void* hip_stream) {
  double e2x2[2] = {0, 0};
  double* pin = pinned_scratch();
  // tt_error returns only after its stream is idle, so its temporaries can come
  // from a per-thread, per-device arena that the next call rewinds
  Arena* ar = error_arena();
  hipError_t e = ar ? arena_begin(ar, (hipStream_t)hip_stream) : hipSuccess;
  if (e != hipSuccess) return hfail(nullptr, e, "tt_error");
  ArenaScope scope(ar);
  if (fn && fn->kind == PSTT2_FN_GAUSS)
    e = tt_error_run_gauss(cores, fn->centers, fn->n_terms, fn->gamma, pin ? pin : e2x2, (hipStream_t)hip_stream);
  else e = tt_error_run(cores, x_dev, dtype, pin ? pin : e2x2, (hipStream_t)hip_stream, fn ? 1 : 0);
  if (pin) {
    e2x2[0] = pin[0];
    e2x2[1] = pin[1];
  }
  if (e != hipSuccess) return hfail(nullptr, e, "tt_error");
  *rel_err = e2x2[1] > 0 ? std::sqrt(e2x2[0] / e2x2[1]) : (e2x2[0] > 0 ? INFINITY : 0.0);
  if (!std::isfinite(*rel_err)) return fail(nullptr, PSTT2_ENUMERIC, "non-finite error");
  return PSTT2_OK;
}

pstt2_status tt_error(const tt_cores* cores, const void* x_dev, pstt2_dtype dtype, double* rel_err, void* hip_stream) {
  pstt2_status st = check_cores(cores);
  if (st != PSTT2_OK) return st;
  if (!x_dev || !rel_err) return fail(nullptr, PSTT2_EINVAL, "null argument");
  return error_common(cores, x_dev, dtype, nullptr, rel_err, hip_stream);
}

pstt2_status tt_error_noalloc(const tt_cores* cores, const void* x_dev, pstt2_dtype dtype, double* err_dev,
                              void* hip_stream) {
  pstt2_status st = check_cores(cores);
  if (st != PSTT2_OK) return st;
  if (!x_dev || !err_dev) return fail(nullptr, PSTT2_EINVAL, "null argument");
  if (dtype != PSTT2_F64 && dtype != PSTT2_F32) return fail(nullptr, PSTT2_EINVAL, "bad dtype");
  const int64_t need = tt_error_scratch_bytes(cores);
  if (need > PSTT2_NOALLOC_SCRATCH_BYTES) {
    char msg[160];
    std::snprintf(msg, sizeof(msg), "tt_error_noalloc needs %lld bytes of scratch; the static buffer holds %lld",
                  (long long)need, (long long)PSTT2_NOALLOC_SCRATCH_BYTES);
    return fail(nullptr, PSTT2_ENOMEM, msg);
  }
  const hipError_t e = tt_error_noalloc_run(cores, x_dev, dtype, err_dev, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hfail(nullptr, e, "tt_error_noalloc");
  return PSTT2_OK;
}

pstt2_status tt_error_fn(const tt_cores* cores, const pstt2_fn* fn, double* rel_err, void* hip_stream) {
  pstt2_status st = check_cores(cores);
  if (st != PSTT2_OK) return st;
  if (!fn || !rel_err) return fail(nullptr, PSTT2_EINVAL, "null argument");
  if (const char* why = fn_invalid(fn)) return fail(nullptr, PSTT2_EINVAL, why);
  return error_common(cores, nullptr, PSTT2_F64, fn, rel_err, hip_stream);
}

pstt2_status tt_reconstruct(const tt_cores* cores, void* x_out_dev, pstt2_dtype dtype, int64_t first, int64_t count,
                            void* hip_stream) {
  pstt2_status st = check_cores(cores);
  if (st != PSTT2_OK) return st;
  int64_t N = 1;
  for (int k = 0; k < cores->d; ++k) N *= cores->n[k];
  if (first < 0 || count < 0 || first + count > N) return fail(nullptr, PSTT2_EINVAL, "range outside the tensor");
  if (!x_out_dev && count > 0) return fail(nullptr, PSTT2_EINVAL, "null output");
  hipError_t e = tt_reconstruct_run(cores, x_out_dev, dtype, first, count, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hfail(nullptr, e, "tt_reconstruct");
  return PSTT2_OK;
}

}  // extern "C"
