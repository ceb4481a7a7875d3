// Internal declarations shared by the translation units of libpstt2.
// Not part of the public ABI (include/pstt2.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/pstt2.h"

namespace pstt2 {

// ---- device memory (workspace.hip) ----
// Every device allocation of the library: counted against the memory budget
// (pstt2_set_memory_limit / PSTT2_MAX_BYTES) and in the live / peak totals.
hipError_t dev_malloc_raw(void** p, size_t bytes);
template <typename T>
inline hipError_t dev_malloc(T** p, size_t bytes) {
  return dev_malloc_raw((void**)p, bytes);
}
hipError_t dev_malloc_async(void** p, size_t bytes, hipStream_t s);
void dev_free(void* p);
void dev_free_async(void* p, hipStream_t s);
void mem_limit_set(int64_t bytes);
void mem_stats(int64_t* live, int64_t* peak, int64_t* limit);
// Launch-failure injection (pstt2_inject_launch_failure): after fault_arm(k)
// the next k launch sites proceed and the one after reports a failure without
// launching; fault_take() is called at each such site.
void fault_arm(int64_t count);
bool fault_take();

// ---- seeded Gaussian factors (rng.hip, host code) ----
// Philox4x32-10 block for (seed, counter); and the standard normals
// first .. first + count - 1 of the stream defined in rng.hip.
void philox_block(uint64_t seed, uint64_t counter, uint32_t out[4]);
void gaussian_fill(uint64_t seed, int64_t first, int64_t count, double* out);

// ---- device workspace (workspace.hip) ----
struct Arena {
  char* base = nullptr;
  size_t cap = 0, off = 0, need = 0;
  std::vector<void*> spill;
};
// the arena ws_alloc / ws_free use on this host thread (nullptr: none)
Arena*& current_arena();
struct ArenaScope {
  Arena* prev;
  explicit ArenaScope(Arena* a);
  ~ArenaScope();
};
// start a pass: release the last pass's overflow, regrow to what it needed, rewind
hipError_t arena_begin(Arena* a, hipStream_t s);
void arena_release(Arena* a, hipStream_t s);
hipError_t ws_alloc(void** p, size_t bytes, hipStream_t s);
void ws_free(void* p, hipStream_t s);

constexpr int kMaxSeg = 48;   // slabs per sketch launch

// One run of whole columns of the middle unfolding X_m held in one buffer.
struct Seg {
  const void* ptr;   // first entry of the run (column gcol0, row 0)
  int64_t gcol0;     // global column index of its first column
  int64_t ncols;     // number of columns
  int64_t chunk0;    // index of its first chunk in the launch's chunk list (sketch_chunk_cols wide)
};

// Everything a sketch launch needs; passed by value as the kernel argument.
struct SketchArgs {
  int64_t R;         // rows of X_m: n_1 ... n_m
  int64_t nchunks;   // chunks in this launch
  int32_t ell;       // sketch size
  int32_t gi_count;  // row blocks
  int32_t gj_count;  // column groups
  int32_t d, m;
  int32_t nseg;
  int32_t n[PSTT2_MAX_D];
  const double* fac;           // FP64 factors, device
  int64_t psi_off[PSTT2_MAX_D];    // offset of psi_q (q = 1..d-1) at index q-1
  int64_t omega_off[PSTT2_MAX_D];  // offset of omega_q (q = 2..d) at index q-1
  void* ypart;       // [gj][c][row], ell columns
  // FP64 kernel with one column group only: when set, the kernel adds its Y
  // tile straight into this R x ell column-major sketch (and raises *yflag on
  // a non-finite sum) instead of writing ypart; the reduction then skips Y.
  double* ydirect;
  int* yflag;
  int32_t ystore;    // with ydirect: Y holds no data yet and stands for zero, so
                     // the tile is stored (0 + y) instead of added
  void* tpart;       // tlp == 0: [gi][a][gcol], ell rows; tlp > 0: [gi][gcol][tlp] (sketch index
                     // contiguous); indexed by global column; then kTPartPad spare entries
  int32_t tlp;       // layout of tpart (see above)
  int32_t x32;       // FP64 kernel: the segments hold FP32 entries (widened as loaded)
  int64_t C;         // columns of X_m (for the tpart stride)
  const double* om_tab;  // Omega_m(col, c) table, C x L4, FP64
  int32_t L4;            // its row stride: ell rounded up to a multiple of 4
  const double* psi_tab; // optional Psi(row, a) table, R x L4 (else products of the factors)
  const uint16_t* om16;  // 16-bit precisions: Omega_m rounded per plane, [plane][c < LP][col]
  Seg seg[kMaxSeg];
  // Tensor given by a formula (FP64 kernel only): 0 = X read from the
  // segments; 1 = Hilbert tensor, X(row, col) = fn_rec[fn_row[row] + fn_col[col]]
  int32_t fn;
  const double* fn_rec;   // 1/k, k = 0 .. 1 + sum_q (n_q - 1) (entry 0 unused)
  const int32_t* fn_row;  // 1 + digit sum of each row of X_m (0-based mode indices)
  const int32_t* fn_col;  // digit sum of each column of X_m
};

// Index tables of the Hilbert tensor X(i) = 1 / (1 - d + i_1 + ... + i_d)
// (1-based i) on the split X_m = rows (modes 1..m) x columns (modes m+1..d):
// X(row, col) = rec[row_t[row] + col_t[col]].  rec holds 2 + sum (n_q - 1)
// entries, row_t R and col_t C.
hipError_t hilbert_tables(const int64_t* n, int d, int m, int64_t R, int64_t C, double* rec, int32_t* row_t,
                          int32_t* col_t, hipStream_t s);
// Columns [c0, c0 + nc) of X_m of the Hilbert tensor from its tables into W
// (R x nc column-major, dtype F64 or F32).
hipError_t hilbert_columns(const double* rec, const int32_t* row_t, const int32_t* col_t, int64_t R, int64_t c0,
                           int64_t nc, int dtype, void* W, hipStream_t s);
inline int64_t hilbert_rec_len(const int64_t* n, int d) {
  int64_t k = 2;
  for (int q = 0; q < d; ++q) k += n[q] - 1;
  return k;
}

// Gaussian-bump tensor X(i) = sum_j exp(-gamma sum_q (x_q - c_{j,q})^2) on the
// split X_m: X(row, col) = sum_j e1(i_1, j) ahi(row / n_1, j) bc(col, j), the
// per-mode factors multiplied out over modes 1, 2..m and m+1..d.  Tables are
// j-major: e1[j * n1 + i_1], ahi[j * rhi + row / n_1], bc[j * bstride + col]
// with bstride = C + kGaussCols and zero padding after column C - 1.
constexpr int kGaussCols = 32;   // columns of X_m per thread in gauss_columns
struct GaussTabs {
  const double* e1;
  const double* ahi;
  const double* bc;
  int32_t nterms;
  int64_t n1, rhi, R, C, bstride;
};
// doubles of the buffer gauss_tables fills (centers, then the three tables)
int64_t gauss_table_doubles(const int64_t* n, int d, int m, int nterms);
// Copy the centers (host, nterms x d row-major) into buf and build the tables;
// returns after stream s is idle.
hipError_t gauss_tables(const int64_t* n, int d, int m, const double* centers_host, int nterms, double gamma,
                        double* buf, GaussTabs* out, hipStream_t s);
// Columns of X_m per workspace chunk: at most PSTT2_GAUSS_CHUNK_BYTES (one column
// if larger; a multiple of kGaussCols when above it), at most 65535 column blocks, at most C.
int64_t gauss_chunk_cols(const GaussTabs& g, int elem_bytes);
// Evaluate columns [c0, c0 + nc) of X_m into W (R x nc column-major, dtype F64 or F32).
hipError_t gauss_columns(const GaussTabs& g, int64_t c0, int64_t nc, int dtype, void* W, hipStream_t s);

// Launch the streaming dual-sketch kernel for the configured precision.
hipError_t launch_sketch(int prec, int lp, const SketchArgs& a, hipStream_t s);
// Entries after the T partials that the sketch kernels' idle lanes store to (never
// read): every memory operation in the chunk loop is then unconditional, which
// lets the compiler wait only for the loads it needs.
constexpr int64_t kTPartPad = 2048;
// 16-bit sketch precisions (plain BF16, FP16: 1 plane; split BF16: 3 planes; else 0)
int omega16_planes(int prec);
// Layout of the 16-bit Omega table: row stride (C rounded up to a multiple of
// four) and entries to allocate (LP rows plus kOmega16Slack zeroed entries
// that the 8-byte operand loads of the last columns may reach).
constexpr int64_t kOmega16Slack = 64;
__host__ __device__ inline int64_t omega16_stride(int64_t C) { return (C + 3) / 4 * 4; }
__host__ __device__ inline int64_t omega16_entries(int64_t C, int LP) {
  return (int64_t)LP * omega16_stride(C) + kOmega16Slack;
}
// Columns per chunk of the precision's sketch kernel (Seg::chunk0 counts these).
int sketch_chunk_cols(int prec);
// om16[(q LP + c) C + col] = plane q of Omega_m(col, c) rounded as the kernel uses it.
hipError_t build_omega16_table(const double* om_tab, int64_t C, int L4, int ell, int LP, int prec, uint16_t* om16,
                               hipStream_t s);
// Build the Omega_m table (C x L4, FP64) from the factors.
hipError_t build_omega_table(const SketchArgs& a, int L4, double* tab, hipStream_t s);
// Per-precision launch geometry: rows of X_m per workgroup, threads per
// workgroup, workgroups resident per CU.
void sketch_geometry(int prec, int ell, int* rows_per_block, int* threads, int* wg_per_cu);
// Sum the tile partials of one launch into the FP64 accumulators (fixed order).
hipError_t launch_reduce(int prec, const SketchArgs& a, double* Y, double* Tt, int* flag, hipStream_t s);
// FP64 contribution of one partial column (rows [r0, r1) of global column gcol).
hipError_t launch_partial_col(int dtype, const void* x, int64_t r0, int64_t r1, int64_t gcol,
                              const SketchArgs& a, double* Y, double* Tt, hipStream_t s);

// Recovery building blocks (recover.hip); all FP64, column-major.
hipError_t derive_left(const double* Sin, double* Sout, int64_t Rk, int nk1, int ell, const double* omega,
                       hipStream_t s);
hipError_t derive_right(const double* Tin, double* Tout, int64_t Ck, int nk, int ell, const double* psi,
                        hipStream_t s);

// Orthonormal bases of range(A_p) for n independent M_p x ell matrices by
// TSQR + pivoted QR of the final R; every tree level, the pivoted QRs and the
// singular values run as one launch over all problems.
struct BasisBatch;
// Phase 1 (async): factor every A_p; pivots into piv[p] (ell ints); singular
// values of R when want_sv.
hipError_t basis_factor_batch(int n, const double* const* A, const int64_t* M, int ell, int* const* piv,
                              bool want_sv, BasisBatch** w, hipStream_t s);
// Device pointer to problem p's ell singular values (descending), or null.
const double* basis_batch_sv(BasisBatch* w, int p);
// Phase 2 (async): Q_p (M_p x r_p) = first r_p columns of the sign-fixed pivoted factor.
hipError_t basis_form_q_batch(BasisBatch* w, const int* r, double* const* Q, hipStream_t s);
// Release (stream-ordered).
void basis_batch_free(BasisBatch* w);

hipError_t core_left(const double* Qprev, int64_t Rprev, int rprev, const double* Qk, int nk, int rk, double* G,
                     hipStream_t s);
hipError_t core_right(const double* Pprev, int64_t Cprev, int rprev, const double* Pk, int64_t Ck, int nk, int rk,
                      double* G, hipStream_t s);
hipError_t middle_z(const double* Qprev, int64_t Rprev, int rprev, const double* Y, int64_t Rm, int nm, int ell,
                    double* Z, hipStream_t s);
hipError_t middle_a(const double* Pm, int64_t Cm, int rm, const SketchArgs& geo, int prec, double* A,
                    hipStream_t s);
hipError_t middle_ls(const double* Z, int64_t nz, const double* A, int rm, int ell, double* G, int* flag,
                     hipStream_t s);
// Khatri-Rao DRM over a run of consecutive modes: entry (row, u) is the product
// of f_q(i_q, u) over the chain's modes, with row = i_1 + n_1 (i_2 + n_2 (...))
// (first listed mode fastest); factor f_q sits at fac + off[q], n[q] x ell,
// ell fastest.
struct KRChain {
  int32_t cnt;
  int32_t n[PSTT2_MAX_D];
  int64_t off[PSTT2_MAX_D];
};
// out (rows x ell, column-major) = the chain's DRM; rows = prod n[q]
hipError_t kr_table(const double* fac, const KRChain& ch, int64_t rows, int ell, double* out, hipStream_t s);
// Two-sided sketches of several splits (recover.hip): entry p is split
// split[p], operand S[p] (K[p] x ell, column-major) = S_k (right = 0, DRM
// Psi_k over modes 1..k) or T_k^T (right = 1, DRM Omega_k over modes k+1..d);
// out[p] receives B_k (ell x ell, column-major).  chain holds the factor
// offsets of split k's left (slot 0) and right (slot 1) chains at
// chain[(2 k + slot) d + j], then the d mode sizes.
struct TwoSidedBatch {
  int n, d, ell;
  const double* fac;
  const int64_t* chain;
  const double* S[PSTT2_MAX_D];
  int64_t K[PSTT2_MAX_D];
  int split[PSTT2_MAX_D], right[PSTT2_MAX_D];
  int scols[PSTT2_MAX_D];   // columns of S (0: ell; fewer: the rest of the product is zero)
  int steps[PSTT2_MAX_D];   // TS_ROWS-row slices per workgroup (set by two_sided_batch)
  int64_t nmode[PSTT2_MAX_D];   // mode sizes n_1 .. n_d (host copy; zero: the per-slice path)
  const double* H[PSTT2_MAX_D];  // whole H tables (set by two_sided_batch)
  double* out[PSTT2_MAX_D];
  int64_t blk0[PSTT2_MAX_D + 1];
};
hipError_t two_sided_batch(TwoSidedBatch& B, hipStream_t s);
// out (k x k) = identity
hipError_t eye(int k, double* out, hipStream_t s);
hipError_t middle_twopass(int dtype, const void* x, int64_t first, int64_t count, int64_t Rprev, int nm,
                          int64_t Cm, const double* Qprev, int rprev, const double* Pm, int rm, double* G,
                          hipStream_t s);

// Adjoint building blocks (adjoint.hip); FP64, column-major.
hipError_t adj_gemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                    const double* B, int64_t ldb, double beta, double* C, int64_t ldc, hipStream_t s);
// C_i = A^T B_i for i < nbatch (B_i = B + i sb, C_i = C + i sc, each M x N with
// leading dimension ldc): the same products as nbatch calls of adj_gemm with
// ta, alpha = 1, beta = 0, bitwise, in one pair of launches where the tall-skinny
// path applies.
hipError_t adj_gemm_tn_batch(int64_t M, int64_t N, int64_t K, int nbatch, const double* A, int64_t lda,
                             const double* B, int64_t ldb, int64_t sb, double* C, int64_t ldc, int64_t sc,
                             hipStream_t s);
hipError_t adj_table(const double* in, int64_t rows, int cnt, int64_t si, int64_t sc, int L4, double* out,
                     hipStream_t s);
hipError_t adj_transpose(const double* A, int64_t arows, int64_t acols, double* B, hipStream_t s);
hipError_t adj_axpy(int64_t n, double alpha, const double* X, double* Y, hipStream_t s);
hipError_t adj_ls(const double* G, const double* Gb, const double* Z, const double* A, int64_t p, int r, int ell,
                  double* Zb, double* Ab, hipStream_t s);
hipError_t adj_core_right(const double* Gb, const double* Pp, const double* Pk, int64_t Ck, int nk, int rp, int rk,
                          double* Ppb, double* Pkb, hipStream_t s);
hipError_t adj_pbar(const double* om_tab, int L4, int64_t Cm, int rm, int ell, int prec, const double* Ab, double* Pb,
                    hipStream_t s);
hipError_t adj_qr(const double* S, const double* Q, const double* Qb, int64_t M, int ell, int r, const int* piv,
                  double* Sb, hipStream_t s);
hipError_t adj_derive_left(const double* Sbk, double* Sbk1, int64_t Rk, int nk1, int ell, const double* om,
                           hipStream_t s);
hipError_t adj_derive_right(const double* Tbk, double* Tbp, int64_t Ck, int nk, int ell, const double* ps,
                            hipStream_t s);
hipError_t adj_out(int dtype, const SketchArgs& g, int prec, const double* Yb, const double* Tbt, const double* L,
                   const double* Rt, int r, const void* x, void* gx, bool acc, hipStream_t s);

// Parallel-TTSVD building blocks (ttsvd.hip).  W is the L x sp work matrix of
// an unfolding (X_k^T when R_k <= C_k, else X_k; sp = the short side rounded up
// to even, zero columns past it), J its sp x sp rotation accumulator.
hipError_t svd_load(const double* x, int64_t R, int64_t C, int sp, double* W, hipStream_t s);
hipError_t svd_init(double* J, int sp, int* counter, hipStream_t s);
// one sweep of the round-robin schedule; *counter receives the rotations made
hipError_t svd_sweep(double* W, int64_t L, double* J, int sp, double tol, int* counter, hipStream_t s);
hipError_t svd_colnorms(const double* W, int64_t L, int scols, double* sig, hipStream_t s);
hipError_t svd_gather(const double* src, int64_t ld, int64_t rows, const int* idx, const double* sig, int r,
                      double* dst, hipStream_t s);
hipError_t svd_last_core(const double* src, int64_t ld, const int* idx, const double* sig, int r, int nd, double* G,
                         hipStream_t s);

// TT evaluation (tt_eval.hip).
hipError_t tt_interfaces(const tt_cores* c, int split, double** L, double** Rt, double** base, hipStream_t s);
// Bytes of the static scratch the allocation-free error pass of these cores needs.
int64_t tt_error_scratch_bytes(const tt_cores* c);
// The error pass in the static scratch; err_dev receives (relative error,
// sum (x - x~)^2, sum x^2).  async.
hipError_t tt_error_noalloc_run(const tt_cores* c, const void* x, int dtype, double* err_dev, hipStream_t s);
}  // namespace pstt2

// Thread-local error text for calls without a context.
void pstt2_set_tls_error(const std::string& msg);
