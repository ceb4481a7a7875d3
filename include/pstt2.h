/*
 * pstt2.h -- C ABI of the MI355X PSTT2 library (libpstt2.so).
 *
 * What it computes (Shi, Ruth, Townsend, "Parallel Algorithms for computing the
 * Tensor-train decomposition"):
 *   input  a dense d-way tensor X (n_1 x ... x n_d, column-major, i_1 fastest;
 *          Section 2.1) and either target TT ranks r_1..r_{d-1} or a tolerance eps;
 *   output TT cores G_k (r_{k-1} x n_k x r_k, r_0 = r_d = 1) with
 *          ||X - X~||_F <= eps ||X||_F in the tolerance form of the problem
 *          statement (Section 1, equation "FrobeniusNorm").
 * The method is PSTT2-onepass (Section 3.2, final paragraphs; Section 4.2):
 * a single streaming pass over X forms, with Khatri-Rao Gaussian DRMs
 * (Section 3.2, equation "sketch_orig"), the right sketch Y_R = X_m Omega_m and
 * the left sketch T_m = Psi_m^T X_m of the middle unfolding (m = ceil(d/2)),
 * from which every other split's sketch S_k = X_k Omega_k (k < m) and
 * T_k = Psi_k^T X_k (k > m) follows by contracting one mode at a time (the
 * nested DRM scheme: one Gaussian factor per mode, shared by every split).
 * Column bases Q_k (k < m) and row bases P_k (k >= m) come from column-pivoted
 * QR of those sketches (Algorithm PSTT, CPQR step), outer cores from
 * neighbouring bases (Theorem 2, equation "core", and its row-space mirror),
 * and the middle core from two small products and a least-squares solve
 * (equation "onepass_final_core" applied to the middle unfolding).
 *
 * Conventions
 *   - Every pointer named *_dev is device memory on the current HIP device;
 *     every other pointer is host memory.
 *   - Every call returns a pstt2_status; nothing throws across the ABI.  On an
 *     error the outputs are left untouched and pstt2_last_error() describes it.
 *     The exception: a call that adds data into a context's sketches (or into
 *     a two-pass middle core) in several launches and fails after the first of
 *     them has run leaves those sums partial.  The context is then poisoned:
 *     every later sketch, recover, middle-pass and vjp call on it returns
 *     PSTT2_ESTATE until pstt2_reset (and a middle core being accumulated by
 *     pstt2_middle_pass_fn must be recomputed).  Nothing is double-counted by
 *     retrying after the reset.
 *   - Every device allocation of the library counts against an optional
 *     memory budget (pstt2_set_memory_limit; initial value from the
 *     environment variable PSTT2_MAX_BYTES, in bytes).  A request past it
 *     fails with PSTT2_ENOMEM, like a failed hipMalloc.
 *   - Calls marked "async" enqueue work on the context's (or the given) HIP
 *     stream and return before it runs; device-side failures of async work are
 *     reported by the next synchronising call.  Calls marked "sync" block the
 *     host until their stream is idle.
 *   - A context is bound to one stream and is not thread-safe.
 *   - Sizes are int64; flat indices and byte offsets exceed 2^31.
 */
#ifndef PSTT2_H
#define PSTT2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PSTT2_MAX_D 32   /* largest supported order d */
#define PSTT2_MAX_ELL 32 /* largest supported sketch size ell */

typedef enum {
  PSTT2_OK = 0,
  PSTT2_EINVAL = -1,   /* bad argument or descriptor field */
  PSTT2_ESHAPE = -2,   /* sizes inconsistent with the context */
  PSTT2_ENOMEM = -3,   /* device or host allocation failed */
  PSTT2_EDEVICE = -4,  /* a HIP runtime call failed */
  PSTT2_ENUMERIC = -5, /* non-finite values in X or a singular sketch */
  PSTT2_ESTATE = -6    /* call out of order (e.g. overlapping or missing slabs) */
} pstt2_status;

/* Element type of X in device memory. */
typedef enum { PSTT2_F64 = 0, PSTT2_F32 = 1 } pstt2_dtype;

/* Arithmetic of the sketch contractions.  Recovery is always FP64.
 *   F64     FP64 products and sums (FP64 matrix cores); with dtype F32 the
 *           FP32 entries are widened to FP64 as they are loaded (products
 *           of the stored values, exact up to FP64 summation)
 *   F32     FP32 products, FP32 accumulation within a tile, FP64 across tiles
 *   BF16    X and the DRM rounded to bfloat16, FP32 accumulation
 *   BF16X3  split precision: X and the DRM each split into three bfloat16
 *           terms t0 + t1 + t2 (exact for FP32 values), the six products
 *           t_i * t_j with i + j <= 2 on bfloat16 matrix cores, FP32
 *           accumulation; about FP32 accuracy
 *   F16     X and the DRM rounded to IEEE half precision (round to nearest
 *           even), FP32 accumulation on the f16 matrix cores: eight times
 *           finer rounding than BF16 at the same rate.  Half precision spans
 *           6.1e-5 .. 65504 (with gradual underflow below): entries of X or of
 *           the DRM past 65504 in magnitude become infinite and recover
 *           reports ENUMERIC; tensors whose entries sit far below 6e-5 lose
 *           relative precision and should be scaled by the caller.
 * F32 / BF16 / BF16X3 / F16 need dtype F32; F64 takes either dtype. */
typedef enum {
  PSTT2_P_F64 = 0,
  PSTT2_P_F32 = 1,
  PSTT2_P_BF16 = 2,
  PSTT2_P_BF16X3 = 3,
  PSTT2_P_F16 = 4
} pstt2_prec;

/* Middle-core rule.  ONEPASS: least squares from the extra right sketch of the
 * middle unfolding (PSTT2-onepass).  TWOPASS: second stream over X,
 * G_m = reshape(X, R_{m-1}, n_m, C_m) x_1 Q_{m-1}^T x_3 P_m^T
 * (equation "PSTT2_final_core"); see pstt2_middle_pass.  TWOSIDED: still one
 * pass; Y_R is sketched once more on its leading m-1 modes with split (m-1)'s
 * left DRM Psi' (R_{m-1} x ell), H = reshape(Y_R) x_1 Psi'^T (ell x n_m x ell),
 * and G_m = H x_1 (Psi'^T Q_{m-1})^+ x_3 (Omega_m^T P_m)^+: the pseudo-inverse
 * step of equation "onepass_final_core" taken on both outer modes.  For d = 2
 * (m = 1) TWOSIDED is ONEPASS. */
typedef enum { PSTT2_MID_ONEPASS = 0, PSTT2_MID_TWOPASS = 1, PSTT2_MID_TWOSIDED = 2 } pstt2_mid;

/* Khatri-Rao DRM scheme (Section 3.2, equation "sketch_orig").
 *   NESTED       one Gaussian factor per mode, shared by every split: the
 *                pass forms the two sketches of the middle unfolding and every
 *                other split's sketch follows by contracting modes (2 products
 *                per tile of X).
 *   INDEPENDENT  every split draws its own factors (the paper's Psi^(j)): the
 *                pass forms one right sketch per split k <= m and one left
 *                sketch per split k >= m (d products per tile), each slab read
 *                once per pair of them.
 * The adjoint (pstt2_vjp) covers both. */
typedef enum { PSTT2_DRM_NESTED = 0, PSTT2_DRM_INDEPENDENT = 1 } pstt2_drm;

/* Algorithm.
 *   PSTT2  two-sided (default): column bases Q_k for k < m = ceil(d/2), row
 *          bases P_k for k >= m, and a middle core (see pstt2_mid).
 *   PSTT   one-sided (Algorithm PSTT): column bases Q_1..Q_{d-1} of every
 *          unfolding, cores by equation "core", and the last core either from
 *          the extra left sketch T_{d-1} = Psi_{d-1}^T X_{d-1} by the one-pass
 *          rule G_d = (Psi_{d-1}^T Q_{d-1})^+ T_{d-1} (mid ONEPASS, PSTT-onepass,
 *          equation "onepass_final_core") or by a second pass
 *          G_d = Q_{d-1}^T X_{d-1} (mid TWOPASS, pstt2_middle_pass).  The pass
 *          sketches the split d-1, so the right sketch is R_{d-1} x ell
 *          (N / n_d rows: the one-sided method's storage cost, Section 4.3).
 *          TWOSIDED is refused; pstt2_vjp reports ESTATE. */
typedef enum { PSTT2_ALGO_PSTT2 = 0, PSTT2_ALGO_PSTT = 1 } pstt2_algo;

typedef struct {
  int32_t d;                  /* order, 2 <= d <= PSTT2_MAX_D */
  int64_t n[PSTT2_MAX_D];     /* mode sizes n_1..n_d in n[0..d-1], each >= 1 */
  pstt2_dtype dtype;          /* element type of X */
  pstt2_prec prec;            /* sketch arithmetic */
  pstt2_mid mid;              /* middle-core rule */
  int32_t ranks[PSTT2_MAX_D]; /* r_1..r_{d-1} in ranks[0..d-2]; ranks[0] <= 0 selects tolerance mode */
  double eps;                 /* tolerance mode: target relative Frobenius error, 0 < eps < 1 */
  int32_t rmax;               /* tolerance mode: rank cap (<= 0: ell - 2) */
  int32_t ell;                /* sketch size r + p, 1 <= ell <= PSTT2_MAX_ELL */
  const double* drm_factors;  /* host, copied at create, or NULL (drawn from seed); factor q is n_q x ell with ell fastest
                                 (element (i, c) at i*ell + c), iid standard Gaussian in the
                                 paper's DRMs (Section 3.2).  NESTED: psi_1..psi_{d-1} then
                                 omega_2..omega_d.  INDEPENDENT: for split k = 1..d-1 in turn,
                                 psi^(k)_1..psi^(k)_k then omega^(k)_{k+1}..omega^(k)_d */
  pstt2_drm drm;              /* factor scheme */
  pstt2_algo algo;            /* two-sided PSTT2 (0) or one-sided PSTT */
  uint64_t seed;              /* drm_factors == NULL: the library draws the factors from this
                                 seed (see pstt2_drm_factors) */
} pstt2_desc;

/* A tensor train.  Core k (0-based) is r[k] x n[k] x r[k+1], column-major
 * (element (a, i, b) at a + r[k]*(i + n[k]*b)), FP64, device memory. */
typedef struct {
  int32_t d;
  int64_t n[PSTT2_MAX_D];
  int32_t r[PSTT2_MAX_D + 1];  /* r[0] = r[d] = 1 */
  double* core[PSTT2_MAX_D];   /* device pointers */
  int32_t owned;               /* 1: allocated by the library, release with tt_cores_free */
  void* stream;                /* owned cores: the HIP stream that orders their release */
} tt_cores;

typedef struct pstt2_ctx pstt2_ctx;

/* Create a context: validate the descriptor, upload the DRM factors, allocate
 * the sketch accumulators (R_m x ell and ell x C_m, FP64) and the tile
 * partials.  hip_stream may be NULL (the null stream).  sync.
 * Errors: EINVAL (descriptor), ENOMEM, EDEVICE. */
pstt2_status pstt2_create(const pstt2_desc* desc, void* hip_stream, pstt2_ctx** out);

/* Stream one slab of X into the sketches (Algorithm "parsketch": every sketch
 * from one read of each sub-tensor).  x_dev points at the slab's first entry,
 * which is flat column-major index `first` of X; the slab holds `count`
 * entries of the context's dtype.  first and count must be multiples of n_1
 * (whole mode-1 fibres); slabs may arrive in any order, each entry exactly
 * once.  x_dev must stay valid until the context's stream passes the work.
 * async.  Errors: EINVAL (alignment, range), ESTATE (overlaps an earlier slab). */
pstt2_status pstt2_sketch(pstt2_ctx* ctx, const void* x_dev, int64_t first, int64_t count);

/* The same for nslabs slabs in one launch (slab s at xs_dev[s], flat range
 * [firsts[s], firsts[s] + counts[s])).  Host arrays; async. */
pstt2_status pstt2_sketch_slabs(pstt2_ctx* ctx, int32_t nslabs, const void* const* xs_dev,
                                const int64_t* firsts, const int64_t* counts);

/* Tensors given by a formula of their indices: the streaming setting of
 * Section 4.2, where each sub-tensor comes from a function of its indices and
 * the whole tensor is never stored.
 *   HILBERT  X(i_1, ..., i_d) = 1 / (1 - d + i_1 + ... + i_d), 1 <= i_q <= n_q
 *            (the Hilbert tensor of Section 4.3 and Table 1), evaluated in
 *            FP64 inside the sketch and error kernels: the reciprocal of the
 *            integer index sum, correctly rounded.  Other fields unused.
 *   GAUSS    X(i_1, ..., i_d) = sum_{j < n_terms} exp(-gamma sum_q (x_q - c_{j,q})^2),
 *            x_q = 2 i_q / n_q - 1 with 1 <= i_q <= n_q (the Gaussian-bump
 *            tensor of Section 4.4, for any d).  centers is host memory,
 *            n_terms x d row-major (c_{j,q} at centers[j * d + q]), read during
 *            the call only; 1 <= n_terms <= PSTT2_GAUSS_MAX_TERMS, gamma > 0.
 *            Each bump is a product of one factor per mode, so the library
 *            tabulates those factors (FP64 exp) and evaluates chunks of whole
 *            columns of X_m into a workspace of at most PSTT2_GAUSS_CHUNK_BYTES
 *            (one column if that is larger), which the memory kernels then
 *            stream: the tensor is never stored whole.  The bumps are added in
 *            increasing j. */
typedef enum { PSTT2_FN_HILBERT = 0, PSTT2_FN_GAUSS = 1 } pstt2_fn_kind;
#define PSTT2_GAUSS_MAX_TERMS 1024
#define PSTT2_GAUSS_CHUNK_BYTES (1LL << 32)
typedef struct {
  pstt2_fn_kind kind;
  int32_t n_terms;         /* GAUSS: number of bumps */
  double gamma;            /* GAUSS: width parameter */
  const double* centers;   /* GAUSS: host, n_terms x d, row-major */
} pstt2_fn;

/* Stream the entries [first, first + count) of the tensor fn (flat
 * column-major, the context's mode sizes) into the sketches, as pstt2_sketch
 * does for a slab in memory.  HILBERT needs a context with dtype F64 and prec
 * F64; GAUSS takes any context (its entries are evaluated in FP64 and rounded
 * to the context's dtype, as a stored tensor of that dtype would be).
 * first and count must be multiples of R_m = n_1...n_m (whole columns of the
 * middle unfolding X_m); the same coverage rules as pstt2_sketch apply, and
 * slabs from memory and from fn may be mixed.  HILBERT builds small index
 * tables (R_m + C_m int32 and sum_q n_q doubles) on first use and keeps them
 * with the context; GAUSS builds its tables on every call.  async (GAUSS first
 * waits for the stream's earlier work and its own table set-up, so the centers
 * may be freed on return, then queues the chunks).  Errors: EINVAL (kind, fields,
 * dtype / prec, alignment, range), ESTATE (overlap, after recover), ENOMEM, EDEVICE. */
pstt2_status pstt2_sketch_fn(pstt2_ctx* ctx, const pstt2_fn* fn, int64_t first, int64_t count);

/* Recover the TT cores from the accumulated sketches: derive every split's
 * sketch and its two-sided sketch B_k = Psi_k^T X_k Omega_k (ell x ell; as
 * Psi_k^T S_k for k < m and T_k Omega_k for k >= m, FP64 DRM entries), bases
 * by TSQR + column-pivoted QR of the small R factor (sign fixed
 * so that diag(R) >= 0), outer cores, middle core.  In tolerance mode the
 * ranks follow the rule sum_{i>r} sigma_i(S_k)^2 <= eps^2/(d-1) ||S_k||_F^2
 * capped at rmax.  out->core[k] are library-allocated (out->owned = 1).  sync.
 * For PSTT2_MID_TWOPASS the middle core is computed by pstt2_middle_pass calls
 * made after this one; until then out->core[m-1] is allocated and zero.
 * Errors: ESTATE (not every entry of X was streamed exactly once),
 * ENUMERIC (non-finite sketch, rank-deficient least-squares system), ENOMEM, EDEVICE. */
pstt2_status pstt2_recover(pstt2_ctx* ctx, tt_cores* out);

/* Tolerance mode with a certificate.  The eps rule reads the ranks off the
 * sketches, and its bound is probabilistic; Section 4.1 measures the error of
 * every trial.  This call recovers, measures ||X - X~||_F / ||X||_F in a
 * second pass over X (x_dev, the tensor that was sketched, in the context's
 * dtype) or over the tensor function fn (give exactly one), and while the
 * error exceeds eps recovers again from the same sketches (no new pass for
 * them), with the rule's tolerance halved until at least one rank grows.  It
 * stops when the error is at most eps, after max_tries recoveries, or when
 * every rank is at its cap (rmax, ell - 2, the unfolding's size): then only a
 * larger sketch size can help.  *out receives the last recovery's cores and
 * *rel_err its measured error, which the caller compares with eps; the ranks
 * are in out->r.  sync.  Errors: EINVAL (arguments), ESTATE (fixed-rank or
 * two-pass context, or not every entry streamed), and those of pstt2_recover
 * and tt_error. */
pstt2_status pstt2_recover_certified(pstt2_ctx* ctx, const void* x_dev, const pstt2_fn* fn, int32_t max_tries,
                                     tt_cores* out, double* rel_err);

/* Two-pass middle core (equation "PSTT2_final_core"): add the contribution of a
 * slab of X to out->core[m-1] of the cores returned by pstt2_recover.  Same slab
 * rules as pstt2_sketch.  async.  Errors: ESTATE (context not in two-pass mode or
 * recover not called), EINVAL. */
pstt2_status pstt2_middle_pass(pstt2_ctx* ctx, tt_cores* cores, const void* x_dev, int64_t first,
                               int64_t count);

/* The same second pass over the tensor function fn (see pstt2_fn): Section
 * 4.4's PSTT2 evaluates the function a second time for its middle core (the
 * one-sided algorithm: its last core), which the one-pass cores avoid.  The
 * entries [first, first + count) are evaluated in FP64 into workspace chunks of
 * whole columns of the pass's unfolding (at most PSTT2_GAUSS_CHUNK_BYTES each,
 * in the context's dtype) that pstt2_middle_pass then reads; first and count
 * must be multiples of that unfolding's row count (n_1...n_m, or
 * n_1...n_{d-1} for PSTT2_ALGO_PSTT).  Like pstt2_sketch_fn it waits for the
 * table set-up and returns once the last chunk's work is queued.  Errors:
 * those of pstt2_middle_pass, EINVAL (fn fields, alignment), ENOMEM, EDEVICE. */
pstt2_status pstt2_middle_pass_fn(pstt2_ctx* ctx, tt_cores* cores, const pstt2_fn* fn, int64_t first,
                                  int64_t count);

/* Vector-Jacobian product of the one-pass map X -> X~ (the cores returned by
 * the last pstt2_recover of this context, reconstructed by the entry formula
 * of Section 2.2), with the pivots and ranks of that recovery held fixed.
 * NESTED: X~ depends on X only through the two sketches of the middle
 * unfolding, so
 *   J^T gbar = Ybar Omega_m^T + Psi_m Tbar_m,
 * where (Ybar, Tbar_m) are the cotangents of Y_R and T_m obtained by running
 * the recovery (least squares or the two-sided pseudo-inverse products, outer
 * cores, QR of the pivoted sketch columns, derived sketches) backwards in FP64
 * on the GPU.  INDEPENDENT: the same with one such pair of terms per pass
 * group, each with the factors that group sketched with.
 *   gbar_dev != NULL: gx_dev = J^T gbar (gbar and gx have X's shape and dtype);
 *                     x_dev is not read and may be NULL.
 *   gbar_dev == NULL: gx_dev = gradient of ||X - X~||_F^2 with respect to X,
 *                     i.e. 2 (X - X~) + J^T (-2 (X - X~)); x_dev must be the
 *                     tensor that was sketched.
 * gx_dev is caller-owned device memory of N entries of the context's dtype.
 * The cotangent is never stored: gbar (or X, for the Frobenius loss, whose
 * -2 X~ part is applied through two r_m x r_m Gram matrices of the interfaces)
 * is streamed from caller memory.  Uses stream-ordered device workspace of
 * O((R_m + C_m) r_m) doubles plus the workgroup partials of that stream
 * (8 (gi C_m + gj R_m) r_m bytes), nothing tensor-sized.  sync.
 * Errors: ESTATE (no successful pstt2_recover; a two-pass middle core),
 * EINVAL (null pointers, cores not from this context), ENOMEM, EDEVICE. */
pstt2_status pstt2_vjp(pstt2_ctx* ctx, const tt_cores* cores, const void* x_dev, const void* gbar_dev,
                       void* gx_dev);

/* Copy an accumulated or derived sketch to host memory (FP64, column-major).
 * which = 0: the right sketch of split k (1 <= k <= m; k = m is Y_R), R_k x ell.
 * which = 1: the transposed left sketch T_k^T of split k (m <= k <= d-1), C_k x ell.
 * which = 2: the two-sided sketch B_k = Psi_k^T X_k Omega_k (1 <= k <= d-1), ell x ell.
 * which = 3: the two-sided middle sketch H (PSTT2_MID_TWOSIDED, d >= 3; k ignored),
 *            (ell n_m) x ell, row a + ell i_m.
 * Valid after pstt2_recover.  *rows and *cols receive the shape; host_out must hold
 * rows*cols doubles (pass host_out = NULL to query the shape).  sync. */
pstt2_status pstt2_get_sketch(pstt2_ctx* ctx, int32_t which, int32_t k, double* host_out, int64_t* rows,
                              int64_t* cols);

/* Pivot order chosen for split k's basis (0-based column indices, ell of them). sync. */
pstt2_status pstt2_get_pivots(pstt2_ctx* ctx, int32_t k, int32_t* host_piv);

/* Kernel timing: with enable = 1 every later sketch launch of this context is
 * bracketed by HIP events recorded on the context's stream (around the
 * streaming sketch kernel only, not its partial reduction).  enable = 0 stops
 * and clears the record.  Host-side; async.  Errors: EINVAL. */
pstt2_status pstt2_profile(pstt2_ctx* ctx, int32_t enable);

/* Sum of the recorded sketch-kernel durations (milliseconds) and the number of
 * launches, then clear the record.  sync.  Errors: EINVAL, EDEVICE. */
pstt2_status pstt2_profile_read(pstt2_ctx* ctx, double* total_ms, int64_t* launches);

/* Forget all streamed data (zero the sketches and the coverage record); the DRM
 * factors are kept, so the same context sketches the next tensor.  async. */
pstt2_status pstt2_reset(pstt2_ctx* ctx);

/* Release the context.  sync.  NULL is ignored. */
void pstt2_destroy(pstt2_ctx* ctx);

/* Relative error ||X - X~||_F / ||X||_F by entrywise differences over one
 * streaming pass, sums in FP64 (Section 4.1: the error measured for every
 * trial).  For X = 0 the result is 0 when X~ = 0 too, and ENUMERIC otherwise.
 * cores may point at caller memory.  sync.  Errors: EINVAL, ENUMERIC, ENOMEM,
 * EDEVICE. */
pstt2_status tt_error(const tt_cores* cores, const void* x_dev, pstt2_dtype dtype, double* rel_err,
                      void* hip_stream);

/* tt_error without allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same pass and the same sums in the same order as tt_error,
 * but every temporary (interface tables, padded right interface, workgroup
 * partials) lives in one static device buffer of PSTT2_NOALLOC_SCRATCH_BYTES
 * that the library holds on each device it runs on until the process ends; no
 * allocation of any kind is made.  err_dev is caller-owned device memory of
 * three doubles: err_dev[0] = ||X - X~||_F / ||X||_F (0 for X = 0 = X~, +inf
 * for X = 0 != X~), err_dev[1] = sum (x - x~)^2, err_dev[2] = sum x^2.  async:
 * the result is in err_dev once the stream passes the work; nothing is
 * synchronised.  Every call on a device shares that device's buffer (nothing
 * in it needs clearing, each call writes what it reads), so calls that overlap
 * on one device, on any streams, race: serialise them.  Errors: EINVAL
 * (cores, null pointers, dtype), ENOMEM (the pass would need more than
 * PSTT2_NOALLOC_SCRATCH_BYTES: about 8 (R_m r_m + 16 C_m) bytes at the
 * middle split, e.g. 10 MB for d = 6, n = 32, rank 10), EDEVICE. */
#define PSTT2_NOALLOC_SCRATCH_BYTES (64LL << 20)
pstt2_status tt_error_noalloc(const tt_cores* cores, const void* x_dev, pstt2_dtype dtype, double* err_dev,
                              void* hip_stream);

/* The same for the tensor fn (see pstt2_fn), evaluated in FP64 instead of read
 * from memory; the mode sizes are the cores'.  sync.
 * Errors: EINVAL, ENUMERIC, ENOMEM, EDEVICE. */
pstt2_status tt_error_fn(const tt_cores* cores, const pstt2_fn* fn, double* rel_err, void* hip_stream);

/* Write entries [first, first + count) of X~ (flat column-major, entry formula
 * of Section 2.2) to x_out_dev in the given dtype.  sync.  Errors: EINVAL, EDEVICE. */
pstt2_status tt_reconstruct(const tt_cores* cores, void* x_out_dev, pstt2_dtype dtype, int64_t first,
                            int64_t count, void* hip_stream);

/* Copy the core values of src into the buffers of dst (same d, n, r; dst's
 * core pointers are caller-provided device memory).  sync.  Errors: EINVAL, EDEVICE. */
pstt2_status tt_cores_copy(const tt_cores* src, tt_cores* dst, void* hip_stream);

/* Release library-owned cores (owned == 1), stream-ordered after the work
 * already enqueued on the stream that produced them, and clear the struct.
 * NULL is ignored. */
void tt_cores_free(tt_cores* cores);

/* Parallel-TTSVD (Section 3.1, Algorithm Parallel-TTSVD, Theorem perf_alg1):
 * the deterministic compress-then-combine TT of a dense FP64 tensor.  For
 * every split k = 1..d-1 a truncated SVD X_k ~ U_k Sigma_k V_k^T keeps the
 * smallest rank r_k with sum_{i > r_k} sigma_i(X_k)^2 <= eps^2 ||X||_F^2 / (d-1)
 * (capped at rmax when rmax > 0, and at PSTT2_MAX_ELL); then G_1 = U_1,
 * G_k = reshape(U_{k-1}^T reshape(U_k, R_{k-1}, n_k r_k)) (equation "core")
 * and G_d = Sigma_{d-1} V_{d-1}^T, so that ||X - X~||_F <= eps ||X||_F
 * (Theorem perf_alg1) when no cap binds.  The SVDs run on the GPU by one-sided
 * Jacobi on each unfolding's short side, directly on the data (no Gram
 * matrix: singular values keep their relative accuracy), FP64 throughout.
 * Scope: every unfolding's short side min(R_k, C_k) must be at most
 * PSTT2_TTSVD_MAX_SIDE; the work is about 10 sweeps of short side x N
 * products per split.  x_dev: N = n_1...n_d FP64 entries, column-major,
 * read-only.  out receives library-owned cores (release with tt_cores_free).
 * X = 0 gives ranks 1 and X~ = 0.  sync.  Errors: EINVAL (arguments, scope),
 * ENUMERIC (non-finite X, no convergence in 40 sweeps), ENOMEM, EDEVICE. */
#define PSTT2_TTSVD_MAX_SIDE 1024
pstt2_status pstt2_parallel_ttsvd(int32_t d, const int64_t* n, const double* x_dev, double eps, int32_t rmax,
                                  void* hip_stream, tt_cores* out);

/* The DRM factors a context draws when desc->drm_factors is NULL (Algorithm
 * PSTT: i.i.d. standard Gaussian entries, Section 3.2), in the packed layout of
 * pstt2_desc.drm_factors for desc's d, n, ell and drm (other fields unused).
 * Entry j of the buffer is the standard normal
 *   p = j / 2, (x0..x3) = Philox4x32-10(counter (p mod 2^32, p div 2^32, 0, 0),
 *                                       key (seed mod 2^32, seed div 2^32))
 *   u1 = 1 - ((x0 >> 5) 2^26 + (x1 >> 6)) / 2^53,  u2 = ((x2 >> 5) 2^26 + (x3 >> 6)) / 2^53
 *   entry 2p = sqrt(-2 ln u1) cos(2 pi u2),   entry 2p + 1 = sqrt(-2 ln u1) sin(2 pi u2)
 * (Philox4x32-10: Salmon, Moraes, Dror, Shaw, SC 2011; Box-Muller transform).
 * host_out == NULL: *count receives the number of doubles.  Otherwise *count
 * must hold the capacity of host_out and receives the number written.  Host
 * only, needs no GPU.  Errors: EINVAL. */
pstt2_status pstt2_drm_factors(const pstt2_desc* desc, double* host_out, int64_t* count);

/* Device-memory budget of the library in bytes (<= 0: none).  Buffers already
 * allocated are kept; a later request that would take the live total past the
 * budget fails with PSTT2_ENOMEM.  Process-wide, all devices.  Never fails. */
pstt2_status pstt2_set_memory_limit(int64_t bytes);

/* Live and peak bytes of device memory held by the library (contexts,
 * workspaces, cores not yet released) and the budget (-1: none).  Any pointer
 * may be NULL.  Never fails. */
pstt2_status pstt2_memory_stats(int64_t* live_bytes, int64_t* peak_bytes, int64_t* limit_bytes);

/* Testing hook for the failure paths: after this call the next `count` kernel
 * launches of the library's streaming stages (sketch, partial reduction,
 * partial column, tensor-function columns, two-pass middle core) go ahead and
 * the one after them is reported as a failed launch (PSTT2_EDEVICE) without
 * running; then the hook disarms.  count < 0 disarms it.  Host-side only: no
 * kernel is altered.  Process-wide.  Never fails. */
pstt2_status pstt2_inject_launch_failure(int64_t count);

/* Message for the last failing call on ctx, or (ctx == NULL) on this thread. */
const char* pstt2_last_error(const pstt2_ctx* ctx);

/* Library version string. */
const char* pstt2_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PSTT2_H */
