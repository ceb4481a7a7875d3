"""Plain FP64 PSTT2 oracle (paper Section 3.2) -- TEST INFRASTRUCTURE ONLY.

Imported only by tests, the smoke check and the benchmark's CPU-baseline leg.
Everything here is written for a reader checking it against the paper: no
blocking, fusion or reordering beyond what the paper's own formulas state.

Conventions (Section 2.1): a tensor is a flat FP64 vector in column-major
order (i_1 fastest); the k-th unfolding X_k = reshape(X, n_1...n_k, n_{k+1}...n_d)
is a column-major view of it.  Real arithmetic throughout (the paper's ^* is
the transpose here).  All indices in code are 0-based.

Khatri-Rao DRMs (Section 3.2, equation "sketch_orig"): the right DRM of split k
is Omega_k = omega_d (.) ... (.) omega_{k+1}, the column-wise Kronecker product
with the last-listed factor varying fastest, so that its rows line up with the
columns of X_k.  The left DRM is Psi_k = psi_k (.) ... (.) psi_1, rows lined up
with the rows of X_k.  In the *nested* scheme every split uses the same
per-mode factors; in the *independent* scheme (the paper's Psi^{(j)}) each
split draws its own.

PSTT2 (Section 3.2, end; equation "PSTT2_final_core"), m = ceil(d/2):
  * column bases Q_k of X_k for k = 1..m-1 from CPQR of S_k = X_k Omega_k;
  * row bases P_k of X_k for k = m..d-1 from CPQR of T_k^T, T_k = Psi_k^T X_k
    (the paper's "P_j" read as the row basis of X_{j-1}, the only index
    reading consistent with the three-way reshape of its middle-core formula);
  * outer cores from neighbouring bases (equation "core" and its row mirror);
  * the middle core either from a second pass over X (two-pass PSTT2) or from
    the extra sketch Y_R = X_m Omega_m and a least-squares solve (PSTT2-onepass,
    equation "onepass_final_core" applied to the middle unfolding), or from
    the same Y_R sketched once more on its leading modes and a pseudo-inverse
    on each side ("twosided");
  * the two-sided sketches B_k = Psi_k^T X_k Omega_k of every split.

Parity pins (tests/test_oracle_*.py):
  unfold, khatri_rao, right/left sketches .... brute-force index loops, np.kron,
                                               the eq. sketch_orig block form, a
                                               rank-one closed form
  cpqr_basis ................................. LAPACK geqp3 invariants, pivots of R
  two_sided_sketch ........................... brute-force index loops, a rank-one
                                               closed form, Psi_k^T S_k = T_k Omega_k
  pstt2 (all middle-core forms) .............. exact recovery of exact-rank TTs,
                                               the deterministic projection bound
                                               (eq. proj_acc), Thm 3/4 expectation
                                               bounds by Monte Carlo
  tt_full / tt_error ......................... brute-force entry formula (Sec. 2.2)
  tt_storage ................................. Table 1 printed sizes
  rank_from_tolerance ........................ closed-form spectra
"""
from __future__ import annotations

import math
import time
from typing import Dict, List, Optional, Sequence

import numpy as np
import scipy.linalg

__all__ = [
    "middle_index", "rows_of", "cols_of", "unfold", "khatri_rao", "NestedKR", "IndependentKR",
    "DenseDRM", "sketch_right_dense", "sketch_left_dense", "sketch_right_modewise",
    "sketch_left_modewise", "cpqr_basis", "rank_from_tolerance", "outer_core_left",
    "outer_core_right", "middle_core_twopass", "middle_core_onepass", "middle_core_twosided",
    "two_sided_sketch", "pstt2", "pstt",
    "tt_full", "tt_entry", "tt_error", "tt_storage", "kmode_product", "tt_ranks",
]


# ----------------------------------------------------------------------------
# Section 2.1: unfoldings and the k-mode product
# ----------------------------------------------------------------------------

def middle_index(d: int) -> int:
    """d_* = ceil(d/2) (Section 3.2, PSTT2)."""
    return (d + 1) // 2


def rows_of(n: Sequence[int], k: int) -> int:
    """Number of rows n_1...n_k of the k-th unfolding."""
    return int(np.prod(n[:k], dtype=np.int64))


def cols_of(n: Sequence[int], k: int) -> int:
    """Number of columns n_{k+1}...n_d of the k-th unfolding."""
    return int(np.prod(n[k:], dtype=np.int64))


def unfold(x: np.ndarray, n: Sequence[int], k: int) -> np.ndarray:
    """X_k = reshape(X, prod_{s<=k} n_s, prod_{s>k} n_s), column-major (Section 2.1)."""
    return np.reshape(x, (rows_of(n, k), cols_of(n, k)), order="F")


def kmode_product(x: np.ndarray, n: Sequence[int], k: int, a: np.ndarray) -> np.ndarray:
    """X x_k A (Section 2.1, equation "kfold"), k 1-based; returns the new flat tensor."""
    t = np.reshape(x, tuple(n), order="F")
    t = np.moveaxis(np.tensordot(a, t, axes=([1], [k - 1])), 0, k - 1)
    return np.reshape(t, -1, order="F")


# ----------------------------------------------------------------------------
# Section 3.2: Khatri-Rao dimension reduction maps
# ----------------------------------------------------------------------------

def khatri_rao(mats: Sequence[np.ndarray]) -> np.ndarray:
    """A_1 (.) A_2 (.) ... (.) A_p: column c is A_1(:,c) kron ... kron A_p(:,c).

    Written out as the definition: row index (i_1, ..., i_p) with i_p fastest.
    """
    ell = mats[0].shape[1]
    out = np.ones((1, ell))
    for a in mats:
        # (out (.) a)(i_out * n_a + i_a, c) = out(i_out, c) * a(i_a, c)
        out = (out[:, None, :] * a[None, :, :]).reshape(-1, ell)
    return out


class NestedKR:
    """Nested Khatri-Rao factors: psi[q] (q = 1..d-1) and omega[q] (q = 2..d), each (n_q, ell)."""

    def __init__(self, psi: Dict[int, np.ndarray], omega: Dict[int, np.ndarray]):
        self.psi = psi
        self.omega = omega

    def right_factors(self, k: int, d: int) -> List[np.ndarray]:
        """[omega_{k+1}, ..., omega_d] for the right DRM of split k."""
        return [self.omega[q] for q in range(k + 1, d + 1)]

    def left_factors(self, k: int) -> List[np.ndarray]:
        """[psi_1, ..., psi_k] for the left DRM of split k."""
        return [self.psi[q] for q in range(1, k + 1)]

    def omega_dense(self, k: int, d: int) -> np.ndarray:
        """Omega_k = omega_d (.) ... (.) omega_{k+1} (prod_{q>k} n_q x ell)."""
        return khatri_rao(self.right_factors(k, d)[::-1])

    def psi_dense(self, k: int) -> np.ndarray:
        """Psi_k = psi_k (.) ... (.) psi_1 (prod_{q<=k} n_q x ell)."""
        return khatri_rao(self.left_factors(k)[::-1])


class IndependentKR(NestedKR):
    """Independent Khatri-Rao factors per split: psi[k][q], omega[k][q] (the paper's Psi^{(j)})."""

    def right_factors(self, k: int, d: int) -> List[np.ndarray]:
        return [self.omega[k][q] for q in range(k + 1, d + 1)]

    def left_factors(self, k: int) -> List[np.ndarray]:
        return [self.psi[k][q] for q in range(1, k + 1)]


class DenseDRM:
    """Unstructured DRMs: omega[k] (C_k x ell) and psi[k] (R_k x ell) given as full matrices."""

    def __init__(self, psi: Dict[int, np.ndarray], omega: Dict[int, np.ndarray]):
        self.psi = psi
        self.omega = omega

    def omega_dense(self, k: int, d: int) -> np.ndarray:
        return self.omega[k]

    def psi_dense(self, k: int) -> np.ndarray:
        return self.psi[k]


def sketch_right_dense(x: np.ndarray, n: Sequence[int], k: int, omega_k: np.ndarray) -> np.ndarray:
    """S_k = X_k Omega_k (Algorithm PSTT, sketch step), with a dense DRM."""
    return unfold(x, n, k) @ omega_k


def sketch_left_dense(x: np.ndarray, n: Sequence[int], k: int, psi_k: np.ndarray) -> np.ndarray:
    """T_k = Psi_k^T X_k: the row-space sketch "using X_j^T" (Section 4.2)."""
    return psi_k.T @ unfold(x, n, k)


def two_sided_sketch(x: np.ndarray, n: Sequence[int], k: int, drm) -> np.ndarray:
    """B_k = Psi_k^T X_k Omega_k (ell x ell): the split-k unfolding sketched from both sides.

    Section 3.2 sketches X_k from the right (column space, Algorithm PSTT) and,
    for PSTT2, from the left (row space); B_k applies both DRMs of split k at
    once.  Written from the definition with the dense Khatri-Rao DRMs.
    """
    d = len(n)
    return drm.psi_dense(k).T @ unfold(x, n, k) @ drm.omega_dense(k, d)


def sketch_right_modewise(x: np.ndarray, n: Sequence[int], k: int, factors: Sequence[np.ndarray]) -> np.ndarray:
    """X_k (omega_d (.) ... (.) omega_{k+1}) via the block form of equation "sketch_orig".

    The columns of X_k are grouped by the slow indices (i_{k+2}..i_d); each block
    is multiplied by omega_{k+1} and scaled by the diagonal matrices D built from
    the rows of the slower factors.  Here the scalings are applied one mode at a
    time, slowest mode first.  factors = [omega_{k+1}, ..., omega_d].
    """
    d = len(n)
    ell = factors[0].shape[1]
    rk = rows_of(n, k)
    # contract the slowest mode first: Z(row, i_{k+1}..i_{d-1}, c)
    z = unfold(x, n, d - 1) @ factors[-1]                  # (R_{d-1} x ell)
    for q in range(d - 1, k, -1):                           # modes d-1 .. k+1
        nq = n[q - 1]
        z = z.reshape(rows_of(n, q - 1), nq, ell, order="F")
        z = np.einsum("rjc,jc->rc", z, factors[q - k - 1])
    return z.reshape(rk, ell)


def sketch_left_modewise(x: np.ndarray, n: Sequence[int], k: int, factors: Sequence[np.ndarray]) -> np.ndarray:
    """Psi_k^T X_k with Psi_k = psi_k (.) ... (.) psi_1, contracting mode 1 first.

    factors = [psi_1, ..., psi_k].  Returns the ell x C_k matrix T_k.
    """
    ell = factors[0].shape[1]
    ck = cols_of(n, k)
    z = factors[0].T @ unfold(x, n, 1)                      # (ell x C_1)
    for q in range(2, k + 1):
        nq = n[q - 1]
        z = z.reshape(ell, nq, cols_of(n, q), order="F")
        z = np.einsum("cjr,jc->cr", z, factors[q - 1])
    return z.reshape(ell, ck)


def _right_sketch(x, n, k, drm, dense_limit):
    d = len(n)
    if isinstance(drm, DenseDRM) or cols_of(n, k) * drm_ell(drm, k, d) <= dense_limit:
        return sketch_right_dense(x, n, k, drm.omega_dense(k, d))
    return sketch_right_modewise(x, n, k, drm.right_factors(k, d))


def _left_sketch(x, n, k, drm, dense_limit):
    d = len(n)
    if isinstance(drm, DenseDRM) or rows_of(n, k) * drm_ell(drm, k, d) <= dense_limit:
        return sketch_left_dense(x, n, k, drm.psi_dense(k))
    return sketch_left_modewise(x, n, k, drm.left_factors(k))


def drm_ell(drm, k, d):
    if isinstance(drm, DenseDRM):
        return drm.omega[k].shape[1] if k in drm.omega else drm.psi[k].shape[1]
    f = drm.right_factors(k, d) if k < d else drm.left_factors(k)
    return f[0].shape[1]


# ----------------------------------------------------------------------------
# Bases: CPQR truncation (Algorithm PSTT, CPQR step)
# ----------------------------------------------------------------------------

def cpqr_basis(s: np.ndarray, r: int):
    """First r columns of Q from a column-pivoted QR of S, sign-fixed so diag(R) >= 0.

    Returns (Q_r, R, piv) with S[:, piv] = Q R.  LAPACK geqp3 picks, at each
    step, the first column of largest remaining norm.
    """
    q, rr, piv = scipy.linalg.qr(s, mode="economic", pivoting=True)
    sgn = np.where(np.diag(rr) < 0.0, -1.0, 1.0)
    q = q * sgn[None, :]
    rr = rr * sgn[:, None]
    return q[:, :r].copy(), rr, piv


def rank_from_tolerance(s: np.ndarray, eps: float, d: int, rmax: int) -> int:
    """Smallest r with sum_{i>r} sigma_i(S)^2 <= (eps^2/(d-1)) ||S||_F^2, capped at rmax.

    The per-unfolding share eps/sqrt(d-1) is the TT-SVD truncation rule of
    Section 2.2 applied to the sketch.  Also capped at min(rows, cols) of S.
    """
    sig = np.linalg.svd(s, compute_uv=False)
    tot = float(np.sum(sig ** 2))
    thr = (eps * eps / (d - 1)) * tot
    r = len(sig)
    tail = 0.0
    # walk down from the smallest singular value
    for i in range(len(sig) - 1, -1, -1):
        if tail + sig[i] ** 2 <= thr:
            tail += sig[i] ** 2
            r = i
        else:
            break
    r = max(1, r)
    return int(min(r, rmax, min(s.shape)))


# ----------------------------------------------------------------------------
# Cores (Theorem 2, equation "core", and its row-space mirror)
# ----------------------------------------------------------------------------

def outer_core_left(q_prev: np.ndarray, q_k: np.ndarray, n_k: int) -> np.ndarray:
    """G_k = reshape(Q_{k-1}^T reshape(Q_k, R_{k-1}, n_k r_k), r_{k-1}, n_k, r_k)."""
    r_prev = q_prev.shape[1]
    r_k = q_k.shape[1]
    r_rows = q_prev.shape[0]
    w = q_prev.T @ np.reshape(q_k, (r_rows, n_k * r_k), order="F")
    return np.reshape(w, (r_prev, n_k, r_k), order="F")


def outer_core_right(p_prev: np.ndarray, p_k: np.ndarray, n_k: int) -> np.ndarray:
    """Row-space mirror of equation "core": G_k(a, i, b) = sum_c P_{k-1}(i + n_k c, a) P_k(c, b).

    P_{k-1} is the row basis of X_{k-1} (C_{k-1} x r_{k-1}), P_k that of X_k.
    """
    r_prev = p_prev.shape[1]
    c_k = p_k.shape[0]
    p3 = np.reshape(p_prev, (n_k, c_k, r_prev), order="F")     # (i, c, a)
    return np.einsum("ica,cb->aib", p3, p_k)


def middle_core_twopass(x: np.ndarray, n: Sequence[int], q_prev: np.ndarray, p_m: np.ndarray, m: int) -> np.ndarray:
    """Equation "PSTT2_final_core": reshape(X, R_{m-1}, n_m, C_m) x_1 Q_{m-1}^T x_3 P_m^T."""
    r_rows = rows_of(n, m - 1)
    x3 = np.reshape(x, (r_rows, n[m - 1], cols_of(n, m)), order="F")
    return np.einsum("ra,rjc,cb->ajb", q_prev, x3, p_m)


def middle_core_onepass(y_r: np.ndarray, omega_m: np.ndarray, q_prev: np.ndarray, p_m: np.ndarray,
                        n_m: int) -> np.ndarray:
    """One-pass middle core from Y_R = X_m Omega_m (Section 3.2 end, Section 4.2 "PSTT2-onepass").

    Z = (I_{n_m} kron Q_{m-1})^T Y_R and A = P_m^T Omega_m; the core's second
    unfolding G (r_{m-1} n_m x r_m) solves min ||G A - Z||_F, i.e.
    G = Z A^+ as in equation "onepass_final_core".
    """
    r_prev = q_prev.shape[1]
    r_m = p_m.shape[1]
    r_rows = q_prev.shape[0]
    ell = y_r.shape[1]
    y3 = np.reshape(y_r, (r_rows, n_m, ell), order="F")           # (row', i_m, c)
    z = np.einsum("ra,rjc->ajc", q_prev, y3).reshape(r_prev * n_m, ell, order="F")
    a = p_m.T @ omega_m                                           # (r_m x ell)
    g_t, *_ = np.linalg.lstsq(a.T, z.T, rcond=None)               # (r_m x r_prev n_m)
    return np.reshape(g_t.T, (r_prev, n_m, r_m), order="F")


def middle_core_twosided(y_r: np.ndarray, psi_prev: np.ndarray, q_prev: np.ndarray, omega_m: np.ndarray,
                         p_m: np.ndarray, n_m: int) -> np.ndarray:
    """Two-sided one-pass middle core (Section 3.2, PSTT2-onepass, with both outer modes sketched).

    The middle core of equation "PSTT2_final_core" is X3 x_1 Q_{m-1}^T x_3 P_m^T
    with X3 = reshape(X, R_{m-1}, n_m, C_m).  Sketch X3 on both outer modes,
        H = X3 x_1 Psi'^T x_3 Omega_m^T   (ell x n_m x ell),
    where Psi' = Psi_{m-1} (R_{m-1} x ell) and H is the leading-mode
    contraction of Y_R = X_m Omega_m.  With X3 ~ G x_1 Q_{m-1} x_3 P_m,
    H ~ G x_1 (Psi'^T Q_{m-1}) x_3 (Omega_m^T P_m), so
        G = H x_1 (Psi'^T Q_{m-1})^+ x_3 (Omega_m^T P_m)^+,
    the pseudo-inverse step of equation "onepass_final_core" taken on both
    sides.
    """
    r_rows = q_prev.shape[0]
    ell = y_r.shape[1]
    y3 = np.reshape(y_r, (r_rows, n_m, ell), order="F")          # (row', i_m, c)
    h = np.einsum("ra,rjc->ajc", psi_prev, y3)                   # (a, i_m, c)
    a1 = psi_prev.T @ q_prev                                     # ell x r_{m-1}
    a3 = omega_m.T @ p_m                                         # ell x r_m
    return np.einsum("pa,ajc,qc->pjq", np.linalg.pinv(a1), h, np.linalg.pinv(a3))


# ----------------------------------------------------------------------------
# The top-level routine
# ----------------------------------------------------------------------------

def _clamp_ranks(n, ranks, ell):
    d = len(n)
    out = []
    for k in range(1, d):
        out.append(int(min(ranks[k - 1], rows_of(n, k), cols_of(n, k), ell)))
    return out


def pstt2(x: np.ndarray, n: Sequence[int], drm, ranks: Optional[Sequence[int]] = None,
          eps: Optional[float] = None, rmax: int = 0, middle: str = "onepass",
          dense_limit: int = 1 << 22, timings: Optional[dict] = None) -> dict:
    """PSTT2 (two-pass) or PSTT2-onepass on a flat column-major FP64 tensor.

    drm: NestedKR / IndependentKR / DenseDRM.  Give ranks r_1..r_{d-1} (fixed
    rank) or eps (tolerance mode, ranks from the sketches' spectra, capped at
    rmax and at ell - 2 so that the oversampling p >= 2 of Theorem 3 holds).

    Returns a dict with cores, ranks, bases Q (k < m) and P (k >= m), the
    sketches S_k, T_k, Y_R and the middle index m.  With a `timings` dict, the
    wall time of the sketches and of the recovery (seconds) is stored in it
    under "sketch_s" and "recover_s" (measurement only).
    """
    t_start = time.perf_counter()
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    n = tuple(int(v) for v in n)
    d = len(n)
    m = middle_index(d)
    ell = drm_ell(drm, 1 if d > 1 else 1, d)

    s_sk = {k: _right_sketch(x, n, k, drm, dense_limit) for k in range(1, m)}
    t_sk = {k: _left_sketch(x, n, k, drm, dense_limit) for k in range(m, d)}
    y_r = _right_sketch(x, n, m, drm, dense_limit) if middle in ("onepass", "twosided") else None
    t_sketched = time.perf_counter()

    if ranks is None:
        if eps is None:
            raise ValueError("give ranks or eps")
        cap = rmax if rmax > 0 else ell
        cap = min(cap, max(1, ell - 2))
        rk = []
        for k in range(1, d):
            sk = s_sk[k] if k < m else t_sk[k].T
            rk.append(rank_from_tolerance(sk, eps, d, cap))
        ranks = rk
    ranks = _clamp_ranks(n, ranks, ell)
    r = [1] + list(ranks) + [1]

    q = {0: np.ones((1, 1))}
    piv = {}
    for k in range(1, m):
        q[k], _, piv[k] = cpqr_basis(s_sk[k], r[k])
    p = {d: np.ones((1, 1))}
    for k in range(m, d):
        p[k], _, piv[k] = cpqr_basis(t_sk[k].T, r[k])

    cores: List[np.ndarray] = [None] * d
    for k in range(1, m):
        if k == 1:
            cores[0] = np.reshape(q[1], (1, n[0], r[1]), order="F")
        else:
            cores[k - 1] = outer_core_left(q[k - 1], q[k], n[k - 1])
    for k in range(m + 1, d + 1):
        if k == d:
            cores[d - 1] = np.reshape(p[d - 1].T, (r[d - 1], n[d - 1], 1), order="F")
        else:
            cores[k - 1] = outer_core_right(p[k - 1], p[k], n[k - 1])
    if middle == "onepass" or (middle == "twosided" and m == 1):
        om = drm.omega_dense(m, d) if not isinstance(drm, DenseDRM) else drm.omega[m]
        cores[m - 1] = middle_core_onepass(y_r, om, q[m - 1], p[m], n[m - 1])
    elif middle == "twosided":
        # d >= 3: Psi' is split (m-1)'s left DRM, drawn independently of Q_{m-1}
        om = drm.omega_dense(m, d) if not isinstance(drm, DenseDRM) else drm.omega[m]
        cores[m - 1] = middle_core_twosided(y_r, drm.psi_dense(m - 1), q[m - 1], om, p[m], n[m - 1])
    elif middle == "twopass":
        cores[m - 1] = middle_core_twopass(x, n, q[m - 1], p[m], m)
    else:
        raise ValueError(middle)
    if timings is not None:
        timings["sketch_s"] = t_sketched - t_start
        timings["recover_s"] = time.perf_counter() - t_sketched
    return {"cores": cores, "ranks": ranks, "m": m, "Q": q, "P": p, "S": s_sk, "T": t_sk,
            "Y": y_r, "piv": piv}


def pstt(x: np.ndarray, n: Sequence[int], drm, ranks: Sequence[int], onepass_psi: Optional[np.ndarray] = None,
         dense_limit: int = 1 << 22) -> dict:
    """One-sided PSTT (Algorithm PSTT) and, with onepass_psi given, PSTT-onepass.

    Column bases Q_j of every unfolding from S_j = X_j Omega_j; cores by
    equation "core"; last core G_d = Q_{d-1}^T X_{d-1} (two-pass) or
    (Psi^T Q_{d-1})^+ Psi^T X_{d-1} (equation "onepass_final_core").
    """
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    n = tuple(int(v) for v in n)
    d = len(n)
    ell = drm_ell(drm, 1, d)
    ranks = _clamp_ranks(n, ranks, ell)
    r = [1] + list(ranks) + [1]
    q = {}
    for j in range(1, d):
        q[j], _, _ = cpqr_basis(_right_sketch(x, n, j, drm, dense_limit), r[j])
    cores: List[np.ndarray] = [None] * d
    cores[0] = np.reshape(q[1], (1, n[0], r[1]), order="F")
    for k in range(2, d):
        cores[k - 1] = outer_core_left(q[k - 1], q[k], n[k - 1])
    xd = unfold(x, n, d - 1)
    if onepass_psi is None:
        last = q[d - 1].T @ xd
    else:
        t = onepass_psi.T @ xd
        last, *_ = np.linalg.lstsq(onepass_psi.T @ q[d - 1], t, rcond=None)
    cores[d - 1] = np.reshape(last, (r[d - 1], n[d - 1], 1), order="F")
    return {"cores": cores, "ranks": ranks, "Q": q}


# ----------------------------------------------------------------------------
# TT evaluation (Section 2.2)
# ----------------------------------------------------------------------------

def tt_ranks(cores: Sequence[np.ndarray]) -> List[int]:
    return [c.shape[0] for c in cores] + [cores[-1].shape[2]]


def tt_entry(cores: Sequence[np.ndarray], idx: Sequence[int]) -> float:
    """X_{i_1..i_d} = G_1(:, i_1, :) G_2(:, i_2, :) ... G_d(:, i_d, :)."""
    v = np.ones((1, 1))
    for g, i in zip(cores, idx):
        v = v @ g[:, i, :]
    return float(v[0, 0])


def tt_full(cores: Sequence[np.ndarray]) -> np.ndarray:
    """Dense column-major flat tensor of a TT, by sweeping the entry formula left to right."""
    m = np.ones((1, 1))
    for g in cores:
        a, nk, b = g.shape
        # M_new(row + R * i, b) = sum_a M(row, a) G(a, i, b)
        m = np.einsum("ra,aib->rib", m, g).reshape(m.shape[0] * nk, b, order="F")
    return m.reshape(-1)


def tt_error(x: np.ndarray, cores: Sequence[np.ndarray]) -> float:
    """||X - X~||_F / ||X||_F by entrywise difference (equation "FrobeniusNorm")."""
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    xt = tt_full(cores)
    return float(np.linalg.norm(x - xt) / np.linalg.norm(x))


def tt_storage(n: Sequence[int], r: Sequence[int]) -> int:
    """Degrees of freedom sum_k s_{k-1} n_k s_k of a TT with core sizes s (Section 2.2)."""
    return int(sum(r[k] * n[k] * r[k + 1] for k in range(len(n))))
