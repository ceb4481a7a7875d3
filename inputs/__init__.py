"""Seeded synthetic inputs shared by the oracle-side tests, the benchmark and the
GPU parity tests.

This module only *draws* data: dense tensors built from random tensor-train
cores, smooth function samples on Chebyshev grids, Gaussian noise, and the
Gaussian factors of the Khatri-Rao dimension reduction maps.  It holds none of
the sketching / recovery arithmetic of the method itself; both the CPU oracle
and the GPU library receive the arrays produced here as plain inputs.

Layout convention (Section 2.1 of the paper): a tensor X of size n_1 x ... x n_d
is a flat vector in column-major order, i_1 varying fastest.  Every unfolding
X_k is then a zero-copy column-major view with leading dimension
n_1 * ... * n_k.

Seeds: base seed 211110448; a workload with index c draws four independent
streams SeedSequence([211110448, c]).spawn(4) -> (cores, noise, left factors,
right factors), NumPy PCG64.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

BASE_SEED = 211110448


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload: shape, data recipe and sketch parameters."""
    name: str
    index: int                 # seed stream index c
    n: tuple                   # mode sizes n_1..n_d
    dtype: str                 # "f64" or "f32": element type of X in memory
    kind: str                  # "tt" (random Gaussian TT + noise) or "invsum" (Chebyshev 1/sum)
    tt_rank: int = 0           # ranks of the random TT (kind == "tt")
    noise: float = 0.0         # standard deviation of iid Gaussian noise
    unit_norm: bool = False    # scale the TT so that ||TT||_F = 1 before noise
    ell: int = 0               # sketch size (rank + oversampling)
    rank: Optional[int] = None  # target TT rank (fixed-rank mode)
    eps: Optional[float] = None  # tolerance (tolerance mode)
    rmax: int = 0              # rank cap in tolerance mode
    nslabs: int = 1            # number of contiguous slabs the tensor is delivered in
    rank_list: tuple = ()      # per-split target ranks r_1..r_{d-1} (overrides rank)
    terms: int = 0             # number of Gaussian bumps (kind == "gauss")
    gamma: float = 0.0         # their width parameter (kind == "gauss")

    @property
    def d(self) -> int:
        return len(self.n)

    @property
    def numel(self) -> int:
        return int(np.prod(self.n, dtype=np.int64))

    @property
    def itemsize(self) -> int:
        return 8 if self.dtype == "f64" else 4

    def ranks(self) -> Optional[List[int]]:
        """Target ranks r_1..r_{d-1} in fixed-rank mode, clamped to the unfolding sizes."""
        if self.rank is None and not self.rank_list:
            return None
        out = []
        for k in range(1, self.d):
            rk = int(np.prod(self.n[:k]))
            ck = int(np.prod(self.n[k:]))
            want = self.rank_list[k - 1] if self.rank_list else self.rank
            out.append(min(want, rk, ck, self.ell))
        return out


# The five workloads of the benchmark description plus scaled-down parity twins.
WORKLOADS = {
    # d=4, n=16, TT ranks 3, noise 1e-10, sketch rank 3, sketch size 6, FP64
    "c1": Workload("c1", 0, (16,) * 4, "f64", "tt", tt_rank=3, noise=1e-10, ell=6, rank=3),
    "c1_exact": Workload("c1_exact", 0, (16,) * 4, "f64", "tt", tt_rank=3, noise=0.0, ell=6, rank=3),
    # d=6, n=32 (1.07e9 entries, 8.6 GB), TT ranks 10, ||X||_F = 1, noise 1e-8, rank 10, sketch size 20, FP64
    "c2": Workload("c2", 1, (32,) * 6, "f64", "tt", tt_rank=10, noise=1e-8, unit_norm=True, ell=20, rank=10),
    # the same tensor without noise: exact-rank, recovered to rounding at full size
    "c2_exact": Workload("c2_exact", 1, (32,) * 6, "f64", "tt", tt_rank=10, noise=0.0, unit_norm=True, ell=20,
                         rank=10),
    # d=5, n=64 FP32 samples of 1/(x1+..+x5) on a Chebyshev grid over [1,2]^5, eps=1e-5, ranks <= 16, sketch size 32
    "c3": Workload("c3", 2, (64,) * 5, "f32", "invsum", ell=32, eps=1e-5, rmax=16),
    # the same samples kept in FP64 (the plain-FP64 comparator of the precision study)
    "c3_f64": Workload("c3_f64", 2, (64,) * 5, "f64", "invsum", ell=32, eps=1e-5, rmax=16),
    # d=8, n=12 FP32, TT ranks 8, noise 1e-4, rank 8, sketch size 16, 64 contiguous slabs
    "c4": Workload("c4", 3, (12,) * 8, "f32", "tt", tt_rank=8, noise=1e-4, ell=16, rank=8, nslabs=64),
    # d=4, n=48 FP32, TT ranks 6, noise 1e-3, rank 6, sketch size 12 (differentiation workload)
    "c5": Workload("c5", 4, (48,) * 4, "f32", "tt", tt_rank=6, noise=1e-3, ell=12, rank=6),
    # finite-difference instance of the differentiation workload: d=4, n=8, FP64
    "c5_fd": Workload("c5_fd", 5, (8,) * 4, "f64", "tt", tt_rank=6, noise=1e-3, ell=12, rank=6),
    # scaled-down twins: same recipe, sizes the oracle finishes in seconds, several
    # kernel tiles and a ragged tail
    "c2_small": Workload("c2_small", 11, (9, 10, 11, 8, 7, 6), "f64", "tt", tt_rank=5, noise=1e-8,
                         unit_norm=True, ell=10, rank=5),
    "c3_small": Workload("c3_small", 12, (24, 20, 19, 18, 17), "f32", "invsum", ell=32, eps=1e-5, rmax=16),
    "c4_small": Workload("c4_small", 13, (6, 5, 7, 6, 5, 6, 4, 5), "f32", "tt", tt_rank=4, noise=1e-4,
                         ell=8, rank=4, nslabs=7),
    "c5_small": Workload("c5_small", 14, (20, 17, 19, 21), "f32", "tt", tt_rank=6, noise=1e-3, ell=12, rank=6),
    # twins of the d=6 FP64 recipe at the benchmark's own sketch parameters (rank 10,
    # sketch size 20; the tests also set 24, 28, 32): 1716 x 990 middle unfolding,
    # so 7 (or 4) row blocks with a ragged last one and 62 column chunks, the last
    # with 14 columns.  The _odd twin has an odd row count (1287 x 770): its columns
    # are not 16-byte aligned, which selects the kernel's unaligned loads.
    "c2_twin": Workload("c2_twin", 15, (12, 11, 13, 10, 9, 11), "f64", "tt", tt_rank=10, noise=1e-8,
                        unit_norm=True, ell=20, rank=10),
    "c2_twin_odd": Workload("c2_twin_odd", 16, (13, 11, 9, 10, 7, 11), "f64", "tt", tt_rank=10, noise=1e-8,
                            unit_norm=True, ell=20, rank=10, nslabs=9),
    # the d=8 FP32 slab recipe at sketch size 24: a 32-wide sketch tile with 8 padding columns
    "c4_twin24": Workload("c4_twin24", 17, (6, 5, 7, 6, 5, 6, 4, 5), "f32", "tt", tt_rank=8, noise=1e-4,
                          ell=24, rank=8, nslabs=7),
    # Table 1 (Section 4.3): Hilbert tensors of order 3, 5 and 9 with the printed TT
    # ranks (6.59 GB, 60.8 GB and 38.4 GB in FP64).  Sketch size 32 (the library's
    # largest): oversampling 7 to 20.  The GPU evaluates them inside its kernels.
    "t1_d3": Workload("t1_d3", 21, (960,) * 3, "f64", "hilbert", ell=32, rank_list=(25, 25)),
    "t1_d5": Workload("t1_d5", 22, (96,) * 5, "f64", "hilbert", ell=32, rank_list=(17, 18, 18, 17)),
    "t1_d9": Workload("t1_d9", 23, (12,) * 9, "f64", "hilbert", ell=32,
                      rank_list=(12, 18, 18, 19, 19, 18, 18, 12)),
    # scaled-down Hilbert twins (ragged modes) that the oracle finishes in seconds
    "t1_small3": Workload("t1_small3", 24, (61, 47, 53), "f64", "hilbert", ell=16, rank_list=(8, 8)),
    "t1_small5": Workload("t1_small5", 25, (13, 11, 12, 9, 10), "f64", "hilbert", ell=14,
                          rank_list=(6, 7, 7, 6)),
    # Section 4.4: a sum of 100 Gaussian bumps (width parameter 10, centers uniform on
    # [-1, 1]^d) on the order-3 shape of Table 1 (n = 960, 6.59 GB in FP64, never
    # stored).  The paper prints no ranks for it; the unfoldings' singular values
    # fall below 1e-10 of the norm past about 22, so ranks 24 and sketch size 32.
    "gb_d3": Workload("gb_d3", 26, (960,) * 3, "f64", "gauss", ell=32, rank_list=(24, 24), terms=100,
                      gamma=10.0),
    # scaled-down twins (ragged modes) that the oracle finishes in seconds
    "gb_small3": Workload("gb_small3", 27, (45, 38, 41), "f64", "gauss", ell=16, rank_list=(10, 10), terms=100,
                          gamma=10.0),
    "gb_small4": Workload("gb_small4", 28, (13, 11, 12, 9), "f64", "gauss", ell=14, rank_list=(7, 9, 7),
                          terms=100, gamma=10.0),
}


def seed_streams(index: int):
    """Four independent generators (cores, noise, left factors, right factors)."""
    ss = np.random.SeedSequence([BASE_SEED, int(index)]).spawn(4)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss]


def random_tt_cores(rng: np.random.Generator, n: Sequence[int], rank: int) -> List[np.ndarray]:
    """Cores G_k of shape (s_{k-1}, n_k, s_k) with iid N(0,1) entries, s_0 = s_d = 1.

    Interior core sizes are min(rank, n_1..n_k, n_{k+1}..n_d) so that the cores
    are not trivially rank-deficient.
    """
    d = len(n)
    s = [1]
    for k in range(1, d):
        left = int(np.prod(n[:k]))
        right = int(np.prod(n[k:]))
        s.append(min(rank, left, right))
    s.append(1)
    return [rng.standard_normal((s[k], n[k], s[k + 1])) for k in range(d)]


def dense_from_cores(cores: Sequence[np.ndarray]) -> np.ndarray:
    """Column-major flat tensor whose entries are the products G_1(i_1) ... G_d(i_d).

    Built left to right: the running matrix M has one row per multi-index
    (i_1..i_k), i_1 fastest, and one column per rank index.
    """
    g0 = cores[0]
    m = g0.reshape(g0.shape[1], g0.shape[2], order="F")
    for g in cores[1:-1]:
        a, nk, b = g.shape
        m = (m @ g.reshape(a, nk * b, order="F")).reshape(m.shape[0] * nk, b, order="F")
    g = cores[-1]
    a, nk, _ = g.shape
    # X_{d-1} = M @ G_d(:, :) is R_{d-1} x n_d; its transpose in C order is the
    # column-major flat vector of X.
    xt = g.reshape(a, nk, order="F").T @ m.T
    return np.ascontiguousarray(xt).reshape(-1)


def chebyshev_points(n: int, lo: float = 1.0, hi: float = 2.0) -> np.ndarray:
    """Second-kind Chebyshev points on [lo, hi], ascending."""
    if n == 1:
        return np.array([(lo + hi) / 2.0])
    j = np.arange(n, dtype=np.float64)
    return (lo + hi) / 2.0 - (hi - lo) / 2.0 * np.cos(np.pi * j / (n - 1))


def inverse_sum_tensor(n: Sequence[int]) -> np.ndarray:
    """Samples of f(x) = 1/(x_1 + ... + x_d) on the tensor Chebyshev grid over [1,2]^d (FP64)."""
    d = len(n)
    pts = [chebyshev_points(nk) for nk in n]
    inner = np.zeros(1)
    for k in range(d - 1):  # column-major: earlier modes vary fastest
        inner = (inner[:, None] + pts[k][None, :]).reshape(-1, order="F")
    out = np.empty(int(np.prod(n)), dtype=np.float64)
    blk = inner.size
    for i, t in enumerate(pts[d - 1]):
        np.divide(1.0, inner + t, out=out[i * blk:(i + 1) * blk])
    return out


def hilbert_tensor(n: Sequence[int]) -> np.ndarray:
    """Hilbert tensor 1/(i_1 + ... + i_d - d + 1) with 1-based indices (Section 4.3)."""
    d = len(n)
    inner = np.zeros(1)
    for k in range(d - 1):
        inner = (inner[:, None] + np.arange(1, n[k] + 1, dtype=np.float64)[None, :]).reshape(-1, order="F")
    out = np.empty(int(np.prod(n)), dtype=np.float64)
    blk = inner.size
    for i in range(n[d - 1]):
        np.divide(1.0, inner + (i + 1) - d + 1, out=out[i * blk:(i + 1) * blk])
    return out


def hilbert_entries(n: Sequence[int], m: int, rows, cols) -> np.ndarray:
    """Entries X_m(rows[i], cols[j]) of the Hilbert tensor's m-th unfolding (rows: flat
    indices over modes 1..m, cols: over modes m+1..d), from the formula, as an FP64
    len(rows) x len(cols) array."""
    def index_sum(f, modes):
        f = np.asarray(f, dtype=np.int64).copy()
        s = np.zeros(f.shape, dtype=np.int64)
        for nq in modes:
            s += f % nq + 1
            f //= nq
        return s
    d = len(n)
    sr = index_sum(rows, n[:m])
    sc = index_sum(cols, n[m:])
    return 1.0 / (sr[:, None] + sc[None, :] - d + 1).astype(np.float64)


def gauss_centers(w: Workload) -> np.ndarray:
    """Centers of the Gaussian-bump tensor (Section 4.4): terms x d, iid uniform on [-1, 1],
    drawn from the workload's first stream."""
    rc, _, _, _ = seed_streams(w.index)
    return rc.uniform(-1.0, 1.0, size=(w.terms, w.d))


def gauss_grid(nq: int) -> np.ndarray:
    """Grid points x = 2 i / n - 1 of one mode, i = 1..n (Section 4.4; 1-based i)."""
    return 2.0 * np.arange(1, nq + 1, dtype=np.float64) / nq - 1.0


def gauss_tensor(n: Sequence[int], centers: np.ndarray, gamma: float) -> np.ndarray:
    """X(i) = sum_j exp(-gamma * sum_q (x_q - c_{j,q})^2), flat column-major, FP64.
    The bumps are added in increasing j; each exponent sums its modes in increasing q."""
    d = len(n)
    out = np.zeros(int(np.prod(n)), dtype=np.float64)
    for c in centers:
        e = np.zeros(1)
        for q in range(d):
            e = (e[:, None] + ((gauss_grid(n[q]) - c[q]) ** 2)[None, :]).reshape(-1, order="F")
        out += np.exp(-gamma * e)
    return out


def gauss_entries(n: Sequence[int], m: int, rows, cols, centers: np.ndarray, gamma: float) -> np.ndarray:
    """Entries X_m(rows[i], cols[j]) of the Gaussian-bump tensor's m-th unfolding, from the
    formula, as an FP64 len(rows) x len(cols) array."""
    def sq_dist(f, modes, cq):
        f = np.asarray(f, dtype=np.int64).copy()
        s = np.zeros(f.shape, dtype=np.float64)
        for nq, c in zip(modes, cq):
            s += (2.0 * (f % nq + 1) / nq - 1.0 - c) ** 2
            f //= nq
        return s
    out = np.zeros((len(rows), len(cols)), dtype=np.float64)
    for c in centers:
        out += np.exp(-gamma * (sq_dist(rows, n[:m], c[:m])[:, None] + sq_dist(cols, n[m:], c[m:])[None, :]))
    return out


def add_noise(x: np.ndarray, rng: np.random.Generator, sigma: float, chunk: int = 1 << 24) -> None:
    """In place: x += sigma * N(0,1), drawn in fixed-size chunks (deterministic for a seed)."""
    if sigma == 0.0:
        return
    for s in range(0, x.size, chunk):
        e = min(x.size, s + chunk)
        x[s:e] += sigma * rng.standard_normal(e - s)


def make_tensor(w: Workload) -> np.ndarray:
    """The workload's tensor as a flat column-major array of its dtype."""
    rc, rn, _, _ = seed_streams(w.index)
    if w.kind == "tt":
        cores = random_tt_cores(rc, w.n, w.tt_rank)
        x = dense_from_cores(cores)
        del cores
        if w.unit_norm:
            x *= 1.0 / float(np.linalg.norm(x))
        add_noise(x, rn, w.noise)
    elif w.kind == "invsum":
        x = inverse_sum_tensor(w.n)
    elif w.kind == "hilbert":
        x = hilbert_tensor(w.n)
    elif w.kind == "gauss":
        x = gauss_tensor(w.n, gauss_centers(w), w.gamma)
    else:
        raise ValueError(f"unknown tensor kind {w.kind!r}")
    if w.dtype == "f32":
        x = x.astype(np.float32)
    return x


def drm_factors(w: Workload, n: Optional[Sequence[int]] = None, ell: Optional[int] = None):
    """Gaussian Khatri-Rao factors for the nested sketch.

    Returns (psi, omega): psi[q] for modes q = 1..d-1 and omega[q] for modes
    q = 2..d (1-based keys), each an (n_q, ell) FP64 array with iid N(0,1)
    entries.  Left and right factors come from independent streams.
    """
    n = tuple(w.n if n is None else n)
    ell = w.ell if ell is None else ell
    _, _, rl, rr = seed_streams(w.index)
    d = len(n)
    psi = {q: rl.standard_normal((n[q - 1], ell)) for q in range(1, d)}
    omega = {q: rr.standard_normal((n[q - 1], ell)) for q in range(2, d + 1)}
    return psi, omega


def drm_factors_independent(w: Workload, n: Optional[Sequence[int]] = None, ell: Optional[int] = None):
    """Independent Khatri-Rao factors: one factor set per split (the paper's Psi^{(j)}).

    Returns (psi, omega) with psi[k][q] (split k, mode q <= k) and omega[k][q]
    (split k, mode q > k), 1-based, each (n_q, ell).
    """
    n = tuple(w.n if n is None else n)
    ell = w.ell if ell is None else ell
    _, _, rl, rr = seed_streams(w.index)
    d = len(n)
    psi = {k: {q: rl.standard_normal((n[q - 1], ell)) for q in range(1, k + 1)} for k in range(1, d)}
    omega = {k: {q: rr.standard_normal((n[q - 1], ell)) for q in range(k + 1, d + 1)} for k in range(1, d)}
    return psi, omega


def pack_factors(psi: dict, omega: dict, d: int) -> np.ndarray:
    """Flat FP64 buffer: psi_1..psi_{d-1} then omega_2..omega_d, each n_q x ell with ell fastest."""
    parts = [np.ascontiguousarray(psi[q], dtype=np.float64).reshape(-1) for q in range(1, d)]
    parts += [np.ascontiguousarray(omega[q], dtype=np.float64).reshape(-1) for q in range(2, d + 1)]
    return np.concatenate(parts)


def pack_factors_independent(psi: dict, omega: dict, d: int) -> np.ndarray:
    """Flat FP64 buffer for per-split factors: for split k = 1..d-1, psi[k][1..k] then omega[k][k+1..d],
    each n_q x ell with ell fastest."""
    parts = []
    for k in range(1, d):
        parts += [np.ascontiguousarray(psi[k][q], dtype=np.float64).reshape(-1) for q in range(1, k + 1)]
        parts += [np.ascontiguousarray(omega[k][q], dtype=np.float64).reshape(-1) for q in range(k + 1, d + 1)]
    return np.concatenate(parts)


# ---- counter-based Gaussian stream (the library's seeded factors) ----
# Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
# as 1, 2, 3", SC 2011) and the Box-Muller transform, written from their
# published definitions.  Entry j of the stream: p = j // 2, four 32-bit words
# x = Philox4x32-10(counter (p mod 2^32, p div 2^32, 0, 0), key (seed mod 2^32,
# seed div 2^32)); u1 = 1 - ((x0 >> 5) 2^26 + (x1 >> 6)) / 2^53,
# u2 = ((x2 >> 5) 2^26 + (x3 >> 6)) / 2^53; entry 2p = sqrt(-2 ln u1) cos(2 pi u2)
# and entry 2p + 1 = sqrt(-2 ln u1) sin(2 pi u2).
_PHILOX_M = (0xD2511F53, 0xCD9E8D57)     # round multipliers
_PHILOX_W = (0x9E3779B9, 0xBB67AE85)     # Weyl key increments
_U32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(counters: np.ndarray, seed: int) -> np.ndarray:
    """Philox4x32-10 of 64-bit block counters (words (c mod 2^32, c div 2^32, 0, 0)) under a 64-bit key.

    Returns an (len(counters), 4) uint64 array of the four 32-bit output words.
    """
    c = np.asarray(counters, dtype=np.uint64)
    w0, w1 = c & _U32, c >> np.uint64(32)
    w2 = np.zeros_like(c)
    w3 = np.zeros_like(c)
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _PHILOX_W[0]) & 0xFFFFFFFF
            k1 = (k1 + _PHILOX_W[1]) & 0xFFFFFFFF
        p0 = np.uint64(_PHILOX_M[0]) * w0          # < 2^64: exact in uint64
        p1 = np.uint64(_PHILOX_M[1]) * w2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _U32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _U32
        w0, w1, w2, w3 = hi1 ^ w1 ^ np.uint64(k0), lo1, hi0 ^ w3 ^ np.uint64(k1), lo0
    return np.stack([w0, w1, w2, w3], axis=1)


def philox_normals(seed: int, count: int, first: int = 0) -> np.ndarray:
    """Entries first .. first + count - 1 of the seeded standard-normal stream above."""
    j = np.arange(first, first + count, dtype=np.uint64)
    x = philox4x32_10(j >> np.uint64(1), seed)
    def unit53(a, b):
        return ((a >> np.uint64(5)).astype(np.float64) * 67108864.0 + (b >> np.uint64(6)).astype(np.float64)) \
            / 9007199254740992.0
    u1 = 1.0 - unit53(x[:, 0], x[:, 1])
    u2 = unit53(x[:, 2], x[:, 3])
    two_pi = 2.0 * math.pi
    out = np.empty(count)
    # the C library's log / sqrt / cos / sin, one value at a time (as the host code does)
    for t in range(count):
        rad = math.sqrt(-2.0 * math.log(float(u1[t])))
        ang = two_pi * float(u2[t])
        out[t] = rad * (math.sin(ang) if (first + t) & 1 else math.cos(ang))
    return out


def seeded_factors(n: Sequence[int], ell: int, seed: int, drm: str = "nested"):
    """The factors a context draws from `seed` (no caller factors): the stream cut into
    the packed layout.  Returns (psi, omega) like drm_factors / drm_factors_independent."""
    d = len(n)
    if drm == "nested":
        sizes = [("psi", q) for q in range(1, d)] + [("omega", q) for q in range(2, d + 1)]
    else:
        sizes = []
        for k in range(1, d):
            sizes += [("psi", k, q) for q in range(1, k + 1)] + [("omega", k, q) for q in range(k + 1, d + 1)]
    total = sum(n[key[-1] - 1] * ell for key in sizes)
    z = philox_normals(seed, total)
    psi, omega, o = {}, {}, 0
    for key in sizes:
        nq = n[key[-1] - 1]
        blk = z[o:o + nq * ell].reshape(nq, ell)
        o += nq * ell
        tgt = psi if key[0] == "psi" else omega
        if drm == "nested":
            tgt[key[1]] = blk
        else:
            tgt.setdefault(key[1], {})[key[2]] = blk
    return psi, omega


def slab_bounds(numel: int, fiber: int, nslabs: int):
    """Split [0, numel) into nslabs contiguous runs of whole fibers of length `fiber`.

    Returns a list of (first, count).  Slab sizes differ by at most one fiber.
    """
    nf = numel // fiber
    out = []
    start = 0
    for s in range(nslabs):
        nf_s = nf // nslabs + (1 if s < nf % nslabs else 0)
        out.append((start * fiber, nf_s * fiber))
        start += nf_s
    return out
