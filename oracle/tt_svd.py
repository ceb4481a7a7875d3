"""TT-SVD and Parallel-TTSVD (paper Sections 2.2 and 3.1) -- TEST INFRASTRUCTURE ONLY.

A deterministic second reference for the PSTT2 oracle: reference ranks and
errors on the same inputs.

Parity pins (tests/test_oracle_pstt2.py: test_ttsvd_exact_and_bound and
test_inverse_sum_is_low_rank): exact recovery of exact-rank TTs; the error
bound ||X - X~||_F <= eps ||X||_F of Section 2.2; Parallel-TTSVD (Algorithm
Parallel-TTSVD) reaching the same bound (Theorem 2).  The GPU Parallel-TTSVD
is compared with parallel_ttsvd in tests/test_gpu_ttsvd.py.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np


def _trunc_rank(sig: np.ndarray, delta: float) -> int:
    """Smallest r with sqrt(sum_{i>r} sigma_i^2) <= delta (at least 1)."""
    tail2 = np.concatenate([np.cumsum((sig ** 2)[::-1])[::-1], [0.0]])  # tail2[r] = sum_{i>=r}
    r = int(np.argmax(tail2 <= delta * delta))
    return max(1, r)


def ttsvd(x: np.ndarray, n: Sequence[int], eps: Optional[float] = None,
          ranks: Optional[Sequence[int]] = None) -> List[np.ndarray]:
    """Sequential TT-SVD: truncate each SVD to eps ||X||_F / sqrt(d-1) (Section 2.2).

    With `ranks` given, truncate to those ranks instead.
    """
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    d = len(n)
    delta = None
    if ranks is None:
        delta = eps * np.linalg.norm(x) / np.sqrt(max(d - 1, 1))
    cores = []
    r_prev = 1
    c = x.copy()
    for k in range(d - 1):
        c = c.reshape(r_prev * n[k], -1, order="F")
        u, s, vt = np.linalg.svd(c, full_matrices=False)
        r = _trunc_rank(s, delta) if ranks is None else min(int(ranks[k]), len(s))
        cores.append(u[:, :r].reshape(r_prev, n[k], r, order="F"))
        c = (s[:r, None] * vt[:r, :]).reshape(-1, order="F")
        r_prev = r
    cores.append(c.reshape(r_prev, n[d - 1], 1, order="F"))
    return cores


def parallel_ttsvd(x: np.ndarray, n: Sequence[int], eps: float) -> List[np.ndarray]:
    """Algorithm Parallel-TTSVD: SVD of every unfolding, then cores from neighbouring bases.

    U_j from a truncated SVD of X_j with ||X_j - U_j S_j V_j^T||_F <= eps ||X|| / sqrt(d-1);
    G_1 = U_1, G_{k+1} = reshape(U_k^T reshape(U_{k+1}, ...)), G_d = S_{d-1} V_{d-1}^T.
    """
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    d = len(n)
    delta = eps * np.linalg.norm(x) / np.sqrt(max(d - 1, 1))
    u = {}
    last = None
    for j in range(1, d):
        xj = x.reshape(int(np.prod(n[:j])), -1, order="F")
        uu, s, vt = np.linalg.svd(xj, full_matrices=False)
        r = _trunc_rank(s, delta)
        u[j] = uu[:, :r]
        if j == d - 1:
            last = s[:r, None] * vt[:r, :]
    cores = [u[1].reshape(1, n[0], u[1].shape[1], order="F")]
    for k in range(1, d - 1):
        rk = u[k].shape[1]
        rk1 = u[k + 1].shape[1]
        w = u[k].T @ u[k + 1].reshape(u[k].shape[0], n[k] * rk1, order="F")
        cores.append(w.reshape(rk, n[k], rk1, order="F"))
    cores.append(last.reshape(last.shape[0], n[d - 1], 1, order="F"))
    return cores
