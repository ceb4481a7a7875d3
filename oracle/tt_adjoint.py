"""Adjoint of PSTT2-onepass for the oracle -- TEST INFRASTRUCTURE ONLY.

Imported only by tests (and the smoke check).  The product path never calls it.

The one-pass approximation X~ depends on X only through the sketches, which
are linear in X.  The discrete choices (CPQR pivots and ranks) are piecewise
constant, so the derivative is taken with them frozen at the values of the
forward pass: each basis is then the thin QR factor (sign-fixed, diag R >= 0)
of the first r_k pivoted columns of its sketch, which is the leading part of
the pivoted factor that the forward pass uses (Algorithm PSTT, CPQR step).

Both DRM schemes (nested and independent Khatri-Rao factors) are covered
through the DRM object, and both one-pass middle-core rules: the rule of
equation "onepass_final_core" (middle="onepass") and the two-sided rule that
also sketches the leading outer mode with split (m-1)'s left DRM
(middle="twosided", oracle.tt_sketch.middle_core_twosided).

Contents
  pstt2_frozen   numpy forward X -> TT cores with given pivots and ranks; every
                 step is a call into oracle.tt_sketch (sketches of Section 3.2,
                 cores by equation "core" and its row mirror, middle core by
                 equation "onepass_final_core" or the two-sided rule).
  pstt2_vjp      J^T gbar and the gradient of ||X - X~||_F^2, by torch CPU FP64
                 autograd of an independent torch transcription of the same
                 forward pass.

Parity pins (tests/test_oracle_adjoint.py): pstt2_frozen reproduces pstt2's
cores; pstt2_vjp agrees with central finite differences of pstt2_frozen in
random directions and, on a 4096-entry tensor, entry by entry, for each
middle-core rule and DRM scheme.
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence

import numpy as np

from . import tt_sketch as O

__all__ = ["pstt2_frozen", "pstt2_vjp"]


def _frozen_basis(s: np.ndarray, piv: np.ndarray, r: int) -> np.ndarray:
    """Thin QR basis of the first r pivoted columns of S, sign-fixed (diag R >= 0)."""
    q, rr = np.linalg.qr(s[:, np.asarray(piv[:r])], mode="reduced")
    sgn = np.where(np.diag(rr) < 0.0, -1.0, 1.0)
    return q * sgn[None, :]


def pstt2_frozen(x: np.ndarray, n: Sequence[int], drm, ranks: Sequence[int], piv: Dict[int, np.ndarray],
                 middle: str = "onepass"):
    """PSTT2-onepass cores of X with the pivots and ranks of an earlier pass held fixed."""
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    n = tuple(int(v) for v in n)
    d = len(n)
    m = O.middle_index(d)
    r = [1] + list(ranks) + [1]
    q = {0: np.ones((1, 1))}
    for k in range(1, m):
        q[k] = _frozen_basis(O.sketch_right_dense(x, n, k, drm.omega_dense(k, d)), piv[k], r[k])
    p = {}
    for k in range(m, d):
        p[k] = _frozen_basis(O.sketch_left_dense(x, n, k, drm.psi_dense(k)).T, piv[k], r[k])
    cores = [None] * d
    for k in range(1, m):
        cores[k - 1] = (np.reshape(q[1], (1, n[0], r[1]), order="F") if k == 1
                        else O.outer_core_left(q[k - 1], q[k], n[k - 1]))
    for k in range(m + 1, d + 1):
        cores[k - 1] = (np.reshape(p[d - 1].T, (r[d - 1], n[d - 1], 1), order="F") if k == d
                        else O.outer_core_right(p[k - 1], p[k], n[k - 1]))
    om = drm.omega_dense(m, d)
    y_r = O.sketch_right_dense(x, n, m, om)
    if middle == "twosided" and m >= 2:
        cores[m - 1] = O.middle_core_twosided(y_r, drm.psi_dense(m - 1), q[m - 1], om, p[m], n[m - 1])
    elif middle in ("onepass", "twosided"):
        cores[m - 1] = O.middle_core_onepass(y_r, om, q[m - 1], p[m], n[m - 1])
    else:
        raise ValueError(middle)
    return cores


def _torch_forward(xt, n, drm, ranks, piv, middle="onepass"):
    """Torch transcription of pstt2_frozen (same steps, differentiable in X)."""
    import torch
    d = len(n)
    m = O.middle_index(d)
    r = [1] + list(ranks) + [1]

    def unfold(k):
        return xt.reshape(int(np.prod(n[k:])), int(np.prod(n[:k]))).T   # column-major X_k

    def basis(s, pv, rk):
        qq, rr = torch.linalg.qr(s[:, torch.as_tensor(np.asarray(pv[:rk]), dtype=torch.long)], mode="reduced")
        sgn = torch.where(torch.diagonal(rr) < 0, -1.0, 1.0).to(qq.dtype)
        return qq * sgn[None, :]

    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)
    q = {0: torch.ones((1, 1), dtype=torch.float64)}
    for k in range(1, m):
        q[k] = basis(unfold(k) @ t(drm.omega_dense(k, d)), piv[k], r[k])
    p = {}
    for k in range(m, d):
        p[k] = basis((t(drm.psi_dense(k)).T @ unfold(k)).T, piv[k], r[k])

    def fres(a, shape):   # column-major reshape
        at = a.permute(*reversed(range(a.dim()))).reshape(tuple(reversed(shape)))
        return at.permute(*reversed(range(len(shape))))

    cores = [None] * d
    for k in range(1, m):
        if k == 1:
            cores[0] = fres(q[1], (1, n[0], r[1]))
        else:
            w = q[k - 1].T @ fres(q[k], (q[k - 1].shape[0], n[k - 1] * r[k]))
            cores[k - 1] = fres(w, (r[k - 1], n[k - 1], r[k]))
    for k in range(m + 1, d + 1):
        if k == d:
            cores[d - 1] = fres(p[d - 1].T, (r[d - 1], n[d - 1], 1))
        else:
            p3 = fres(p[k - 1], (n[k - 1], p[k].shape[0], r[k - 1]))
            cores[k - 1] = torch.einsum("ica,cb->aib", p3, p[k])
    om = t(drm.omega_dense(m, d))
    y_r = unfold(m) @ om
    ell = om.shape[1]
    rp = q[m - 1].shape[0]
    y3 = fres(y_r, (rp, n[m - 1], ell))
    if middle == "twosided" and m >= 2:
        # H = Y3 x_1 Psi'^T; G = H x_1 (Psi'^T Q)^+ x_3 (Omega^T P)^+, each
        # pseudo-inverse of a full-column-rank B written as (B^T B)^{-1} B^T
        psi = t(drm.psi_dense(m - 1))
        h = torch.einsum("ra,rjc->ajc", psi, y3)
        b1 = psi.T @ q[m - 1]
        b3 = om.T @ p[m]
        w1 = torch.linalg.solve(b1.T @ b1, b1.T)
        w3 = torch.linalg.solve(b3.T @ b3, b3.T)
        g = fres(torch.einsum("pa,ajc,qc->pjq", w1, h, w3), (r[m - 1] * n[m - 1], r[m]))
    else:
        z = fres(torch.einsum("ra,rjc->ajc", q[m - 1], y3), (r[m - 1] * n[m - 1], ell))
        a = p[m].T @ om
        # G = Z A^+ with A^+ = A^T (A A^T)^{-1} (A has full row rank r_m <= ell)
        g = torch.linalg.solve(a @ a.T, a @ z.T).T
    cores[m - 1] = fres(g, (r[m - 1], n[m - 1], r[m]))
    # X~ by the entry formula, swept left to right (Section 2.2)
    mm = torch.ones((1, 1), dtype=torch.float64)
    for gk in cores:
        a_, nk, b_ = gk.shape
        mm = fres(torch.einsum("ra,aib->rib", mm, gk), (mm.shape[0] * nk, b_))
    return mm[:, 0]


def pstt2_vjp(x: np.ndarray, n: Sequence[int], drm, ranks: Sequence[int], piv: Dict[int, np.ndarray],
              gbar: Optional[np.ndarray] = None, middle: str = "onepass") -> np.ndarray:
    """J^T gbar (J = dX~/dX, pivots and ranks frozen), or with gbar None the gradient of ||X - X~||_F^2.

    All arrays are flat column-major FP64.
    """
    import torch
    n = tuple(int(v) for v in n)
    xt = torch.tensor(np.asarray(x, dtype=np.float64).reshape(-1), requires_grad=True)
    xtil = _torch_forward(xt, n, drm, ranks, piv, middle)
    if gbar is None:
        loss = torch.sum((xt - xtil) ** 2)
        (gx,) = torch.autograd.grad(loss, xt)
    else:
        (gx,) = torch.autograd.grad(xtil, xt, grad_outputs=torch.as_tensor(np.asarray(gbar, dtype=np.float64)))
    return gx.detach().numpy().copy()


def reconstruct_frozen_torch(x, n, drm, ranks, piv, middle="onepass") -> np.ndarray:
    """X~ from the torch transcription (no gradient): ties the two forward passes together."""
    import torch
    with torch.no_grad():
        xt = torch.as_tensor(np.asarray(x, dtype=np.float64).reshape(-1))
        return _torch_forward(xt, tuple(int(v) for v in n), drm, ranks, piv, middle).numpy().copy()
