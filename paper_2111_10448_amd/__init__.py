"""MI355X PSTT2: streaming two-sided sketching tensor-train decomposition.

Thin Python binding of libpstt2 (C ABI in include/pstt2.h).  Every step of the
method runs in the library's HIP kernels; this module only marshals
arguments.  PyTorch provides device memory (tensors) and the current HIP
stream.

    import paper_2111_10448_amd as P
    ctx = P.PSTT2(n, ell, factors, dtype="f32", prec="bf16x3", eps=1e-5, rmax=16)
    ctx.sketch(x_gpu)              # one pass over X (or several slabs)
    tt = ctx.recover()             # TT cores on the GPU
    err = tt.error(x_gpu)          # ||X - X~||_F / ||X||_F
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np

from . import _lib as L
from ._lib import PSTT2Error  # noqa: F401

__all__ = ["PSTT2", "TT", "PSTT2Error", "GaussBumps", "decompose", "tt_error", "tt_error_fn", "tt_reconstruct", "version", "cores_struct",
           "PSTT2Reconstruct", "pstt2_reconstruct", "set_memory_limit", "memory_stats", "inject_launch_failure",
           "drm_factors_from_seed", "parallel_ttsvd"]


def _torch():
    import torch
    return torch


def _stream_handle(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return L.F64
    if t.dtype == torch.float32:
        return L.F32
    raise TypeError(f"X must be float64 or float32, got {t.dtype}")


def _check_dev(t):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor (flat column-major slab)")


def version() -> str:
    return L.lib().pstt2_version().decode()


def parallel_ttsvd(x, n: Sequence[int], eps: float, rmax: int = 0, stream=None) -> "TT":
    """Algorithm Parallel-TTSVD on the GPU: truncated SVDs of every unfolding (one-sided
    Jacobi), cores by equation "core".  x: flat column-major FP64 CUDA tensor."""
    _check_dev(x)
    if _dtype_code(x) != L.F64:
        raise TypeError("Parallel-TTSVD takes an FP64 tensor")
    nn = (ctypes.c_int64 * len(n))(*[int(v) for v in n])
    cs = L.TTCores()
    L.check(L.lib().pstt2_parallel_ttsvd(len(n), nn, ctypes.c_void_p(x.data_ptr()), float(eps), int(rmax),
                                         ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(cs)))
    return TT(cs, stream)


def drm_factors_from_seed(n: Sequence[int], ell: int, seed: int, drm: str = "nested") -> np.ndarray:
    """The packed factors a context with no caller factors draws from `seed` (host only)."""
    desc = L.Desc()
    desc.d = len(n)
    for k, v in enumerate(n):
        desc.n[k] = int(v)
    desc.ell = int(ell)
    desc.drm = L.DRM[drm]
    desc.seed = int(seed)
    cnt = ctypes.c_int64(0)
    L.check(L.lib().pstt2_drm_factors(ctypes.byref(desc), None, ctypes.byref(cnt)))
    out = np.empty(cnt.value)
    L.check(L.lib().pstt2_drm_factors(ctypes.byref(desc), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      ctypes.byref(cnt)))
    return out


def set_memory_limit(nbytes: int) -> None:
    """Device-memory budget of the library in bytes (<= 0: none)."""
    L.check(L.lib().pstt2_set_memory_limit(int(nbytes)))


def memory_stats() -> dict:
    """Live and peak device bytes held by the library, and the budget (-1: none)."""
    live, peak, lim = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    L.check(L.lib().pstt2_memory_stats(ctypes.byref(live), ctypes.byref(peak), ctypes.byref(lim)))
    return {"live": live.value, "peak": peak.value, "limit": lim.value}


def inject_launch_failure(count: int) -> None:
    """Testing hook: the launch after the next `count` streaming launches is reported as failed."""
    L.check(L.lib().pstt2_inject_launch_failure(int(count)))


class TT:
    """Tensor-train cores produced by the library (device memory)."""

    def __init__(self, cs: L.TTCores, stream=None):
        self._c = cs
        self._stream = stream

    @property
    def d(self) -> int:
        return self._c.d

    @property
    def n(self) -> List[int]:
        return [int(self._c.n[k]) for k in range(self._c.d)]

    @property
    def ranks(self) -> List[int]:
        return [int(self._c.r[k]) for k in range(self._c.d + 1)]

    def struct(self) -> L.TTCores:
        return self._c

    def cores_torch(self):
        """Copies of the cores as flat FP64 CUDA tensors (column-major r_{k-1} x n_k x r_k)."""
        torch = _torch()
        out = []
        dst = L.TTCores()
        dst.d = self._c.d
        for k in range(self._c.d):
            dst.n[k] = self._c.n[k]
            sz = self._c.r[k] * self._c.n[k] * self._c.r[k + 1]
            t = torch.empty(int(sz), dtype=torch.float64, device="cuda")
            out.append(t)
            dst.core[k] = t.data_ptr()
        for k in range(self._c.d + 1):
            dst.r[k] = self._c.r[k]
        L.check(L.lib().tt_cores_copy(ctypes.byref(self._c), ctypes.byref(dst), _stream_handle(self._stream)))
        return out

    def cores_numpy(self) -> List[np.ndarray]:
        """Host copies shaped (r_{k-1}, n_k, r_k)."""
        r = self.ranks
        n = self.n
        return [t.cpu().numpy().reshape((r[k], n[k], r[k + 1]), order="F")
                for k, t in enumerate(self.cores_torch())]

    def error(self, x) -> float:
        return tt_error(self, x, stream=self._stream)

    def error_fn(self, fn="hilbert") -> float:
        """Relative error against a tensor given by a formula (see PSTT2.sketch_fn)."""
        return tt_error_fn(self, fn, stream=self._stream)

    def reconstruct(self, first: int = 0, count: Optional[int] = None, dtype=None):
        return tt_reconstruct(self, first, count, dtype, stream=self._stream)

    def free(self) -> None:
        if self._c is not None and self._c.owned:
            L.lib().tt_cores_free(ctypes.byref(self._c))
        self._c = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def cores_struct(cores: Sequence, n: Sequence[int], ranks: Sequence[int]) -> L.TTCores:
    """A non-owning tt_cores view of caller cores.

    cores[k] is a contiguous FP64 CUDA tensor holding core k column-major
    (element (a, i, b) at a + r_k (i + n_k b)); ranks = (1, r_1, ..., r_{d-1}, 1).
    Keep the tensors alive while the struct is used.
    """
    torch = _torch()
    cs = L.TTCores()
    d = len(n)
    if len(ranks) != d + 1 or ranks[0] != 1 or ranks[d] != 1:
        raise ValueError("ranks must be (1, r_1, ..., r_{d-1}, 1)")
    cs.d = d
    cs.owned = 0
    for k in range(d):
        t = cores[k]
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise TypeError("cores must be contiguous float64 CUDA tensors")
        if t.numel() != ranks[k] * n[k] * ranks[k + 1]:
            raise ValueError(f"core {k} has {t.numel()} entries, expected {ranks[k] * n[k] * ranks[k + 1]}")
        cs.n[k] = int(n[k])
        cs.core[k] = t.data_ptr()
    for k in range(d + 1):
        cs.r[k] = int(ranks[k])
    return cs


class PSTT2:
    """A PSTT2-onepass (or two-pass) context: DRM factors, sketches, slab coverage."""

    def __init__(self, n: Sequence[int], ell: int, factors: Optional[np.ndarray] = None, *, dtype: str = "f64",
                 prec: Optional[str] = None, ranks: Optional[Sequence[int]] = None, eps: Optional[float] = None,
                 rmax: int = 0, mid: str = "onepass", drm: str = "nested", algo: str = "pstt2", stream=None,
                 seed: int = 0):
        """factors: the packed DRM factors (host), or None to have the library draw
        them from `seed` (see drm_factors_from_seed)."""
        self.n = [int(v) for v in n]
        self.d = len(self.n)
        self.ell = int(ell)
        self.dtype = dtype
        prec = prec or dtype
        self._stream = stream
        desc = L.Desc()
        desc.d = self.d
        for k, v in enumerate(self.n):
            desc.n[k] = v
        desc.dtype = L.F64 if dtype == "f64" else L.F32
        desc.prec = L.PREC[prec]
        desc.mid = L.MID[mid]
        desc.drm = L.DRM[drm]
        desc.algo = L.ALGO[algo]
        if ranks is not None:
            for k, v in enumerate(ranks):
                desc.ranks[k] = int(v)
        else:
            desc.ranks[0] = 0
            desc.eps = float(eps if eps is not None else 0.0)
            desc.rmax = int(rmax)
        desc.ell = self.ell
        desc.seed = int(seed)
        if factors is None:
            self._fac = None
            desc.drm_factors = None
        else:
            self._fac = np.ascontiguousarray(factors, dtype=np.float64)
            desc.drm_factors = self._fac.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self._ctx = ctypes.c_void_p()
        L.check(L.lib().pstt2_create(ctypes.byref(desc), ctypes.c_void_p(_stream_handle(stream)),
                                     ctypes.byref(self._ctx)))
        self._keep = []   # slabs kept alive until the stream passes them

    def _c(self):
        if not self._ctx:
            raise RuntimeError("context closed")
        return self._ctx

    def sketch(self, x, first: int = 0) -> None:
        """Stream a flat column-major slab of X starting at flat index `first` (async)."""
        _check_dev(x)
        self._keep.append(x)
        L.check(L.lib().pstt2_sketch(self._c(), ctypes.c_void_p(x.data_ptr()), int(first), int(x.numel())),
                self._ctx)

    def sketch_fn(self, fn="hilbert", first: int = 0, count: Optional[int] = None) -> None:
        """Stream entries [first, first + count) of a tensor given by a formula of its
        indices: "hilbert" (1 / (1 - d + i_1 + ... + i_d), evaluated inside the kernel)
        or a GaussBumps.  first and count are multiples of n_1...n_m; count defaults to
        the rest (async)."""
        f = _fn_struct(fn, len(self.n))
        if count is None:
            count = int(np.prod(self.n)) - int(first)
        L.check(L.lib().pstt2_sketch_fn(self._c(), ctypes.byref(f), int(first), int(count)), self._ctx)

    def sketch_slabs(self, xs: Sequence, firsts: Sequence[int]) -> None:
        """Stream several slabs in one launch (async)."""
        ns = len(xs)
        ptrs = (ctypes.c_void_p * ns)()
        fs = (ctypes.c_int64 * ns)()
        cs = (ctypes.c_int64 * ns)()
        for i, (x, f) in enumerate(zip(xs, firsts)):
            _check_dev(x)
            ptrs[i] = x.data_ptr()
            fs[i] = int(f)
            cs[i] = int(x.numel())
        self._keep.extend(xs)
        L.check(L.lib().pstt2_sketch_slabs(self._c(), ns, ptrs, fs, cs), self._ctx)

    def recover(self) -> TT:
        cs = L.TTCores()
        L.check(L.lib().pstt2_recover(self._c(), ctypes.byref(cs)), self._ctx)
        self._keep = []
        return TT(cs, self._stream)

    def recover_certified(self, x=None, fn: Optional[str] = None, max_tries: int = 8):
        """Tolerance mode: recover, measure the error against x (or the tensor function
        fn), and recover again from the same sketches with a tighter rank rule while it
        exceeds eps.  Returns (TT, relative error)."""
        if (x is None) == (fn is None):
            raise ValueError("give exactly one of x and fn")
        if x is not None:
            _check_dev(x)
        fp = None
        if fn is not None:
            fs = _fn_struct(fn, len(self.n))
            fp = ctypes.byref(fs)
        cs = L.TTCores()
        err = ctypes.c_double()
        L.check(L.lib().pstt2_recover_certified(self._c(), ctypes.c_void_p(x.data_ptr() if x is not None else 0), fp,
                                                int(max_tries), ctypes.byref(cs), ctypes.byref(err)), self._ctx)
        self._keep = []
        return TT(cs, self._stream), err.value

    def middle_pass(self, tt: TT, x, first: int = 0) -> None:
        _check_dev(x)
        L.check(L.lib().pstt2_middle_pass(self._c(), ctypes.byref(tt.struct()), ctypes.c_void_p(x.data_ptr()),
                                          int(first), int(x.numel())), self._ctx)
        self._keep.append(x)

    def middle_pass_fn(self, tt: TT, fn="hilbert", first: int = 0, count: Optional[int] = None) -> None:
        """The two-pass middle core's second pass over a tensor function ("hilbert" or a
        GaussBumps), evaluated in workspace chunks; count defaults to the rest."""
        f = _fn_struct(fn, len(self.n))
        if count is None:
            count = int(np.prod(self.n)) - int(first)
        L.check(L.lib().pstt2_middle_pass_fn(self._c(), ctypes.byref(tt.struct()), ctypes.byref(f), int(first),
                                             int(count)), self._ctx)

    def vjp(self, tt: "TT", x=None, gbar=None):
        """J^T gbar for X~ = the one-pass approximation (either one-pass middle-core
        rule, either DRM scheme; pivots and ranks of the last recover held fixed);
        with gbar None, the gradient of ||X - X~||_F^2 (needs x).
        Returns a flat CUDA tensor of the context's dtype."""
        torch = _torch()
        ref = gbar if gbar is not None else x
        if ref is None:
            raise ValueError("give gbar, or x for the Frobenius-loss gradient")
        for t in (x, gbar):
            if t is not None:
                _check_dev(t)
        gx = torch.empty(ref.numel(), dtype=ref.dtype, device=ref.device)
        L.check(L.lib().pstt2_vjp(self._c(), ctypes.byref(tt.struct()),
                                  ctypes.c_void_p(x.data_ptr() if x is not None else 0),
                                  ctypes.c_void_p(gbar.data_ptr() if gbar is not None else 0),
                                  ctypes.c_void_p(gx.data_ptr())), self._ctx)
        return gx

    def get_sketch(self, which: int, k: int) -> np.ndarray:
        """which = 0: right sketch of split k (R_k x ell); 1: transposed left sketch (C_k x ell);
        2: two-sided sketch B_k = Psi_k^T X_k Omega_k (ell x ell); 3: two-sided middle sketch H
        ((ell n_m) x ell, mid="twosided")."""
        rows = ctypes.c_int64()
        cols = ctypes.c_int64()
        L.check(L.lib().pstt2_get_sketch(self._c(), which, k, None, ctypes.byref(rows), ctypes.byref(cols)),
                self._ctx)
        out = np.empty(rows.value * cols.value, dtype=np.float64)
        L.check(L.lib().pstt2_get_sketch(self._c(), which, k, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         ctypes.byref(rows), ctypes.byref(cols)), self._ctx)
        return out.reshape((rows.value, cols.value), order="F")

    def pivots(self, k: int) -> np.ndarray:
        out = (ctypes.c_int32 * self.ell)()
        L.check(L.lib().pstt2_get_pivots(self._c(), k, out), self._ctx)
        return np.array(out[:], dtype=np.int64)

    def profile(self, enable: bool = True) -> None:
        """Bracket every later sketch-kernel launch with HIP events on the context's stream."""
        L.check(L.lib().pstt2_profile(self._c(), 1 if enable else 0), self._ctx)

    def profile_read(self):
        """(total milliseconds, launches) of the sketch kernel since the last read."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        L.check(L.lib().pstt2_profile_read(self._c(), ctypes.byref(ms), ctypes.byref(n)), self._ctx)
        return ms.value, n.value

    def reset(self) -> None:
        L.check(L.lib().pstt2_reset(self._c()), self._ctx)
        self._keep = []

    def close(self) -> None:
        if self._ctx:
            L.lib().pstt2_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()
        self._keep = []

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tt_error(tt, x, stream=None) -> float:
    """||X - X~||_F / ||X||_F over one streaming pass (FP64 sums)."""
    _check_dev(x)
    cs = tt.struct() if isinstance(tt, TT) else tt
    out = ctypes.c_double()
    L.check(L.lib().tt_error(ctypes.byref(cs), ctypes.c_void_p(x.data_ptr()), _dtype_code(x), ctypes.byref(out),
                             ctypes.c_void_p(_stream_handle(stream))))
    return out.value


class GaussBumps:
    """The Gaussian-bump tensor X(i) = sum_j exp(-gamma sum_q (x_q - c_{j,q})^2),
    x_q = 2 i_q / n_q - 1 with 1-based i_q (Section 4.4).  centers: n_terms x d."""

    def __init__(self, centers, gamma: float):
        self.centers = np.ascontiguousarray(np.asarray(centers, dtype=np.float64))
        if self.centers.ndim != 2 or not 1 <= self.centers.shape[0] <= L.GAUSS_MAX_TERMS:
            raise ValueError("centers must be n_terms x d with 1 <= n_terms <= %d" % L.GAUSS_MAX_TERMS)
        self.gamma = float(gamma)


def _fn_struct(fn, d: int) -> "L.Fn":
    """The C description of a tensor function of order d: "hilbert" or a GaussBumps
    (whose centers array the struct points into; the library copies it during the call)."""
    if isinstance(fn, GaussBumps):
        if fn.centers.shape[1] != d:
            raise ValueError(f"centers have {fn.centers.shape[1]} coordinates, the tensor has order {d}")
        return L.Fn(L.FN["gauss"], fn.centers.shape[0], fn.gamma, fn.centers.ctypes.data)
    if fn != "hilbert":
        raise ValueError(f"unknown tensor function {fn!r}")
    return L.Fn(L.FN["hilbert"])


def tt_error_fn(tt, fn="hilbert", stream=None) -> float:
    """||X - X~||_F / ||X||_F for a tensor given by a formula ("hilbert" or a GaussBumps)."""
    cs = tt.struct() if isinstance(tt, TT) else tt
    f = _fn_struct(fn, cs.d)
    out = ctypes.c_double()
    L.check(L.lib().tt_error_fn(ctypes.byref(cs), ctypes.byref(f), ctypes.byref(out),
                                ctypes.c_void_p(_stream_handle(stream))))
    return out.value


def tt_reconstruct(tt, first: int = 0, count: Optional[int] = None, dtype=None, stream=None):
    """Entries [first, first+count) of X~ as a flat CUDA tensor (FP64 by default)."""
    torch = _torch()
    cs = tt.struct() if isinstance(tt, TT) else tt
    n = [int(cs.n[k]) for k in range(cs.d)]
    total = int(np.prod(n))
    if count is None:
        count = total - first
    dtype = dtype or torch.float64
    out = torch.empty(int(count), dtype=dtype, device="cuda")
    L.check(L.lib().tt_reconstruct(ctypes.byref(cs), ctypes.c_void_p(out.data_ptr()), _dtype_code(out), int(first),
                                   int(count), ctypes.c_void_p(_stream_handle(stream))))
    return out


def decompose(x, n: Sequence[int], ell: int, factors: np.ndarray, *, prec: Optional[str] = None,
              ranks: Optional[Sequence[int]] = None, eps: Optional[float] = None, rmax: int = 0,
              mid: str = "onepass", drm: str = "nested") -> TT:
    """One-shot PSTT2 of a whole flat column-major CUDA tensor."""
    dtype = "f64" if _dtype_code(x) == L.F64 else "f32"
    with PSTT2(n, ell, factors, dtype=dtype, prec=prec, ranks=ranks, eps=eps, rmax=rmax, mid=mid,
               drm=drm) as ctx:
        ctx.sketch(x.reshape(-1))
        tt = ctx.recover()
        if mid == "twopass":
            ctx.middle_pass(tt, x.reshape(-1))
            _torch().cuda.synchronize()
        return tt


def _make_function():
    torch = _torch()

    class PSTT2Reconstruct(torch.autograd.Function):
        """X -> X~ (PSTT2-onepass then the entry formula) with the hand-written adjoint.

        forward(x, n, ell, factors, prec, ranks, eps, rmax, mid, drm): x is a flat
        column-major CUDA tensor; mid is "onepass" or "twosided", drm "nested" or
        "independent"; returns X~ in x's dtype.  backward runs pstt2_vjp with the
        forward pass's pivots and ranks held fixed; gradients flow to x only.
        """

        @staticmethod
        def forward(ctx, x, n, ell, factors, prec=None, ranks=None, eps=None, rmax=0, mid="onepass",
                    drm="nested"):
            if mid == "twopass":
                raise ValueError("the differentiable path covers the one-pass middle cores (onepass, twosided)")
            dtype = "f64" if _dtype_code(x) == L.F64 else "f32"
            p = PSTT2(n, ell, factors, dtype=dtype, prec=prec, ranks=ranks, eps=eps, rmax=rmax, mid=mid, drm=drm)
            xf = x.detach().reshape(-1)
            p.sketch(xf)
            tt = p.recover()
            ctx.pstt2 = p
            ctx.tt = tt
            return tt.reconstruct(dtype=x.dtype).view_as(x)

        @staticmethod
        def backward(ctx, gout):
            gx = ctx.pstt2.vjp(ctx.tt, gbar=gout.contiguous().reshape(-1))
            ctx.tt.free()
            ctx.pstt2.close()
            return gx.view_as(gout), None, None, None, None, None, None, None, None, None

    return PSTT2Reconstruct


_fn = None


def __getattr__(name):
    global _fn
    if name == "PSTT2Reconstruct":
        if _fn is None:
            _fn = _make_function()
        return _fn
    raise AttributeError(name)


def pstt2_reconstruct(x, n: Sequence[int], ell: int, factors: np.ndarray, *, prec: Optional[str] = None,
                      ranks: Optional[Sequence[int]] = None, eps: Optional[float] = None, rmax: int = 0,
                      mid: str = "onepass", drm: str = "nested"):
    """Differentiable X~ = PSTT2-onepass approximation of x (see PSTT2Reconstruct)."""
    return __getattr__("PSTT2Reconstruct").apply(x, list(n), int(ell), factors, prec, ranks, eps, rmax, mid, drm)
