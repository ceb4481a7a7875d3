"""GPU parity of the hand-written adjoint (pstt2_vjp, PSTT2Reconstruct).

The reference gradient is the oracle's (torch CPU FP64 autograd of an
independent transcription of PSTT2-onepass with frozen pivots, itself pinned
by finite differences); the FP64 instance is also checked against central
finite differences of the GPU's own forward pass.
"""
import numpy as np
import pytest

import inputs
from oracle import tt_adjoint as OA
from oracle import tt_sketch as O

from gpu_common import rel, say

pytestmark = pytest.mark.gpu


def _instance(name, n=None, middle="onepass", scheme="nested"):
    w = inputs.WORKLOADS[name]
    if n is not None:
        w = inputs.Workload(w.name, w.index, tuple(n), w.dtype, w.kind, tt_rank=w.tt_rank, noise=w.noise,
                            ell=w.ell, rank=w.rank)
    x = inputs.make_tensor(w)
    if scheme == "nested":
        psi, om = inputs.drm_factors(w)
        fac = inputs.pack_factors(psi, om, w.d)
        drm = O.NestedKR(psi, om)
    else:
        psi, om = inputs.drm_factors_independent(w)
        fac = inputs.pack_factors_independent(psi, om, w.d)
        drm = O.IndependentKR(psi, om)
    ref = O.pstt2(np.asarray(x, dtype=np.float64), w.n, drm, ranks=w.ranks(), middle=middle)
    ref["middle"] = middle
    ref["scheme"] = scheme
    return w, x, fac, drm, ref


def _gpu(w, x, fac, prec, middle="onepass", scheme="nested"):
    import torch
    import paper_2111_10448_amd as P
    xg = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    ctx = P.PSTT2(w.n, w.ell, fac, dtype=w.dtype, prec=prec, ranks=w.ranks(), mid=middle, drm=scheme)
    ctx.sketch(xg)
    tt = ctx.recover()
    return ctx, tt, xg


def _check(w, x, fac, drm, ref, prec, tol, seed=3):
    import torch
    middle = ref["middle"]
    ctx, tt, xg = _gpu(w, x, fac, prec, middle, ref["scheme"])
    x64 = np.asarray(x, dtype=np.float64)
    for k in range(1, w.d):
        rk = ref["ranks"][k - 1]
        assert list(ctx.pivots(k)[:rk]) == list(ref["piv"][k][:rk]), k
    rng = np.random.default_rng(seed)
    gb = rng.standard_normal(x.size).astype(x.dtype)
    jt = ctx.vjp(tt, gbar=torch.from_numpy(gb).cuda()).cpu().numpy()
    jt_ref = OA.pstt2_vjp(x64, w.n, drm, ref["ranks"], ref["piv"], gbar=gb.astype(np.float64), middle=middle)
    e1 = rel(jt, jt_ref)
    g = ctx.vjp(tt, x=xg).cpu().numpy()
    # loss gradient 2 r + J^T(-2 r) at the GPU's own residual r = X - X~: the
    # residual is ~1e-4 of X here, so FP32 sketch rounding in X~ would swamp
    # a comparison against the oracle's residual without testing the adjoint
    r = x64 - tt.reconstruct().cpu().numpy()
    g_ref = 2.0 * r + OA.pstt2_vjp(x64, w.n, drm, ref["ranks"], ref["piv"], gbar=-2.0 * r, middle=middle)
    e2 = rel(g, g_ref)
    say(f"    J^T gbar rel {e1:.2e}, loss gradient rel {e2:.2e}")
    assert e1 < tol and e2 < tol, (e1, e2)
    tt.free()
    ctx.close()


@pytest.mark.parametrize("n", [None, (6, 5, 7), (5, 4, 6, 3, 4), (4, 3, 5, 4, 3, 4), (9, 7)])
def test_vjp_fp64_matches_oracle(n):
    """FP64, d = 2..6 (middle index 1..3), ragged modes: J^T gbar and the loss gradient."""
    w, x, fac, drm, ref = _instance("c5_fd", n)
    say(f"[gpu] vjp f64 n={w.n}")
    _check(w, x, fac, drm, ref, "f64", 1e-9)


@pytest.mark.parametrize("n,middle,scheme", [
    (None, "twosided", "nested"), ((6, 5, 7), "twosided", "nested"), ((5, 4, 6, 3, 4), "twosided", "nested"),
    ((4, 3, 5, 4, 3, 4), "twosided", "nested"),
    (None, "onepass", "independent"), ((5, 4, 6, 3, 4), "onepass", "independent"),
    ((4, 3, 5, 4, 3, 4), "onepass", "independent"), ((9, 7), "onepass", "independent"),
    ((5, 4, 6, 3, 4), "twosided", "independent"), ((4, 3, 5, 4, 3, 4), "twosided", "independent")])
def test_vjp_fp64_variants_match_oracle(n, middle, scheme):
    """FP64, the two-sided middle core and the independent DRM scheme, d = 2..6."""
    w, x, fac, drm, ref = _instance("c5_fd", n, middle, scheme)
    say(f"[gpu] vjp f64 n={w.n} middle={middle} drm={scheme}")
    _check(w, x, fac, drm, ref, "f64", 1e-9)


@pytest.mark.parametrize("prec,tol", [("f32", 2e-5), ("bf16x3", 2e-5)])
def test_vjp_fp32_matches_oracle(prec, tol):
    """FP32 tensor (20, 17, 19, 21), FP32 and split-BF16 sketches."""
    w, x, fac, drm, ref = _instance("c5_small")
    say(f"[gpu] vjp {prec} n={w.n}")
    _check(w, x, fac, drm, ref, prec, tol)


@pytest.mark.parametrize("middle,scheme", [("twosided", "nested"), ("onepass", "independent"),
                                           ("twosided", "independent")])
def test_vjp_fp32_variants_match_oracle(middle, scheme):
    """FP32 tensor (20, 17, 19, 21), FP32 sketches, the other middle-core rule and DRM scheme."""
    w, x, fac, drm, ref = _instance("c5_small", None, middle, scheme)
    say(f"[gpu] vjp f32 n={w.n} middle={middle} drm={scheme}")
    _check(w, x, fac, drm, ref, "f32", 2e-5)


def test_gradient_matches_finite_differences_n8():
    """d=4, n=8 FP64: 20 random directions, central differences of the GPU forward loss."""
    import torch
    import paper_2111_10448_amd as P
    w, x, fac, drm, ref = _instance("c5_fd")
    say("[gpu] vjp vs finite differences, c5_fd")
    ctx, tt, xg = _gpu(w, x, fac, "f64")
    g = ctx.vjp(tt, x=xg).cpu().numpy()
    piv0 = [list(ctx.pivots(k)) for k in range(1, w.d)]

    def loss(xx):
        c2 = P.PSTT2(w.n, w.ell, fac, dtype="f64", prec="f64", ranks=w.ranks())
        t = torch.from_numpy(xx).cuda()
        c2.sketch(t)
        t2 = c2.recover()
        assert [list(c2.pivots(k)) for k in range(1, w.d)] == piv0
        xt = t2.reconstruct().cpu().numpy()
        t2.free()
        c2.close()
        return float(np.sum((xx - xt) ** 2))

    rng = np.random.default_rng(11)
    h = 1e-4 * np.linalg.norm(x) / np.sqrt(x.size)
    worst = 0.0
    for _ in range(20):
        v = rng.standard_normal(x.size)
        v /= np.linalg.norm(v)
        fd = (loss(x + h * v) - loss(x - h * v)) / (2 * h)
        worst = max(worst, abs(fd - g @ v) / np.linalg.norm(g))
    say(f"    worst directional FD mismatch {worst:.2e}")
    assert worst < 1e-6
    tt.free()
    ctx.close()


@pytest.mark.parametrize("middle,scheme", [("onepass", "nested"), ("twosided", "independent")])
def test_autograd_function_backpropagates_frobenius_loss(middle, scheme):
    """PSTT2Reconstruct under torch autograd: d/dX ||X - X~||^2 equals the oracle gradient."""
    import torch
    import paper_2111_10448_amd as P
    w, x, fac, drm, ref = _instance("c5_fd", (7, 6, 5, 6), middle, scheme)
    say(f"[gpu] PSTT2Reconstruct autograd middle={middle} drm={scheme}")
    xg = torch.from_numpy(x).cuda().requires_grad_(True)
    xt = P.pstt2_reconstruct(xg, w.n, w.ell, fac, prec="f64", ranks=w.ranks(), mid=middle, drm=scheme)
    loss = torch.sum((xg - xt) ** 2)
    loss.backward()
    g_ref = OA.pstt2_vjp(x, w.n, drm, ref["ranks"], ref["piv"], middle=middle)
    e = rel(xg.grad.cpu().numpy(), g_ref)
    say(f"    autograd gradient rel {e:.2e}")
    assert e < 1e-9


@pytest.mark.slow
def test_vjp_c5_full_size():
    """d=4, n=48 FP32 (5.3e6 entries), FP32 sketches: loss gradient against the oracle."""
    w, x, fac, drm, ref = _instance("c5")
    say("[gpu] vjp c5 full size")
    _check(w, x, fac, drm, ref, "f32", 5e-5)


@pytest.mark.slow
def test_vjp_workspace_is_not_tensor_sized():
    """C5 (5.3e6 FP32 entries): the loss gradient and J^T gbar run under a device budget of the
    library's live bytes plus 4 bytes per entry.  The cotangent is never stored (as FP64 it alone
    would take 8 bytes per entry); the results match the unbudgeted run bitwise."""
    import torch
    import paper_2111_10448_amd as P
    w, x, fac, drm, ref = _instance("c5")
    say("[gpu] vjp c5 workspace under a budget of 4 bytes per entry")
    ctx, tt, xg = _gpu(w, x, fac, "f32")
    gbar = torch.from_numpy(np.random.default_rng(7).standard_normal(x.size).astype(np.float32)).cuda()
    torch.cuda.synchronize()
    P.set_memory_limit(P.memory_stats()["live"] + 4 * x.size)
    try:
        g = ctx.vjp(tt, x=xg)
        jt = ctx.vjp(tt, gbar=gbar)
        torch.cuda.synchronize()
    finally:
        P.set_memory_limit(0)
    assert torch.equal(g, ctx.vjp(tt, x=xg)) and torch.equal(jt, ctx.vjp(tt, gbar=gbar))
    assert torch.isfinite(g).all() and torch.isfinite(jt).all()
    tt.free()
    ctx.close()
