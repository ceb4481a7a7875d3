"""Shared helpers for the GPU parity tests: run the HIP path and the oracle on
the same seeded inputs and compare what is unique (sketches, pivots, ranks,
the reconstructed tensor, the error)."""
import sys

import numpy as np

import inputs
from oracle import tt_sketch as O

# parity tolerances on the reconstructed tensor, relative Frobenius norm.  FP16
# (no bound stated for it) takes the one-term 16-bit bound on X~, whose
# sensitivity to the sketches' rounding depends on the tensor's conditioning,
# and on the sketches, which are plain sums, BF16's bound scaled by the ratio of
# the two formats' unit roundoffs, 2^-11 / 2^-8 = 1/8 (so FP16 sketches that
# rounded like BF16 would fail).
TOL_XT = {"f64": 1e-10, "f32": 1e-5, "bf16x3": 1e-5, "bf16": 5e-3, "f16": 5e-3}
# tolerances on the sketches themselves (relative Frobenius norm)
TOL_SK = {"f64": 1e-12, "f32": 1e-6, "bf16x3": 1e-6, "bf16": 1e-2, "f16": 1e-2 / 8}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def setup(w, n=None, ell=None):
    x = inputs.make_tensor(w)
    psi, omega = inputs.drm_factors(w, n=n, ell=ell)
    fac = inputs.pack_factors(psi, omega, w.d)
    return x, psi, omega, fac


def oracle_run(x, w, psi, omega, middle="onepass", drm="nested"):
    x64 = np.asarray(x, dtype=np.float64)
    drm = O.NestedKR(psi, omega) if drm == "nested" else O.IndependentKR(psi, omega)
    if w.ranks() is not None:
        ref = O.pstt2(x64, w.n, drm, ranks=w.ranks(), middle=middle)
    else:
        ref = O.pstt2(x64, w.n, drm, eps=w.eps, rmax=w.rmax, middle=middle)
    ref["drm"] = drm
    return ref


def gpu_run(x, w, fac, prec, slabs=None, middle="onepass", batched=False, ranks=None, drm="nested"):
    import torch
    import paper_2111_10448_amd as P
    xg = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    kw = dict(dtype=w.dtype, prec=prec, mid=middle, drm=drm)
    if ranks is not None:
        kw["ranks"] = list(ranks)
    elif w.ranks() is not None:
        kw["ranks"] = w.ranks()
    else:
        kw["eps"] = w.eps
        kw["rmax"] = w.rmax
    ctx = P.PSTT2(w.n, w.ell, fac, **kw)
    if slabs is None:
        ctx.sketch(xg)
    elif batched:
        ctx.sketch_slabs([xg[f:f + c] for f, c in slabs], [f for f, _ in slabs])
    else:
        for f, c in slabs:
            ctx.sketch(xg[f:f + c], f)
    tt = ctx.recover()
    if middle == "twopass":
        if slabs is None:
            ctx.middle_pass(tt, xg)
        else:
            for f, c in slabs:
                ctx.middle_pass(tt, xg[f:f + c], f)
        torch.cuda.synchronize()
    return ctx, tt, xg


def compare(ctx, tt, xg, x, w, ref, prec, check_pivots=True, check_cores=False):
    """Assert parity; returns a dict of measured deltas."""
    d = w.d
    m = O.middle_index(d)
    out = {}
    tol_sk = TOL_SK[prec]
    # sketches: Y_R, T_m and every derived split
    if ref["Y"] is not None:
        y = ctx.get_sketch(0, m)
        out["Y"] = rel(y, ref["Y"])
        assert out["Y"] < tol_sk, ("Y_R", out["Y"])
    for k in range(1, m):
        s = ctx.get_sketch(0, k)
        out[f"S{k}"] = rel(s, ref["S"][k])
        assert out[f"S{k}"] < tol_sk, (f"S_{k}", out[f"S{k}"])
    for k in range(m, d):
        t = ctx.get_sketch(1, k)
        out[f"T{k}"] = rel(t, ref["T"][k].T)
        assert out[f"T{k}"] < tol_sk, (f"T_{k}", out[f"T{k}"])
    # two-sided sketches B_k = Psi_k^T X_k Omega_k, from their definition
    x64 = np.asarray(x, dtype=np.float64)
    for k in range(1, d):
        b = ctx.get_sketch(2, k)
        out[f"B{k}"] = rel(b, O.two_sided_sketch(x64, w.n, k, ref["drm"]))
        assert out[f"B{k}"] < tol_sk, (f"B_{k}", out[f"B{k}"])
    # ranks
    assert tt.ranks == [1] + list(ref["ranks"]) + [1], (tt.ranks, ref["ranks"])
    # pivots (the first r_k decide the basis)
    if check_pivots:
        for k in range(1, d):
            pg = ctx.pivots(k)
            po = ref["piv"][k]
            rk = ref["ranks"][k - 1]
            assert list(pg[:rk]) == list(po[:rk]), (k, pg, po)
    # reconstructed tensor
    xt_gpu = tt.reconstruct().cpu().numpy()
    xt_ref = O.tt_full(ref["cores"])
    out["Xt"] = rel(xt_gpu, xt_ref)
    assert out["Xt"] < TOL_XT[prec], ("X~", out["Xt"])
    if check_cores:
        for k, (a, b) in enumerate(zip(tt.cores_numpy(), ref["cores"])):
            out[f"G{k + 1}"] = rel(a, b)
            assert out[f"G{k + 1}"] < 1e-8, (k, out[f"G{k + 1}"])
    # error
    e_gpu = tt.error(xg)
    e_ref = O.tt_error(np.asarray(x, dtype=np.float64), ref["cores"])
    out["err_gpu"] = e_gpu
    out["err_ref"] = e_ref
    assert abs(e_gpu - e_ref) <= TOL_XT[prec] * 1.01 + 1e-3 * e_ref, (e_gpu, e_ref)
    return out
