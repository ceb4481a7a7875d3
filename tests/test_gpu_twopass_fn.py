"""GPU parity of the second pass over a tensor function (pstt2_middle_pass_fn):
the two-pass middle core of equation "PSTT2_final_core" (and the one-sided
algorithm's last core Q^T X) with the tensor evaluated again instead of read.
Section 4.4 contrasts this second round of function evaluations with the
one-pass cores, which need none.

Against the oracle run on the stored tensor: every sketch, rank, pivot, X~ and
the error, with the second pass split in two calls, for the Gaussian bumps
(d = 3, 4; FP64 and FP32 contexts) and the Hilbert tensor (d = 3).
"""
import ctypes

import numpy as np
import pytest

import inputs
from oracle import tt_sketch as O

from gpu_common import TOL_XT, compare, oracle_run, rel, say

pytestmark = pytest.mark.gpu


def _fn(w):
    import paper_2111_10448_amd as P
    return P.GaussBumps(inputs.gauss_centers(w), w.gamma) if w.kind == "gauss" else "hilbert"


@pytest.mark.parametrize("name,prec", [("gb_small3", "f64"), ("gb_small4", "f64"), ("gb_small4", "f32"),
                                       ("t1_small3", "f64")])
def test_twopass_middle_core_over_function(name, prec):
    import torch
    import paper_2111_10448_amd as P
    w = inputs.WORKLOADS[name]
    dtype = "f64" if prec == "f64" else "f32"
    say(f"[gpu] two-pass middle core over {w.kind} n={w.n} prec={prec}")
    x = inputs.make_tensor(w)
    if dtype == "f32":
        x = x.astype(np.float32)
    psi, om = inputs.drm_factors(w)
    fac = inputs.pack_factors(psi, om, w.d)
    ref = oracle_run(x, w, psi, om, middle="twopass")
    fn = _fn(w)
    ctx = P.PSTT2(w.n, w.ell, fac, dtype=dtype, prec=prec, ranks=w.ranks(), mid="twopass")
    if w.kind == "gauss" or dtype == "f64":
        ctx.sketch_fn(fn)
    tt = ctx.recover()
    m = O.middle_index(w.d)
    R = int(np.prod(w.n[:m]))
    C = x.size // R
    half = (C // 2) * R
    ctx.middle_pass_fn(tt, fn, half)          # second half first
    ctx.middle_pass_fn(tt, fn, 0, half)
    torch.cuda.synchronize()
    xg = torch.from_numpy(x).cuda()
    out = compare(ctx, tt, xg, x, w, ref, prec)
    say(f"    {out}")
    tt.free()
    ctx.close()


def test_pstt_last_core_over_function():
    """The one-sided algorithm's two-pass last core Q_{d-1}^T X_{d-1} over the Gaussian bumps,
    in two calls; a second run gives bitwise the same cores (no atomics in the last-core pass)."""
    import torch
    import paper_2111_10448_amd as P
    w = inputs.WORKLOADS["gb_small4"]
    say(f"[gpu] PSTT two-pass last core over gauss n={w.n}")
    x = inputs.make_tensor(w)
    psi, om = inputs.drm_factors(w)
    fac = inputs.pack_factors(psi, om, w.d)
    D = O.NestedKR(psi, om)
    ref = O.pstt(x, w.n, D, w.ranks())
    fn = _fn(w)
    half = (w.n[-1] // 2) * int(np.prod(w.n[:-1]))

    def run():
        ctx = P.PSTT2(w.n, w.ell, fac, dtype="f64", prec="f64", ranks=w.ranks(), mid="twopass", algo="pstt")
        ctx.sketch_fn(fn)
        tt = ctx.recover()
        ctx.middle_pass_fn(tt, fn, half)
        ctx.middle_pass_fn(tt, fn, 0, half)
        torch.cuda.synchronize()
        return ctx, tt

    ctx, tt = run()
    assert tt.ranks == [1] + list(ref["ranks"]) + [1]
    xt = tt.reconstruct().cpu().numpy()
    ctx2, tt2 = run()
    assert np.array_equal(tt2.reconstruct().cpu().numpy(), xt), "last core not bitwise repeatable"
    tt2.free()
    ctx2.close()
    d_xt = rel(xt, O.tt_full(ref["cores"]))
    xg = torch.from_numpy(x).cuda()
    e_gpu, e_ref = tt.error(xg), O.tt_error(x, ref["cores"])
    say(f"    X~ {d_xt:.2e}  error {e_gpu:.3e} (oracle {e_ref:.3e})")
    assert d_xt < TOL_XT["f64"]
    assert abs(e_gpu - e_ref) <= TOL_XT["f64"] * 1.01 + 1e-3 * e_ref
    tt.free()
    ctx.close()


def test_middle_pass_fn_refusals():
    import paper_2111_10448_amd as P
    from paper_2111_10448_amd import _lib as L
    w = inputs.WORKLOADS["gb_small3"]
    say("[gpu] middle_pass_fn error handling")
    psi, om = inputs.drm_factors(w)
    fac = inputs.pack_factors(psi, om, w.d)
    fn = _fn(w)
    with P.PSTT2(w.n, w.ell, fac, dtype="f64", prec="f64", ranks=w.ranks()) as ctx:
        ctx.sketch_fn(fn)
        tt = ctx.recover()
        with pytest.raises(P.PSTT2Error) as e:       # one-pass context
            ctx.middle_pass_fn(tt, fn)
        assert e.value.status == L.ESTATE
        tt.free()
    with P.PSTT2(w.n, w.ell, fac, dtype="f64", prec="f64", ranks=w.ranks(), mid="twopass") as ctx:
        ctx.sketch_fn(fn)
        tt = ctx.recover()
        with pytest.raises(P.PSTT2Error) as e:       # not whole columns of X_m
            ctx.middle_pass_fn(tt, fn, w.n[0], w.n[0] * w.n[1])
        assert e.value.status == L.EINVAL
        bad = L.Fn(L.FN["gauss"], 0, 10.0, None)
        st = L.lib().pstt2_middle_pass_fn(ctx._c(), ctypes.byref(tt.struct()), ctypes.byref(bad), 0, 0)
        assert st == L.EINVAL
        tt.free()
