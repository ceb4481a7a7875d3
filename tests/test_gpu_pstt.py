"""GPU parity of the one-sided algorithm (Algorithm PSTT and PSTT-onepass) on
the same kernels: the pass sketches split d-1, every column basis Q_k comes
from a right sketch derived from it, and the last core comes from the extra
left sketch T_{d-1} by the one-pass rule or from a second pass.  The oracle is
oracle.tt_sketch.pstt (pinned by the expectation bounds of Theorems 3 and 4).
"""
import numpy as np
import pytest

import inputs
from oracle import tt_sketch as O

from gpu_common import TOL_SK, TOL_XT, rel, say

pytestmark = pytest.mark.gpu


def _run(name, n, prec, mid, drm, slabs=1, fibres=False, repeat=False):
    import dataclasses
    import torch
    import paper_2111_10448_amd as P
    w = inputs.WORKLOADS[name]
    if n is not None:
        w = dataclasses.replace(w, n=tuple(n))
    say(f"[gpu] PSTT {name} n={w.n} prec={prec} mid={mid} drm={drm} slabs={slabs}")
    x = inputs.make_tensor(w)
    x64 = np.asarray(x, dtype=np.float64)
    if drm == "nested":
        psi, om = inputs.drm_factors(w)
        fac = inputs.pack_factors(psi, om, w.d)
        D = O.NestedKR(psi, om)
    else:
        psi, om = inputs.drm_factors_independent(w)
        fac = inputs.pack_factors_independent(psi, om, w.d)
        D = O.IndependentKR(psi, om)
    d = w.d
    ranks = w.ranks()
    ref = O.pstt(x64, w.n, D, ranks, onepass_psi=D.psi_dense(d - 1) if mid == "onepass" else None)
    xg = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    ctx = P.PSTT2(w.n, w.ell, fac, dtype=w.dtype, prec=prec, ranks=ranks, mid=mid, drm=drm, algo="pstt")
    # whole columns of X_{d-1}, or mode-1 fibres (slabs that cut columns)
    bounds = inputs.slab_bounds(x.size, w.n[0] if fibres else int(np.prod(w.n[:d - 1])), slabs)
    for f, c in bounds:
        ctx.sketch(xg[f:f + c], f)
    tt = ctx.recover()
    if repeat:
        # a reset and the same pass again reproduce every sketch bitwise
        first = [ctx.get_sketch(0, k) for k in range(1, d)] + [ctx.get_sketch(1, d - 1)]
        tt.free()
        ctx.reset()
        for f, c in bounds:
            ctx.sketch(xg[f:f + c], f)
        tt = ctx.recover()
        again = [ctx.get_sketch(0, k) for k in range(1, d)] + [ctx.get_sketch(1, d - 1)]
        for a, b in zip(first, again):
            assert np.array_equal(a, b)
    if mid == "twopass":
        for f, c in bounds:
            ctx.middle_pass(tt, xg[f:f + c], f)
        torch.cuda.synchronize()
    out = {}
    for k in range(1, d):
        s_ref = O.sketch_right_dense(x64, w.n, k, D.omega_dense(k, d))
        out[f"S{k}"] = rel(ctx.get_sketch(0, k), s_ref)
        assert out[f"S{k}"] < TOL_SK[prec], (k, out[f"S{k}"])
    t_ref = O.sketch_left_dense(x64, w.n, d - 1, D.psi_dense(d - 1))
    out["T"] = rel(ctx.get_sketch(1, d - 1), t_ref.T)
    assert out["T"] < TOL_SK[prec]
    assert tt.ranks == [1] + list(ref["ranks"]) + [1]
    xt = tt.reconstruct().cpu().numpy()
    xr = O.tt_full(ref["cores"])
    out["Xt"] = rel(xt, xr)
    e_gpu, e_ref = tt.error(xg), O.tt_error(x64, ref["cores"])
    say(f"    {out}  error {e_gpu:.3e} (oracle {e_ref:.3e})")
    assert out["Xt"] < TOL_XT[prec]
    assert abs(e_gpu - e_ref) <= TOL_XT[prec] * 1.01 + 1e-3 * e_ref
    tt.free()
    ctx.close()
    return e_gpu


@pytest.mark.parametrize("name,n,prec,mid,drm,slabs", [
    ("c1", None, "f64", "onepass", "nested", 1),
    ("c2_small", None, "f64", "onepass", "nested", 1),
    ("c2_small", None, "f64", "twopass", "nested", 3),
    ("c1", (9, 7, 8), "f64", "onepass", "nested", 1),
    ("c1", (37, 29), "f64", "onepass", "nested", 1),
    ("c1", (6, 5, 7, 6), "f64", "onepass", "independent", 1),
    ("c5_small", None, "f32", "onepass", "nested", 5),
])
def test_pstt_matches_oracle(name, n, prec, mid, drm, slabs):
    _run(name, n, prec, mid, drm, slabs)


@pytest.mark.parametrize("slabs,fibres", [(1, False), (3, False), (5, True)])
def test_pstt_tall_rows(slabs, fibres):
    """X_{d-1} with 2^19 rows: more row blocks than the GPU holds workgroups, so
    every sketch launch has one column group and adds its Y tile directly, and
    the first launch after a reset stores it (Y is not zeroed at reset).  The
    whole tensor, three whole-column slabs (the later launches add), and five
    slabs that cut columns (the partial columns zero Y first), each against the
    oracle, then reset and streamed again, bitwise equal."""
    _run("c1", (128, 64, 64, 2), "f64", "onepass", "nested", slabs, fibres=fibres, repeat=True)


def test_pstt_exact_recovery():
    """Exact-rank TT, no noise: one-sided one-pass recovers X to rounding."""
    e = _run("c1_exact", None, "f64", "onepass", "nested")
    assert e < 1e-11


def test_pstt_refusals():
    import paper_2111_10448_amd as P
    from paper_2111_10448_amd import _lib as L
    import torch
    w = inputs.WORKLOADS["c1"]
    say("[gpu] PSTT refusals")
    psi, om = inputs.drm_factors(w)
    fac = inputs.pack_factors(psi, om, w.d)
    with pytest.raises(P.PSTT2Error) as e:
        P.PSTT2(w.n, w.ell, fac, ranks=w.ranks(), mid="twosided", algo="pstt")
    assert e.value.status == L.EINVAL
    x = inputs.make_tensor(w)
    xg = torch.from_numpy(x).cuda()
    with P.PSTT2(w.n, w.ell, fac, ranks=w.ranks(), algo="pstt") as ctx:
        ctx.sketch(xg)
        tt = ctx.recover()
        with pytest.raises(P.PSTT2Error) as e:
            ctx.vjp(tt, x=xg)
        assert e.value.status == L.ESTATE
        tt.free()
