"""GPU parity of the Gaussian-bump tensor function (Section 4.4), streamed by
pstt2_sketch_fn and measured by tt_error_fn without the tensor being stored.

- Small ragged shapes (d = 3, 4): every sketch, rank, pivot, X~ and the error
  against the oracle run on the stored tensor, for both Khatri-Rao schemes, the
  two-sided middle core and FP32 contexts (entries rounded to FP32 as a stored
  FP32 tensor would be).
- Slabs from memory and from the function mix, in any order.
- The order-3 shape of Table 1 (n = 960, 6.59 GB in FP64, never stored), which
  the library evaluates in several workspace chunks: sampled Y_R and T_m
  entries against their definition and the relative error at ranks 24.
"""
import ctypes

import numpy as np
import pytest

import inputs
from oracle import tt_sketch as O

from gpu_common import compare, oracle_run, rel, say

pytestmark = pytest.mark.gpu


def _bumps(w):
    import paper_2111_10448_amd as P
    return P.GaussBumps(inputs.gauss_centers(w), w.gamma)


def _factors(w, drm):
    if drm == "nested":
        psi, om = inputs.drm_factors(w)
        return psi, om, inputs.pack_factors(psi, om, w.d)
    psi, om = inputs.drm_factors_independent(w)
    return psi, om, inputs.pack_factors_independent(psi, om, w.d)


@pytest.mark.parametrize("name,middle,drm,prec", [
    ("gb_small3", "onepass", "nested", "f64"), ("gb_small4", "onepass", "nested", "f64"),
    ("gb_small4", "twosided", "nested", "f64"), ("gb_small3", "onepass", "independent", "f64"),
    ("gb_small4", "onepass", "nested", "f32"), ("gb_small3", "onepass", "nested", "bf16x3")])
def test_gauss_fn_matches_oracle(name, middle, drm, prec):
    import torch
    import paper_2111_10448_amd as P
    w = inputs.WORKLOADS[name]
    dtype = "f64" if prec == "f64" else "f32"
    say(f"[gpu] Gaussian bumps n={w.n} middle={middle} drm={drm} prec={prec}")
    x64 = inputs.make_tensor(w)
    x = x64 if dtype == "f64" else x64.astype(np.float32)
    psi, om, fac = _factors(w, drm)
    ref = oracle_run(x, w, psi, om, middle=middle, drm=drm)
    fn = _bumps(w)
    ctx = P.PSTT2(w.n, w.ell, fac, dtype=dtype, prec=prec, ranks=w.ranks(), mid=middle, drm=drm)
    ctx.sketch_fn(fn)
    tt = ctx.recover()
    xg = torch.from_numpy(x).cuda()
    out = compare(ctx, tt, xg, x, w, ref, prec)
    e_fn = tt.error_fn(fn)
    e_ref = O.tt_error(x64, ref["cores"])
    say(f"    {out}  error_fn={e_fn:.3e} oracle on the FP64 tensor {e_ref:.3e}")
    tol = 1e-10 if prec == "f64" else 1e-5
    assert abs(e_fn - e_ref) <= tol + 1e-3 * e_ref
    tt.free()
    ctx.close()


def test_gauss_slabs_mix_with_memory_slabs():
    """Half the columns from memory, half evaluated, in the other order: the same
    sketches as the whole tensor from memory, to rounding."""
    import torch
    import paper_2111_10448_amd as P
    w = inputs.WORKLOADS["gb_small4"]
    say(f"[gpu] Gaussian bumps, mixed slabs n={w.n}")
    x = inputs.make_tensor(w)
    xg = torch.from_numpy(x).cuda()
    _, _, fac = _factors(w, "nested")
    m = O.middle_index(w.d)
    R = int(np.prod(w.n[:m]))
    C = x.size // R
    a = P.PSTT2(w.n, w.ell, fac, dtype="f64", prec="f64", ranks=w.ranks())
    a.sketch(xg)
    a.recover().free()
    b = P.PSTT2(w.n, w.ell, fac, dtype="f64", prec="f64", ranks=w.ranks())
    half = (C // 2) * R
    b.sketch(xg[half:], half)
    b.sketch_fn(_bumps(w), 0, half)
    b.recover().free()
    for which in (0, 1):
        d_ = rel(b.get_sketch(which, m), a.get_sketch(which, m))
        say(f"    sketch {which}: {d_:.2e}")
        assert d_ < 1e-14
    a.close()
    b.close()


def test_gauss_error_paths():
    """Bad bump parameters are refused before any launch; the order of the centers
    must match the tensor's."""
    import paper_2111_10448_amd as P
    from paper_2111_10448_amd import _lib as L
    w = inputs.WORKLOADS["gb_small3"]
    say("[gpu] Gaussian bumps error handling")
    _, _, fac = _factors(w, "nested")
    ctr = np.ascontiguousarray(inputs.gauss_centers(w))
    with P.PSTT2(w.n, w.ell, fac, dtype="f64", prec="f64", ranks=w.ranks()) as ctx:
        for nt, g, p in ((0, 10.0, ctr.ctypes.data), (L.GAUSS_MAX_TERMS + 1, 10.0, ctr.ctypes.data),
                         (100, 0.0, ctr.ctypes.data), (100, float("nan"), ctr.ctypes.data), (100, 10.0, None)):
            f = L.Fn(L.FN["gauss"], nt, g, p)
            st = L.lib().pstt2_sketch_fn(ctx._c(), ctypes.byref(f), 0, int(np.prod(w.n)))
            assert st == L.EINVAL, (nt, g, st)
        with pytest.raises(ValueError):
            ctx.sketch_fn(P.GaussBumps(ctr[:, :2], 10.0))
        with pytest.raises(P.PSTT2Error) as e:
            ctx.sketch_fn(_bumps(w), w.n[0], w.n[0] * w.n[1])     # not a whole column of X_m
        assert e.value.status == L.EINVAL


def test_gauss_table1_shape_full_size():
    """n = 960, d = 3 (8.8e8 entries, never stored; two workspace chunks of columns):
    sampled sketch entries match their definition and the relative error at ranks 24
    is below 1e-10."""
    import paper_2111_10448_amd as P
    w = inputs.WORKLOADS["gb_d3"]
    say(f"[gpu] Gaussian bumps n={w.n[0]}^{w.d} ranks={w.ranks()} ell={w.ell}")
    ctr = inputs.gauss_centers(w)
    fn = _bumps(w)
    _, _, fac = _factors(w, "nested")
    ctx = P.PSTT2(w.n, w.ell, fac, dtype="f64", prec="f64", ranks=w.ranks())
    ctx.sketch_fn(fn)
    tt = ctx.recover()
    assert tt.ranks == [1] + w.ranks() + [1]
    m = O.middle_index(w.d)
    R = int(np.prod(w.n[:m]))
    C = int(np.prod(w.n[m:]))
    psi, om = inputs.drm_factors(w)
    drm = O.NestedKR(psi, om)
    rng = np.random.default_rng(6)
    y = ctx.get_sketch(0, m)
    t = ctx.get_sketch(1, m)
    rows = np.unique(np.concatenate([[0, R - 1], rng.integers(0, R, 6)]))
    cols = np.unique(np.concatenate([[0, C - 1], rng.integers(0, C, 2)]))
    omega = drm.omega_dense(m, w.d)
    xr = inputs.gauss_entries(w.n, m, rows, np.arange(C), ctr, w.gamma)
    worst_y = float(np.max(np.abs(y[rows] - xr @ omega) / (np.abs(xr) @ np.abs(omega))))
    psi_m = drm.psi_dense(m)
    xc = inputs.gauss_entries(w.n, m, np.arange(R), cols, ctr, w.gamma)
    worst_t = float(np.max(np.abs(t[cols] - xc.T @ psi_m) / (np.abs(xc.T) @ np.abs(psi_m))))
    err = tt.error_fn(fn)
    say(f"    sampled Y_R {worst_y:.2e}, T_m {worst_t:.2e} (of the absolute sums); relative error {err:.3e}")
    assert worst_y < 1e-13 and worst_t < 1e-13
    assert err < 1e-10
    tt.free()
    ctx.close()
