"""Full-size GPU checks in the launch configuration the benchmark times.

The noisy d=6 tensor runs through the oracle on the host and is compared with
it split by split.  The others compare sampled sketch entries computed one by one
from their definition (Y_R(i, c) = sum_j X_m(i, j) Omega_m(j, c), T_m(a, j) =
sum_i Psi_m(i, a) X_m(i, j), Khatri-Rao DRM columns built with np.kron), and
properties that hold at any size: exact recovery of the noiseless exact-rank
tensor, the error level of the noisy one, and ranks.
"""
import numpy as np
import pytest

import inputs
from oracle import tt_sketch as O

from gpu_common import say

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _kr_col(factors, c):
    """Column c of the Khatri-Rao product with the first listed factor fastest."""
    v = np.ones(1)
    for f in factors:
        v = np.kron(f[:, c], v)
    return v


def _check_sampled(x, w, psi, omega, y_gpu, tt_gpu, nsamp, tol, seed):
    n = w.n
    d = w.d
    m = O.middle_index(d)
    R = O.rows_of(n, m)
    C = O.cols_of(n, m)
    rng = np.random.default_rng(seed)
    xm = x.reshape((R, C), order="F")
    worst = 0.0
    for _ in range(nsamp):
        i = int(rng.integers(R))
        c = int(rng.integers(w.ell))
        om = _kr_col([omega[q] for q in range(m + 1, d + 1)], c)
        row = np.asarray(xm[i, :], dtype=np.float64)
        ref = float(row @ om)
        scale = float(np.abs(row) @ np.abs(om))
        worst = max(worst, abs(y_gpu[i, c] - ref) / scale)
        j = int(rng.integers(C))
        a = int(rng.integers(w.ell))
        ps = _kr_col([psi[q] for q in range(1, m + 1)], a)
        col = np.asarray(xm[:, j], dtype=np.float64)
        ref = float(ps @ col)
        scale = float(np.abs(ps) @ np.abs(col))
        worst = max(worst, abs(tt_gpu[j, a] - ref) / scale)
    assert worst < tol, worst
    return worst


_TENSORS = {}


def _tensor(w):
    """The workload's tensor, kept for the next test of the same workload only."""
    if w.name not in _TENSORS:
        _TENSORS.clear()
        _TENSORS[w.name] = inputs.make_tensor(w)
    return _TENSORS[w.name]


def _run(w, prec, slabs=None, mid="onepass", drm="nested", extra=None):
    import torch
    import paper_2111_10448_amd as P
    x = _tensor(w)
    if drm == "nested":
        psi, omega = inputs.drm_factors(w)
        fac = inputs.pack_factors(psi, omega, w.d)
    else:
        psi, omega = inputs.drm_factors_independent(w)
        fac = inputs.pack_factors_independent(psi, omega, w.d)
    if slabs:
        bounds = inputs.slab_bounds(x.size, w.n[0], slabs)
        xs = [torch.from_numpy(x[f:f + c]).cuda() for f, c in bounds]
        xg = None
    else:
        xg = torch.from_numpy(x).cuda()
    kw = dict(dtype=w.dtype, prec=prec, mid=mid, drm=drm)
    if w.rank is not None:
        kw["ranks"] = w.ranks()
    else:
        kw.update(eps=w.eps, rmax=w.rmax)
    ctx = P.PSTT2(w.n, w.ell, fac, **kw)
    if slabs:
        ctx.sketch_slabs(xs, [f for f, _ in bounds])
    else:
        ctx.sketch(xg)
    tt = ctx.recover()
    m = O.middle_index(w.d)
    y = ctx.get_sketch(0, m)
    t = ctx.get_sketch(1, m)
    if extra is not None:
        extra["B"] = {k: ctx.get_sketch(2, k) for k in range(1, w.d)}
    if slabs:
        xg = torch.cat(xs)
        del xs
    err = tt.error(xg)
    ranks = tt.ranks
    ctx.close()
    del xg
    torch.cuda.empty_cache()
    return x, psi, omega, y, t, err, ranks


def test_c2_exact_rank_full_size():
    """Noiseless d=6, n=32 rank-10 TT (8.6 GB FP64): recovered to rounding."""
    w = inputs.WORKLOADS["c2_exact"]
    say("[gpu] full size c2_exact")
    x, psi, omega, y, t, err, ranks = _run(w, "f64")
    worst = _check_sampled(x, w, psi, omega, y, t, 16, 1e-13, 1)
    say(f"    sampled sketch max rel {worst:.2e}, tt_error {err:.3e}, ranks {ranks}")
    assert ranks == [1] + [10] * 5 + [1]
    assert err < 1e-11


def test_c2_noisy_full_size_against_oracle():
    """d=6, n=32 with N(0, 1e-8) noise (8.6 GB FP64), the benchmark's launch: the oracle's
    PSTT2-onepass runs on the same tensor on the host, and every sketch of every split,
    B_k, pivots, ranks, the gauge-fixed FP64 cores and the error are compared with it."""
    import time
    import torch
    import paper_2111_10448_amd as P
    w = inputs.WORKLOADS["c2"]
    say("[gpu] full size c2 against the oracle")
    x = _tensor(w)
    psi, omega = inputs.drm_factors(w)
    fac = inputs.pack_factors(psi, omega, w.d)
    d, m = w.d, O.middle_index(w.d)
    xg = torch.from_numpy(x).cuda()
    ctx = P.PSTT2(w.n, w.ell, fac, dtype="f64", prec="f64", ranks=w.ranks())
    ctx.sketch(xg)
    tt = ctx.recover()
    got = {"S": {k: ctx.get_sketch(0, k) for k in range(1, m + 1)},
           "T": {k: ctx.get_sketch(1, k) for k in range(m, d)},
           "B": {k: ctx.get_sketch(2, k) for k in range(1, d)},
           "piv": {k: ctx.pivots(k) for k in range(1, d)}}
    cores = tt.cores_numpy()
    err = tt.error(xg)
    ranks = tt.ranks
    tt.free()
    ctx.close()
    del xg
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    drm = O.NestedKR(psi, omega)
    ref = O.pstt2(x, w.n, drm, ranks=w.ranks())
    e_ref = O.tt_error(x, ref["cores"])
    say(f"    oracle on the host: {time.perf_counter() - t0:.1f} s")

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))
    worst = {"Y": rel(got["S"][m], ref["Y"])}
    for k in range(1, m):
        worst[f"S{k}"] = rel(got["S"][k], ref["S"][k])
    for k in range(m, d):
        worst[f"T{k}"] = rel(got["T"][k], ref["T"][k].T)
    # B_k from the oracle's own one-sided sketches and the dense Khatri-Rao DRMs
    for k in range(1, d):
        b = drm.psi_dense(k).T @ ref["S"][k] if k < m else ref["T"][k] @ drm.omega_dense(k, d)
        worst[f"B{k}"] = rel(got["B"][k], b)
    assert max(worst.values()) < 1e-12, worst
    assert ranks == [1] + list(ref["ranks"]) + [1]
    for k in range(1, d):
        rk = ref["ranks"][k - 1]
        assert list(got["piv"][k][:rk]) == list(ref["piv"][k][:rk]), k
    dg = [rel(a, b) for a, b in zip(cores, ref["cores"])]
    noise_rel = w.noise * np.sqrt(x.size) / np.linalg.norm(x)
    say(f"    sketches {max(worst.values()):.2e}, cores {max(dg):.2e}, tt_error {err:.6e} "
        f"(oracle {e_ref:.6e}, noise level {noise_rel:.3e})")
    assert max(dg) < 1e-8, dg
    assert abs(err - e_ref) <= 1e-10 * 1.01 + 1e-6 * e_ref, (err, e_ref)
    # the projection of the noise is the floor; the one-pass sketch stays within
    # a small factor of it (Theorem 4 with p = r)
    assert noise_rel * 0.5 < err < 10 * noise_rel


@pytest.mark.parametrize("prec,tol", [("f32", 2e-6), ("bf16x3", 2e-6), ("bf16", 2e-2)])
def test_c3_precisions_full_size(prec, tol):
    """d=5, n=64 FP32 1/sum on a Chebyshev grid (1.07e9 entries): sampled sketches, error."""
    w = inputs.WORKLOADS["c3"]
    say(f"[gpu] full size c3 prec={prec}")
    x, psi, omega, y, t, err, ranks = _run(w, prec)
    worst = _check_sampled(x, w, psi, omega, y, t, 8, tol, 3)
    say(f"    sampled sketch max rel {worst:.2e}, tt_error {err:.3e}, ranks {ranks}")
    if prec != "bf16":
        assert err <= 1e-5


def test_c4_slabs_full_size():
    """d=8, n=12 FP32 in 64 slabs of whole mode-1 fibres: sampled sketches, error level."""
    w = inputs.WORKLOADS["c4"]
    say("[gpu] full size c4 (64 slabs)")
    x, psi, omega, y, t, err, ranks = _run(w, "f32", slabs=w.nslabs)
    worst = _check_sampled(x, w, psi, omega, y, t, 8, 2e-6, 4)
    say(f"    sampled sketch max rel {worst:.2e}, tt_error {err:.3e}, ranks {ranks}")
    assert ranks == [1] + [8] * 7 + [1]
    assert err < 1e-5


def test_c2_two_sided_sketches_full_size():
    """d=6, n=32: B_m against Psi_m^T Y_R formed on the host from the GPU's Y_R, and the error level."""
    w = inputs.WORKLOADS["c2"]
    say("[gpu] full size c2 two-sided sketches")
    ex = {}
    x, psi, omega, y, t, err, ranks = _run(w, "f64", extra=ex)
    m = O.middle_index(w.d)
    psi_m = O.khatri_rao([psi[q] for q in range(m, 0, -1)])      # R_m x ell, first mode fastest
    om_m = O.khatri_rao([omega[q] for q in range(w.d, m, -1)])   # C_m x ell
    b_left = psi_m.T @ y                                         # Psi_m^T (X_m Omega_m)
    b_right = t.T @ om_m                                         # (Psi_m^T X_m) Omega_m
    e1 = np.linalg.norm(ex["B"][m] - b_left) / np.linalg.norm(b_left)
    e2 = np.linalg.norm(ex["B"][m] - b_right) / np.linalg.norm(b_right)
    say(f"    B_m vs Psi^T Y_R {e1:.2e}, vs T_m Omega_m {e2:.2e}")
    assert e1 < 1e-10 and e2 < 1e-10


@pytest.mark.parametrize("mid,drm", [("twosided", "nested"), ("onepass", "independent")])
def test_c2_exact_rank_variants_full_size(mid, drm):
    """Noiseless d=6, n=32: the two-sided middle core and the independent DRM scheme recover X to rounding."""
    w = inputs.WORKLOADS["c2_exact"]
    say(f"[gpu] full size c2_exact mid={mid} drm={drm}")
    x, psi, omega, y, t, err, ranks = _run(w, "f64", mid=mid, drm=drm)
    say(f"    tt_error {err:.3e}, ranks {ranks}")
    assert ranks == [1] + [10] * 5 + [1]
    assert err < 1e-11
