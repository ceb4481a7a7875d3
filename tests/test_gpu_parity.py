"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle.

Same seeded inputs on both sides; compared element by element: the sketches
(Y_R, T_m and every derived split), CPQR pivots, ranks, the reconstructed
tensor X~ and the relative error.  Tolerances: 1e-10 (FP64), 1e-5 (FP32,
split-BF16), 5e-3 (BF16) on X~.
"""
import numpy as np
import pytest

import inputs
from oracle import tt_sketch as O

from gpu_common import TOL_SK, TOL_XT, compare, gpu_run, oracle_run, rel, say, setup

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["c1", "c1_exact", "c2_small", "c5_small", "c5_fd"])
def test_fp64_and_fp32_workloads(name):
    w = inputs.WORKLOADS[name]
    say(f"[gpu] parity {name} n={w.n} ell={w.ell} dtype={w.dtype}")
    x, psi, omega, fac = setup(w)
    ref = oracle_run(x, w, psi, omega)
    prec = "f64" if w.dtype == "f64" else "f32"
    ctx, tt, xg = gpu_run(x, w, fac, prec)
    out = compare(ctx, tt, xg, x, w, ref, prec, check_cores=(prec == "f64"))
    say(f"    {out}")
    if name == "c1_exact":
        assert out["err_gpu"] < 1e-12
    ctx.close()


@pytest.mark.parametrize("name,slabs", [("c3_small", 1), ("c5_small", 1), ("c4_small", 7)])
def test_fp32_data_fp64_arithmetic(name, slabs):
    """FP32 tensors sketched in FP64 (the entries widened as loaded): the oracle upcasts the
    same FP32 values exactly, so every quantity is held to the FP64 tolerances, including
    the gauge-fixed cores; the 7-slab case runs multi-segment launches with ragged edges."""
    w = inputs.WORKLOADS[name]
    say(f"[gpu] parity {name} n={w.n} FP32 data, FP64 arithmetic, slabs={slabs}")
    assert w.dtype == "f32"
    x, psi, omega, fac = setup(w)
    ref = oracle_run(x, w, psi, omega)
    sl = inputs.slab_bounds(x.size, w.n[0], slabs) if slabs > 1 else None
    ctx, tt, xg = gpu_run(x, w, fac, "f64", slabs=sl)
    out = compare(ctx, tt, xg, x, w, ref, "f64", check_cores=True)
    say(f"    {out}")
    ctx.close()


@pytest.mark.parametrize("prec", ["f32", "bf16x3", "bf16"])
def test_mixed_precision_invsum(prec):
    w = inputs.WORKLOADS["c3_small"]
    say(f"[gpu] parity c3_small prec={prec}")
    x, psi, omega, fac = setup(w)
    ref = oracle_run(x, w, psi, omega)
    # plain BF16 sketches sit ~1e-3 above the 1e-5 tolerance rule, so that run
    # uses the oracle's ranks (fixed-rank mode); the others choose their own.
    ranks = ref["ranks"] if prec == "bf16" else None
    ctx, tt, xg = gpu_run(x, w, fac, prec, ranks=ranks)
    out = compare(ctx, tt, xg, x, w, ref, prec, check_pivots=(prec != "bf16"))
    say(f"    {out}")
    assert out["err_gpu"] <= 1e-5 or prec == "bf16"
    ctx.close()


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
@pytest.mark.parametrize("batched", [False, True])
def test_slab_streaming(prec, batched):
    """Slabs of whole mode-1 fibres (edges cut columns of X_m) in scrambled order."""
    w = inputs.WORKLOADS["c4_small"]
    say(f"[gpu] slabs c4_small prec={prec} batched={batched}")
    x, psi, omega, fac = setup(w)
    ref = oracle_run(x, w, psi, omega)
    slabs = inputs.slab_bounds(x.size, w.n[0], w.nslabs)
    order = np.random.default_rng(5).permutation(len(slabs))
    slabs = [slabs[i] for i in order]
    ctx, tt, xg = gpu_run(x, w, fac, prec, slabs=slabs, batched=batched)
    out = compare(ctx, tt, xg, x, w, ref, prec)
    say(f"    {out}")
    ctx.close()


@pytest.mark.parametrize("name,n,prec,nslabs", [
    ("c2_small", None, "f64", 0),           # d = 6: m = 3, three pass groups
    ("c4_small", None, "f32", 7),           # d = 8 in 7 slabs: four groups, multi-segment launches
    ("c1", (9, 7, 8), "f64", 0),            # d = 3: right splits 1, 2; left split 2
    ("c1", (6, 5, 7, 4, 5), "f64", 0),      # d = 5: m = 3, left splits 3, 4
])
def test_independent_drm_scheme(name, n, prec, nslabs):
    """Per-split factors (the paper's Psi^(j)): every split's sketch, pivots, ranks and X~ vs the oracle."""
    import dataclasses
    w = inputs.WORKLOADS[name]
    if n is not None:
        w = dataclasses.replace(w, name="indep", index=70 + len(n), n=tuple(n))
    say(f"[gpu] independent DRMs {w.name} n={w.n} prec={prec} slabs={nslabs}")
    x = inputs.make_tensor(w)
    psi, omega = inputs.drm_factors_independent(w)
    fac = inputs.pack_factors_independent(psi, omega, w.d)
    ref = oracle_run(x, w, psi, omega, drm="independent")
    slabs = inputs.slab_bounds(x.size, w.n[0], nslabs) if nslabs else None
    ctx, tt, xg = gpu_run(x, w, fac, prec, slabs=slabs, batched=bool(nslabs), drm="independent")
    out = compare(ctx, tt, xg, x, w, ref, prec, check_cores=(prec == "f64"))
    say(f"    {out}")
    ctx.close()


@pytest.mark.parametrize("name,n,prec,drm", [
    ("c2_small", None, "f64", "nested"),
    ("c2_small", None, "f64", "independent"),
    ("c3_small", None, "f32", "nested"),      # tolerance-mode ranks
    ("c1", (6, 5, 7, 4, 5), "f64", "nested"),  # d = 5, m = 3
    ("c1", (9, 7, 8), "f64", "independent"),   # d = 3, m = 2: Psi' is split 1's left DRM
    ("c1", (37, 41), "f64", "nested"),         # d = 2: the rule is the one-pass rule
])
def test_twosided_middle_core(name, n, prec, drm):
    """Middle core from the two-sided middle sketch H: H, cores / X~ and ranks vs the oracle."""
    import dataclasses
    w = inputs.WORKLOADS[name]
    if n is not None:
        w = dataclasses.replace(w, name="twosided", index=110 + len(n), n=tuple(n))
    say(f"[gpu] two-sided middle core {w.name} n={w.n} prec={prec} drm={drm}")
    x = inputs.make_tensor(w)
    if drm == "nested":
        psi, omega = inputs.drm_factors(w)
        fac = inputs.pack_factors(psi, omega, w.d)
    else:
        psi, omega = inputs.drm_factors_independent(w)
        fac = inputs.pack_factors_independent(psi, omega, w.d)
    ref = oracle_run(x, w, psi, omega, middle="twosided", drm=drm)
    ctx, tt, xg = gpu_run(x, w, fac, prec, middle="twosided", drm=drm)
    m = O.middle_index(w.d)
    if m >= 2:
        h = ctx.get_sketch(3, 0)
        rp = O.rows_of(w.n, m - 1)
        y3 = np.reshape(ref["Y"], (rp, w.n[m - 1], w.ell), order="F")
        h_ref = np.einsum("ra,rjc->ajc", ref["drm"].psi_dense(m - 1), y3).reshape(-1, w.ell, order="F")
        e_h = rel(h, h_ref)
        say(f"    H rel {e_h:.2e}")
        assert e_h < TOL_SK[prec]
    out = compare(ctx, tt, xg, x, w, ref, prec, check_cores=(prec == "f64"))
    say(f"    {out}")
    ctx.close()


def test_twopass_middle_core():
    w = inputs.WORKLOADS["c2_small"]
    say("[gpu] two-pass middle core c2_small")
    x, psi, omega, fac = setup(w)
    ref = oracle_run(x, w, psi, omega, middle="twopass")
    ctx, tt, xg = gpu_run(x, w, fac, "f64", middle="twopass")
    out = compare(ctx, tt, xg, x, w, ref, "f64", check_cores=True)
    say(f"    {out}")
    # the adjoint covers the one-pass middle cores only
    import paper_2111_10448_amd as P
    from paper_2111_10448_amd import _lib as L
    with pytest.raises(P.PSTT2Error) as e:
        ctx.vjp(tt, x=xg)
    assert e.value.status == L.ESTATE
    ctx.close()


@pytest.mark.parametrize("n,rank,ell", [((37, 41), 4, 7), ((5, 6, 7), 3, 6), ((3, 4, 5, 4, 3, 2, 3), 2, 5),
                                         ((2, 2, 2, 2, 2, 2, 2, 2, 2), 2, 4)])
def test_exact_recovery_shapes(n, rank, ell):
    """d = 2, 3, 7, 9; exact-rank TT, noise 0: both sides recover X to ~1e-12."""
    import dataclasses
    w = dataclasses.replace(inputs.WORKLOADS["c1_exact"], name="shape", index=90 + len(n), n=tuple(n),
                            tt_rank=rank, ell=ell, rank=rank)
    say(f"[gpu] exact recovery n={n}")
    x, psi, omega, fac = setup(w)
    ref = oracle_run(x, w, psi, omega)
    ctx, tt, xg = gpu_run(x, w, fac, "f64")
    out = compare(ctx, tt, xg, x, w, ref, "f64", check_cores=True)
    assert out["err_gpu"] < 1e-11
    say(f"    {out}")
    ctx.close()


def test_repeatable_bitwise_and_slab_order():
    """Same call sequence -> bitwise-identical sketches; another slab order -> equal to rounding."""
    import torch
    w = inputs.WORKLOADS["c2_small"]
    say("[gpu] determinism c2_small")
    x, psi, omega, fac = setup(w)
    import paper_2111_10448_amd as P
    xg = torch.from_numpy(x).cuda()
    m = O.middle_index(w.d)
    ys = []
    for rep in range(2):
        with P.PSTT2(w.n, w.ell, fac, ranks=w.ranks()) as ctx:
            ctx.sketch(xg)
            ctx.recover()
            ys.append((ctx.get_sketch(0, m), ctx.get_sketch(1, m)))
    assert np.array_equal(ys[0][0], ys[1][0]) and np.array_equal(ys[0][1], ys[1][1])
    slabs = inputs.slab_bounds(x.size, w.n[0], 9)[::-1]
    with P.PSTT2(w.n, w.ell, fac, ranks=w.ranks()) as ctx:
        for f, c in slabs:
            ctx.sketch(xg[f:f + c], f)
        ctx.recover()
        assert rel(ctx.get_sketch(0, m), ys[0][0]) < 1e-13
        assert rel(ctx.get_sketch(1, m), ys[0][1]) < 1e-13


def test_error_paths():
    """Overlap / missing coverage / misalignment / NaN are reported, not run."""
    import torch
    import paper_2111_10448_amd as P
    from paper_2111_10448_amd import _lib as L
    w = inputs.WORKLOADS["c1"]
    say("[gpu] error paths")
    x, psi, omega, fac = setup(w)
    xg = torch.from_numpy(x).cuda()
    with P.PSTT2(w.n, w.ell, fac, ranks=w.ranks()) as ctx:
        ctx.sketch(xg[:1024], 0)
        with pytest.raises(P.PSTT2Error) as e:
            ctx.sketch(xg[512:2048], 512)
        assert e.value.status == L.ESTATE
        with pytest.raises(P.PSTT2Error) as e:
            ctx.sketch(xg[1030:1040], 1030)    # not a multiple of n_1 = 16
        assert e.value.status == L.EINVAL
        with pytest.raises(P.PSTT2Error) as e:
            ctx.recover()                      # entries 1024.. never streamed
        assert e.value.status == L.ESTATE
        ctx.sketch(xg[1024:1024], 1024)        # empty slab is a no-op
        ctx.sketch(xg[1024:], 1024)
        tt = ctx.recover()
        assert tt.ranks[1] == 3
    xn = x.copy()
    xn[777] = np.nan
    with P.PSTT2(w.n, w.ell, fac, ranks=w.ranks()) as ctx:
        ctx.sketch(torch.from_numpy(xn).cuda())
        with pytest.raises(P.PSTT2Error) as e:
            ctx.recover()
        assert e.value.status == L.ENUMERIC
        ctx.reset()
        ctx.sketch(xg)
        ctx.recover()


def test_tt_error_and_reconstruct_on_given_cores():
    """tt_error / tt_reconstruct of caller-provided cores vs the entry formula."""
    import torch
    import paper_2111_10448_amd as P
    say("[gpu] tt_error on given cores")
    n = (7, 6, 5, 8, 3)
    rng = np.random.default_rng(3)
    cores = inputs.random_tt_cores(rng, n, 4)
    ranks = [1] + [c.shape[2] for c in cores[:-1]]
    tc = [torch.from_numpy(np.ascontiguousarray(c.reshape(-1, order="F"))).cuda() for c in cores]
    cs = P.cores_struct(tc, n, ranks + [1])
    xt = O.tt_full(cores)
    got = P.tt_reconstruct(cs).cpu().numpy()
    assert rel(got, xt) < 1e-14
    part = P.tt_reconstruct(cs, 35, 700, dtype=torch.float32).cpu().numpy()
    assert rel(part, xt[35:735]) < 1e-6
    noise = 1e-3 * rng.standard_normal(xt.size)
    xg = torch.from_numpy(xt + noise).cuda()
    e = P.tt_error(cs, xg)
    ref = np.linalg.norm(noise) / np.linalg.norm(xt + noise)
    assert abs(e - ref) < 1e-9 * ref
    e32 = P.tt_error(cs, xg.float())
    ref32 = np.linalg.norm((xt + noise).astype(np.float32).astype(np.float64) - xt) / \
        np.linalg.norm((xt + noise).astype(np.float32).astype(np.float64))
    assert abs(e32 - ref32) < 1e-6 * ref32


@pytest.mark.parametrize("ell", [20, 24, 28, 32])
@pytest.mark.parametrize("name", ["c2_twin", "c2_twin_odd"])
def test_fp64_benchmark_sketch_sizes(name, ell):
    """The FP64 kernel at every sketch size the FP64 workloads use (20 = the d=6 benchmark,
    its 16-wide plus 4-wide tile mix; 24 and 28 mix 16 + 8 and 16 + 12; 32 = the 8-wave
    workgroup of the memory path), element by element against the oracle: every sketch,
    B_k, pivots, ranks, gauge-fixed FP64 cores, X~ and the error.  c2_twin streams the
    whole tensor (one segment, 16-byte loads); c2_twin_odd has an odd row count (scalar
    loads) and arrives in 9 scrambled slabs in one launch (multi-segment launch, slab
    edges through the partial-column kernel)."""
    import dataclasses
    w = dataclasses.replace(inputs.WORKLOADS[name], ell=ell)
    say(f"[gpu] FP64 parity {w.name} n={w.n} ell={ell} slabs={w.nslabs}")
    x, psi, omega, fac = setup(w)
    ref = oracle_run(x, w, psi, omega)
    slabs = None
    if w.nslabs > 1:
        slabs = inputs.slab_bounds(x.size, w.n[0], w.nslabs)
        order = np.random.default_rng(ell).permutation(len(slabs))
        slabs = [slabs[i] for i in order]
    ctx, tt, xg = gpu_run(x, w, fac, "f64", slabs=slabs, batched=slabs is not None)
    out = compare(ctx, tt, xg, x, w, ref, "f64", check_cores=True)
    say(f"    {out}")
    ctx.close()


@pytest.mark.parametrize("name,prec", [("c4_twin24", "f32"), ("c4_twin24", "bf16x3"), ("c3_small", "bf16")])
def test_fp32_family_padded_sketch_size(name, prec):
    """Sketch size 24 in the FP32-family kernels: a 32-wide sketch tile whose last 8
    columns are padding; 7 slabs in scrambled order, one launch.  Plain BF16 runs on
    the smooth 1/sum twin (the workload it is benchmarked on) with the oracle's
    ranks: on the random-TT twin its rounding (2^-9 per operand) is amplified past
    the 5e-3 X~ tolerance by the spread of the sketch's singular values."""
    import dataclasses
    w = dataclasses.replace(inputs.WORKLOADS[name], ell=24, nslabs=7)
    say(f"[gpu] padded sketch size {w.name} ell={w.ell} prec={prec}")
    x, psi, omega, fac = setup(w)
    ref = oracle_run(x, w, psi, omega)
    slabs = inputs.slab_bounds(x.size, w.n[0], w.nslabs)
    order = np.random.default_rng(24).permutation(len(slabs))
    slabs = [slabs[i] for i in order]
    ranks = ref["ranks"] if prec == "bf16" else None
    ctx, tt, xg = gpu_run(x, w, fac, prec, slabs=slabs, batched=True, ranks=ranks)
    out = compare(ctx, tt, xg, x, w, ref, prec, check_pivots=(prec != "bf16"))
    say(f"    {out}")
    ctx.close()


@pytest.mark.parametrize("rank,ell", [(20, 24), (28, 32)])
def test_twopass_wide_ranks_split_pass(rank, ell):
    """Two-pass middle core with middle ranks 20 and 28 (the 24- and 32-wide register
    tiles of the pair-load Z pass: FP64, even row count, whole columns), the second pass
    given as two whole-column halves, the second half first, so the later launch starts
    at a column offset."""
    import dataclasses
    import torch
    w = dataclasses.replace(inputs.WORKLOADS["c2_twin"], tt_rank=rank, rank=rank, ell=ell)
    say(f"[gpu] two-pass ranks {rank} ell {ell} {w.n}")
    x, psi, omega, fac = setup(w)
    ref = oracle_run(x, w, psi, omega, middle="twopass")
    import paper_2111_10448_amd as P
    xg = torch.from_numpy(x).cuda()
    ctx = P.PSTT2(w.n, w.ell, fac, dtype="f64", prec="f64", ranks=w.ranks(), mid="twopass")
    ctx.sketch(xg)
    tt = ctx.recover()
    m = O.middle_index(w.d)
    R = int(np.prod(w.n[:m]))
    half = (x.size // R // 2) * R
    ctx.middle_pass(tt, xg[half:], half)
    ctx.middle_pass(tt, xg[:half], 0)
    torch.cuda.synchronize()
    out = compare(ctx, tt, xg, x, w, ref, "f64", check_cores=True)
    say(f"    {out}")
    ctx.close()


@pytest.mark.parametrize("name,slabs", [("c3_small", False), ("c4_small", True), ("c4_twin24", True)])
def test_fp16_sketches(name, slabs):
    """FP16 sketch arithmetic (IEEE half, FP32 accumulation) against the oracle, at the
    one-term 16-bit tolerances scaled to half precision.  The 1/sum twin runs in
    tolerance mode with the oracle's ranks (as plain BF16); the TT twins in fixed rank,
    streamed as scrambled slabs (16- and 32-wide sketch tiles)."""
    w = inputs.WORKLOADS[name]
    say(f"[gpu] FP16 sketches {name} ell={w.ell} slabs={slabs}")
    x, psi, omega, fac = setup(w)
    ref = oracle_run(x, w, psi, omega)
    sl = None
    if slabs:
        sl = inputs.slab_bounds(x.size, w.n[0], w.nslabs)
        order = np.random.default_rng(16).permutation(len(sl))
        sl = [sl[i] for i in order]
    ranks = ref["ranks"] if w.ranks() is None else None
    ctx, tt, xg = gpu_run(x, w, fac, "f16", slabs=sl, batched=slabs, ranks=ranks)
    out = compare(ctx, tt, xg, x, w, ref, "f16", check_pivots=False)
    say(f"    {out}")
    ctx.close()


def test_fp16_range_overflow_reports_enumeric():
    """FP16 sketches: an entry past half precision's largest finite value (65504) becomes
    infinite, and recover reports ENUMERIC instead of returning cores; after reset the
    same context decomposes the in-range tensor.  Split BF16 (FP32's range) takes the
    out-of-range entry as it is."""
    import torch
    import paper_2111_10448_amd as P
    from paper_2111_10448_amd import _lib as L
    w = inputs.WORKLOADS["c5_small"]
    say("[gpu] FP16 range overflow")
    x, psi, omega, fac = setup(w)
    xb = x.copy()
    xb[123] = np.float32(1.0e5)
    xg = torch.from_numpy(x).cuda()
    with P.PSTT2(w.n, w.ell, fac, dtype="f32", prec="f16", ranks=w.ranks()) as ctx:
        ctx.sketch(torch.from_numpy(xb).cuda())
        with pytest.raises(P.PSTT2Error) as e:
            ctx.recover()
        assert e.value.status == L.ENUMERIC
        ctx.reset()
        ctx.sketch(xg)
        tt = ctx.recover()
        assert np.isfinite(tt.error(xg))
        tt.free()
    with P.PSTT2(w.n, w.ell, fac, dtype="f32", prec="bf16x3", ranks=w.ranks()) as ctx:
        ctx.sketch(torch.from_numpy(xb).cuda())
        tt = ctx.recover()
        tt.free()


@pytest.mark.parametrize("name,n,drm", [("c2_small", None, "nested"), ("c1", (9, 7, 8), "independent"),
                                        ("c4_small", None, "nested")])
def test_seeded_factors(name, n, drm):
    """A context with no caller factors draws them from its seed (Philox4x32-10 +
    Box-Muller in the library's host code); the oracle gets the same stream from the
    independent implementation in inputs and must agree as with caller factors."""
    import dataclasses
    import torch
    import paper_2111_10448_amd as P
    w = inputs.WORKLOADS[name]
    if n is not None:
        w = dataclasses.replace(w, name="seeded", index=120 + len(n), n=tuple(n))
    seed = 0x5EED0000 + w.index
    say(f"[gpu] seeded factors {w.name} n={w.n} drm={drm} seed={seed:#x}")
    x = inputs.make_tensor(w)
    psi, omega = inputs.seeded_factors(w.n, w.ell, seed, drm)
    ref = oracle_run(x, w, psi, omega, drm=drm)
    prec = "f64" if w.dtype == "f64" else "f32"
    xg = torch.from_numpy(x).cuda()
    ctx = P.PSTT2(w.n, w.ell, None, dtype=w.dtype, prec=prec, ranks=w.ranks(), drm=drm, seed=seed)
    ctx.sketch(xg)
    tt = ctx.recover()
    out = compare(ctx, tt, xg, x, w, ref, prec, check_cores=(prec == "f64"))
    say(f"    {out}")
    ctx.close()
