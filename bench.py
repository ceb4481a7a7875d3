#!/usr/bin/env python3
"""PSTT2-onepass benchmark on one MI355X.

One step = the whole hot path over the resident tensor: reset the context,
stream X once through the dual-sketch kernel (right and left sketches of the
middle unfolding), recover the TT cores in FP64 on the GPU (derived sketches,
TSQR + pivoted QR bases, outer cores, least-squares middle core), and
evaluate the relative error ||X - X~||_F / ||X||_F in a second streaming pass.

Default workload: FP64 d=6, n=32 (1.07e9 entries, 8.6 GB), X = random Gaussian
TT with ranks 10 scaled to ||X||_F = 1 plus N(0, 1e-8) noise, target ranks 10,
sketch size 20.  Inputs are synthetic and seeded (inputs/).

Prints one JSON line.  `value` is whole-step throughput (bytes of X per step
time; X is read twice per step: sketch and error).  `roofline` covers the
dominant kernel (the streaming sketch), timed with HIP events on the stream it
runs on, with the rate of a plain read-and-sum over the same bytes beside it.
`cpu_baseline` times the CPU FP64 oracle on a bounded sub-tensor (sketches,
recovery and error pass separately), runs the GPU path on the same sub-tensor
and reports the element-wise sketch differences, ranks and error against the
oracle's, and times the oracle on C1 and C5 with one thread.
Unless --no-variants: the two-sided middle core, the independent DRM scheme,
the precision study (FP64 data; FP32 data in FP64, FP32, split BF16, BF16 and
FP16 arithmetic), the 64-slab stream,
C1 and C5, the adjoint, Table 1's Hilbert tensors evaluated inside the kernels
(never stored) and the Gaussian bumps.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 (vector = matrix)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the sketch kernels' source (all of csrc/sketch.hip): stored counter figures
    are used only while it is unchanged."""
    with open(os.path.join(ROOT, "paper_2111_10448_amd", "csrc", "sketch.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_from_profiles(workload: str, prec: str):
    """HBM bytes per sketch launch (FETCH_SIZE + WRITE_SIZE, calibrated) from the committed
    counter summary of this workload and precision, if it matches this kernel source."""
    path = os.path.join(ROOT, "profiles", f"k_sketch_{workload}_{prec}_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel source sha256\[:16\]:\s*`?([0-9a-f]{16})", txt)
    b = re.search(r"HBM bytes per launch \(scaled\):\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != kernel_source_hash():
        return None
    return float(b.group(1))


def cpu_baseline(x: np.ndarray, w, psi, omega, prec: str, target_s: float = 30.0):
    """Time the oracle (sketches, recovery, error pass) on a leading block of the same tensor.

    The sample keeps modes 1..d-1 whole and the first s slices of mode d (a
    contiguous prefix of the column-major array).  A short probe at s = 1
    sizes s so that the timed oracle run takes about `target_s` seconds.  The
    GPU path then runs on the same sample: its right and left sketches of the
    middle unfolding, ranks and relative error are compared with the oracle's
    (parity on the benchmarked configuration).  Last, the oracle on the small
    configurations C1 and C5 with one BLAS thread.
    """
    from oracle import tt_sketch as O
    try:
        import threadpoolctl
        threads = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] + [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    n = list(w.n)
    slab = int(np.prod(n[:-1]))

    def run(s):
        ns = n[:-1] + [s]
        sub = np.asarray(x[:slab * s], dtype=np.float64)
        psi_s = {q: psi[q][:ns[q - 1]] for q in psi}
        om_s = {q: omega[q][:ns[q - 1]] for q in omega}
        tm = {}
        out = O.pstt2(sub, ns, O.NestedKR(psi_s, om_s), ranks=w.ranks(), timings=tm)
        t1 = time.perf_counter()
        err = O.tt_error(sub, out["cores"])
        tm["error_s"] = time.perf_counter() - t1
        return ns, sub, psi_s, om_s, out, tm, err

    _, sub1, _, _, _, tm1, _ = run(1)
    per_byte = sum(tm1.values()) / sub1.nbytes
    s = int(max(1, min(n[-1], round(target_s / (per_byte * sub1.nbytes)))))
    ns, sub, psi_s, om_s, out, tm, err = run(s)
    total = sum(tm.values())
    nb = sub.nbytes
    rec = {"value": round(nb / total / 1e9, 4), "unit": "GB/s", "cores": int(threads), "kind": "oracle",
           "sample": f"leading block n={tuple(ns)} ({nb // 8} entries, {nb / 1e9:.2f} GB FP64) of the same "
                     f"tensor: oracle sketches {tm['sketch_s']:.1f} s, recovery {tm['recover_s']:.2f} s, "
                     f"error pass {tm['error_s']:.1f} s, rel. error {err:.3e}",
           "phases_s": {k: round(v, 3) for k, v in tm.items()}}
    try:
        rec["parity_on_sample"] = _sample_parity(x[:slab * s], ns, w, psi_s, om_s, out, err, prec)
    except Exception as e:   # report, keep the baseline
        rec["parity_on_sample"] = {"error": str(e)}
    del sub
    rec["one_thread"] = {}
    for name in ("c1", "c5"):
        try:
            rec["one_thread"][name] = _oracle_one_thread(name)
        except Exception as e:
            rec["one_thread"][name] = {"error": str(e)}
    return rec


def _sample_parity(xs, ns, w, psi_s, om_s, ref, err_ref, prec):
    """The GPU path on the oracle's sample: sketches of the middle unfolding element by
    element, ranks, and the relative error, against the oracle's run on the same block."""
    import torch
    import inputs
    import paper_2111_10448_amd as P
    from oracle import tt_sketch as O
    fac = inputs.pack_factors(psi_s, om_s, len(ns))
    xg = torch.from_numpy(np.ascontiguousarray(xs)).to("cuda:0")
    ctx = P.PSTT2(ns, w.ell, fac, dtype=w.dtype, prec=prec, ranks=w.ranks())
    ctx.sketch(xg)
    tt = ctx.recover()
    e = tt.error(xg)
    m = O.middle_index(len(ns))
    y_ref, t_ref = ref["Y"], ref["T"][m].T
    y, t = ctx.get_sketch(0, m), ctx.get_sketch(1, m)
    out = {"Y_R_max_rel": float(np.max(np.abs(y - y_ref)) / np.max(np.abs(y_ref))),
           "T_m_max_rel": float(np.max(np.abs(t - t_ref)) / np.max(np.abs(t_ref))),
           "ranks_equal": list(tt.ranks[1:-1]) == [int(v) for v in ref["ranks"]],
           "tt_rel_error_gpu": e, "tt_rel_error_oracle": err_ref, "tt_rel_error_abs_diff": abs(e - err_ref)}
    tt.free()
    ctx.close()
    del xg
    torch.cuda.empty_cache()
    return out


def _oracle_one_thread(name):
    """The oracle on a whole small configuration with one BLAS thread (phases in ms)."""
    import inputs
    from oracle import tt_sketch as O
    from threadpoolctl import threadpool_limits
    w = inputs.WORKLOADS[name]
    x = np.asarray(inputs.make_tensor(w), dtype=np.float64)
    psi, omega = inputs.drm_factors(w)
    with threadpool_limits(1):
        tm = {}
        out = O.pstt2(x, w.n, O.NestedKR(psi, omega), ranks=w.ranks(), timings=tm)
        t1 = time.perf_counter()
        err = O.tt_error(x, out["cores"])
        tm["error_s"] = time.perf_counter() - t1
    return {"workload": f"{name}: d={w.d} n={w.n[0]} ({x.size} entries)", "threads": 1,
            "sketch_ms": round(tm["sketch_s"] * 1e3, 3), "recover_ms": round(tm["recover_s"] * 1e3, 3),
            "error_ms": round(tm["error_s"] * 1e3, 3), "tt_rel_error": err}


def read_reduce_gbs(nbytes: int, reps: int = 5) -> float:
    """Achievable HBM read rate of a plain read-and-sum (torch's reduction) over nbytes, GB/s."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    a.sum()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        a.sum()
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    del a
    torch.cuda.empty_cache()
    return nbytes / (ms * 1e-3) / 1e9


_HOST = {}


def run_workload(name, prec, steps, warmup, ranks_from=None, mid="onepass", drm="nested", algo="pstt2"):
    import torch
    import inputs
    import paper_2111_10448_amd as P

    w = inputs.WORKLOADS[name]
    t0 = time.perf_counter()
    if _HOST.get("name") != name:     # keep the last workload's host tensor for the next precision
        _HOST.clear()
        x = inputs.make_tensor(w)
        psi, omega = inputs.drm_factors(w)
        _HOST.update(name=name, x=x, psi=psi, omega=omega)
        log(f"[bench] {name}: generated {x.nbytes / 1e9:.2f} GB on the host in {time.perf_counter() - t0:.1f} s")
    x, psi, omega = _HOST["x"], _HOST["psi"], _HOST["omega"]
    if drm == "independent":   # the paper's per-split factors
        ipsi, iomega = inputs.drm_factors_independent(w)
        fac = inputs.pack_factors_independent(ipsi, iomega, w.d)
    else:
        fac = inputs.pack_factors(psi, omega, w.d)
    log(f"[bench] {name} {prec}: timing {steps} steps")
    xg = torch.from_numpy(x).to("cuda:0")
    torch.cuda.synchronize()
    kw = dict(dtype=w.dtype, prec=prec, mid=mid, drm=drm, algo=algo)
    if ranks_from is not None:
        kw["ranks"] = ranks_from
    elif w.rank is not None:
        kw["ranks"] = w.ranks()
    else:
        kw["eps"] = w.eps
        kw["rmax"] = w.rmax
    ctx = P.PSTT2(w.n, w.ell, fac, **kw)
    if w.nslabs > 1:
        # contiguous runs of whole mode-1 fibres, views of the resident tensor
        bounds = inputs.slab_bounds(x.size, w.n[0], w.nslabs)
        xs = [xg[f:f + c] for f, c in bounds]
        firsts = [f for f, _ in bounds]

    def sketch():
        if w.nslabs > 1:
            ctx.sketch_slabs(xs, firsts)
        else:
            ctx.sketch(xg)

    def second_pass(tt):
        # the two-pass middle core reads X again (equation "PSTT2_final_core")
        if mid != "twopass":
            return
        if w.nslabs > 1:
            for xv, f in zip(xs, firsts):
                ctx.middle_pass(tt, xv, f)
        else:
            ctx.middle_pass(tt, xg)

    def step():
        ctx.reset()
        sketch()
        tt = ctx.recover()
        second_pass(tt)
        e = tt.error(xg)
        return tt, e

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read()
    t_dec = 0.0
    t0 = time.perf_counter()
    tt = err = None
    for _ in range(steps):
        a = time.perf_counter()
        ctx.reset()
        sketch()
        tt = ctx.recover()
        if mid == "twopass":
            second_pass(tt)
            torch.cuda.synchronize()
        b = time.perf_counter()
        err = tt.error(xg)
        t_dec += b - a
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, launches = ctx.profile_read()
    ctx.profile(False)
    res = {
        "workload": w, "x": x, "psi": psi, "omega": omega, "ranks": tt.ranks, "err": err,
        "ms_per_step": (t1 - t0) * 1e3 / steps, "decomp_ms": t_dec * 1e3 / steps,
        "kernel_ms": kms / max(launches, 1), "launches_per_step": launches // max(steps, 1),
        "bytes": x.nbytes,
    }
    ctx.close()
    del xg
    torch.cuda.empty_cache()
    return res


def run_function(name, steps, warmup, prec="f64", mid="onepass"):
    """Tensors given by a formula, never stored: Table 1's Hilbert tensors (evaluated
    inside the sketch and error kernels) or the Gaussian bumps of Section 4.4
    (evaluated into workspace chunks of columns that the memory kernels stream).
    Reset, sketch, recover and the error pass against the same formula.  prec other
    than f64 (Gaussian bumps only): an FP32 context, the evaluated chunks rounded to
    FP32 and sketched in that precision.  mid="twopass": the paper's PSTT2, whose
    middle core evaluates the function a second time (pstt2_middle_pass_fn)."""
    import torch
    import inputs
    import paper_2111_10448_amd as P

    w = inputs.WORKLOADS[name]
    psi, omega = inputs.drm_factors(w)
    fac = inputs.pack_factors(psi, omega, w.d)
    fn = P.GaussBumps(inputs.gauss_centers(w), w.gamma) if w.kind == "gauss" else "hilbert"
    dtype = "f64" if prec == "f64" else "f32"
    ctx = P.PSTT2(w.n, w.ell, fac, dtype=dtype, prec=prec, ranks=w.ranks(), mid=mid)
    log(f"[bench] {name}: {w.kind} tensor n={w.n[0]}^{w.d}, {prec} sketches, {mid} middle core, timing {steps} steps")
    t_err = t_sk = 0.0
    for it in range(warmup + steps):
        if it == warmup:
            torch.cuda.synchronize()
            ctx.profile(True)
            ctx.profile_read()
            t0 = time.perf_counter()
        ctx.reset()
        a = time.perf_counter()
        ctx.sketch_fn(fn)
        torch.cuda.synchronize()
        if it >= warmup:
            t_sk += time.perf_counter() - a
        tt = ctx.recover()
        if mid == "twopass":
            ctx.middle_pass_fn(tt, fn)
        a = time.perf_counter()
        err = tt.error_fn(fn)
        if it >= warmup:
            t_err += time.perf_counter() - a
        ranks = tt.ranks
        tt.free()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, launches = ctx.profile_read()
    ctx.profile(False)
    ctx.close()
    kms /= max(launches, 1)
    flops = 4.0 * w.ell * w.numel
    size = f"{w.numel} entries, {8 * w.numel / 2**30:.2f} GiB in FP64, never stored"
    if w.kind == "gauss":
        desc = (f"{name}: Gaussian-bump tensor ({w.terms} bumps, width parameter {w.gamma:g}) d={w.d} n={w.n[0]} "
                f"({size}), ranks {w.ranks()}, sketch size {w.ell}, {prec} sketches, {mid} middle core")
    else:
        desc = f"{name}: Hilbert tensor d={w.d} n={w.n[0]} ({size}), Table 1 ranks, sketch size {w.ell}"
    out = {"workload": desc, "ranks": ranks, "tt_rel_error": err,
           "ms_per_step": round((t1 - t0) * 1e3 / steps, 4), "sketch_fn_ms": round(t_sk * 1e3 / steps, 4),
           "sketch_kernel_ms": round(kms, 4), "error_pass_ms": round(t_err * 1e3 / steps, 4)}
    if w.kind == "gauss":
        # evaluation at 2 x terms FP64 flops per entry, then the memory sketch of the chunks
        ev = 2.0 * w.terms * w.numel
        out["evaluation_fp64_tflops_in_sketch_fn"] = round(ev / (t_sk / steps) / 1e12, 2)
    else:
        out.update({"sketch_entries_per_s": round(w.numel / (kms * 1e-3), 1),
                    "sketch_fp64_tflops": round(flops / (kms * 1e-3) / 1e12, 2),
                    "sketch_fp64_frac": round(flops / (kms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)})
    return out


def run_adjoint(steps, warmup):
    """Forward PSTT2 + X~ and the hand-written gradient of ||X - X~||_F^2 on the d=4, n=48 FP32 tensor."""
    import torch
    import inputs
    import paper_2111_10448_amd as P

    w = inputs.WORKLOADS["c5"]
    x = inputs.make_tensor(w)
    psi, omega = inputs.drm_factors(w)
    fac = inputs.pack_factors(psi, omega, w.d)
    xg = torch.from_numpy(x).to("cuda:0")
    ctx = P.PSTT2(w.n, w.ell, fac, dtype=w.dtype, prec="f32", ranks=w.ranks())
    fwd = bwd = 0.0
    for it in range(warmup + steps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        ctx.reset()
        ctx.sketch(xg)
        tt = ctx.recover()
        xt = tt.reconstruct(dtype=xg.dtype)
        torch.cuda.synchronize()
        b = time.perf_counter()
        g = ctx.vjp(tt, x=xg)
        torch.cuda.synchronize()
        c = time.perf_counter()
        if it >= warmup:
            fwd += b - a
            bwd += c - b
        tt.free()
    loss = float(torch.sum((xg.double() - xt.double()) ** 2))
    out = {"workload": f"c5: d={w.d} n={w.n[0]} ({w.numel} entries, f32), TT rank {w.tt_rank} + noise "
                       f"{w.noise:g}, ranks {w.rank}, sketch size {w.ell}",
           "forward_ms": round(fwd * 1e3 / steps, 4), "vjp_ms": round(bwd * 1e3 / steps, 4),
           "loss": loss, "grad_norm": float(torch.linalg.vector_norm(g.double()))}
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--prec", default=None)
    ap.add_argument("--algo", default="pstt2", choices=["pstt2", "pstt"],
                    help="two-sided PSTT2 (default) or the one-sided PSTT for the main line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the two-sided middle core, the precision study (1/sum tensor in FP64, FP32, "
                         "split BF16, BF16), the 64-slab stream, the adjoint and Table 1's Hilbert tensors")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run a 2 GiB device copy (counter calibration under rocprofv3) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path (asked for {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calib:
        a = torch.empty(1 << 28, dtype=torch.float64, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8, "launches": 3}))
        return

    import inputs
    name = args.workload
    w = inputs.WORKLOADS[name]
    prec = args.prec or ("f64" if w.dtype == "f64" else "f32")
    r = run_workload(name, prec, args.steps, args.warmup, algo=args.algo)
    w = r["workload"]
    value = r["bytes"] / (r["ms_per_step"] * 1e-3) / 1e9
    kb = r["bytes"] / r["launches_per_step"] if r["launches_per_step"] else r["bytes"]
    achieved = kb / (r["kernel_ms"] * 1e-3) / 1e9
    flops = 4.0 * w.ell * w.numel
    record = {
        "metric": "PSTT2 sketch GB/s & % HBM roofline, FP64 vs mixed-prec at stated TT error",
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": f"{name}: d={w.d} n={w.n[0]} ({w.numel} entries, {w.dtype}), random Gaussian TT "
                               f"rank {w.tt_rank}, noise {w.noise:g}, target rank {w.rank}, sketch size {w.ell}",
                   "ranks": r["ranks"], "tt_rel_error": r["err"], "decompose_ms": round(r["decomp_ms"], 4),
                   "sketch_kernel_ms": round(r["kernel_ms"], 4),
                   "sketch_gbs": round(achieved, 2), "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_profiles(name, prec),
                     "fp64_frac": round(flops / (r["kernel_ms"] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)},
    }
    if not args.no_variants:
        var = {}
        for wn, vp, mid, drm, algo in (("c2", "f64", "twosided", "nested", "pstt2"),
                                       ("c2", "f64", "twopass", "nested", "pstt2"),
                                       ("c2", "f64", "onepass", "independent", "pstt2"),
                                       ("c2", "f64", "onepass", "nested", "pstt"),
                                       ("c3_f64", "f64", "onepass", "nested", "pstt2"),
                                       ("c3", "f64", "onepass", "nested", "pstt2"),   # FP32 data, FP64 arithmetic
                                       ("c3", "f32", "onepass", "nested", "pstt2"),
                                       ("c3", "bf16x3", "onepass", "nested", "pstt2"),
                                       ("c3", "bf16", "onepass", "nested", "pstt2"),
                                       ("c3", "f16", "onepass", "nested", "pstt2"),
                                       ("c4", "f32", "onepass", "nested", "pstt2"),
                                       ("c4", "bf16x3", "onepass", "nested", "pstt2"),
                                       ("c4", "f16", "onepass", "nested", "pstt2")):
            key = (f"{wn}_{vp}" + ("" if mid == "onepass" else f"_{mid}") + ("" if drm == "nested" else f"_{drm}")
                   + ("" if algo == "pstt2" else f"_{algo}"))
            try:
                rv = run_workload(wn, vp, max(3, args.steps // 2), 1, mid=mid, drm=drm, algo=algo)
                wv = rv["workload"]
                # the independent scheme streams X once per pass group (max(m, d - m) groups)
                groups = max((wv.d + 1) // 2, wv.d - (wv.d + 1) // 2) if drm == "independent" else 1
                kbv = rv["bytes"] * groups / max(rv["launches_per_step"], 1)
                var[key] = {"workload": wn, "sketch_arithmetic": vp, "middle_core": mid, "drm": drm, "algorithm": algo,
                            "sketch_launches_per_step": rv["launches_per_step"],
                           "sketch_kernel_ms": round(rv["kernel_ms"], 4),
                           "sketch_gbs": round(kbv / (rv["kernel_ms"] * 1e-3) / 1e9, 2),
                           "traffic": traffic_from_profiles(wn, vp) if (mid, drm, algo) == ("onepass", "nested", "pstt2")
                           else None,
                           "ms_per_step": round(rv["ms_per_step"], 4), "ranks": rv["ranks"],
                           "tt_rel_error": rv["err"]}
            except Exception as e:   # report, keep the headline line
                var[key] = {"error": str(e)}
        record["variants"] = var
        small = {}
        for wn, vp in (("c1", "f64"), ("c5", "f32")):   # latency-bound: time only
            try:
                rv = run_workload(wn, vp, max(3, args.steps // 2), 1)
                small[wn] = {"sketch_arithmetic": vp, "ms_per_step": round(rv["ms_per_step"], 4),
                             "decompose_ms": round(rv["decomp_ms"], 4), "ranks": rv["ranks"],
                             "tt_rel_error": rv["err"]}
            except Exception as e:
                small[wn] = {"error": str(e)}
        record["small_configs"] = small
        try:
            record["adjoint"] = run_adjoint(max(3, args.steps // 2), 1)
        except Exception as e:
            record["adjoint"] = {"error": str(e)}
        t1 = {}
        for wn in ("t1_d3", "t1_d5", "t1_d9"):
            try:
                t1[wn] = run_function(wn, max(3, args.steps // 2), 1)
            except Exception as e:
                t1[wn] = {"error": str(e)}
        record["table1_hilbert"] = t1
        try:
            record["gauss_bumps"] = run_function("gb_d3", max(3, args.steps // 2), 1)
        except Exception as e:
            record["gauss_bumps"] = {"error": str(e)}
        try:
            record["gauss_bumps_twopass"] = run_function("gb_d3", max(3, args.steps // 2), 1, mid="twopass")
        except Exception as e:
            record["gauss_bumps_twopass"] = {"error": str(e)}
        for pr in ("f32", "bf16x3"):
            try:
                record[f"gauss_bumps_{pr}"] = run_function("gb_d3", max(3, args.steps // 2), 1, prec=pr)
            except Exception as e:
                record[f"gauss_bumps_{pr}"] = {"error": str(e)}
    try:
        record["roofline"]["read_reduce_gbs"] = round(read_reduce_gbs(r["bytes"]), 1)
    except Exception as e:
        record["roofline"]["read_reduce_gbs"] = str(e)
    if not args.no_cpu_baseline:
        record["cpu_baseline"] = cpu_baseline(r["x"], w, r["psi"], r["omega"], prec)
    print(json.dumps(record), flush=True)


if __name__ == "__main__":
    main()
