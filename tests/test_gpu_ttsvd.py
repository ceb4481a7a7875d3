"""Parallel-TTSVD (Section 3.1) on the GPU against the oracle's
oracle.tt_svd.parallel_ttsvd on the same tensor: equal ranks, X~ to the FP64
tolerance, the error bound of Theorem perf_alg1 (||X - X~|| <= eps ||X||), and
the refused and degenerate cases."""
import time

import numpy as np
import pytest

import inputs
from oracle import tt_sketch as O
from oracle import tt_svd as TS

from gpu_common import TOL_XT, rel, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,n,eps", [
    ("c1", None, 1e-6),                   # d = 4, n = 16: rank 3 plus 1e-10 noise
    ("c5_fd", None, 1e-2),                # d = 4, n = 8, rank 6 plus 1e-3 noise
    ("c2_small", None, 3e-5),             # d = 6 ragged: 990 x 336 middle unfolding (noise floor 5.7e-6)
    ("c1", (37, 41), 1e-3),               # d = 2
    ("c1", (61, 47, 53), 1e-4),           # d = 3, long unfoldings both ways
])
def test_parallel_ttsvd_against_oracle(name, n, eps):
    import dataclasses
    import torch
    import paper_2111_10448_amd as P
    w = inputs.WORKLOADS[name]
    if n is not None:
        w = dataclasses.replace(w, name="ttsvd", index=130 + len(n), n=tuple(n), tt_rank=3)
    say(f"[gpu] Parallel-TTSVD {w.name} n={w.n} eps={eps:g}")
    x = np.asarray(inputs.make_tensor(w), dtype=np.float64)
    ref = TS.parallel_ttsvd(x, w.n, eps)
    xg = torch.from_numpy(x).cuda()
    t0 = time.perf_counter()
    tt = P.parallel_ttsvd(xg, w.n, eps)
    t1 = time.perf_counter()
    ranks_ref = [1] + [g.shape[2] for g in ref[:-1]] + [1]
    e_gpu, e_ref = tt.error(xg), O.tt_error(x, ref)
    d_xt = rel(tt.reconstruct().cpu().numpy(), O.tt_full(ref))
    say(f"    ranks {tt.ranks} (oracle {ranks_ref}), X~ {d_xt:.2e}, error {e_gpu:.3e} (oracle {e_ref:.3e}), "
        f"{(t1 - t0) * 1e3:.1f} ms")
    assert tt.ranks == ranks_ref
    assert d_xt < TOL_XT["f64"]
    assert e_gpu <= eps * (1 + 1e-9)
    assert abs(e_gpu - e_ref) <= 1e-10 + 1e-6 * e_ref
    tt.free()


def test_parallel_ttsvd_exact_rank_and_zero():
    import torch
    import paper_2111_10448_amd as P
    w = inputs.WORKLOADS["c1_exact"]
    say("[gpu] Parallel-TTSVD exact rank and X = 0")
    x = inputs.make_tensor(w)
    tt = P.parallel_ttsvd(torch.from_numpy(x).cuda(), w.n, 1e-10)
    assert tt.ranks == [1, 3, 3, 3, 1]
    assert tt.error(torch.from_numpy(x).cuda()) < 1e-13
    tt.free()
    z = torch.zeros(w.numel, dtype=torch.float64, device="cuda")
    tt = P.parallel_ttsvd(z, w.n, 1e-3)
    assert tt.ranks == [1] * (w.d + 1)
    assert not torch.any(tt.reconstruct())
    tt.free()


def test_parallel_ttsvd_rank_cap():
    """eps below the noise wants ranks past 32 at the middle split: the cap (rmax, else the
    library's rank limit of 32) binds and the cores are still a valid truncation."""
    import torch
    import paper_2111_10448_amd as P
    w = inputs.WORKLOADS["c1"]
    say("[gpu] Parallel-TTSVD rank caps")
    x = inputs.make_tensor(w)
    xg = torch.from_numpy(x).cuda()
    for rmax, want in ((0, [1, 16, 32, 16, 1]), (8, [1, 8, 8, 8, 1])):
        tt = P.parallel_ttsvd(xg, w.n, 1e-12, rmax=rmax)
        assert tt.ranks == want
        assert tt.error(xg) < 1e-9
        tt.free()


def test_parallel_ttsvd_refusals():
    import ctypes
    import torch
    import paper_2111_10448_amd as P
    from paper_2111_10448_amd import _lib as L
    say("[gpu] Parallel-TTSVD refusals")
    x = torch.zeros(16, dtype=torch.float64, device="cuda")
    for n, eps, why in [((2048, 2048), 1e-3, "short side"), ((4, 4), 0.0, "eps"), ((4, 4), 1.0, "eps")]:
        with pytest.raises(P.PSTT2Error) as e:
            P.parallel_ttsvd(x, n, eps)
        assert e.value.status == L.EINVAL and why in str(e.value)
    with pytest.raises(TypeError):
        P.parallel_ttsvd(x.float(), (4, 4), 1e-3)
