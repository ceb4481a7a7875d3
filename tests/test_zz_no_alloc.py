"""tt_error_noalloc (the error pass in the library's static scratch, no
allocation of any kind) through the C ABI against tt_error on the same cores
and tensor: two calls in a row, the second on a smaller tensor, then FP32
data, and a pass too large for the static buffer, which is refused before
anything runs.  The library's device-memory count must not move."""
import ctypes

import numpy as np
import pytest

import inputs

from gpu_common import say

pytestmark = pytest.mark.gpu


def _noalloc(cs, xg, out):
    import torch
    import paper_2111_10448_amd as P
    from paper_2111_10448_amd import _lib as L
    code = L.F64 if xg.dtype == torch.float64 else L.F32
    return L.lib().tt_error_noalloc(ctypes.byref(cs), ctypes.c_void_p(xg.data_ptr()), code,
                                    ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(P._stream_handle()))


def _decomposed(name):
    import torch
    import paper_2111_10448_amd as P
    w = inputs.WORKLOADS[name]
    x = inputs.make_tensor(w)
    psi, omega = inputs.drm_factors(w)
    fac = inputs.pack_factors(psi, omega, w.d)
    xg = torch.from_numpy(x).cuda()
    with P.PSTT2(w.n, w.ell, fac, dtype=w.dtype, prec=w.dtype, ranks=w.ranks()) as ctx:
        ctx.sketch(xg)
        tt = ctx.recover()
    return x, xg, tt


def test_noalloc_error_matches_tt_error():
    import torch
    import paper_2111_10448_amd as P
    from paper_2111_10448_amd import _lib as L
    out = torch.full((3,), -1.0, dtype=torch.float64, device="cuda")
    for name in ("c2_twin", "c1", "c5_small"):      # larger, then smaller; the last one FP32
        x, xg, tt = _decomposed(name)
        ref = tt.error(xg)                      # the allocating entry point (host result)
        torch.cuda.synchronize()
        live = P.memory_stats()["live"]
        cs = tt.struct()
        say(f"[gpu] tt_error_noalloc {name} n={list(x.shape)} dtype={xg.dtype}")
        L.check(_noalloc(cs, xg, out))
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert P.memory_stats()["live"] == live, "the no-allocation pass allocated"
        x64 = np.asarray(x, dtype=np.float64)
        say(f"    noalloc {got[0]:.15e}  tt_error {ref:.15e}")
        assert abs(got[0] - ref) <= 1e-14 * ref, (got[0], ref)
        assert abs(got[2] - float(x64 @ x64)) <= 1e-12 * float(x64 @ x64)
        assert abs(np.sqrt(got[1] / got[2]) - got[0]) <= 1e-15 * got[0]
        tt.free()


def test_noalloc_error_refuses_oversized_pass():
    import torch
    import paper_2111_10448_amd as P
    from paper_2111_10448_amd import _lib as L
    # d = 4, n = (4096, 4096, 8, 8), rank 4: the left interface alone is 4096^2 x 4 doubles (512 MiB)
    n, r = (4096, 4096, 8, 8), [1, 4, 4, 4, 1]
    cores = [torch.zeros(r[k] * n[k] * r[k + 1], dtype=torch.float64, device="cuda") for k in range(4)]
    cs = P.cores_struct(cores, n, r)
    xg = torch.zeros(16, dtype=torch.float64, device="cuda")   # never read: refused first
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    say("[gpu] tt_error_noalloc oversized pass")
    st = _noalloc(cs, xg, out)
    assert st == L.ENOMEM
    assert "static buffer" in L.lib().pstt2_last_error(None).decode()
