"""Pins for the oracle's recovery path: bases, cores, middle core, TT evaluation (CPU only).

What fixes the expected values here (none of them is the oracle itself):
  * exact recovery: a tensor that is exactly a TT with ranks r_k has unfoldings of
    rank r_k (equation "TT_trivial"); with sketch size >= r_k the sketch spans the
    column/row space, so Theorem 2 with a zero tail gives X~ = X, and the
    pseudo-inverse of the one-pass middle core exists with probability one;
  * the deterministic bound "proj_acc" (proof of Theorem 2) for two-pass PSTT2;
  * the expectation bounds of Theorems 3 and 4 (Monte Carlo over Gaussian DRMs);
  * LAPACK's pivoted QR invariants; closed-form spectra for the tolerance rule;
  * the entry formula of Section 2.2 evaluated by brute force;
  * Table 1's printed tensor and TT sizes.
"""
import itertools
import json
import os

import numpy as np
import pytest

import inputs
from oracle import tt_sketch as O
from oracle import tt_svd as TS

HERE = os.path.dirname(os.path.abspath(__file__))


def _exact_tt(n, rank, seed):
    rng = np.random.default_rng(seed)
    cores = inputs.random_tt_cores(rng, n, rank)
    return inputs.dense_from_cores(cores), cores


def _kr(n, ell, seed):
    rng = np.random.default_rng(seed)
    d = len(n)
    psi = {q: rng.standard_normal((n[q - 1], ell)) for q in range(1, d)}
    omega = {q: rng.standard_normal((n[q - 1], ell)) for q in range(2, d + 1)}
    return O.NestedKR(psi, omega)


def _ind(n, ell, seed):
    rng = np.random.default_rng(seed)
    d = len(n)
    psi = {k: {q: rng.standard_normal((n[q - 1], ell)) for q in range(1, k + 1)} for k in range(1, d)}
    omega = {k: {q: rng.standard_normal((n[q - 1], ell)) for q in range(k + 1, d + 1)} for k in range(1, d)}
    return O.IndependentKR(psi, omega)


def _dense(n, ell, seed):
    rng = np.random.default_rng(seed)
    d = len(n)
    psi = {k: rng.standard_normal((O.rows_of(n, k), ell)) for k in range(1, d)}
    omega = {k: rng.standard_normal((O.cols_of(n, k), ell)) for k in range(1, d)}
    return O.DenseDRM(psi, omega)


CASES = [
    ((7, 9), 3, 5),
    ((5, 6, 4), 3, 6),
    ((4, 5, 3, 6), 3, 6),
    ((16, 16, 16, 16), 3, 6),
    ((3, 4, 5, 4, 3), 2, 5),
    ((4, 3, 3, 4, 3, 2), 3, 7),
    ((3, 2, 3, 2, 3, 2, 2), 2, 4),
    ((8, 8, 8, 8), 6, 12),       # sketch size larger than n: wide first/last sketches
]


@pytest.mark.parametrize("n,rank,ell", CASES)
@pytest.mark.parametrize("middle", ["onepass", "twosided", "twopass"])
@pytest.mark.parametrize("scheme", ["nested", "independent", "dense"])
def test_exact_recovery(n, rank, ell, middle, scheme):
    x, cores = _exact_tt(n, rank, 100 + len(n))
    ranks = [c.shape[2] for c in cores[:-1]]
    drm = {"nested": _kr, "independent": _ind, "dense": _dense}[scheme](n, ell, 7)
    out = O.pstt2(x, n, drm, ranks=ranks, middle=middle)
    err = O.tt_error(x, out["cores"])
    assert err < 1e-11, err
    assert [g.shape for g in out["cores"]] == [c.shape for c in cores]


def test_onepass_equals_twopass_on_exact_rank():
    n = (6, 5, 7, 4, 5)
    x, cores = _exact_tt(n, 3, 3)
    drm = _kr(n, 8, 4)
    a = O.pstt2(x, n, drm, ranks=[3] * 4, middle="onepass")
    b = O.pstt2(x, n, drm, ranks=[3] * 4, middle="twopass")
    # same bases, so the middle cores agree up to rounding
    np.testing.assert_allclose(a["cores"][2], b["cores"][2], rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(O.tt_full(a["cores"]), O.tt_full(b["cores"]), rtol=1e-9, atol=1e-11)


def _proj_bound(x, n, out):
    m = out["m"]
    d = len(n)
    tot = 0.0
    for k in range(1, m):
        xk = O.unfold(x, n, k)
        q = out["Q"][k]
        tot += np.linalg.norm(xk - q @ (q.T @ xk)) ** 2
    for k in range(m, d):
        xk = O.unfold(x, n, k)
        p = out["P"][k]
        tot += np.linalg.norm(xk - (xk @ p) @ p.T) ** 2
    return tot


@pytest.mark.parametrize("seed", range(5))
def test_projection_bound_twopass(seed):
    """Equation "proj_acc" with column bases for k < m and row bases for k >= m."""
    n = (5, 4, 6, 3, 4)
    x, _ = _exact_tt(n, 4, seed)
    rng = np.random.default_rng(50 + seed)
    x = x + 0.05 * np.linalg.norm(x) / np.sqrt(x.size) * rng.standard_normal(x.size)
    out = O.pstt2(x, n, _kr(n, 6, seed), ranks=[2, 3, 3, 2], middle="twopass")
    err2 = np.linalg.norm(x - O.tt_full(out["cores"])) ** 2
    assert err2 <= _proj_bound(x, n, out) * (1 + 1e-10)


def _tails(x, n, ranks):
    out = []
    for j in range(1, len(n)):
        s = np.linalg.svd(O.unfold(x, n, j), compute_uv=False)
        out.append(float(np.sum(s[ranks[j - 1]:] ** 2)))
    return out


def test_theorem3_expectation_bound_monte_carlo():
    """E||X - X~||^2 <= sum_j (1 + r_j/(p-1)) tail_j  (Theorem 3, Gaussian DRMs, p >= 2).

    The theorem holds for PSTT and, as stated at the end of Section 3.2, for PSTT2.
    """
    n = (4, 5, 4, 5)
    rng = np.random.default_rng(9)
    x, _ = _exact_tt(n, 3, 9)
    x = x + 0.3 * np.linalg.norm(x) / np.sqrt(x.size) * rng.standard_normal(x.size)
    ranks = [2, 2, 2]
    p = 3
    ell = 2 + p
    tails = _tails(x, n, ranks)
    bound = sum((1 + r / (p - 1)) * t for r, t in zip(ranks, tails))
    errs_pstt2, errs_pstt = [], []
    for s in range(300):
        drm = _dense(n, ell, 1000 + s)
        out = O.pstt2(x, n, drm, ranks=ranks, middle="twopass")
        errs_pstt2.append(np.linalg.norm(x - O.tt_full(out["cores"])) ** 2)
        out = O.pstt(x, n, drm, ranks=ranks)
        errs_pstt.append(np.linalg.norm(x - O.tt_full(out["cores"])) ** 2)
    assert np.mean(errs_pstt2) <= bound
    assert np.mean(errs_pstt) <= bound
    # and the error is not trivially zero: the bound is exercised
    assert np.mean(errs_pstt) > 0.3 * sum(tails)


def test_theorem4_onepass_expectation_bound_monte_carlo():
    """PSTT-onepass: E||X - X~~||^2 <= sum_{j<d-1} (1+r_j/(p-1)) tail_j + (1+r_{d-1}/(p-1))^2 tail_{d-1}."""
    n = (4, 5, 4, 5)
    rng = np.random.default_rng(19)
    x, _ = _exact_tt(n, 3, 19)
    x = x + 0.3 * np.linalg.norm(x) / np.sqrt(x.size) * rng.standard_normal(x.size)
    ranks = [2, 2, 2]
    p = 3
    ell = 2 + p
    tails = _tails(x, n, ranks)
    bound = sum((1 + r / (p - 1)) * t for r, t in zip(ranks[:-1], tails[:-1]))
    bound += (1 + ranks[-1] / (p - 1)) ** 2 * tails[-1]
    errs = []
    rr = O.rows_of(n, len(n) - 1)
    for s in range(300):
        drm = _dense(n, ell, 5000 + s)
        psi = np.random.default_rng(9000 + s).standard_normal((rr, ell))
        out = O.pstt(x, n, drm, ranks=ranks, onepass_psi=psi)
        errs.append(np.linalg.norm(x - O.tt_full(out["cores"])) ** 2)
    assert np.mean(errs) <= bound
    assert np.mean(errs) > 0.3 * sum(tails)


def test_cpqr_invariants_and_pivots_of_r():
    """geqp3 invariants; the pivots of S equal the pivots of the R of an unpivoted QR of S."""
    rng = np.random.default_rng(3)
    s = rng.standard_normal((200, 12)) @ np.diag(np.logspace(0, -8, 12)) @ rng.standard_normal((12, 12))
    q, r, piv = O.cpqr_basis(s, 12)
    np.testing.assert_allclose(q.T @ q, np.eye(12), atol=1e-13)
    np.testing.assert_allclose(q @ r, s[:, piv], atol=1e-12 * np.abs(s).max())
    dg = np.diag(r)
    assert np.all(dg >= 0)
    assert np.all(np.diff(dg) <= 1e-12 * dg[0])
    r0 = np.linalg.qr(s, mode="r")
    _, _, piv_r = O.cpqr_basis(r0, 12)
    assert list(piv_r) == list(piv)


@pytest.mark.parametrize("sig,eps,d,rmax,expect", [
    ([1.0, 0.5, 1e-3, 1e-6, 1e-9], 1e-2, 2, 10, 2),
    ([1.0, 0.5, 1e-3, 1e-6, 1e-9], 1e-2, 5, 10, 2),
    ([1.0, 0.5, 1e-3, 1e-6, 1e-9], 2e-3, 2, 10, 2),
    ([1.0, 0.5, 1e-3, 1e-6, 1e-9], 4e-4, 2, 10, 3),
    ([1.0, 0.5, 1e-3, 1e-6, 1e-9], 1e-4, 2, 10, 3),
    ([1.0, 0.5, 1e-3, 1e-6, 1e-9], 1e-7, 2, 10, 4),
    ([1.0, 0.5, 1e-3, 1e-6, 1e-9], 1e-7, 2, 2, 2),
    ([1.0, 1.0, 1.0, 1.0], 0.49, 2, 10, 4),
    ([1.0, 1.0, 1.0, 1.0], 0.51, 2, 10, 3),
])
def test_rank_from_tolerance_closed_form(sig, eps, d, rmax, expect):
    """r = min{r : sum_{i>r} sigma_i^2 <= eps^2/(d-1) * sum sigma_i^2}, capped."""
    rng = np.random.default_rng(0)
    k = len(sig)
    u, _ = np.linalg.qr(rng.standard_normal((30, k)))
    v, _ = np.linalg.qr(rng.standard_normal((k, k)))
    s = u @ np.diag(sig) @ v.T
    assert O.rank_from_tolerance(s, eps, d, rmax) == expect


def test_tt_full_matches_entry_formula():
    n = (3, 4, 2, 3)
    rng = np.random.default_rng(1)
    cores = inputs.random_tt_cores(rng, n, 3)
    full = O.tt_full(cores)
    for idx in itertools.product(*[range(v) for v in n]):
        f = idx[0] + 3 * (idx[1] + 4 * (idx[2] + 2 * idx[3]))
        # entry formula written out with explicit sums over rank indices
        ref = 0.0
        for a in range(cores[0].shape[2]):
            for b in range(cores[1].shape[2]):
                for c in range(cores[2].shape[2]):
                    ref += (cores[0][0, idx[0], a] * cores[1][a, idx[1], b]
                            * cores[2][b, idx[2], c] * cores[3][c, idx[3], 0])
        assert abs(full[f] - ref) < 1e-12
        assert abs(O.tt_entry(cores, idx) - ref) < 1e-12
    # the input generator's dense builder agrees with the entry formula too
    np.testing.assert_allclose(inputs.dense_from_cores(cores), full, rtol=1e-13, atol=1e-13)


def test_tt_error_known_perturbation():
    n = (4, 5, 3)
    rng = np.random.default_rng(2)
    cores = inputs.random_tt_cores(rng, n, 2)
    x = O.tt_full(cores)
    e = np.zeros_like(x)
    e[7] = 0.25
    assert abs(O.tt_error(x + e, cores) - 0.25 / np.linalg.norm(x + e)) < 1e-15


def test_table1_sizes():
    """Table 1: tensor size 8 n^d / 2^30 and TT size 8 sum r_{k-1} n r_k / 2^20 (3 significant digits)."""
    with open(os.path.join(HERE, "golden", "table1.json")) as f:
        t1 = json.load(f)
    for case in t1["cases"]:
        n = [case["n"]] * case["d"]
        ts = 8.0 * float(case["n"]) ** case["d"] / 2 ** 30
        tt = 8.0 * O.tt_storage(n, case["r"]) / 2 ** 20
        assert float(f"{ts:.3g}") == case["tensor_size_gb"]
        assert float(f"{tt:.3g}") == case["tt_size_mb"]
    assert O.tt_storage([960] * 3, [1, 25, 25, 1]) == 648000
    assert O.tt_storage([96] * 5, [1, 17, 18, 18, 17, 1]) == 93120
    assert O.tt_storage([12] * 9, [1, 12, 18, 18, 19, 19, 18, 18, 12, 1]) == 25788


@pytest.mark.parametrize("n,rank", [((5, 6, 4, 3), 3), ((4, 4, 4, 4, 4), 2)])
def test_ttsvd_exact_and_bound(n, rank):
    x, cores = _exact_tt(n, rank, 21)
    c = TS.ttsvd(x, n, eps=1e-12)
    assert O.tt_error(x, c) < 1e-12
    assert [g.shape[2] for g in c[:-1]] == [g.shape[2] for g in cores[:-1]]
    rng = np.random.default_rng(22)
    y = x + 1e-3 * np.linalg.norm(x) / np.sqrt(x.size) * rng.standard_normal(x.size)
    for eps in (1e-1, 1e-2, 1e-4):
        for fn in (TS.ttsvd, TS.parallel_ttsvd):
            cc = fn(y, n, eps=eps)
            assert O.tt_error(y, cc) <= eps * (1 + 1e-12)


def test_inverse_sum_is_low_rank():
    """The Chebyshev 1/sum workload has rapidly decaying unfolding spectra (low numerical TT rank)."""
    w = inputs.WORKLOADS["c3_small"]
    x = inputs.make_tensor(w).astype(np.float64)
    c = TS.ttsvd(x, w.n, eps=1e-5)
    assert max(g.shape[2] for g in c[:-1]) <= 8
    assert O.tt_error(x, c) <= 1e-5


def test_planted_mistakes_are_caught(monkeypatch):
    """A transposed operand or dropped index in the core formulas breaks exact recovery."""
    n = (4, 5, 3, 4, 5)
    x, cores = _exact_tt(n, 3, 31)
    drm = _kr(n, 6, 32)

    def bad_right(p_prev, p_k, n_k):
        r_prev = p_prev.shape[1]
        c_k = p_k.shape[0]
        p3 = np.reshape(p_prev, (c_k, n_k, r_prev), order="F")   # wrong index order
        return np.einsum("cia,cb->aib", p3, p_k)

    monkeypatch.setattr(O, "outer_core_right", bad_right)
    out = O.pstt2(x, n, drm, ranks=[3] * 4)
    assert O.tt_error(x, out["cores"]) > 1e-3
    monkeypatch.undo()

    def bad_left(q_prev, q_k, n_k):
        w = q_prev.T @ np.reshape(q_k, (q_prev.shape[0], n_k * q_k.shape[1]), order="C")
        return np.reshape(w, (q_prev.shape[1], n_k, q_k.shape[1]), order="F")

    monkeypatch.setattr(O, "outer_core_left", bad_left)
    out = O.pstt2(x, n, drm, ranks=[3] * 4)
    assert O.tt_error(x, out["cores"]) > 1e-3
