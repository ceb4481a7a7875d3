"""Pins of the oracle adjoint (oracle/tt_adjoint.py) by finite differences.

The loss is L(X) = ||X - X~(X)||_F^2, X~ the PSTT2-onepass approximation with
the CPQR pivots and ranks of the forward pass held fixed.  Central differences
of the numpy forward pass (oracle.tt_sketch steps) pin the torch-autograd
gradient and the vector-Jacobian product J^T gbar.
"""
import numpy as np
import pytest

import inputs
from oracle import tt_adjoint as A
from oracle import tt_sketch as O


def _setup(name, n=None, middle="onepass", scheme="nested"):
    w = inputs.WORKLOADS[name]
    if n is not None:
        w = inputs.Workload(w.name, w.index, tuple(n), "f64", w.kind, tt_rank=w.tt_rank, noise=w.noise,
                            ell=w.ell, rank=w.rank)
    x = inputs.make_tensor(w).astype(np.float64)
    if scheme == "nested":
        psi, om = inputs.drm_factors(w)
        drm = O.NestedKR(psi, om)
    else:
        psi, om = inputs.drm_factors_independent(w)
        drm = O.IndependentKR(psi, om)
    ref = O.pstt2(x, w.n, drm, ranks=w.ranks(), middle=middle)
    ref["middle"] = middle
    return w, x, drm, ref


def _frozen(x, w, drm, ref):
    return A.pstt2_frozen(x, w.n, drm, ref["ranks"], ref["piv"], middle=ref["middle"])


def _vjp(x, w, drm, ref, gbar=None):
    return A.pstt2_vjp(x, w.n, drm, ref["ranks"], ref["piv"], gbar=gbar, middle=ref["middle"])


def _loss(x, w, drm, ref):
    return float(np.sum((x - O.tt_full(_frozen(x, w, drm, ref))) ** 2))


# (workload, modes, middle-core rule, DRM scheme); d = 3..5 so the two-sided
# rule is exercised with m = 2 and m = 3, and d = 2 covers its one-pass limit
CASES = [("c5_fd", None, "onepass", "nested"), ("c5_fd", (6, 5, 7), "onepass", "nested"),
         ("c5_fd", (5, 4, 6, 3, 4), "onepass", "nested"),
         ("c5_fd", None, "twosided", "nested"), ("c5_fd", (6, 5, 7), "twosided", "nested"),
         ("c5_fd", (5, 4, 6, 3, 4), "twosided", "nested"), ("c5_fd", (9, 7), "twosided", "nested"),
         ("c5_fd", None, "onepass", "independent"), ("c5_fd", (5, 4, 6, 3, 4), "onepass", "independent"),
         ("c5_fd", (5, 4, 6, 3, 4), "twosided", "independent")]


@pytest.mark.parametrize("name,n,middle,scheme", CASES)
def test_frozen_forward_reproduces_pstt2(name, n, middle, scheme):
    w, x, drm, ref = _setup(name, n, middle, scheme)
    cores = _frozen(x, w, drm, ref)
    for a, b in zip(cores, ref["cores"]):
        assert np.abs(a - b).max() < 1e-10 * max(1.0, np.abs(b).max())
    xt = A.reconstruct_frozen_torch(x, w.n, drm, ref["ranks"], ref["piv"], middle)
    assert np.linalg.norm(xt - O.tt_full(cores)) < 1e-11 * np.linalg.norm(xt)


@pytest.mark.parametrize("name,n,middle,scheme", CASES)
def test_gradient_matches_directional_differences(name, n, middle, scheme):
    """20 random unit directions v: (L(x + hv) - L(x - hv)) / 2h = <grad L, v>."""
    w, x, drm, ref = _setup(name, n, middle, scheme)
    g = _vjp(x, w, drm, ref)
    rng = np.random.default_rng(7)
    # the mismatch falls as h^2 (truncation) down to h ~ 3e-6 of the entry scale,
    # where it is still ~1e-10: this step keeps it below 1e-7 on every case
    h = 2e-5 * np.linalg.norm(x) / np.sqrt(x.size)
    worst = 0.0
    for _ in range(20):
        v = rng.standard_normal(x.size)
        v /= np.linalg.norm(v)
        fd = (_loss(x + h * v, w, drm, ref) - _loss(x - h * v, w, drm, ref)) / (2 * h)
        worst = max(worst, abs(fd - g @ v) / np.linalg.norm(g))
    assert worst < 1e-6, worst


@pytest.mark.parametrize("name,n,middle,scheme", CASES)
def test_vjp_matches_directional_differences(name, n, middle, scheme):
    """For a random cotangent gbar: d/dh <gbar, X~(x + hv)> = <J^T gbar, v>."""
    w, x, drm, ref = _setup(name, n, middle, scheme)
    rng = np.random.default_rng(8)
    gb = rng.standard_normal(x.size)
    jt = _vjp(x, w, drm, ref, gbar=gb)

    def f(xx):
        return float(gb @ O.tt_full(_frozen(xx, w, drm, ref)))

    h = 1e-3 * np.linalg.norm(x) / np.sqrt(x.size)
    worst = 0.0
    for _ in range(20):
        v = rng.standard_normal(x.size)
        v /= np.linalg.norm(v)
        fd = (f(x + h * v) - f(x - h * v)) / (2 * h)
        worst = max(worst, abs(fd - jt @ v) / np.linalg.norm(jt))
    assert worst < 1e-6, worst


@pytest.mark.parametrize("middle,scheme", [("onepass", "nested"), ("twosided", "independent")])
def test_gradient_every_entry_n8(middle, scheme):
    """All 4096 entries of the d=4, n=8 gradient by central differences."""
    w, x, drm, ref = _setup("c5_fd", None, middle, scheme)
    g = _vjp(x, w, drm, ref)
    # single-entry directions move the bases the most: the O(h^2) term needs a small step
    h = 1e-5 * np.linalg.norm(x) / np.sqrt(x.size)
    fd = np.empty_like(g)
    e = np.zeros_like(x)
    for i in range(x.size):
        e[i] = h
        fd[i] = (_loss(x + e, w, drm, ref) - _loss(x - e, w, drm, ref)) / (2 * h)
        e[i] = 0.0
    assert np.abs(fd - g).max() < 1e-6 * np.abs(g).max()


def test_planted_mistakes_are_caught():
    """Dropping the Jacobian term, or transposing the cotangent's layout, breaks the FD check."""
    w, x, drm, ref = _setup("c5_fd")
    g = _vjp(x, w, drm, ref)
    xt = O.tt_full(_frozen(x, w, drm, ref))
    assert np.linalg.norm(2 * (x - xt) - g) > 1e-2 * np.linalg.norm(g)
    rng = np.random.default_rng(9)
    gb = rng.standard_normal(x.size)
    jt = A.pstt2_vjp(x, w.n, drm, ref["ranks"], ref["piv"], gbar=gb)
    gbt = gb.reshape(w.n, order="F").transpose(3, 2, 1, 0).reshape(-1, order="F")
    jt_wrong = A.pstt2_vjp(x, w.n, drm, ref["ranks"], ref["piv"], gbar=gbt)
    assert np.linalg.norm(jt_wrong - jt) > 1e-2 * np.linalg.norm(jt)
