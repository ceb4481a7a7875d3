"""Pins for the oracle's unfoldings, Khatri-Rao DRMs and sketches (CPU only).

Each check compares the oracle with something other than itself: explicit
index loops over multi-indices, numpy's Kronecker product, the paper's block
form of the Khatri-Rao sketch (equation "sketch_orig", Section 3.2) and the
closed form for a rank-one tensor.
"""
import itertools

import numpy as np
import pytest

import inputs
from oracle import tt_sketch as O


def _flat_index(idx, n):
    f, s = 0, 1
    for i, nk in zip(idx, n):
        f += i * s
        s *= nk
    return f


def _tiny(n, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(int(np.prod(n)))


def _factors(n, ell, seed=1):
    rng = np.random.default_rng(seed)
    d = len(n)
    psi = {q: rng.standard_normal((n[q - 1], ell)) for q in range(1, d)}
    omega = {q: rng.standard_normal((n[q - 1], ell)) for q in range(2, d + 1)}
    return psi, omega


@pytest.mark.parametrize("n", [(2, 3, 4, 2), (3, 1, 2, 5), (4, 3)])
def test_unfold_matches_multi_index(n):
    """X_k(row, col) with row = (i_1..i_k), col = (i_{k+1}..i_d), i_1 fastest (Section 2.1)."""
    x = _tiny(n)
    d = len(n)
    for k in range(1, d):
        xk = O.unfold(x, n, k)
        assert xk.shape == (O.rows_of(n, k), O.cols_of(n, k))
        for idx in itertools.product(*[range(v) for v in n]):
            row = _flat_index(idx[:k], n[:k])
            col = _flat_index(idx[k:], n[k:])
            assert xk[row, col] == x[_flat_index(idx, n)]


def test_kmode_product_definition():
    """Equation "kfold": (X x_k A)_{..j..} = sum_{i_k} X_{..i_k..} A_{j,i_k}."""
    n = (3, 4, 2)
    x = _tiny(n)
    a = np.random.default_rng(5).standard_normal((5, 4))
    y = O.kmode_product(x, n, 2, a)
    nn = (3, 5, 2)
    for i1, j, i3 in itertools.product(range(3), range(5), range(2)):
        ref = sum(x[_flat_index((i1, i2, i3), n)] * a[j, i2] for i2 in range(4))
        assert abs(y[_flat_index((i1, j, i3), nn)] - ref) < 1e-13


def test_khatri_rao_matches_kron():
    rng = np.random.default_rng(2)
    mats = [rng.standard_normal((nk, 4)) for nk in (3, 2, 5)]
    kr = O.khatri_rao(mats)
    assert kr.shape == (30, 4)
    for c in range(4):
        ref = np.kron(np.kron(mats[0][:, c], mats[1][:, c]), mats[2][:, c])
        np.testing.assert_array_equal(kr[:, c], ref)


@pytest.mark.parametrize("n", [(3, 2, 4, 3), (2, 3, 2, 2, 3), (5, 4)])
def test_sketches_bruteforce(n):
    """S_k = X_k Omega_k and T_k = Psi_k^T X_k against explicit multi-index sums."""
    ell = 3
    d = len(n)
    x = _tiny(n)
    psi, omega = _factors(n, ell)
    drm = O.NestedKR(psi, omega)
    for k in range(1, d):
        rk, ck = O.rows_of(n, k), O.cols_of(n, k)
        s_ref = np.zeros((rk, ell))
        t_ref = np.zeros((ell, ck))
        for idx in itertools.product(*[range(v) for v in n]):
            row = _flat_index(idx[:k], n[:k])
            col = _flat_index(idx[k:], n[k:])
            xv = x[_flat_index(idx, n)]
            for c in range(ell):
                w = np.prod([omega[q][idx[q - 1], c] for q in range(k + 1, d + 1)])
                s_ref[row, c] += xv * w
                v = np.prod([psi[q][idx[q - 1], c] for q in range(1, k + 1)])
                t_ref[c, col] += v * xv
        s_dense = O.sketch_right_dense(x, n, k, drm.omega_dense(k, d))
        s_mode = O.sketch_right_modewise(x, n, k, drm.right_factors(k, d))
        t_dense = O.sketch_left_dense(x, n, k, drm.psi_dense(k))
        t_mode = O.sketch_left_modewise(x, n, k, drm.left_factors(k))
        for a in (s_dense, s_mode):
            np.testing.assert_allclose(a, s_ref, rtol=1e-12, atol=1e-12)
        for a in (t_dense, t_mode):
            np.testing.assert_allclose(a, t_ref, rtol=1e-12, atol=1e-12)


def test_sketch_orig_block_form():
    """Equation "sketch_orig": X_j Omega_j = sum over blocks (X_j)_I Psi_{j+1} D_{l_d} ... D_{l_{j+2}}.

    (X_j)_I are the blocks of n_{j+1} consecutive columns of X_j; D_{l_q} is the
    diagonal matrix of row l_q of the q-th factor.
    """
    n = (2, 3, 4, 3, 2)
    d = len(n)
    ell = 4
    x = _tiny(n, 7)
    psi, omega = _factors(n, ell, 8)
    drm = O.NestedKR(psi, omega)
    for j in range(1, d - 1):
        xj = O.unfold(x, n, j)
        nb = n[j]                       # block width n_{j+1}
        slow = n[j + 1:]                 # modes j+2..d
        acc = np.zeros((xj.shape[0], ell))
        for blk, lidx in enumerate(itertools.product(*[range(v) for v in slow[::-1]])):
            lidx = lidx[::-1]            # (l_{j+2}, ..., l_d), l_{j+2} fastest
            b = _flat_index(lidx, slow)
            dprod = np.ones(ell)
            for q, lq in zip(range(j + 2, d + 1), lidx):
                dprod = dprod * omega[q][lq, :]
            acc += (xj[:, b * nb:(b + 1) * nb] @ omega[j + 1]) @ np.diag(dprod)
        ref = O.sketch_right_dense(x, n, j, drm.omega_dense(j, d))
        np.testing.assert_allclose(acc, ref, rtol=1e-12, atol=1e-12)


def test_rank_one_closed_form():
    """X = a_1 o ... o a_d: S_k(row, c) = (a_1..a_k)(row) prod_{q>k} <a_q, omega_q(:, c)>."""
    n = (4, 3, 5, 2, 3)
    d = len(n)
    ell = 5
    rng = np.random.default_rng(11)
    a = [rng.standard_normal(nk) for nk in n]
    x = a[0]
    for v in a[1:]:
        x = np.kron(v, x)       # earlier modes fastest
    psi, omega = _factors(n, ell, 12)
    drm = O.NestedKR(psi, omega)
    for k in range(1, d):
        left = a[0]
        for v in a[1:k]:
            left = np.kron(v, left)
        right = a[k]
        for v in a[k + 1:]:
            right = np.kron(v, right)
        wr = np.prod([a[q - 1] @ omega[q] for q in range(k + 1, d + 1)], axis=0)
        wl = np.prod([a[q - 1] @ psi[q] for q in range(1, k + 1)], axis=0)
        np.testing.assert_allclose(O.sketch_right_modewise(x, n, k, drm.right_factors(k, d)),
                                   np.outer(left, wr), rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(O.sketch_left_modewise(x, n, k, drm.left_factors(k)),
                                   np.outer(wl, right), rtol=1e-11, atol=1e-12)


def test_two_sided_invariant_and_linearity():
    """Psi_m^T Y_R = T_m Omega_m; sketches are linear and additive over column slabs."""
    w = inputs.WORKLOADS["c2_small"]
    x = inputs.make_tensor(w)
    n = w.n
    d = len(n)
    m = O.middle_index(d)
    psi, omega = inputs.drm_factors(w)
    drm = O.NestedKR(psi, omega)
    y = O.sketch_right_modewise(x, n, m, drm.right_factors(m, d))
    t = O.sketch_left_modewise(x, n, m, drm.left_factors(m))
    lhs = drm.psi_dense(m).T @ y
    rhs = t @ drm.omega_dense(m, d)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10, atol=1e-12 * np.abs(lhs).max())
    # linearity
    x2 = _tiny(n, 3)
    y2 = O.sketch_right_modewise(x2, n, m, drm.right_factors(m, d))
    y12 = O.sketch_right_modewise(2.0 * x - 0.5 * x2, n, m, drm.right_factors(m, d))
    np.testing.assert_allclose(y12, 2.0 * y - 0.5 * y2, rtol=1e-11, atol=1e-13)
    # slab additivity: zero out everything but one run of whole fibres
    slabs = inputs.slab_bounds(x.size, n[0], 5)
    acc = np.zeros_like(y)
    for first, count in slabs:
        xs = np.zeros_like(x)
        xs[first:first + count] = x[first:first + count]
        acc += O.sketch_right_modewise(xs, n, m, drm.right_factors(m, d))
    np.testing.assert_allclose(acc, y, rtol=1e-11, atol=1e-13)


def test_independent_factors_differ_per_split():
    """The independent scheme gives each split its own factors; the nested one shares them."""
    w = inputs.WORKLOADS["c1"]
    psi, omega = inputs.drm_factors_independent(w)
    ind = O.IndependentKR(psi, omega)
    d = w.d
    assert not np.allclose(ind.right_factors(1, d)[-1], ind.right_factors(2, d)[-1])
    x = inputs.make_tensor(w)
    for k in range(1, d):
        np.testing.assert_allclose(O.sketch_right_modewise(x, w.n, k, ind.right_factors(k, d)),
                                   O.sketch_right_dense(x, w.n, k, ind.omega_dense(k, d)),
                                   rtol=1e-11, atol=1e-10)
