"""Pins for the oracle's two-sided pieces (CPU only): the sketches B_k = Psi_k^T X_k Omega_k
of every split and the two-sided one-pass middle core.

What fixes the expected values here (none of them is the formula under test
retyped):
  * B_k by brute force over every entry of small tensors, with the DRM entries
    formed as products of factor entries (equation "sketch_orig");
  * a rank-one tensor, where B_k factors into per-mode inner products;
  * B_k = Psi_k^T (X_k Omega_k) = (Psi_k^T X_k) Omega_k with the one-sided
    sketches taken mode by mode (a different code path);
  * exact recovery of exact-rank TTs, where every middle-core rule must give
    the two-pass core of equation "PSTT2_final_core";
  * the special case Psi' = Q_{m-1}: the mode-1 pseudo-inverse is then the
    identity and the rule reduces to the one-pass least-squares core;
  * planted mistakes in the rule, each caught.
"""
import itertools

import numpy as np
import pytest

from oracle import tt_sketch as O

from test_oracle_pstt2 import _exact_tt, _ind, _kr


def _brute_b(x, n, k, drm):
    d = len(n)
    psi = drm.left_factors(k)          # psi_1..psi_k
    om = drm.right_factors(k, d)       # omega_{k+1}..omega_d
    ell = psi[0].shape[1]
    b = np.zeros((ell, ell))
    xf = x.reshape(n, order="F")
    for idx in itertools.product(*[range(v) for v in n]):
        for a in range(ell):
            pa = 1.0
            for q in range(k):
                pa *= psi[q][idx[q], a]
            for c in range(ell):
                oc = 1.0
                for q in range(k, d):
                    oc *= om[q - k][idx[q], c]
                b[a, c] += xf[idx] * pa * oc
    return b


@pytest.mark.parametrize("scheme", ["nested", "independent"])
def test_two_sided_sketch_brute_force(scheme):
    n = (3, 4, 2, 3)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(int(np.prod(n)))
    drm = (_kr if scheme == "nested" else _ind)(n, 3, 6)
    for k in range(1, len(n)):
        np.testing.assert_allclose(O.two_sided_sketch(x, n, k, drm), _brute_b(x, n, k, drm), rtol=1e-12, atol=1e-12)


def test_two_sided_sketch_rank_one_closed_form():
    """X = u_1 o ... o u_d: B_k(a, c) = prod_{q<=k} <psi_q(:, a), u_q> * prod_{q>k} <omega_q(:, c), u_q>."""
    n = (5, 3, 4, 6, 2)
    rng = np.random.default_rng(11)
    us = [rng.standard_normal(v) for v in n]
    x = us[0]
    for u in us[1:]:
        x = np.kron(u, x)                      # column-major: the first mode varies fastest
    drm = _kr(n, 7, 12)
    d = len(n)
    for k in range(1, d):
        left = np.prod([drm.psi[q].T @ us[q - 1] for q in range(1, k + 1)], axis=0)
        right = np.prod([drm.omega[q].T @ us[q - 1] for q in range(k + 1, d + 1)], axis=0)
        np.testing.assert_allclose(O.two_sided_sketch(x, n, k, drm), np.outer(left, right), rtol=1e-11,
                                   atol=1e-12)


@pytest.mark.parametrize("scheme", ["nested", "independent"])
def test_two_sided_equals_both_one_sided_products(scheme):
    n = (4, 3, 5, 3, 4)
    rng = np.random.default_rng(21)
    x = rng.standard_normal(int(np.prod(n)))
    drm = (_kr if scheme == "nested" else _ind)(n, 6, 22)
    d = len(n)
    for k in range(1, d):
        s_k = O.sketch_right_modewise(x, n, k, drm.right_factors(k, d))
        t_k = O.sketch_left_modewise(x, n, k, drm.left_factors(k))
        b = O.two_sided_sketch(x, n, k, drm)
        np.testing.assert_allclose(b, drm.psi_dense(k).T @ s_k, rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(b, t_k @ drm.omega_dense(k, d), rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("n,rank,ell", [((5, 6, 4), 3, 6), ((4, 5, 3, 6), 3, 6), ((4, 3, 3, 4, 3, 2), 3, 7)])
@pytest.mark.parametrize("scheme", ["nested", "independent"])
def test_twosided_core_equals_twopass_on_exact_rank(n, rank, ell, scheme):
    x, cores = _exact_tt(n, rank, 40 + len(n))
    ranks = [c.shape[2] for c in cores[:-1]]
    drm = (_kr if scheme == "nested" else _ind)(n, ell, 41)
    a = O.pstt2(x, n, drm, ranks=ranks, middle="twosided")
    b = O.pstt2(x, n, drm, ranks=ranks, middle="twopass")
    m = a["m"]
    np.testing.assert_allclose(a["cores"][m - 1], b["cores"][m - 1], rtol=1e-9, atol=1e-11)
    assert O.tt_error(x, a["cores"]) < 1e-11


def test_twosided_with_basis_as_sketch_is_the_onepass_core():
    """Psi' = Q_{m-1} makes Psi'^T Q_{m-1} = I; on a noisy tensor the rule is then the LS core."""
    n = (5, 4, 6, 3, 5)
    rng = np.random.default_rng(3)
    x, _ = _exact_tt(n, 3, 3)
    x = x + 0.1 * np.linalg.norm(x) / np.sqrt(x.size) * rng.standard_normal(x.size)
    drm = _kr(n, 7, 4)
    out = O.pstt2(x, n, drm, ranks=[3] * 4, middle="onepass")
    m = out["m"]
    om = drm.omega_dense(m, len(n))
    q, p = out["Q"][m - 1], out["P"][m]
    g1 = O.middle_core_onepass(out["Y"], om, q, p, n[m - 1])
    g2 = O.middle_core_twosided(out["Y"], q, q, om, p, n[m - 1])
    np.testing.assert_allclose(g2, g1, rtol=1e-9, atol=1e-12)


def test_twosided_d2_is_the_onepass_rule():
    n = (7, 9)
    x, _ = _exact_tt(n, 3, 8)
    rng = np.random.default_rng(8)
    x = x + 0.05 * rng.standard_normal(x.size)
    drm = _kr(n, 5, 9)
    a = O.pstt2(x, n, drm, ranks=[3], middle="twosided")
    b = O.pstt2(x, n, drm, ranks=[3], middle="onepass")
    np.testing.assert_allclose(O.tt_full(a["cores"]), O.tt_full(b["cores"]), rtol=1e-12, atol=1e-13)


def test_twosided_noisy_error_is_near_twopass():
    """With noise the two-sided rule stays within a small factor of the two-pass core's error."""
    n = (4, 5, 4, 5, 4)
    rng = np.random.default_rng(17)
    x, _ = _exact_tt(n, 3, 17)
    x = x + 0.05 * np.linalg.norm(x) / np.sqrt(x.size) * rng.standard_normal(x.size)
    e2, e1 = [], []
    for s in range(20):
        drm = _kr(n, 8, 300 + s)
        e2.append(O.tt_error(x, O.pstt2(x, n, drm, ranks=[3] * 4, middle="twosided")["cores"]))
        e1.append(O.tt_error(x, O.pstt2(x, n, drm, ranks=[3] * 4, middle="twopass")["cores"]))
    assert np.mean(e2) <= 3.0 * np.mean(e1)
    assert np.mean(e2) >= np.mean(e1) * (1 - 1e-9)   # the two-pass core is the projection optimum


def test_planted_mistakes_are_caught(monkeypatch):
    n = (4, 5, 3, 4, 5)
    x, cores = _exact_tt(n, 3, 31)
    drm = _kr(n, 6, 32)
    good = O.middle_core_twosided

    def no_pinv(y_r, psi_prev, q_prev, omega_m, p_m, n_m):
        # treats Psi'^T Q as if it had orthonormal columns
        r_rows, ell = q_prev.shape[0], y_r.shape[1]
        h = np.einsum("ra,rjc->ajc", psi_prev, np.reshape(y_r, (r_rows, n_m, ell), order="F"))
        return np.einsum("ap,ajc,qc->pjq", psi_prev.T @ q_prev, h, np.linalg.pinv(omega_m.T @ p_m))

    def wrong_reshape(y_r, psi_prev, q_prev, omega_m, p_m, n_m):
        r_rows, ell = q_prev.shape[0], y_r.shape[1]
        y3 = np.reshape(y_r, (n_m, r_rows, ell), order="F").transpose(1, 0, 2)
        return good(np.reshape(y3, (-1, ell), order="F"), psi_prev, q_prev, omega_m, p_m, n_m)

    for bad in (no_pinv, wrong_reshape):
        monkeypatch.setattr(O, "middle_core_twosided", bad)
        out = O.pstt2(x, n, drm, ranks=[3] * 4, middle="twosided")
        assert O.tt_error(x, out["cores"]) > 1e-3, bad.__name__
        monkeypatch.undo()
