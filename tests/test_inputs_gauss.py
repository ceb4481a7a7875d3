"""Pins of the Gaussian-bump tensor inputs (Section 4.4) that the function path is checked against."""
import itertools
import math

import numpy as np

import inputs


def test_gauss_tensor_is_the_formula_entry_by_entry():
    """X(i) = sum_j exp(-gamma sum_q (x_q - c_jq)^2), x_q = 2 i_q / n_q - 1 (1-based), column-major."""
    n = (4, 3, 5)
    rng = np.random.default_rng(3)
    ctr = rng.uniform(-1, 1, size=(7, 3))
    x = inputs.gauss_tensor(n, ctr, 10.0)
    for idx in itertools.product(*[range(1, k + 1) for k in n]):
        f = sum((i - 1) * int(np.prod(n[:q])) for q, i in enumerate(idx))
        want = sum(math.exp(-10.0 * sum((2.0 * i / nq - 1.0 - c[q]) ** 2 for q, (i, nq) in enumerate(zip(idx, n))))
                   for c in ctr)
        assert abs(x[f] - want) <= 1e-15 * abs(want)


def test_one_bump_is_separable_and_n_bumps_have_rank_at_most_n():
    """A single bump is a product of one function per mode: every unfolding has rank 1.
    A sum of three has rank at most 3 at every split."""
    n = (9, 8, 7, 6)
    rng = np.random.default_rng(4)
    for nb in (1, 3):
        x = inputs.gauss_tensor(n, rng.uniform(-1, 1, size=(nb, 4)), 2.0)
        for k in range(1, 4):
            R = int(np.prod(n[:k]))
            s = np.linalg.svd(x.reshape(-1, R).T, compute_uv=False)
            assert s[nb - 1] > 1e-8 * s[0] and s[nb] < 1e-13 * s[0], (nb, k, s[:nb + 1])


def test_gauss_entries_match_the_unfoldings():
    w = inputs.WORKLOADS["gb_small4"]
    ctr = inputs.gauss_centers(w)
    assert ctr.shape == (100, 4) and ctr.min() >= -1 and ctr.max() <= 1
    x = inputs.make_tensor(w)
    for m in range(1, 4):
        R = int(np.prod(w.n[:m]))
        xm = x.reshape(-1, R).T
        rows = np.array([0, 5, R - 1])
        cols = np.array([0, 2, xm.shape[1] - 1])
        e = inputs.gauss_entries(w.n, m, rows, cols, ctr, w.gamma)
        assert np.allclose(e, xm[np.ix_(rows, cols)], rtol=1e-14, atol=0)
