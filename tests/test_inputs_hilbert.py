"""Pins of the Hilbert-tensor inputs (Section 4.3) that the function path is checked against.

The generator and the entry sampler are the only things that define the
tensor on the host; the GPU evaluates its own entries inside the kernels.
"""
import itertools
import json
import os

import numpy as np

import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def test_hilbert_tensor_is_the_formula_entry_by_entry():
    """X(i_1, ..., i_d) = 1 / (1 - d + i_1 + ... + i_d), 1-based, column-major (mode 1 fastest)."""
    n = (4, 3, 5, 2)
    x = inputs.hilbert_tensor(n)
    d = len(n)
    for idx in itertools.product(*[range(1, k + 1) for k in n]):
        f = sum((i - 1) * int(np.prod(n[:q])) for q, i in enumerate(idx))
        assert x[f] == 1.0 / (1 - d + sum(idx))


def test_hilbert_entries_match_the_unfoldings():
    n = (5, 4, 6, 3)
    x = inputs.hilbert_tensor(n)
    for m in range(1, len(n)):
        R = int(np.prod(n[:m]))
        xm = x.reshape(-1, R).T                   # X_m, R x C column-major view
        rows = np.array([0, 3, R - 1])
        cols = np.array([0, 1, xm.shape[1] - 1])
        e = inputs.hilbert_entries(n, m, rows, cols)
        assert np.array_equal(e, xm[np.ix_(rows, cols)])


def test_table1_workloads_carry_the_printed_shapes_and_ranks():
    """The t1_* workloads are Table 1's tensors: sizes 8 n^d / 2^30 GB and the printed ranks."""
    g = json.load(open(os.path.join(HERE, "golden", "table1.json")))
    for case, name in zip(g["cases"], ("t1_d3", "t1_d5", "t1_d9")):
        w = inputs.WORKLOADS[name]
        assert w.kind == "hilbert" and w.n == (case["n"],) * case["d"]
        assert [1] + w.ranks() + [1] == case["r"]
        assert round(8 * w.numel / 2 ** 30, 2 if case["tensor_size_gb"] < 10 else 1) == case["tensor_size_gb"]
