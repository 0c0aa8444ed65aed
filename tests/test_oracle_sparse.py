"""Pins of the oracle's sparse-to-MPO conversion (Algorithm 4.1)."""

import json
import os

import numpy as np

from oracle import tnrsvd_oracle as o

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def coo(A):
    r, c = np.nonzero(A)
    return r, c, A[r, c]


def test_paper_2x6_example():
    """The 2 x 6 matrix of Sec. 4.2 with I = (1, 1, 2), J = (1, 3, 2): two nonzero
    1 x 1 blocks, so rank 2, and the sum of the paper's two Kronecker terms."""
    g = json.load(open(os.path.join(GOLD, "sparse_2x6_example.json")))
    A = np.array(g["matrix"], dtype=float)
    M = o.sparse_to_mpo(*coo(A), g["dims_I"], g["dims_J"])
    assert [c.shape for c in M] == [(1, 1, 1, 2), (2, 1, 3, 2), (2, 2, 2, 1)]
    np.testing.assert_array_equal(o.mpo_to_dense(M), A)


def test_rank_is_number_of_nonzero_blocks_and_densifies_exactly():
    rng = np.random.default_rng(0)
    rows, cols = [4, 2, 2, 2], [4, 2, 2, 2]            # 32 x 32, blocks of 4 x 4
    A = np.zeros((32, 32))
    for _ in range(40):                                  # a random banded pattern
        i = int(rng.integers(0, 32))
        j = min(31, max(0, i + int(rng.integers(-5, 6))))
        A[i, j] = rng.standard_normal()
    M = o.sparse_to_mpo(*coo(A), rows, cols)
    nb = len({(i // 4, j // 4) for i, j in zip(*np.nonzero(A))})
    assert M[0].shape == (1, 4, 4, nb) and M[-1].shape == (nb, 2, 2, 1)
    np.testing.assert_array_equal(o.mpo_to_dense(M), A)


def test_duplicates_add_and_zero_matrix():
    rows, cols = [2, 2], [2, 2]
    r = np.array([0, 0, 3]); c = np.array([1, 1, 2]); v = np.array([1.5, 2.0, -1.0])
    M = o.sparse_to_mpo(r, c, v, rows, cols)
    D = o.mpo_to_dense(M)
    assert D[0, 1] == 3.5 and D[3, 2] == -1.0 and np.count_nonzero(D) == 2
    Z = o.sparse_to_mpo(np.array([], int), np.array([], int), np.array([]), rows, cols)
    assert np.all(o.mpo_to_dense(Z) == 0.0)
