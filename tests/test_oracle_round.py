"""Pins of the oracle's MPO rounding (Sec. 3), used on the output of Algorithm 4.1.

Each pin checks the oracle against something it does not compute itself: the
ranks of the dense unfoldings (numpy's matrix_rank), the dense matrix, the
rounding error bound, orthonormality, and a Kronecker product whose MPO has
rank 1.
"""

import numpy as np

from oracle import tnrsvd_oracle as o


def dense(cores):
    return o.mpo_to_dense(cores)


def unfolding_ranks(A, rows, cols):
    """Ranks of the unfoldings (i_1 j_1 ... i_k j_k) x (rest) of the dense
    matrix, with the eq. (1) index order (i_1 fastest)."""
    d = len(rows)
    T = A.reshape(list(reversed(rows)) + list(reversed(cols)))
    # axes: i_d .. i_1, j_d .. j_1 -> i_1 j_1 i_2 j_2 ...
    perm = []
    for k in range(d):
        perm += [d - 1 - k, 2 * d - 1 - k]
    T = T.transpose(perm)
    out = []
    for k in range(1, d):
        m = int(np.prod([rows[l] * cols[l] for l in range(k)]))
        out.append(int(np.linalg.matrix_rank(T.reshape(m, -1), tol=1e-10 * np.linalg.norm(A))))
    return out


def random_mpo(rng, rows, cols, ranks):
    return [rng.standard_normal((ranks[k], rows[k], cols[k], ranks[k + 1]))
            for k in range(len(rows))]


def test_exact_rounding_reaches_the_unfolding_ranks():
    rng = np.random.default_rng(1)
    rows, cols = [3, 2, 2, 3], [2, 3, 2, 2]
    A = random_mpo(rng, rows, cols, [1, 2, 3, 2, 1])
    A2 = o.mpo_add(A, A)                                   # ranks doubled, same matrix x 2
    # eps = 0 would keep the rounding-noise directions of the doubled ranks
    R = o.round_mpo(A2, 1e-12)
    D = dense(A)
    np.testing.assert_allclose(dense(R), 2 * D, atol=1e-12 * np.abs(D).max())
    got = [c.shape[3] for c in R[:-1]]
    assert got == unfolding_ranks(2 * D, rows, cols)
    assert got != [c.shape[3] for c in A2[:-1]]


def test_left_orthonormal_and_error_bound():
    rng = np.random.default_rng(2)
    rows, cols = [2, 2, 2, 2, 2], [2, 2, 2, 2, 2]
    # a sum of terms with decaying weights: truncation has something to drop
    A = random_mpo(rng, rows, cols, [1, 1, 1, 1, 1, 1])
    for w in [1e-1, 1e-2, 1e-3, 1e-4]:
        B = random_mpo(rng, rows, cols, [1, 2, 2, 2, 2, 1])
        B[0] = B[0] * w
        A = o.mpo_add(A, B)
    D = dense(A)
    for eps in [1e-1, 1e-2, 1e-3]:
        R = o.round_mpo(A, eps)
        err = np.linalg.norm(dense(R) - D)
        assert err <= eps * np.linalg.norm(D) * (1 + 1e-10)
        for c in R[:-1]:
            Q = c.reshape(-1, c.shape[3])
            np.testing.assert_allclose(Q.T @ Q, np.eye(Q.shape[1]), atol=1e-12)
    # tighter tolerance keeps more
    assert sum(c.size for c in o.round_mpo(A, 1e-3)) > sum(c.size for c in o.round_mpo(A, 1e-1))


def test_rank_cap():
    rng = np.random.default_rng(3)
    rows, cols = [2, 2, 2, 2], [2, 2, 2, 2]
    A = random_mpo(rng, rows, cols, [1, 4, 6, 4, 1])
    R = o.round_mpo(A, 0.0, rmax=3)
    assert max(c.shape[3] for c in R[:-1]) <= 3


def test_kronecker_matrix_rounds_to_rank_one():
    """A = A_3 (x) A_2 (x) A_1 is a rank-1 MPO (Theorem 1); its Algorithm 4.1 MPO
    has one term per nonzero block, and rounding must find rank 1 again."""
    rng = np.random.default_rng(4)
    rows, cols = [3, 2, 2], [2, 3, 2]
    F = [rng.standard_normal((rows[k], cols[k])) for k in range(3)]
    F[1][0, 1] = 0.0
    K = np.kron(F[2], np.kron(F[1], F[0]))
    r, c = np.nonzero(K)
    S = o.sparse_to_mpo(r, c, K[r, c], rows, cols)
    assert S[0].shape[3] > 1
    R = o.round_mpo(S, 1e-14)
    assert [x.shape[3] for x in R] == [1, 1, 1]
    np.testing.assert_allclose(dense(R), K, atol=1e-13 * np.abs(K).max())


def test_single_core_and_zero_matrix():
    rng = np.random.default_rng(5)
    A = [rng.standard_normal((1, 4, 3, 1))]
    np.testing.assert_allclose(o.round_mpo(A, 0.5)[0], A[0], atol=1e-14)
    Z = [np.zeros((1, 2, 2, 3)), np.zeros((3, 2, 2, 1))]
    R = o.round_mpo(Z, 1e-3)
    assert [c.shape for c in R] == [(1, 2, 2, 1), (1, 2, 2, 1)] and not any(np.any(c) for c in R)


def test_zero_product_of_nonzero_cores_rounds_to_zero_cores():
    """The zero-matrix reading also covers a product that vanishes because
    one core is zero while the others are not."""
    rng = np.random.default_rng(12)
    C = [rng.standard_normal(s) for s in [(1, 2, 3, 3), (3, 2, 3, 3), (3, 2, 3, 3), (3, 2, 3, 1)]]
    C[2] = np.zeros_like(C[2])
    R = o.round_mpo(C, 1e-8)
    assert [x.shape for x in R] == [(1, 2, 3, 1)] * 4 and not any(np.any(x) for x in R)
