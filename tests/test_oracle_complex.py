"""Pins of the oracle's complex-MPO support: the real embedding is, entry by
entry, the block matrix [[Re A, -Im A], [Im A, Re A]] with the component digits
placed as documented, and TNrSVD of it gives the complex matrix's singular
values (LAPACK's complex SVD on the dense matrix)."""

import numpy as np

from oracle import tnrsvd_oracle as o


def complex_mpo(shapes, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(s) + 1j * rng.standard_normal(s) for s in shapes]


def dense_complex(cores):
    """Dense complex matrix of an MPO, little-endian indices as in eq. (1)."""
    T = cores[0][0]
    rows, cols = T.shape[0], T.shape[1]
    for c in cores[1:]:
        _, I, J, r2 = c.shape
        T = np.einsum("ijr,rxyb->xiyjb", T, c).reshape(I * rows, J * cols, r2)
        rows, cols = rows * I, cols * J
    return T[:, :, 0]


def test_embedding_is_the_real_block_form_entry_by_entry():
    C = complex_mpo([(1, 2, 3, 3), (3, 3, 2, 4), (4, 2, 2, 1)], 1)
    A = dense_complex(C)
    B = o.mpo_to_dense(o.complex_to_real_mpo(C))
    M, N = A.shape
    I0 = C[0].shape[1]
    i = np.arange(M)
    j = np.arange(N)
    for s_ in (0, 1):
        for t_ in (0, 1):
            rows = s_ * I0 + (i % I0) + 2 * I0 * (i // I0)
            cols = j + t_ * N
            blk = B[np.ix_(rows, cols)]
            want = {(0, 0): A.real, (0, 1): -A.imag, (1, 0): A.imag, (1, 1): A.real}[(s_, t_)]
            np.testing.assert_allclose(blk, want, rtol=1e-14, atol=1e-14)


def test_single_core_embedding():
    C = complex_mpo([(1, 3, 4, 1)], 2)
    B = o.mpo_to_dense(o.complex_to_real_mpo(C))
    A = C[0][0, :, :, 0]
    np.testing.assert_allclose(np.linalg.svd(B, compute_uv=False)[0::2],
                               np.linalg.svd(A, compute_uv=False), rtol=1e-13)


def test_tnrsvd_complex_matches_lapack_when_K_spans_the_space():
    """16 x 16 complex matrix: its real form is 32 x 32, and K' = 2 (k + p) = 32
    columns span it, so the randomized SVD is exact."""
    C = complex_mpo([(1, 4, 4, 3), (3, 4, 4, 1)], 3)
    A = dense_complex(C)
    ref = np.linalg.svd(A, compute_uv=False)
    s = o.tnrsvd_complex(C, 4, 12, 0, seed=4)
    np.testing.assert_allclose(s, ref[:4], rtol=1e-11)


def test_tnrsvd_complex_power_iterations_on_a_decaying_spectrum():
    """A random complex MPO (2^6 x 2^6, slowly decaying spectrum): q = 4 power
    iterations bring the top three singular values to LAPACK's within 1e-6
    (the error falls by about 50x per iteration here)."""
    rng = np.random.default_rng(5)
    d = 6
    C = []
    r = [1, 3, 3, 3, 3, 3, 1]
    for k in range(d):
        G = rng.standard_normal((r[k], 2, 2, r[k + 1])) + 1j * rng.standard_normal((r[k], 2, 2, r[k + 1]))
        C.append(G)
    A = dense_complex(C)
    ref = np.linalg.svd(A, compute_uv=False)
    s = o.tnrsvd_complex(C, 3, 7, 4, seed=6)
    np.testing.assert_allclose(s, ref[:3], rtol=1e-6)
