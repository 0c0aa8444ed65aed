"""Pins of the oracle's sketched product truncation (sketch_compress), an
opt-in step that is not in the paper.

What the mathematics fixes, whatever Gaussian sketch is drawn:
* the result is the orthogonal projection (U U^T (x) I) Y of the chain onto the
  span of its left-orthonormal cores, so the residual is orthogonal to it
  (Yhat^T (Y - Yhat) = 0) and |Yhat| <= |Y|;
* when ell reaches the chain's true bond ranks (below its formal ranks), the
  projection is exact;
* cores 0 .. d-2 are left-orthonormal with bond ranks <= ell;
* a chain whose bond ranks all fit in ell is returned unchanged.
"""

import numpy as np

from oracle import tnrsvd_oracle as o
import workloads as wl


def chain(shapes, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(s) for s in shapes]


def inflated(true_ranks, n, K, formal, seed):
    """A chain of true bond ranks `true_ranks` written with formal ranks
    `formal`: core k becomes G_k Y_k H_{k+1} with H_k G_k = I."""
    rng = np.random.default_rng(seed)
    r = [1] + list(true_ranks) + [K]
    Y = [rng.standard_normal((r[k], n[k], r[k + 1])) for k in range(len(n))]
    G, H = [np.eye(1)], [np.eye(1)]
    for k in range(1, len(n)):
        g = rng.standard_normal((formal, r[k]))
        G.append(g)
        H.append(np.linalg.pinv(g))              # r_k x formal, H G = I
    G.append(np.eye(K))
    H.append(np.eye(K))
    out = [np.einsum("ab,bic,cd->aid", G[k], Y[k], H[k + 1]) for k in range(len(n))]
    return Y, out


def test_chain_with_ranks_within_ell_is_unchanged():
    Y = chain([(1, 2, 3), (3, 2, 4), (4, 3, 5)], 1)
    out = o.sketch_compress(Y, 4, 7, 0)
    for a, b in zip(out, Y):
        np.testing.assert_array_equal(a, b)


def test_exact_when_ell_reaches_the_true_ranks():
    n = [2, 3, 2, 2, 3]
    Ytrue, Y = inflated([2, 3, 3, 2], n, 4, 9, 2)
    assert max(y.shape[2] for y in Y[:-1]) == 9
    out = o.sketch_compress(Y, 5, 11, 3)
    assert max(c.shape[2] for c in out[:-1]) <= 5
    D, Dh = o.mps_to_dense(Y), o.mps_to_dense(out)
    np.testing.assert_allclose(Dh, D, atol=1e-12 * np.abs(D).max())
    np.testing.assert_allclose(D, o.mps_to_dense(Ytrue), atol=1e-12 * np.abs(D).max())


def test_projection_properties_when_truncating():
    Y = chain([(1, 4, 8), (8, 4, 8), (8, 4, 8), (8, 4, 5)], 3)
    out = o.sketch_compress(Y, 3, 5, 1)
    for c in out[:-1]:
        Q = c.reshape(-1, c.shape[2])
        assert Q.shape[1] <= 3
        np.testing.assert_allclose(Q.T @ Q, np.eye(Q.shape[1]), atol=1e-13)
    D, Dh = o.mps_to_dense(Y), o.mps_to_dense(out)
    scale = np.linalg.norm(D) ** 2
    np.testing.assert_allclose(Dh.T @ (D - Dh), 0.0, atol=1e-13 * scale)
    assert np.linalg.norm(Dh) <= np.linalg.norm(D) * (1 + 1e-14)
    assert np.linalg.norm(D - Dh) > 1e-3 * np.linalg.norm(D)   # it does truncate


def test_sketch_depends_on_seed_and_product_index():
    Y = chain([(1, 4, 8), (8, 4, 8), (8, 4, 5)], 4)
    a = o.mps_to_dense(o.sketch_compress(Y, 2, 5, 0))
    b = o.mps_to_dense(o.sketch_compress(Y, 2, 5, 1))
    c = o.mps_to_dense(o.sketch_compress(Y, 2, 6, 0))
    assert np.abs(a - b).max() > 1e-6 and np.abs(a - c).max() > 1e-6


def test_counter_stream_matches_the_scalar_generator():
    idx = np.array([0, 1, 2, 3, (1 << 40) + 5, (3 << 40) + 12345], dtype=np.uint64)
    ref = [o.gaussian_counter(9, int(i)) for i in idx]
    np.testing.assert_allclose(o.gaussian_counter_array(9, idx), ref, rtol=1e-15, atol=1e-15)


def test_sketched_solve_matches_the_plain_solve_when_ell_covers_the_ranks():
    W = wl.small()
    om = wl.gaussian_omega([c.shape[2] for c in o.merge_tail(W.cores, o.merge_plan(
        [c.shape[1] for c in W.cores], [c.shape[2] for c in W.cores], W.K))], W.K, 3)
    r0 = o.tnrsvd(W.cores, W.k, W.p, 1, omega=om)
    # the products reach formal rank 48 (A's 3 times the basis' 16), true rank <= 16
    r1 = o.tnrsvd(W.cores, W.k, W.p, 1, omega=om, sketch_rank=16, sketch_seed=2)
    np.testing.assert_allclose(r1.sigma, r0.sigma, rtol=1e-12)
    r2 = o.tnrsvd(W.cores, W.k, W.p, 1, omega=om, sketch_rank=8, sketch_seed=2)
    assert np.max(np.abs(r2.sigma - r0.sigma)) > 1e-4 * r0.sigma[0]   # below the true ranks
