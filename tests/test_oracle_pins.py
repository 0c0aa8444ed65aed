"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests touches the GPU library.  Each one is chosen so that a
plausible slip in the oracle (a transposed operand, a wrong index order, a
dropped term, a wrong sign) fails it.
"""

import json
import math
import os

import numpy as np
import pytest

from oracle import tnrsvd_oracle as o
import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- Sec. 2 ----

def test_reshape_examples_multi_index():
    """Examples of Sec. 2: the mode-1 matricisation and vec of the 4x3x2 tensor 1..24."""
    g = _gold("reshape_examples.json")
    dims = g["tensor_dims"]
    # tensor entry (i1,i2,i3) holds 1 + linear index (eq. 1)
    mat = np.zeros((4, 6), dtype=int)
    vec = np.zeros(24, dtype=int)
    for i1 in range(4):
        for i2 in range(3):
            for i3 in range(2):
                val = 1 + o.multi_index([i1, i2, i3], dims)
                mat[i1, o.multi_index([i2, i3], [3, 2])] = val
                vec[o.multi_index([i1, i2, i3], dims)] = val
    assert mat.tolist() == g["mode1_matricization"]
    assert vec.tolist() == g["vec"]


def test_multi_index_rejects_out_of_range():
    with pytest.raises(IndexError):
        o.multi_index([4, 0, 0], [4, 3, 2])


# ---------------------------------------------------------------- Sec. 3 ----

def test_theorem1_rank_one_mpo_is_reversed_kronecker():
    """Theorem 3.1: a unit-rank MPO equals A^(d) kron ... kron A^(1)."""
    rng = np.random.default_rng(0)
    shapes = [(2, 3), (3, 2), (2, 2), (4, 1)]
    mats = [rng.standard_normal(s) for s in shapes]
    cores = [m.reshape(1, *m.shape, 1) for m in mats]
    dense = o.mpo_to_dense(cores)
    ref = mats[0]
    for m in mats[1:]:
        ref = np.kron(m, ref)
    np.testing.assert_allclose(dense, ref, rtol=0, atol=1e-14)
    np.testing.assert_allclose(o.kron_chain(mats), ref, rtol=0, atol=0)


def test_theorem1_entrywise():
    """Entry form of Theorem 3.1: A([i1..id],[j1..jd]) = prod_k A^(k)(i_k, j_k)."""
    rng = np.random.default_rng(1)
    mats = [rng.standard_normal((2, 3)), rng.standard_normal((3, 2)), rng.standard_normal((2, 2))]
    cores = [m.reshape(1, *m.shape, 1) for m in mats]
    dense = o.mpo_to_dense(cores)
    I = [m.shape[0] for m in mats]
    J = [m.shape[1] for m in mats]
    for idx in np.ndindex(*I):
        for jdx in np.ndindex(*J):
            val = np.prod([mats[k][idx[k], jdx[k]] for k in range(3)])
            assert dense[o.multi_index(idx, I), o.multi_index(jdx, J)] == pytest.approx(val, abs=1e-14)


def test_sparse_example_sum_of_rank_one_mpos():
    """Sec. 4.2 2x6 example: two rank-1 MPOs add up to the matrix; the sum has rank 2."""
    g = _gold("sparse_2x6_example.json")
    terms = []
    for t in g["terms"]:
        cores = [np.array(f, dtype=float).reshape(1, len(f), len(f[0]), 1)
                 for f in t["factors_first_core_first"]]
        terms.append(cores)
    summed = o.mpo_add(terms[0], terms[1])
    assert [c.shape for c in summed] == [(1, 1, 1, 2), (2, 1, 3, 2), (2, 2, 2, 1)]
    np.testing.assert_array_equal(o.mpo_to_dense(summed), np.array(g["matrix"], dtype=float))
    assert o.rank_bounds(g["dims_I"], g["dims_J"]) == g["canonical_rank_bounds_R2_R3"]


def test_theorem2_factor_ordering_bounds():
    """Theorem 3.2 bounds for the orderings worked out in Sec. 4.3."""
    for case in _gold("factor_ordering.json")["cases"]:
        assert o.rank_bounds(case["I"], case["J"]) == case["bounds_R2_R3"]


def test_theorem2_bound_holds_for_random_mpo():
    """Numerical ranks of the bond unfoldings of a dense matrix obey Theorem 3.2."""
    rng = np.random.default_rng(2)
    cores = [rng.standard_normal(s) for s in [(1, 2, 2, 6), (6, 2, 3, 6), (6, 2, 1, 1)]]
    bounds = o.rank_bounds([2, 2, 2], [2, 3, 1])
    D = o.mpo_to_dense(cores)
    # unfold at bond 2: rows (i1, j1), cols (i2 j2 i3 j3)
    T = D.reshape(2, 2, 2, 1, 3, 2)  # (i3, i2, i1, j3, j2, j1) in C order
    T = np.transpose(T, (2, 5, 1, 4, 0, 3)).reshape(4, -1)
    assert np.linalg.matrix_rank(T) <= bounds[0]


def test_mpo_addition_densifies_to_sum():
    rng = np.random.default_rng(3)
    a = wl.random_mpo(3, 2, 3, 2, 1.0, 4)
    b = wl.random_mpo(3, 2, 3, 3, 1.0, 5)
    s = o.mpo_add(a, b)
    np.testing.assert_allclose(o.mpo_to_dense(s), o.mpo_to_dense(a) + o.mpo_to_dense(b), atol=1e-12)


def test_merge_preserves_matrix():
    A = wl.random_mpo(6, 2, 3, 3, 1.0, 7)
    for m in (1, 2, 4, 6):
        np.testing.assert_allclose(o.mpo_to_dense(o.merge_tail(A, m)), o.mpo_to_dense(A), atol=1e-12)


def test_merge_plan():
    assert o.merge_plan([2] * 8, [2] * 8, 16) == 4
    assert o.merge_plan([2] * 50, [2] * 50, 20) == 5
    assert o.merge_plan([4] * 30, [4] * 30, 24) == 3
    assert o.merge_plan([2] * 15 + [32], [2] * 15 + [32], 30) == 1
    assert o.merge_plan([4, 2], [2, 8], 8) == 2
    with pytest.raises(ValueError):
        o.merge_plan([2, 2], [2, 2], 5)


# ------------------------------------------------------------- Sec. 5.1 ----

def test_splitmix64_reference_vector():
    g = _gold("splitmix64_vectors.json")
    got = [o.splitmix64(g["seed"], n) for n in range(len(g["outputs"]))]
    assert got == [int(v) for v in g["outputs"]]


def test_box_muller_pair_radius_and_moments():
    """Each Box-Muller pair has squared radius -2 ln u1; the stream is N(0,1)-like."""
    seed = 99
    for k in range(50):
        g0 = o.gaussian_counter(seed, 2 * k)
        g1 = o.gaussian_counter(seed, 2 * k + 1)
        u1 = ((o.splitmix64(seed, 2 * k) >> 11) + 1) * 2.0 ** -53
        assert g0 * g0 + g1 * g1 == pytest.approx(-2.0 * math.log(u1), rel=1e-13)
    x = np.array([o.gaussian_counter(seed, n) for n in range(20000)])
    assert abs(x.mean()) < 0.04 and abs(x.var() - 1.0) < 0.05
    from scipy import stats
    assert stats.kstest(x, "norm").pvalue > 1e-3


@pytest.mark.parametrize("Jlast,K", [(16, 16), (16, 10), (8, 12), (32, 30)])
def test_random_mpo_rank(Jlast, K):
    """Lemma of Sec. 5.1: rank(Omega) = K iff K <= J of the K-core (else J)."""
    cols = [2, 3, Jlast]
    vecs, last = o.omega_from_seed(cols, K, 5)
    D = o.mps_to_dense(o.omega_as_mps(vecs, last))
    assert D.shape == (2 * 3 * Jlast, K)
    assert np.linalg.matrix_rank(D) == min(K, Jlast)
    # Kronecker structure of the lemma: Omega = omega_2 kron omega_1 kron ... (reversed)
    ref = o.kron_chain([vecs[0].reshape(-1, 1), vecs[1].reshape(-1, 1), np.ones((1, 1))])
    np.testing.assert_allclose(D, np.kron(last, ref), atol=1e-14)


# ------------------------------------------------------------- Sec. 5.2 ----

def test_products_match_dense():
    rng = np.random.default_rng(8)
    A = wl.random_mpo(4, 2, 3, 3, 1.0, 9)
    X = [rng.standard_normal(s) for s in [(1, 3, 2), (2, 3, 3), (3, 3, 2), (2, 3, 5)]]
    Xt = [rng.standard_normal(s) for s in [(1, 2, 2), (2, 2, 3), (3, 2, 2), (2, 2, 5)]]
    Ad = o.mpo_to_dense(A)
    np.testing.assert_allclose(o.mps_to_dense(o.mpo_times_mps(A, X)), Ad @ o.mps_to_dense(X), atol=1e-11)
    np.testing.assert_allclose(o.mps_to_dense(o.mpo_t_times_mps(A, Xt)), Ad.T @ o.mps_to_dense(Xt), atol=1e-11)
    Y = o.mpo_times_mps(A, X)
    assert [y.shape[0] for y in Y] == [1, 6, 9, 6]   # ranks multiply


def test_mps_gram_matches_dense():
    rng = np.random.default_rng(10)
    X = [rng.standard_normal(s) for s in [(1, 2, 3), (3, 4, 2), (2, 3, 4)]]
    Y = [rng.standard_normal(s) for s in [(1, 2, 2), (2, 4, 5), (5, 3, 6)]]
    np.testing.assert_allclose(o.mps_gram(X, Y), o.mps_to_dense(X).T @ o.mps_to_dense(Y), atol=1e-12)


# ------------------------------------------------------- rounding (Sec. 3) --

def _mpo_as_mps(cores):
    return [c.reshape(c.shape[0], c.shape[1] * c.shape[2], c.shape[3]) for c in cores]


def test_rounding_example_rank16_to_rank1():
    """Sec. 4.2 example: Kron of three random 2x2 matrices, one rank-1 term per
    2x2 block (16 blocks, uniform rank 16), rounding gives unit ranks."""
    rng = np.random.default_rng(11)
    A1, A2, A3 = (rng.standard_normal((2, 2)) for _ in range(3))
    dense = np.kron(A3, np.kron(A2, A1))
    acc = None
    for i2 in range(2):
        for i3 in range(2):
            for j2 in range(2):
                for j3 in range(2):
                    X = dense[2 * (i2 + 2 * i3):2 * (i2 + 2 * i3) + 2,
                              2 * (j2 + 2 * j3):2 * (j2 + 2 * j3) + 2]
                    E2 = np.zeros((2, 2)); E2[i2, j2] = 1
                    E3 = np.zeros((2, 2)); E3[i3, j3] = 1
                    t = [X.reshape(1, 2, 2, 1), E2.reshape(1, 2, 2, 1), E3.reshape(1, 2, 2, 1)]
                    acc = t if acc is None else o.mpo_add(acc, t)
    assert [c.shape[3] for c in acc[:-1]] == [16, 16]
    np.testing.assert_allclose(o.mpo_to_dense(acc), dense, atol=1e-13)
    r = o.round_sweep(_mpo_as_mps(acc), 1e-12, 0, "qr")
    assert r["ranks"] == [1, 1, 1]
    Yd = (o.mps_to_dense(r["cores"]) @ r["R"])[:, 0]
    # grouped mode of core k is m_k = x_k * J_k + y_k (C order of (I, J))
    for x in np.ndindex(2, 2, 2):
        for y in np.ndindex(2, 2, 2):
            n = o.multi_index([x[k] * 2 + y[k] for k in range(3)], [4, 4, 4])
            row = o.multi_index(x, [2, 2, 2])
            col = o.multi_index(y, [2, 2, 2])
            assert Yd[n] == pytest.approx(dense[row, col], abs=1e-13)


def test_rounding_two_cores_is_eckart_young():
    """One bond: the capped rounding equals the best rank-rho approximation of
    the bond unfolding (Eckart-Young)."""
    rng = np.random.default_rng(12)
    C = [rng.standard_normal((1, 6, 7)), rng.standard_normal((7, 5, 4))]
    D = o.mps_to_dense(C)                     # rows x1 + 6 x2, cols kappa
    M = D.reshape(5, 6, 4).transpose(1, 0, 2).reshape(6, 20)   # [x1] x [x2, kappa]
    U, S, Vt = np.linalg.svd(M)
    for rho in (1, 2, 4):
        r = o.round_sweep(C, 0.0, rho, "qr")
        assert r["ranks"] == [1, rho]
        Dr = o.mps_to_dense(r["cores"]) @ r["R"]
        Mr = Dr.reshape(5, 6, 4).transpose(1, 0, 2).reshape(6, 20)
        best = (U[:, :rho] * S[:rho]) @ Vt[:rho]
        np.testing.assert_allclose(Mr, best, atol=1e-12)


def test_rounding_error_bound_and_tolerance_rule():
    """||Y - round(Y)||_F <= eps ||Y||_F (Oseledets' bound behind the rounding of Sec. 3)."""
    rng = np.random.default_rng(13)
    C = [rng.standard_normal(s) for s in [(1, 2, 4), (4, 2, 6), (6, 2, 6), (6, 2, 5), (5, 4, 3)]]
    D = o.mps_to_dense(C)
    for eps in (0.3, 0.1, 0.03):
        r = o.round_sweep(C, eps, 0, "qr")
        Dr = o.mps_to_dense(r["cores"]) @ r["R"]
        assert np.linalg.norm(D - Dr) <= eps * np.linalg.norm(D) * (1 + 1e-12)
        assert r["norm"] == pytest.approx(np.linalg.norm(D), rel=1e-12)


def test_rounding_without_truncation_is_exact_and_orthonormal():
    rng = np.random.default_rng(14)
    C = [rng.standard_normal(s) for s in [(1, 3, 4), (4, 2, 5), (5, 2, 3), (3, 8, 6)]]
    r = o.round_sweep(C, 0.0, 0, "qr")
    Q, R = r["cores"], r["R"]
    np.testing.assert_allclose(o.mps_to_dense(Q) @ R, o.mps_to_dense(C), atol=1e-12)
    np.testing.assert_allclose(o.mps_gram(Q, Q), np.eye(6), atol=1e-13)
    assert np.all(np.diag(R) >= 0)
    assert np.allclose(R, np.triu(R))
    # each core is left-orthonormal
    for q in Q[:-1]:
        M = q.reshape(-1, q.shape[2])
        np.testing.assert_allclose(M.T @ M, np.eye(M.shape[1]), atol=1e-13)


def test_choose_rank_rule():
    S = np.array([4.0, 2.0, 1.0, 0.5])
    assert o.choose_rank(S, 0.0, 0) == 4
    assert o.choose_rank(S, 0.5, 0) == 3
    assert o.choose_rank(S, math.sqrt(1.25) + 1e-12, 0) == 2
    assert o.choose_rank(S, 100.0, 0) == 1
    assert o.choose_rank(S, 0.0, 2) == 2


# --------------------------------------------------- whole pipeline (Sec. 5) --

@pytest.mark.parametrize("q", [0, 1, 2])
def test_pipeline_equals_dense_rsvd(q):
    """Untruncated TNrSVD equals the dense Algorithm 5.1/5.4 with the same Omega."""
    W = wl.small()
    K = W.K
    rows = [c.shape[1] for c in W.cores]
    cols = [c.shape[2] for c in W.cores]
    m = o.merge_plan(rows, cols, K)
    cols_m = cols[: len(cols) - m] + [int(np.prod(cols[len(cols) - m:]))]
    om = wl.gaussian_omega(cols_m, K, W.omega_seed)
    res = o.tnrsvd(W.cores, W.k, W.p, q, omega=om)
    D = o.mpo_to_dense(W.cores)          # unmerged cores: independent of merge_tail
    Om = o.mps_to_dense(o.omega_as_mps(*om))
    U, S, V = o.dense_rsvd(D, Om, q)
    np.testing.assert_allclose(res.sigma, S[: W.k], rtol=1e-12)
    Ud, Vd = o.mps_to_dense(res.U), o.mps_to_dense(res.V)
    np.testing.assert_allclose(np.abs(np.sum(Ud * U[:, : W.k], 0)), 1.0, atol=1e-10)
    np.testing.assert_allclose(np.abs(np.sum(Vd * V[:, : W.k], 0)), 1.0, atol=1e-10)
    np.testing.assert_allclose(Ud.T @ D @ Vd, np.diag(res.sigma), atol=1e-10 * S[0])
    # interlacing: sigma_j(Q^T A) <= sigma_j(A)
    Sfull = np.linalg.svd(D, compute_uv=False)
    assert np.all(res.sigma_all <= Sfull[: K] * (1 + 1e-12))
    # first product is gauge free: compare densified Y with A Omega
    np.testing.assert_allclose(o.mps_to_dense(res.Y0), D @ Om, atol=1e-11)


def test_pipeline_invariants():
    W = wl.small()
    res = o.tnrsvd(W.cores, W.k, W.p, 1, seed=3)
    np.testing.assert_allclose(o.mps_gram(res.Q, res.Q), np.eye(W.K), atol=1e-13)
    np.testing.assert_allclose(o.mps_gram(res.U, res.U), np.eye(W.k), atol=1e-13)
    np.testing.assert_allclose(o.mps_gram(res.V, res.V), np.eye(W.k), atol=1e-13)
    np.testing.assert_allclose(res.W.T @ res.W, np.eye(W.K), atol=1e-13)
    assert np.all(np.diff(res.sigma_all) <= 0) and np.all(res.sigma_all >= 0)


def test_pipeline_known_spectrum():
    """Prescribed-spectrum family of Sec. 6.3: sigma_j = 10^(-j/4) recovered."""
    W = wl.spectrum(d_inner=9)
    res = o.tnrsvd(W.cores, W.k, W.p, W.q, seed=W.omega_seed, eps=W.eps, rmax=W.rmax)
    np.testing.assert_allclose(res.sigma, W.sigma_exact[: W.k], rtol=1e-12, atol=1e-14)
    assert all(max(r) <= 5 for r in res.ranks)


def test_known_spectrum_generator():
    W = wl.spectrum(d_inner=5, last=16, r=4, n_sig=12, k=6, p=4)
    S = np.linalg.svd(o.mpo_to_dense(W.cores), compute_uv=False)
    np.testing.assert_allclose(S[:12], W.sigma_exact, rtol=1e-12)
    assert S[12] < 1e-13


def test_orientation_mirror_matches_paper_orientation():
    """Reading of the K-leg placement: the mirrored pipeline on A equals the
    paper's orientation (K leg on core 1, right-to-left sweeps) on the
    core-reversed A with the same Omega."""
    W = wl.small()
    K = W.K
    A = o.merge_tail(W.cores, 4)
    om = wl.gaussian_omega([c.shape[2] for c in A], K, 21)
    for q in (0, 1):
        s1 = o.tnrsvd(A, W.k, W.p, q, omega=om, merge=False).sigma
        s2 = o.tnrsvd_paper_orientation(o.reverse_mpo(A), W.k, W.p, q, om[1], om[0][::-1])
        np.testing.assert_allclose(s1, s2, rtol=1e-11)


def test_zero_matrix_is_not_an_error():
    W = wl.small()
    Z = [np.zeros_like(c) for c in W.cores]
    res = o.tnrsvd(Z, W.k, W.p, 1, seed=1)
    assert np.all(res.sigma == 0)
    np.testing.assert_allclose(o.mps_gram(res.Q, res.Q), np.eye(W.K), atol=1e-13)


def test_shape_errors():
    W = wl.small()
    with pytest.raises(ValueError):
        o.tnrsvd(W.cores, 200, 100, 0, seed=1)
    bad = [c.copy() for c in W.cores]
    bad[3] = bad[3][:2]
    with pytest.raises(ValueError):
        o.mpo_to_dense(bad)
