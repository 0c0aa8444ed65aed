"""Pins of the oracle's gradient of sum_j sigma_j (frozen computed subspace).

* The environments and the merge adjoint against the dense bilinear form
  sum_j w_j u_j^T A v_j (u_j, v_j densified from the oracle's U, V cores),
  whose derivative with respect to one core entry is a plain finite
  difference of a function that is linear in that core (exact up to
  rounding).
* In the exact case (rank(A) <= K, no truncation) the frozen-subspace
  gradient is the gradient of the pipeline's output: central finite
  differences of the whole FP64 pipeline with the same Omega, and the
  closed form sum_j u_j v_j^T from LAPACK's SVD of the densified A.
"""

import numpy as np

from oracle import tnrsvd_oracle as o


def rank_r_mpo(d, n, r, seed):
    """MPO of a rank-r matrix: the sum (MPO addition) of r Kronecker products of
    rank-1 factors u v^T, each of which is a rank-1 matrix (Theorem 1)."""
    rng = np.random.default_rng(seed)
    A = None
    for t in range(r):
        term = [np.outer(rng.standard_normal(n), rng.standard_normal(n)).reshape(1, n, n, 1)
                for _ in range(d)]
        A = term if A is None else o.mpo_add(A, term)
    return A


def dense_form(A_cores, res, w):
    Ud = o.mps_to_dense(res.U)
    Vd = o.mps_to_dense(res.V)
    Ad = o.mpo_to_dense(A_cores)
    return float(np.sum(w * np.einsum("ij,ik,kj->j", Ud, Ad, Vd)))


def test_environments_match_dense_bilinear_form():
    rng = np.random.default_rng(3)
    A = [rng.standard_normal(s) for s in [(1, 2, 2, 3), (3, 2, 2, 3), (3, 2, 2, 2), (2, 2, 2, 2),
                                          (2, 2, 2, 1)]]
    res = o.tnrsvd(A, 4, 2, 1, seed=11)          # K = 6: the last 3 cores are merged
    w = rng.standard_normal(4)
    G = o.sigma_sum_grad(A, res, w)
    assert [g.shape for g in G] == [a.shape for a in A]
    base = dense_form(A, res, w)
    h = 1e-3
    for i in range(len(A)):
        for idx in [tuple(rng.integers(0, n) for n in A[i].shape) for _ in range(3)]:
            Ap = [a.copy() for a in A]
            Ap[i][idx] += h
            fd = (dense_form(Ap, res, w) - base) / h     # linear in A_i up to the merge
            assert abs(fd - G[i][idx]) <= 1e-7 * (1 + abs(G[i][idx])), (i, idx)


def test_merge_adjoint_is_the_transpose_of_the_merge():
    rng = np.random.default_rng(4)
    tail = [rng.standard_normal(s) for s in [(2, 2, 3, 3), (3, 3, 2, 2), (2, 2, 2, 1)]]
    M = o.merge_tail(tail, 3)[0]
    dM = rng.standard_normal(M.shape)
    g = o.merge_tail_adjoint(tail, dM)
    for j in range(3):
        D = rng.standard_normal(tail[j].shape)
        h = 1e-6
        tp = [t.copy() for t in tail]
        tp[j] = tp[j] + h * D
        tm = [t.copy() for t in tail]
        tm[j] = tm[j] - h * D
        fd = np.sum(dM * (o.merge_tail(tp, 3)[0] - o.merge_tail(tm, 3)[0])) / (2 * h)
        assert abs(fd - np.sum(g[j] * D)) <= 1e-8 * (1 + abs(fd))


def test_exact_case_equals_pipeline_derivative_and_lapack():
    """rank(A) = 3 <= K = 8, no truncation: the computed subspace is exact."""
    A = rank_r_mpo(6, 2, 3, 5)
    k, p = 3, 5
    om = o.omega_from_seed([c.shape[2] for c in o.merge_tail(A, o.merge_plan(
        [c.shape[1] for c in A], [c.shape[2] for c in A], k + p))], k + p, 21)
    res = o.tnrsvd(A, k, p, 1, omega=om)
    G = o.sigma_sum_grad(A, res)
    # LAPACK closed form: sum_j u_j v_j^T of the dense matrix
    Ad = o.mpo_to_dense(A)
    Ul, S, Vt = np.linalg.svd(Ad)
    np.testing.assert_allclose(S[:k], res.sigma, rtol=1e-12)
    Gd = Ul[:, :k] @ Vt[:k, :]
    rng = np.random.default_rng(8)
    h = 1e-6
    for i in (0, 3, 5):
        D = rng.standard_normal(A[i].shape)
        Ap = [a.copy() for a in A]
        Ap[i] = Ap[i] + h * D
        Am = [a.copy() for a in A]
        Am[i] = Am[i] - h * D
        # pipeline finite difference (same Omega, no truncation)
        fd = (o.tnrsvd(Ap, k, p, 1, omega=om).sigma.sum()
              - o.tnrsvd(Am, k, p, 1, omega=om).sigma.sum()) / (2 * h)
        # closed form: <Gd, dA/dt>
        dA = (o.mpo_to_dense(Ap) - o.mpo_to_dense(Am)) / (2 * h)
        closed = float(np.sum(Gd * dA))
        got = float(np.sum(G[i] * D))
        assert abs(got - closed) <= 1e-7 * (1 + abs(closed)), (i, got, closed)
        assert abs(got - fd) <= 1e-5 * (1 + abs(fd)), (i, got, fd)
