"""Pins of the oracle's derivative of the whole pipeline (``pipeline_grad``):
L = sum_j dsigma_j sigma_j of ``tnrsvd`` with Omega fixed and every
rounding's bond ranks frozen at their forward values.

* The Gram (environment) form of the rounding computes the map of the
  QR/SVD form (``round_sweep``): equal cores, sigma and ranks.
* The QR adjoint and the rounding adjoint against central finite differences
  of ``qr_nonneg`` and ``round_sweep`` themselves (the QR/SVD form, so the
  finite differences do not go through the code under test).
* The whole gradient against central finite differences of ``tnrsvd``
  (h = 1e-6, seeded unit directions, d <= 8; q = 0, 1, 2; truncating ranks;
  a merged tail), each perturbed run checked to keep the forward's ranks.
* Where the computed subspace is exact (rank(A) = K), the gradient against
  the closed form sum_j dsigma_j u_j v_j^T from LAPACK's SVD of the dense A,
  carried to the cores by the exact chain rule through the dense contraction.
A dropped term, a wrong sign or a transposed operand anywhere in the reverse
pass moves these directional derivatives far beyond the tolerances.
"""

import numpy as np
import pytest

from oracle import tnrsvd_oracle as o
import workloads as wl


def omega_for(cores, K, seed):
    rows = [c.shape[1] for c in cores]
    cols = [c.shape[2] for c in cores]
    m = o.merge_plan(rows, cols, K)
    cm = cols[: len(cols) - m] + [int(np.prod(cols[len(cols) - m:]))]
    return wl.gaussian_omega(cm, K, seed)


def random_chain(shapes, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(s) for s in shapes]


CHAIN = [(1, 2, 4), (4, 2, 6), (6, 3, 5), (5, 2, 4), (4, 4, 6)]


@pytest.mark.parametrize("eps,rmax", [(0.0, 0), (0.0, 3), (0.1, 0)])
@pytest.mark.parametrize("last", ["qr", "svd"])
def test_gram_form_is_the_rounding_map(eps, rmax, last):
    Y = random_chain(CHAIN, 1)
    a = o.round_sweep(Y, eps, rmax, last)
    b = o.round_sweep_gram(Y, eps, rmax, last)
    assert b["ranks"] == a["ranks"]
    for x, y in zip(a["cores"], b["cores"]):
        assert x.shape == y.shape
        np.testing.assert_allclose(y, x, atol=1e-12)
    if last == "svd":
        np.testing.assert_allclose(b["sigma"], a["sigma"], rtol=1e-12)
    else:
        np.testing.assert_allclose(b["R"], a["R"], atol=1e-11 * np.abs(a["R"]).max())


def test_qr_adjoint_finite_differences():
    rng = np.random.default_rng(2)
    M = rng.standard_normal((9, 4))
    dQ = rng.standard_normal((9, 4))
    dR = np.triu(rng.standard_normal((4, 4)))
    Q, R = o.qr_nonneg(M)
    dM = o.qr_adjoint(Q, R, dQ, dR)

    def loss(X):
        q, r = o.qr_nonneg(X)
        return float(np.sum(dQ * q) + np.sum(dR * r))

    h = 1e-6
    for _ in range(5):
        D = rng.standard_normal(M.shape)
        fd = (loss(M + h * D) - loss(M - h * D)) / (2 * h)
        assert abs(np.sum(dM * D) - fd) <= 1e-7 * (1 + abs(fd))


@pytest.mark.parametrize("eps,rmax,last", [(0.0, 3, "qr"), (0.0, 0, "qr"), (0.0, 3, "svd"),
                                           (0.0, 2, "svd"), (0.05, 0, "qr")])
def test_rounding_adjoint_finite_differences(eps, rmax, last):
    rng = np.random.default_rng(7)
    Y = random_chain(CHAIN, 3)
    fwd = o.round_sweep(Y, eps, rmax, last)
    ranks = fwd["ranks"]
    W = [rng.standard_normal(c.shape) for c in fwd["cores"]]
    ws = rng.standard_normal(len(fwd["sigma"])) if last == "svd" else None

    def loss(Yp):
        r = o.round_sweep(Yp, eps, rmax, last)
        assert r["ranks"] == ranks
        if last == "qr":
            return sum(float(np.sum(w * c)) for w, c in zip(W, r["cores"]))
        return float(np.sum(ws * r["sigma"]))

    rec = o.round_sweep_gram(Y, eps, rmax, last, ranks=ranks)["rec"]
    if last == "qr":
        dY = o.round_sweep_gram_adjoint(rec, dcores=W[:-1], dlast=W[-1])
    else:
        dY = o.round_sweep_gram_adjoint(rec, dsigma=ws)
    h = 1e-6
    for _ in range(5):
        i = int(rng.integers(0, len(Y)))
        D = rng.standard_normal(Y[i].shape)
        Yp = [y.copy() for y in Y]
        Yp[i] += h * D
        Ym = [y.copy() for y in Y]
        Ym[i] -= h * D
        fd = (loss(Yp) - loss(Ym)) / (2 * h)
        assert abs(np.sum(dY[i] * D) - fd) <= 1e-6 * (1 + abs(fd)), (i, np.sum(dY[i] * D), fd)


def _fd_check(A, k, p, q, eps, rmax, seed, ndir=4, h=1e-6, tol=1e-6):
    rng = np.random.default_rng(seed)
    om = omega_for(A, k + p, seed + 100)
    res = o.tnrsvd(A, k, p, q, omega=om, eps=eps, rmax=rmax)
    w = rng.standard_normal(k)
    G = o.pipeline_grad(A, k, p, q, om, eps, rmax, dsigma=w, ranks=res.ranks)
    assert [g.shape for g in G] == [a.shape for a in A]
    for _ in range(ndir):
        i = int(rng.integers(0, len(A)))
        D = rng.standard_normal(A[i].shape)
        D /= np.linalg.norm(D)
        Ap = [a.copy() for a in A]
        Ap[i] += h * D
        Am = [a.copy() for a in A]
        Am[i] -= h * D
        rp = o.tnrsvd(Ap, k, p, q, omega=om, eps=eps, rmax=rmax)
        rm = o.tnrsvd(Am, k, p, q, omega=om, eps=eps, rmax=rmax)
        assert rp.ranks == res.ranks and rm.ranks == res.ranks
        fd = (np.sum(w * rp.sigma) - np.sum(w * rm.sigma)) / (2 * h)
        got = float(np.sum(G[i] * D))
        assert abs(got - fd) <= tol * (abs(fd) + 1e-3 * np.linalg.norm(G[i])), (i, got, fd)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_pipeline_gradient_finite_differences(q):
    A = random_chain([(1, 2, 2, 3), (3, 2, 2, 3), (3, 2, 2, 2), (2, 2, 2, 2), (2, 2, 2, 1)], 3)
    A = [a for a in A]
    _fd_check(A, 3, 3, q, 0.0, 0, 5 + q)


def test_pipeline_gradient_finite_differences_truncating_and_merged():
    A = random_chain([(1, 2, 2, 3), (3, 2, 2, 3), (3, 2, 2, 2), (2, 2, 2, 2), (2, 2, 2, 1)], 3)
    _fd_check(A, 3, 3, 1, 0.0, 2, 9)                      # rank cap 2 truncates every product
    W = wl.small()                                        # d = 8, last 4 cores merged (K = 16)
    _fd_check(W.cores, W.k, W.p, 1, 0.0, 3, 12)
    _fd_check(W.cores, W.k, W.p, 1, 0.0, 0, 11)


def rank_r_mpo(d, n, r, seed):
    rng = np.random.default_rng(seed)
    A = None
    for _ in range(r):
        term = [np.outer(rng.standard_normal(n), rng.standard_normal(n)).reshape(1, n, n, 1)
                for _ in range(d)]
        A = term if A is None else o.mpo_add(A, term)
    return A


def core_grad_from_dense(A, Gd):
    """dL/dA_i for L = <Gd, dense(A)>: the dense matrix is linear in core i,
    entry ([r, x, r'], [c, y, c']) = Left[r, c, a] A_i[a, x, y, b] Right[b, r', c']
    with little-endian row and column indices (eq. (1))."""
    out = []
    for i in range(len(A)):
        L = np.ones((1, 1, 1))
        for c in A[:i]:
            _, I, J, r2 = c.shape
            L = np.einsum("pqa,axyb->xpyqb", L, c).reshape(L.shape[0] * I, L.shape[1] * J, r2)
        R = np.ones((1, 1, 1))
        for c in A[i + 1:][::-1]:
            r1, I, J, _ = c.shape
            R = np.einsum("axyb,bpq->apxqy", c, R).reshape(r1, R.shape[1] * I, R.shape[2] * J)
        _, I, J, _ = A[i].shape
        G6 = Gd.reshape(R.shape[1], I, L.shape[0], R.shape[2], J, L.shape[1])
        out.append(np.einsum("sxrtyc,rca,bst->axyb", G6, L, R))
    return out


@pytest.mark.parametrize("q", [0, 1])
def test_exact_case_equals_lapack_closed_form(q):
    A = rank_r_mpo(6, 2, 8, 5)            # rank 8 = K: the computed subspace is range(A)
    k, p = 3, 5
    om = omega_for(A, k + p, 21)
    w = np.array([1.0, 0.5, -2.0])
    G = o.pipeline_grad(A, k, p, q, om, 0.0, 0, dsigma=w)
    U, S, Vt = np.linalg.svd(o.mpo_to_dense(A))
    assert np.sum(S > 1e-10 * S[0]) == k + p
    Gd = (U[:, :k] * w[None, :]) @ Vt[:k]
    ref = core_grad_from_dense(A, Gd)
    num = np.sqrt(sum(np.sum((a - b) ** 2) for a, b in zip(G, ref)))
    den = np.sqrt(sum(np.sum(b ** 2) for b in ref))
    assert num / den <= 1e-10


def test_product_adjoints_are_the_transposes():
    rng = np.random.default_rng(4)
    A = [rng.standard_normal(s) for s in [(1, 2, 3, 2), (2, 3, 2, 1)]]
    for op, fwd, adj, nmode in [(0, o.mpo_times_mps, o.mpo_times_mps_adjoint, 2),
                                (1, o.mpo_t_times_mps, o.mpo_t_times_mps_adjoint, 1)]:
        X = [rng.standard_normal((1, A[0].shape[nmode], 2)),
             rng.standard_normal((2, A[1].shape[nmode], 3))]
        Y = fwd(A, X)
        dY = [rng.standard_normal(y.shape) for y in Y]
        dA, dX = adj(A, X, dY)
        DA = [rng.standard_normal(a.shape) for a in A]
        DX = [rng.standard_normal(x.shape) for x in X]
        # bilinear: <dY, Y(DA, X)> = <dA, DA>, <dY, Y(A, DX)> = <dX, DX>
        lhs = sum(np.sum(g * y) for g, y in zip(dY, fwd(DA, X)))
        assert abs(lhs - sum(np.sum(g * d) for g, d in zip(dA, DA))) <= 1e-12 * (1 + abs(lhs))
        lhs = sum(np.sum(g * y) for g, y in zip(dY, fwd(A, DX)))
        assert abs(lhs - sum(np.sum(g * d) for g, d in zip(dX, DX))) <= 1e-12 * (1 + abs(lhs))
