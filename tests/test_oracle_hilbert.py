"""Pins of the Hilbert experiment (Sec. 6.3) on the CPU.

The input MPO (workloads.hilbert_mpo, an exponential sum) is pinned against
the closed form A(i, j) = 1 / (i + j + 1); its rounding by the oracle against
the same closed form within the rounding bound; and the oracle's TNrSVD in the
paper's orientation (first 5 cores merged, K = 32 on the first core) against
LAPACK's singular values of the dense matrix where that fits in memory.
"""

import numpy as np
import pytest

from oracle import tnrsvd_oracle as o
import workloads as wl


def closed_form(i, j):
    return 1.0 / (np.asarray(i, dtype=np.float64) + np.asarray(j, dtype=np.float64) + 1.0)


def entries(cores, i, j):
    """MPO entries at positions (i, j), little-endian digits as in eq. (1)."""
    v = np.ones((len(i), 1))
    ii, jj = np.array(i, dtype=np.int64), np.array(j, dtype=np.int64)
    for G in cores:
        I, J = G.shape[1], G.shape[2]
        v = np.einsum("ea,eab->eb", v, G[:, ii % I, jj % J, :].transpose(1, 0, 2))
        ii //= I
        jj //= J
    return v[:, 0]


def sample(N, n, seed):
    rng = np.random.default_rng(seed)
    i = rng.integers(0, 2 ** N, n, dtype=np.int64)
    j = rng.integers(0, 2 ** (N - 1), n, dtype=np.int64)
    i[:4] = [0, 2 ** N - 1, 0, 2 ** N - 1]          # the corners of the matrix
    j[:4] = [0, 2 ** (N - 1) - 1, 2 ** (N - 1) - 1, 0]
    return i, j


def paper_sigma(P, W):
    """The oracle's TNrSVD in the paper's orientation on the MPO P, with the
    first 5 cores merged (the digits ordered as the library merges them) and
    Omega drawn for the mirrored layout."""
    L = o.reverse_mpo(P)
    m = o.merge_plan([c.shape[1] for c in L], [c.shape[2] for c in L], W.K)
    cols = [c.shape[2] for c in L]
    om = wl.gaussian_omega(cols[: len(L) - m] + [int(np.prod(cols[len(L) - m:]))], W.K,
                           W.omega_seed)
    A1 = o.reverse_mpo(o.merge_tail(L, m))
    return m, o.tnrsvd_paper_orientation(A1, W.k, W.p, W.q, om[1], om[0][::-1], eps=W.eps,
                                            rmax=W.rmax)


def test_exponential_sum_matches_the_closed_form_densely():
    N = 10
    D = o.mpo_to_dense(wl.hilbert_mpo(N))
    H = closed_form(np.arange(2 ** N)[:, None], np.arange(2 ** (N - 1))[None, :])
    assert D.shape == (1024, 512)
    assert np.max(np.abs(D - H) / H) < 5e-13


@pytest.mark.parametrize("N", [20, 50])
def test_exponential_sum_matches_the_closed_form_sampled(N):
    C = wl.hilbert_mpo(N)
    assert len(C) == N and C[-1].shape[2] == 1 and all(c.shape[1] == 2 for c in C)
    i, j = sample(N, 600, N)
    assert np.max(np.abs(entries(C, i, j) - closed_form(i, j)) / closed_form(i, j)) < 5e-13


def test_rounded_mpo_within_the_bound_and_small_ranks():
    N = 10
    R = o.round_mpo(wl.hilbert_mpo(N), wl.HILBERT_MPO_TOL)
    H = closed_form(np.arange(2 ** N)[:, None], np.arange(2 ** (N - 1))[None, :])
    nH = np.linalg.norm(H)
    # rounding bound plus the exponential sum's own error (< 5e-13 relative per entry)
    assert np.linalg.norm(o.mpo_to_dense(R) - H) <= (wl.HILBERT_MPO_TOL + 5e-13) * nH
    assert max(c.shape[3] for c in R[:-1]) <= 12


def test_paper_orientation_merges_five_cores_and_matches_lapack():
    W = wl.hilbert(10)
    P = o.round_mpo(W.cores, wl.HILBERT_MPO_TOL)
    m, s = paper_sigma(P, W)
    assert m == 5                                   # as in the paper: 32 x 32 first core
    H = closed_form(np.arange(1024)[:, None], np.arange(512)[None, :])
    ref = np.linalg.svd(H, compute_uv=False)[:16]
    assert np.linalg.norm(s - ref) / np.linalg.norm(ref) < 1e-8
