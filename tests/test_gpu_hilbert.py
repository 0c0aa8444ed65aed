"""GPU parity of the rounding of a general MPO (tnrsvd_round_mpo) and of the
Hilbert experiment of Sec. 6.3 (round the MPO, then TNrSVD in the paper's
orientation with the first 5 cores merged).

Rounding: both sides compute the same truncated SVDs in FP64 by different
algorithms (Householder QR + Jacobi on the GPU, LAPACK in the oracle) with the
same sign conventions, so ranks are equal and cores agree to 1e-9 of their
scale where singular values are separated and well above the rounding level
(random MPOs); the Hilbert MPO keeps singular values down to 1e-12 |A|_F, so
it is compared through the matrix it represents.  The Hilbert solve: the GPU runs
on its own rounded MPO, the oracle on its own, with the same Omega; singular
values agree to 1e-8 relative (rounding at 1e-12, then 1e-9 inside the
solve), and at N = 10 both match LAPACK on the dense matrix.
"""

import numpy as np
import pytest

from oracle import tnrsvd_oracle as o
import workloads as wl
from gpu_helpers import omega_for, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1707_07803_amd import load_library
    load_library()
    yield


def gpu_round(cores, eps, rmax=0, dtype="f64"):
    from paper_1707_07803_amd import round_mpo
    return [c.cpu().numpy() for c in round_mpo(to_device(cores, dtype), eps, rmax)]


def assert_close_cores(g, ref, tol=1e-9):
    assert [x.shape for x in g] == [x.shape for x in ref]
    scale = np.linalg.norm(ref[-1])
    for k, (a, b) in enumerate(zip(g, ref)):
        s = 1.0 if k < len(g) - 1 else scale      # the last core carries the norm
        np.testing.assert_allclose(a, b, atol=tol * s, rtol=0)


def left_orthonormal(cores):
    for G in cores[:-1]:
        Q = G.reshape(-1, G.shape[3])
        np.testing.assert_allclose(Q.T @ Q, np.eye(Q.shape[1]), atol=1e-11)


def rand_mpo(shapes, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(s) for s in shapes]


def chain(I, J, R):
    d = len(I)
    r = [1] + list(R) + [1]
    return [(r[k], I[k], J[k], r[k + 1]) for k in range(d)]


CASES = {
    "random_d6": (chain([2] * 6, [3] * 6, [4, 5, 6, 5, 4]), 1e-12, 0),
    "truncating": (chain([2] * 6, [3] * 6, [4, 5, 6, 5, 4]), 0.3, 0),
    "rank_cap": (chain([2] * 6, [3] * 6, [4, 5, 6, 5, 4]), 1e-12, 3),
    "mixed_modes": (chain([3, 1, 4, 2], [2, 5, 1, 3], [6, 9, 5]), 1e-10, 0),
    "wide_bonds": (chain([2, 2, 2, 2], [2, 2, 2, 2], [40, 70, 30]), 1e-10, 0),
    "d2": (chain([7, 5], [3, 4], [9]), 1e-10, 0),
    # an LQ panel of 16 * 80 = 1280 rows: too tall for the LDS panel path
    "tall_panel": (chain([4] * 4, [4] * 4, [80, 80, 80]), 1e-10, 0),
}


@pytest.mark.parametrize("case", list(CASES))
def test_random_mpo_against_oracle(case):
    shapes, eps, rmax = CASES[case]
    A = rand_mpo(shapes, 100 + list(CASES).index(case))
    g = gpu_round(A, eps, rmax)
    ref = o.round_mpo(A, eps, rmax)
    print(case, "ranks", [x.shape[3] for x in ref[:-1]])
    assert_close_cores(g, ref)
    left_orthonormal(g)
    if rmax == 0:
        D, Dg = o.mpo_to_dense(A), o.mpo_to_dense(g)
        assert np.linalg.norm(Dg - D) <= max(eps, 1e-13) * np.linalg.norm(D) * 1.0001


def test_float32_input_and_single_core():
    A = rand_mpo(chain([2] * 5, [2] * 5, [3, 4, 4, 3]), 7)
    A32 = [a.astype(np.float32).astype(np.float64) for a in A]
    assert_close_cores(gpu_round(A32, 1e-10, dtype="f32"), o.round_mpo(A32, 1e-10))
    B = rand_mpo([(1, 6, 5, 1)], 8)
    np.testing.assert_array_equal(gpu_round(B, 0.5)[0], B[0])


def test_zero_product_gives_zero_cores():
    A = rand_mpo(chain([2] * 4, [3] * 4, [3, 3, 3]), 9)
    A[2] = np.zeros_like(A[2])
    g = gpu_round(A, 1e-8)
    assert [x.shape for x in g] == [(1, 2, 3, 1)] * 4 and not any(np.any(x) for x in g)


def test_errors():
    import torch
    from paper_1707_07803_amd import TNrSVDError, round_mpo
    A = to_device(rand_mpo(chain([2] * 3, [2] * 3, [2, 2]), 1))
    with pytest.raises(TNrSVDError) as ei:
        round_mpo(A, -1.0)
    assert ei.value.status == -1
    with pytest.raises(TNrSVDError) as ei:
        round_mpo(A, 1e-3, -2)
    assert ei.value.status == -1
    bad = [torch.zeros((2, 2, 2, 2), dtype=torch.float64, device="cuda")] + A[1:]
    with pytest.raises(TNrSVDError) as ei:          # rank[0] != 1
        round_mpo(bad, 1e-3)
    assert ei.value.status == -2


# ----------------------------------------------------------------- Hilbert ----

@pytest.mark.parametrize("N", [10, 20])
def test_hilbert_rounding_against_oracle(N):
    """Ranks equal to the oracle's; the cores themselves are compared through
    the matrix they represent, because the rounding keeps singular values down
    to 1e-12 |A|_F whose vectors FP64 fixes only to about 1e-4."""
    C = wl.hilbert_mpo(N)
    g = gpu_round(C, wl.HILBERT_MPO_TOL)
    ref = o.round_mpo(C, wl.HILBERT_MPO_TOL)
    print(f"hilbert{N} input rank {C[0].shape[3]}, rounded ranks {[x.shape[3] for x in g[:-1]]}")
    assert [x.shape for x in g] == [x.shape for x in ref]
    left_orthonormal(g)
    nA = np.linalg.norm(g[-1])                      # |rounded|_F, given orthonormality
    bound = (wl.HILBERT_MPO_TOL + 5e-13) * nA       # rounding + the exponential sum's error
    if N == 10:
        H = 1.0 / (np.arange(1024)[:, None] + np.arange(512)[None, :] + 1.0)
        assert np.linalg.norm(o.mpo_to_dense(g) - H) <= bound
        assert np.linalg.norm(o.mpo_to_dense(g) - o.mpo_to_dense(ref)) <= 2 * bound
    else:
        rng = np.random.default_rng(N)
        i = rng.integers(0, 2 ** N, 4000, dtype=np.int64)
        j = rng.integers(0, 2 ** (N - 1), 4000, dtype=np.int64)
        exact = 1.0 / (i.astype(np.float64) + j + 1.0)
        assert np.max(np.abs(entries(g, i, j) - exact)) <= bound
        assert np.max(np.abs(entries(g, i, j) - entries(ref, i, j))) <= 2 * bound


def entries(cores, i, j):
    v = np.ones((len(i), 1))
    ii, jj = i.copy(), j.copy()
    for G in cores:
        I, J = G.shape[1], G.shape[2]
        v = np.einsum("ea,eab->eb", v, G[:, ii % I, jj % J, :].transpose(1, 0, 2))
        ii //= I
        jj //= J
    return v[:, 0]


def hilbert_solve_gpu(P, W, seed=0):
    """TNrSVD in the paper's orientation on the device MPO P (first cores
    merged), with Omega drawn as the oracle draws it for the mirrored layout."""
    from paper_1707_07803_amd import TNrSVD, omega_flat
    L_shapes = o.reverse_mpo([np.zeros(tuple(c.shape)) for c in P])
    om = omega_flat(*omega_for(L_shapes, W.K, W.omega_seed))
    h = TNrSVD(P, W.k, W.p, W.q, seed=seed, round_tol=W.eps, max_rank=W.rmax,
               orientation="k_first")
    h.set_omega(om)
    s = h.run()[0]
    return s, h


def hilbert_solve_oracle(Pn, W):
    L = o.reverse_mpo(Pn)
    m = o.merge_plan([c.shape[1] for c in L], [c.shape[2] for c in L], W.K)
    cols = [c.shape[2] for c in L]
    om = wl.gaussian_omega(cols[: len(L) - m] + [int(np.prod(cols[len(L) - m:]))], W.K,
                           W.omega_seed)
    A1 = o.reverse_mpo(o.merge_tail(L, m))
    return m, o.tnrsvd_paper_orientation(A1, W.k, W.p, W.q, om[1], om[0][::-1], eps=W.eps,
                                            rmax=W.rmax)


@pytest.mark.parametrize("N", [10, 30, 50])
def test_hilbert_sigma_against_oracle(N):
    from paper_1707_07803_amd import round_mpo
    W = wl.hilbert(N)
    P = round_mpo(to_device(W.cores), wl.HILBERT_MPO_TOL)
    s, h = hilbert_solve_gpu(P, W)
    assert h.d_merged() == N - 4                    # the first 5 cores merged (32 x 32)
    assert h.ranks()[0] == W.K
    m, ref = hilbert_solve_oracle(o.round_mpo(W.cores, wl.HILBERT_MPO_TOL), W)
    assert m == 5
    err = np.linalg.norm(s - ref) / np.linalg.norm(ref)
    print(f"hilbert{N}: sigma_1 {s[0]:.6f} sigma_16 {s[15]:.3e} rel err vs oracle {err:.2e}")
    assert err < 1e-8
    if N == 10:
        H = 1.0 / (np.arange(1024)[:, None] + np.arange(512)[None, :] + 1.0)
        lap = np.linalg.svd(H, compute_uv=False)[:16]
        assert np.linalg.norm(s - lap) / np.linalg.norm(lap) < 1e-8
