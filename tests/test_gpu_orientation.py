"""GPU tests of the paper's orientation (tnrsvd_opts.orientation = K_FIRST).

In the paper (Sec. 5) Omega, Y, Q, U and V carry their K leg on the FIRST
core and the sweeps run right to left; the library keeps it on the last core.
A K_FIRST handle reads the caller's MPO with its cores reversed and their rank
legs swapped (the same matrix with the row and column digits reversed), so:
- its singular values equal, bit for bit, those of a K_LAST handle on the
  reversed MPO, and match the oracle written in the paper's orientation;
- its factors are digit permutations of the K_LAST factors, and as
  matrices over the caller's own (little-endian, eq. (1)) indices they
  diagonalise the caller's matrix: U^T A V = diag(sigma);
- its gradients are the K_LAST gradients reversed, and their directional
  derivative equals that of sum_j u_j^T A v_j computed densely.
"""

import ctypes

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


def mixed_radix():
    rng = np.random.default_rng(31)
    rows, cols, R = [3, 2, 4, 2, 2, 3], [2, 3, 2, 4, 2, 2], [1, 3, 4, 3, 4, 2, 1]
    return [rng.standard_normal((R[i], rows[i], cols[i], R[i + 1])) for i in range(6)]


CASES = {"small": (lambda: wl.small().cores, 10, 6, 0),
         "small_q1": (lambda: wl.small().cores, 10, 6, 1),
         "mixed": (mixed_radix, 4, 4, 1)}


def k_first_dense(cores):
    """Factor cores in the paper's layout (K, n_0, r_1), ..., (r, n, 1) as a
    (prod n) x K matrix with the little-endian index of eq. (1)."""
    T = cores[0].transpose(0, 1, 2)                      # (K, idx, r)
    for c in cores[1:]:
        K, m, r = T.shape
        T = np.einsum("kir,rjs->kjis", T, c).reshape(K, c.shape[1] * m, c.shape[2])
    return T[:, :, 0].T


def k_last_dense(cores):
    """Factor cores in the library's layout (1, n_0, r_1), ..., (r, n, K)."""
    T = cores[0][0]                                      # (idx, r)
    for c in cores[1:]:
        m, r = T.shape
        T = np.einsum("ir,rjs->jis", T, c).reshape(c.shape[1] * m, c.shape[2])
    return T


def digit_reverse_rows(X, radices):
    """Row i of the result is row rev(i) of X, rev reversing the little-endian
    digits of radices (given in X's own order)."""
    d = len(radices)
    Y = X.reshape(tuple(radices[::-1]) + X.shape[1:])     # C order: most significant first
    Y = Y.transpose(tuple(range(d))[::-1] + tuple(range(d, Y.ndim)))
    return Y.reshape(X.shape)


def perm_close(a, b):
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-13 * np.abs(b).max())


def handles(case, seed=3):
    from paper_1707_07803_amd import TNrSVD, omega_flat
    make, k, p, q = CASES[case]
    L = make()                              # the library-orientation MPO
    P = o.reverse_mpo(L)                    # the same matrix, read as the paper's layout
    om = omega_flat(*omega_for(L, k + p, seed))
    hl = TNrSVD(to_device(L), k, p, q, seed=seed)
    hf = TNrSVD(to_device(P), k, p, q, seed=seed, orientation="k_first")
    hl.set_omega(om)
    hf.set_omega(om)
    return L, P, hl, hf, k, p, q, om


def paper_merged_first(P, m):
    """Merge the first m cores of a paper-layout MPO into one, with the merged
    digits in the order the library merges them (core m-1's least significant)."""
    return o.reverse_mpo(o.merge_tail(o.reverse_mpo(P), m))


@pytest.mark.parametrize("case", list(CASES))
def test_sigma_matches_library_layout_and_paper_oracle(case):
    L, P, hl, hf, k, p, q, om = handles(case)
    sl, sf = hl.run()[0], hf.run()[0]
    np.testing.assert_array_equal(sf, sl)
    # the oracle in the paper's orientation: Omega's K leg on the (merged)
    # first core; the library's merged Omega matrix is indexed by the merged
    # digits of the reversed MPO, which the oracle's merge of reverse(P)'s
    # trailing cores reproduces, and its vectors run in the reversed order
    dm = hf.d_merged()
    m = len(P) - dm + 1
    Km = k + p
    Jm = int(np.prod([c.shape[2] for c in P[:m]]))
    vec_len = [c.shape[2] for c in L[: len(L) - m]]
    offs = np.cumsum([0] + vec_len)
    vecs = [om[offs[i]:offs[i + 1]] for i in range(len(vec_len))]
    last = om[offs[-1]:].reshape(Jm, Km)
    s_or = o.tnrsvd_paper_orientation(paper_merged_first(P, m), k, p, q, last, vecs[::-1])
    np.testing.assert_allclose(sf, s_or, rtol=1e-10, atol=1e-12 * s_or[0])


@pytest.mark.parametrize("case", list(CASES))
def test_factors_are_digit_permutations_and_diagonalise(case):
    L, P, hl, hf, k, p, q, om = handles(case)
    s = hf.run()[0]
    hl.run()
    assert hf.ranks() == hl.ranks()[::-1]
    rows_P = [c.shape[1] for c in P]
    cols_P = [c.shape[2] for c in P]
    Uf = k_first_dense([t.cpu().numpy() for t in hf.factor(0)])
    Vf = k_first_dense([t.cpu().numpy() for t in hf.factor(1)])
    Ul = k_last_dense([t.cpu().numpy() for t in hl.factor(0)])
    Vl = k_last_dense([t.cpu().numpy() for t in hl.factor(1)])
    # (the two dense contractions run in opposite orders: rounding only)
    perm_close(Uf, digit_reverse_rows(Ul, rows_P[::-1]))
    perm_close(Vf, digit_reverse_rows(Vl, cols_P[::-1]))
    # as matrices over the caller's own indices (U and V keep all K columns;
    # the first k belong to the returned singular values)
    Uf, Vf = Uf[:, :k], Vf[:, :k]
    A = o.mpo_to_dense(P)
    np.testing.assert_allclose(Uf.T @ Uf, np.eye(k), atol=1e-12)
    np.testing.assert_allclose(Vf.T @ Vf, np.eye(k), atol=1e-12)
    np.testing.assert_allclose(Uf.T @ A @ Vf, np.diag(s), atol=1e-11 * s[0])
    # Y = A Omega (which 3) keeps its FP64 values, permuted the same way
    Yf = k_first_dense([t.double().cpu().numpy() for t in hf.factor(3)])
    Yl = k_last_dense([t.double().cpu().numpy() for t in hl.factor(3)])
    perm_close(Yf, digit_reverse_rows(Yl, rows_P[::-1]))


def test_get_factor_reports_paper_shape_without_pointer():
    L, P, hl, hf, k, p, q, om = handles("mixed")
    hf.run()
    lib = hf._lib
    dm = hf.d_merged()
    ranks = hf.ranks()
    for core in range(dm):
        ptr = ctypes.c_void_p(1)
        shape = (ctypes.c_int64 * 4)()
        dt = ctypes.c_int()
        assert lib.tnrsvd_get_factor(hf._h, 0, 2, core, ctypes.byref(ptr), shape,
                                     ctypes.byref(dt)) == 0
        assert ptr.value is None
        assert shape[0] == ranks[core] and shape[2] == ranks[core + 1]
    assert ranks[0] == k + p and ranks[-1] == 1


def test_gradient_reversed_and_directional():
    import torch
    L, P, hl, hf, k, p, q, om = handles("small")
    hl.run()
    hf.run()
    gl = [torch.zeros_like(t) for t in to_device(L)]
    gf = [torch.zeros_like(t) for t in to_device(P)]
    w = np.linspace(1.0, 2.0, k)
    hl.backward(w, gl)                 # the pipeline's derivative
    hf.backward(w, gf)
    for a, b in zip([g.cpu().numpy() for g in gf], o.reverse_mpo([g.cpu().numpy() for g in gl])):
        np.testing.assert_array_equal(a, b)
    hl.backward(w, gl, frozen=True)    # the derivative at fixed singular vectors
    hf.backward(w, gf, frozen=True)
    gl = [g.cpu().numpy() for g in gl]
    gf = [g.cpu().numpy() for g in gf]
    for a, b in zip(gf, o.reverse_mpo(gl)):
        np.testing.assert_array_equal(a, b)
    # directional derivative of sum_j w_j u_j^T A v_j at fixed u, v, densely
    Uf = k_first_dense([t.cpu().numpy() for t in hf.factor(0)])[:, :k]
    Vf = k_first_dense([t.cpu().numpy() for t in hf.factor(1)])[:, :k]
    rng = np.random.default_rng(8)
    dG = [rng.standard_normal(c.shape) for c in P]
    dA = sum(o.mpo_to_dense(P[:c] + [dG[c]] + P[c + 1:]) for c in range(len(P)))
    want = float(np.sum(w * np.einsum("ij,ik,kj->j", Uf, dA, Vf)))
    got = float(sum(np.vdot(g, x) for g, x in zip(gf, dG)))
    assert abs(got - want) <= 1e-10 * max(abs(want), 1.0)


def test_unknown_orientation_is_rejected(monkeypatch):
    from paper_1707_07803_amd import TNrSVD, TNrSVDError, tnrsvd as binding
    monkeypatch.setitem(binding.ORIENTATIONS, "sideways", 2)
    with pytest.raises(TNrSVDError) as ei:
        TNrSVD(to_device(wl.small().cores), 10, 6, 0, orientation="sideways")
    assert ei.value.status == -1
