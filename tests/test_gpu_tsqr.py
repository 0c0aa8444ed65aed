"""GPU parity of the tall last-core panel path of the right-to-left sweep.

When the last core's panel has more than 256 and at most 4096 rows (mode
size n times K) and at most 128 columns, it is factorised by TSQR: the 256-row
leaves all at once (one workgroup each), then a binary tree of merges, level
by level.  These cases cover the largest leaf count (16), odd trees (3 and 6
leaves), a ragged last leaf with fewer rows than the panel has columns, and a batch that mixes leaf
counts with an MPO whose last core takes the plain register path.  The
singular values are compared with the FP64 oracle, which factorises the
panels without any tiling.
"""

import numpy as np
import pytest

from oracle import tnrsvd_oracle as o
from tests.gpu_helpers import gpu_solve, omega_for, rel_err, to_device
import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1707_07803_amd import load_library
    load_library()
    yield


def tall_mpo(n_last, seed, R=3):
    """Three 2 x 2 cores, then one n_last x n_last core behind a bond of rank
    4, so the product panels reach 4 x 8 = 32 columns."""
    rng = np.random.default_rng(seed)
    shapes = [(1, 2, 2, R), (R, 2, 2, R), (R, 2, 2, 4), (4, n_last, n_last, 1)]
    return [rng.standard_normal(s) for s in shapes]


@pytest.mark.parametrize("n_last,k,p,q", [
    (64, 40, 24, 1),   # 64 * 64 = 4096 rows: 16 leaves, the most the path takes
    (17, 10, 6, 1),    # 17 * 16 = 272 rows: 2 leaves, the second with 16 rows < 32 columns
    (20, 10, 6, 2),    # 320 rows, ragged second leaf, two power steps
    (40, 10, 6, 1),    # 640 rows: 3 leaves, an odd tree
    (44, 20, 12, 1),   # 1408 rows: 6 leaves, a partial right subtree
])
def test_tall_last_core_against_oracle(n_last, k, p, q):
    A = tall_mpo(n_last, 40 + n_last)
    K = k + p
    assert o.merge_plan([c.shape[1] for c in A], [c.shape[2] for c in A], K) == 1
    om = omega_for(A, K, 7)
    ref = o.tnrsvd(A, k, p, q, omega=om)
    sig, h = gpu_solve(A, k, p, q, omega=om)
    print(f"last core {n_last}x{n_last}, K={K}: {n_last * K} panel rows, "
          f"sigma rel err {rel_err(sig, ref.sigma):.2e}")
    assert rel_err(sig, ref.sigma) <= 1e-10
    h.close()


def test_batch_mixing_leaf_counts_equals_oracle():
    from paper_1707_07803_amd import TNrSVD, omega_flat
    k, p, q = 10, 6, 1
    K = k + p
    mpos = [tall_mpo(64, 1), tall_mpo(17, 2), wl.small().cores, tall_mpo(20, 3)]
    oms = [omega_for(c, K, 60 + b) for b, c in enumerate(mpos)]
    h = TNrSVD([to_device(c) for c in mpos], k, p, q)
    for b, om in enumerate(oms):
        h.set_omega(omega_flat(*om), b)
    for rep in range(2):                 # the leaf workspace is reused between runs
        sig = h.run()
        for b, c in enumerate(mpos):
            ref = o.tnrsvd(c, k, p, q, omega=oms[b]).sigma
            assert rel_err(sig[b], ref) <= 1e-10, (rep, b)
    h.close()


def test_tall_last_core_f32_and_graph_replay():
    import torch
    from paper_1707_07803_amd import TNrSVD, omega_flat
    A = tall_mpo(64, 9)
    om = omega_for(A, 16, 3)
    ref = o.tnrsvd(A, 10, 6, 1, omega=om).sigma
    h = TNrSVD(to_device(A, "f32"), 10, 6, 1, precision="f32")
    h.set_omega(omega_flat(*om))
    eager = h.run()[0]
    assert rel_err(eager, ref) <= 1e-5
    for rep in range(3):
        s = h.run_graph()[0]
        np.testing.assert_array_equal(s, eager)
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()
    h.close()


def test_batch_mixing_tree_depths_equals_oracle():
    """A 16-leaf tree (4096 rows) sharing the level launches with a 6-leaf
    tree (1408 rows, a partial right subtree) and a 3-leaf one (640 rows):
    the smaller trees stop at their own root levels while the big one goes on."""
    from paper_1707_07803_amd import TNrSVD, omega_flat
    k, p, q = 10, 6, 1
    K = k + p
    mpos = [tall_mpo(256, 11), tall_mpo(88, 12), tall_mpo(40, 13)]
    oms = [omega_for(c, K, 70 + b) for b, c in enumerate(mpos)]
    h = TNrSVD([to_device(c) for c in mpos], k, p, q)
    for b, om in enumerate(oms):
        h.set_omega(omega_flat(*om), b)
    sig = h.run()
    for b, c in enumerate(mpos):
        ref = o.tnrsvd(c, k, p, q, omega=oms[b]).sigma
        print(f"tree member {b}: {c[-1].shape[1] * K} rows, sigma rel err {rel_err(sig[b], ref):.2e}")
        assert rel_err(sig[b], ref) <= 1e-10, b
    h.close()


def test_tall_last_core_factors_against_oracle():
    """The singular vectors after the 6-leaf tree's replay in the
    left-to-right pass: U and V densified are orthonormal and match the
    oracle's column by column (sign conventions fixed on both sides)."""
    from tests.gpu_helpers import cores_np
    k, p, q = 20, 12, 1
    A = tall_mpo(44, 84)
    om = omega_for(A, k + p, 7)
    ref = o.tnrsvd(A, k, p, q, omega=om)
    sig, h = gpu_solve(A, k, p, q, omega=om)
    assert rel_err(sig, ref.sigma) <= 1e-10
    for which, R in ((0, ref.U), (1, ref.V)):
        F = cores_np(h.factor(which))
        F[-1] = F[-1][:, :, :k]
        D, Dr = o.mps_to_dense(F), o.mps_to_dense(R)
        assert D.shape == Dr.shape
        np.testing.assert_allclose(D.T @ D, np.eye(k), atol=1e-12)
        np.testing.assert_allclose(D, Dr, atol=1e-8)
    h.close()
