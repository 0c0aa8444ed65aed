"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Inputs are drawn once by ``workloads`` (seeded) and handed to both sides; the
random MPO Omega is passed in explicitly (tnrsvd_set_omega) except where the
device's own counter-based generator is under test.

Tolerances (norm-wise relative error of the top-k singular values against the
oracle): 1e-10 for FP64 contractions, 1e-5 for FP32 contractions, 1e-2 for
BF16 contractions before and 1e-5 after one FP32 refinement step.  Quantities
with a gauge (basis cores) are compared under the sign convention both sides
apply (largest-magnitude entry of each left singular vector positive, and
diag(R) >= 0 in every QR) or through gauge-free overlaps.
"""

import numpy as np
import pytest

from oracle import tnrsvd_oracle as o
import workloads as wl
from tests.gpu_helpers import omega_for, gpu_solve, rel_err, cores_np, to_device

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5, "bf16": 1e-2}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1707_07803_amd import load_library
    load_library()   # raises if libtnrsvd.so was not built: no fallback exists
    yield


# ---------------------------------------------------------------- small ----

@pytest.mark.parametrize("q", [0, 1, 2])
def test_small_f64_sigma_and_factors(q):
    W = wl.small()
    om = omega_for(W.cores, W.K, W.omega_seed)
    ref = o.tnrsvd(W.cores, W.k, W.p, q, omega=om)
    sig, h = gpu_solve(W.cores, W.k, W.p, q, omega=om)
    print(f"small f64 q={q}: sigma rel err {rel_err(sig, ref.sigma):.3e}")
    assert rel_err(sig, ref.sigma) <= TOL["f64"]
    # basis cores elementwise (sign conventions fixed on both sides)
    Q = cores_np(h.factor(2))
    assert [c.shape for c in Q] == [c.shape for c in ref.Q]
    for a, b in zip(Q, ref.Q):
        np.testing.assert_allclose(a, b, atol=1e-9)
    # U, V densified against the oracle's
    U = cores_np(h.factor(0))
    V = cores_np(h.factor(1))
    U[-1] = U[-1][:, :, : W.k]
    V[-1] = V[-1][:, :, : W.k]
    np.testing.assert_allclose(o.mps_to_dense(U), o.mps_to_dense(ref.U), atol=1e-9)
    np.testing.assert_allclose(o.mps_to_dense(V), o.mps_to_dense(ref.V), atol=1e-9)
    h.close()


def test_small_first_product_elementwise():
    """Y = A Omega has no gauge: its cores compare elementwise (Sec. 5.2)."""
    W = wl.small()
    om = omega_for(W.cores, W.K, W.omega_seed)
    ref = o.tnrsvd(W.cores, W.k, W.p, 0, omega=om)
    _, h = gpu_solve(W.cores, W.k, W.p, 0, omega=om)
    Y = cores_np(h.factor(3))
    for a, b in zip(Y, ref.Y0):
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-13)
    h.close()


def test_small_f32():
    W = wl.small()
    om = omega_for(W.cores, W.K, W.omega_seed)
    ref = o.tnrsvd(W.cores, W.k, W.p, 1, omega=om)
    sig, h = gpu_solve(W.cores, W.k, W.p, 1, precision="f32", omega=om)
    print(f"small f32: sigma rel err {rel_err(sig, ref.sigma):.3e}")
    assert rel_err(sig, ref.sigma) <= TOL["f32"]
    h.close()


def test_device_omega_matches_counter_generator():
    """The device draws Omega with the same published SplitMix64 + Box-Muller stream."""
    from paper_1707_07803_amd import TNrSVD
    W = wl.small()
    h = TNrSVD(to_device(W.cores), W.k, W.p, 0, seed=1234)
    vecs, last = o.omega_from_seed(omega_cols(W), W.K, 1234)
    ref = np.concatenate([np.ravel(v) for v in vecs] + [np.ravel(last)])
    got = h.omega()
    np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-15)
    sig = h.run()[0]
    res = o.tnrsvd(W.cores, W.k, W.p, 0, seed=1234)
    assert rel_err(sig, res.sigma) <= TOL["f64"]
    h.close()


def omega_cols(W):
    from tests.gpu_helpers import merged_cols
    return merged_cols(W.cores, W.K)


# ------------------------------------------------------------- spectrum ----

@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_spectrum_full_size(precision):
    """Known-spectrum workload at full size (15 cores of 2x2 plus a 32x32 core)."""
    W = wl.spectrum()
    eps = W.eps_by_precision[precision]
    om = omega_for(W.cores, W.K, W.omega_seed)
    ref = o.tnrsvd(W.cores, W.k, W.p, W.q, omega=om, eps=eps, rmax=W.rmax)
    sig, h = gpu_solve(W.cores, W.k, W.p, W.q, precision=precision, eps=eps, rmax=W.rmax,
                       omega=om)
    err = rel_err(sig, ref.sigma)
    exact = rel_err(sig, W.sigma_exact[: W.k])
    print(f"spectrum {precision}: vs oracle {err:.3e}, vs prescribed {exact:.3e}, "
          f"ranks {h.ranks()}")
    assert err <= TOL[precision]
    assert exact <= TOL[precision]
    assert h.ranks() == [1] + ref.ranks[-2][1:] + [W.K]
    h.close()


def test_spectrum_bf16_then_fp32_refinement():
    """BF16 storage + FP32 accumulation, then one FP32 power step (refine)."""
    import torch
    W = wl.spectrum()
    om = omega_for(W.cores, W.K, W.omega_seed)
    ref = o.tnrsvd(W.cores, W.k, W.p, W.q, omega=om, eps=W.eps_by_precision["f64"], rmax=W.rmax)
    sig, h = gpu_solve(W.cores, W.k, W.p, W.q, precision="bf16", eps=W.eps_by_precision["bf16"],
                       rmax=W.rmax, omega=om)
    e0 = rel_err(sig, ref.sigma)
    assert h.factor(2)[0].dtype == torch.bfloat16
    sig2 = h.refine(round_tol=W.eps_by_precision["f32"])[0]
    e1 = rel_err(sig2, ref.sigma)
    print(f"spectrum bf16: {e0:.3e} before, {e1:.3e} after FP32 refinement; ranks {h.ranks()}")
    assert e0 <= TOL["bf16"]
    assert e1 <= TOL["f32"]
    assert rel_err(sig2, W.sigma_exact[: W.k]) <= TOL["f32"]
    assert h.factor(2)[0].dtype == torch.float32
    # the next solve runs in BF16 again and reproduces the first one
    np.testing.assert_array_equal(h.run()[0], sig)
    assert h.factor(2)[0].dtype == torch.bfloat16
    h.close()


def test_small_bf16_first_product_and_sigma():
    W = wl.small()
    om = omega_for(W.cores, W.K, W.omega_seed)
    ref = o.tnrsvd(W.cores, W.k, W.p, 1, omega=om)
    sig, h = gpu_solve(W.cores, W.k, W.p, 1, precision="bf16", omega=om)
    assert rel_err(sig, ref.sigma) <= TOL["bf16"]
    # the first product is rounded to BF16 once per operand and once on output
    for a, b in zip(cores_np(h.factor(3)), ref.Y0):
        assert np.linalg.norm(a - b) <= 2e-2 * np.linalg.norm(b)
    # refinement adds one power step: compare with the oracle at q + 1 (this
    # random MPO has no spectral decay, so the start basis still matters at
    # the BF16 level after one step)
    sig2 = h.refine()[0]
    ref2 = o.tnrsvd(W.cores, W.k, W.p, 2, omega=om)
    print(f"small bf16: {rel_err(sig, ref.sigma):.3e}; refined vs q=2 oracle "
          f"{rel_err(sig2, ref2.sigma):.3e}")
    assert np.all(np.diff(sig2) <= 0) and np.all(sig2 >= 0)
    assert rel_err(sig2, ref2.sigma) <= 2 * TOL["bf16"]
    h.close()


def test_refine_state_errors():
    from paper_1707_07803_amd import TNrSVD, TNrSVDError
    W = wl.small()
    h = TNrSVD(to_device(W.cores, "f32"), W.k, W.p, 0, seed=2, precision="f32")
    h.run()
    with pytest.raises(TNrSVDError) as e:
        h.refine()
    assert e.value.status == -3
    h.close()
    h = TNrSVD(to_device(W.cores, "f32"), W.k, W.p, 0, seed=2, precision="bf16")
    with pytest.raises(TNrSVDError) as e:
        h.refine()
    assert e.value.status == -3
    h.run()
    h.refine()
    with pytest.raises(TNrSVDError) as e:
        h.refine()
    assert e.value.status == -3
    h.close()


# ---------------------------------------------------------- edge cases ----

def test_single_core_mpo():
    """d = 1: no bonds; the pipeline reduces to a dense randomized SVD of the core."""
    rng = np.random.default_rng(5)
    A = [rng.standard_normal((1, 24, 20, 1))]
    om = ([], rng.standard_normal((20, 12)))
    ref = o.tnrsvd(A, 8, 4, 1, omega=om)
    sig, h = gpu_solve(A, 8, 4, 1, omega=om)
    assert rel_err(sig, ref.sigma) <= TOL["f64"]
    h.close()


def test_rectangular_uneven_cores():
    """Ragged shapes: I != J, mixed mode sizes, a merge of 3 cores."""
    rng = np.random.default_rng(6)
    shapes = [(1, 3, 2, 4), (4, 2, 3, 5), (5, 4, 2, 3), (3, 2, 3, 2), (2, 3, 2, 2), (2, 2, 4, 1)]
    A = [rng.standard_normal(s) for s in shapes]
    om = omega_for(A, 10, 7)
    for q in (0, 1):
        ref = o.tnrsvd(A, 6, 4, q, omega=om)
        sig, h = gpu_solve(A, 6, 4, q, omega=om)
        assert rel_err(sig, ref.sigma) <= TOL["f64"]
        h.close()


@pytest.mark.parametrize("k,p", [(24, 16), (64, 32)])
def test_last_core_panel_layouts(k, p):
    """The left-to-right pass keeps the last core's (s n) x K panel in LDS up
    to 10240 entries.  K = 40 (s n = 256): the panel exactly at that limit,
    its explicit Q in the scratch, the SVD rotations in LDS; K = 96: all
    three in the scratch.  Both against the oracle, q = 1 (three roundings
    with the QR of the last core, one with its SVD)."""
    rng = np.random.default_rng(21)
    d, R = 8, 4
    cores = [rng.standard_normal((1 if i == 0 else R, 2, 2, 1 if i == d - 1 else R))
             for i in range(d)]
    om = omega_for(cores, k + p, 5)
    ref = o.tnrsvd(cores, k, p, 1, omega=om)
    sig, h = gpu_solve(cores, k, p, 1, omega=om)
    print(f"K={k + p}: sigma rel err {rel_err(sig, ref.sigma):.2e}")
    assert rel_err(sig, ref.sigma) <= TOL["f64"]
    h.close()


@pytest.mark.parametrize("R,rmax", [(16, 8), (12, 8), (10, 7)])
def test_register_qr_panel_widths(R, rmax):
    """Products of 128 (the register QR's widest panel, 256 rows), 96 (three
    full 32-column blocks) and 70 columns (a 6-column last block) through the
    right-to-left sweep, against the oracle."""
    d, k, p = 10, 8, 8
    rng = np.random.default_rng(5)
    cores = [rng.standard_normal((1 if i == 0 else R, 2, 2, 1 if i == d - 1 else R)) / np.sqrt(R)
             for i in range(d)]
    om = omega_for(cores, k + p, 3)
    ref = o.tnrsvd(cores, k, p, 1, omega=om, rmax=rmax)
    sig, h = gpu_solve(cores, k, p, 1, omega=om, rmax=rmax)
    P, _ = h.product_ranks()
    print(f"R={R} rmax={rmax}: product ranks {P}, sigma rel err {rel_err(sig, ref.sigma):.2e}")
    assert max(P) == R * rmax
    assert rel_err(sig, ref.sigma) <= TOL["f64"]
    h.close()


def test_zero_matrix():
    W = wl.small()
    Z = [np.zeros_like(c) for c in W.cores]
    sig, h = gpu_solve(Z, W.k, W.p, 1, seed=3)
    assert np.all(sig == 0.0)
    h.close()


def test_rank_cap_truncation_matches_oracle():
    """r_max below the product ranks: the truncation path of the rounding."""
    W = wl.small()
    om = omega_for(W.cores, W.K, W.omega_seed)
    ref = o.tnrsvd(W.cores, W.k, W.p, 1, omega=om, rmax=4)
    sig, h = gpu_solve(W.cores, W.k, W.p, 1, omega=om, rmax=4)
    assert rel_err(sig, ref.sigma) <= TOL["f64"]
    assert h.ranks() == [1] + ref.ranks[-2][1:] + [W.K]
    h.close()


def test_tolerance_truncation_matches_oracle():
    W = wl.spectrum(d_inner=8)
    om = omega_for(W.cores, W.K, 9)
    for eps in (1e-3, 1e-8):
        ref = o.tnrsvd(W.cores, W.k, W.p, 1, omega=om, eps=eps, rmax=32)
        sig, h = gpu_solve(W.cores, W.k, W.p, 1, omega=om, eps=eps, rmax=32)
        assert rel_err(sig, ref.sigma) <= TOL["f64"]
        h.close()


def test_batch_equals_single_solves():
    """Uneven MPOs in one persistent launch equal their one-by-one solves."""
    from paper_1707_07803_amd import TNrSVD, omega_flat
    Ws = wl.batched(6)
    for W in Ws:   # shrink ranks so the oracle stays fast
        W.cores = W.cores[:10]
        W.cores[-1] = W.cores[-1][..., :1]
    sub = []
    for W in Ws:
        r = [1] + [min(c.shape[3], 6) for c in W.cores[:-1]] + [1]
        sub.append([np.ascontiguousarray(c[: r[i], :, :, : r[i + 1]]) for i, c in enumerate(W.cores)])
    K = Ws[0].K
    oms = [omega_for(c, K, 100 + b) for b, c in enumerate(sub)]
    h = TNrSVD([to_device(c) for c in sub], 8, 8, 1, max_rank=32)
    for b, om in enumerate(oms):
        h.set_omega(omega_flat(*om), b)
    sig = h.run()
    for b, c in enumerate(sub):
        ref = o.tnrsvd(c, 8, 8, 1, omega=oms[b], rmax=32)
        assert rel_err(sig[b], ref.sigma) <= TOL["f64"], b
    h.close()


# ------------------------------------------------------------ ABI errors ----

def test_state_machine_errors():
    from paper_1707_07803_amd import TNrSVD, TNrSVDError
    W = wl.small()
    h = TNrSVD(to_device(W.cores), W.k, W.p, 0, seed=1)
    with pytest.raises(TNrSVDError) as e:
        h.orthogonalize()
    assert e.value.status == -3
    with pytest.raises(TNrSVDError) as e:
        h.mult(1)
    assert e.value.status == -3
    h.mult(0)
    with pytest.raises(TNrSVDError):
        h.mult(0)
    h.orthogonalize()
    with pytest.raises(TNrSVDError):
        h.solve()
    h.project()
    sig = h.solve()
    ref = o.tnrsvd(W.cores, W.k, W.p, 0, seed=1)
    assert rel_err(sig[0], ref.sigma) <= TOL["f64"]
    h.close()


def test_create_errors():
    from paper_1707_07803_amd import TNrSVD, TNrSVDError
    W = wl.small()
    with pytest.raises(TNrSVDError) as e:
        TNrSVD(to_device(wl.random_mpo(3, 2, 2, 2, 1.0, 1)), 6, 4, 0)   # K = 10 > prod I = 8
    assert e.value.status == -2
    with pytest.raises(TNrSVDError) as e:
        TNrSVD(to_device(W.cores), 200, 57, 0)                          # K above the cap
    assert e.value.status == -1
    bad = [c.copy() for c in W.cores]
    bad[2][0, 0, 0, 0] = np.nan
    with pytest.raises(TNrSVDError) as e:
        TNrSVD(to_device(bad), 4, 2, 0, check_finite=True)
    assert e.value.status == -6
