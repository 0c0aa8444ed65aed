"""The frozen-subspace gradient (tnrsvd_backward_frozen, TNrSVD.backward(...,
frozen=True)) against the oracle's sigma_sum_grad on the same Omega.

Both sides differentiate sum_j dsigma_j u_j^T A v_j at the computed singular
vectors; the FP64 factors of the two sides agree to ~1e-12, so FP64
gradients must agree to 1e-8 relative (norm-wise over all cores); FP32 ones
to 1e-4 when the singular values are well separated relative to sigma_0 and
to 1e-3 on the known spectrum, whose small singular vectors FP32 rounding
moves by eps32 sigma_0 / gap.  Where the computed subspace is exact (rank(A)
<= K, no truncation) it is the derivative of the pipeline's output, which
finite differences of the whole GPU pipeline check here; the pipeline
derivative (tnrsvd_backward) has its own parity tests beside this file.
"""

import numpy as np
import pytest

from oracle import tnrsvd_oracle as o
import workloads as wl
from tests.gpu_helpers import omega_for, gpu_solve, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1707_07803_amd import load_library
    load_library()
    yield


def gpu_grad(h, cores, dsigma=None, dtype=None, frozen=True):
    import torch
    td = {None: torch.float64, "f64": torch.float64, "f32": torch.float32}[dtype]
    grads = [torch.empty(c.shape, dtype=td, device="cuda") for c in cores]
    h.backward(dsigma, grads, frozen=frozen)
    return [g.double().cpu().numpy() for g in grads]


def rel(gs, rs):
    a = np.concatenate([g.ravel() for g in gs])
    b = np.concatenate([r.ravel() for r in rs])
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rank_r_mpo(d, n, r, seed):
    rng = np.random.default_rng(seed)
    A = None
    for _ in range(r):
        term = [np.outer(rng.standard_normal(n), rng.standard_normal(n)).reshape(1, n, n, 1)
                for _ in range(d)]
        A = term if A is None else o.mpo_add(A, term)
    return A


def test_small_weighted_f64_with_merged_tail():
    W = wl.small()                     # the last 4 cores are merged (K = 16)
    om = omega_for(W.cores, W.K, W.omega_seed)
    ref = o.tnrsvd(W.cores, W.k, W.p, 1, omega=om)
    w = np.random.default_rng(2).standard_normal(W.k)
    G_ref = o.sigma_sum_grad(W.cores, ref, w)
    _, h = gpu_solve(W.cores, W.k, W.p, 1, omega=om)
    G = gpu_grad(h, W.cores, w)
    err = rel(G, G_ref)
    print(f"small f64 weighted gradient: rel err {err:.3e}")
    assert err <= 1e-8
    h.close()


def test_exact_case_gradient_and_pipeline_finite_differences():
    A = rank_r_mpo(6, 2, 3, 5)         # rank 3 <= K = 8: computed subspace is exact
    k, p = 3, 5
    om = omega_for(A, k + p, 21)
    ref = o.tnrsvd(A, k, p, 1, omega=om)
    G_ref = o.sigma_sum_grad(A, ref)
    sig, h = gpu_solve(A, k, p, 1, omega=om)
    G = gpu_grad(h, A)
    assert rel(G, G_ref) <= 1e-8
    h.close()
    rng = np.random.default_rng(8)
    hstep = 1e-6
    for i in (0, 2, 5):
        D = rng.standard_normal(A[i].shape)
        Ap = [a.copy() for a in A]
        Ap[i] = Ap[i] + hstep * D
        Am = [a.copy() for a in A]
        Am[i] = Am[i] - hstep * D
        sp, hp = gpu_solve(Ap, k, p, 1, omega=om)
        sm, hm = gpu_solve(Am, k, p, 1, omega=om)
        hp.close()
        hm.close()
        fd = (sp.sum() - sm.sum()) / (2 * hstep)
        got = float(np.sum(G[i] * D))
        assert abs(got - fd) <= 1e-5 * (1 + abs(fd)), (i, got, fd)


def test_grad_workload_f32_against_oracle():
    """d = 30, 4 x 4 cores, ranks 16, k = 16, p = 8, q = 1 (the last 3 cores merged)."""
    W = wl.grad()
    om = omega_for(W.cores, W.K, W.omega_seed)
    ref = o.tnrsvd(W.cores, W.k, W.p, W.q, omega=om, eps=W.eps, rmax=W.rmax)
    G_ref = o.sigma_sum_grad(W.cores, ref)
    sig, h = gpu_solve(W.cores, W.k, W.p, W.q, precision="f32", eps=W.eps, rmax=W.rmax, omega=om)
    G = gpu_grad(h, W.cores, dtype="f32")
    err = rel(G, G_ref)
    print(f"grad workload f32: sigma rel err "
          f"{np.linalg.norm(sig - ref.sigma) / np.linalg.norm(ref.sigma):.3e}, gradient rel err "
          f"{err:.3e}")
    assert err <= 1e-4
    h.close()


def test_backward_errors():
    import torch
    from paper_1707_07803_amd import TNrSVD, TNrSVDError
    W = wl.small()
    h = TNrSVD(to_device(W.cores), W.k, W.p, 0, seed=4)
    grads = [torch.empty(c.shape, dtype=torch.float64, device="cuda") for c in W.cores]
    with pytest.raises(TNrSVDError) as e:        # no solve yet
        h.backward(None, grads)
    assert e.value.status == -3
    h.run()
    with pytest.raises(TNrSVDError) as e:        # wrong number of weights
        h.backward(np.ones(W.k + 1), grads)
    assert e.value.status == -1
    with pytest.raises(TNrSVDError) as e:
        h.backward(np.ones(W.k + 1), grads, frozen=True)
    assert e.value.status == -1
    h.backward(None, grads, frozen=True)         # all-ones weights
    G = [g.cpu().numpy() for g in grads]
    res = o.tnrsvd(W.cores, W.k, W.p, 0, seed=4)
    assert rel(G, o.sigma_sum_grad(W.cores, res)) <= 1e-8
    h.close()


def test_spectrum_frozen_gradient_matches_pipeline_finite_differences():
    """On the known spectrum (sigma_j = 10^(-j/4), K = 30 > k = 20) the computed
    subspace captures A v_j up to ~sigma_30 / sigma_j, so the derivative at fixed
    singular vectors is the derivative of the FP64 pipeline to ~1e-6."""
    W = wl.spectrum()
    om = omega_for(W.cores, W.K, W.omega_seed)
    eps = W.eps_by_precision["f64"]
    sig, h = gpu_solve(W.cores, W.k, W.p, W.q, eps=eps, rmax=W.rmax, omega=om)
    G = gpu_grad(h, W.cores)
    h.close()
    rng = np.random.default_rng(3)
    step = 1e-5
    for i in (0, 7, len(W.cores) - 1):
        D = rng.standard_normal(W.cores[i].shape)
        D /= np.linalg.norm(D)
        Ap = [c.copy() for c in W.cores]
        Ap[i] = Ap[i] + step * D
        Am = [c.copy() for c in W.cores]
        Am[i] = Am[i] - step * D
        sp, hp = gpu_solve(Ap, W.k, W.p, W.q, eps=eps, rmax=W.rmax, omega=om)
        sm, hm = gpu_solve(Am, W.k, W.p, W.q, eps=eps, rmax=W.rmax, omega=om)
        hp.close()
        hm.close()
        fd = (sp.sum() - sm.sum()) / (2 * step)
        got = float(np.sum(G[i] * D))
        print(f"spectrum core {i}: gradient {got:.9e}, pipeline FD {fd:.9e}")
        assert abs(got - fd) <= 1e-5 * (abs(fd) + np.linalg.norm(G[i]))
