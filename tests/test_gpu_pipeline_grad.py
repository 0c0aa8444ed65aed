"""The pipeline's derivative on the GPU (tnrsvd_backward, TNrSVD.backward,
TNrSVDFunction) against the oracle's pipeline_grad and against central finite
differences of the GPU pipeline itself.

Both sides differentiate sum_j dsigma_j sigma_j of the whole solve (Y = A Omega,
the roundings, Algorithm 5.4's products, the last-core SVD) with Omega and every
rounding's bond ranks held at their forward values.  The GPU recomputes the
forward in FP64 from the (widened) input cores, so FP64 solves must agree with
the oracle to 1e-8 relative (norm-wise over all cores) and FP32 ones to 1e-4,
the FP32 inputs being the same numbers on both sides.
"""

import numpy as np
import pytest

from oracle import tnrsvd_oracle as o
import workloads as wl
from tests.gpu_helpers import omega_for, gpu_solve, to_device, merged_cols

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1707_07803_amd import load_library
    load_library()
    yield


def gpu_grad(h, cores, dsigma=None, dtype="f64"):
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    grads = [torch.empty(c.shape, dtype=td, device="cuda") for c in cores]
    h.backward(dsigma, grads)
    return [g.double().cpu().numpy() for g in grads]


def rel(gs, rs):
    a = np.concatenate([g.ravel() for g in gs])
    b = np.concatenate([r.ravel() for r in rs])
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("q", [0, 1, 2])
def test_small_f64_against_oracle(q):
    """d = 8, 2 x 2 cores, ranks 3, k = 10, p = 6 (the last 4 cores merged)."""
    W = wl.small()
    om = omega_for(W.cores, W.K, W.omega_seed)
    ref = o.tnrsvd(W.cores, W.k, W.p, q, omega=om)
    w = np.random.default_rng(2).standard_normal(W.k)
    G_ref = o.pipeline_grad(W.cores, W.k, W.p, q, omega=om, dsigma=w, ranks=ref.ranks)
    _, h = gpu_solve(W.cores, W.k, W.p, q, omega=om)
    err = rel(gpu_grad(h, W.cores, w), G_ref)
    print(f"small q={q} f64 pipeline gradient: rel err {err:.3e}")
    assert err <= 1e-8
    h.close()


def rank_r_mpo(d, n, r, seed):
    rng = np.random.default_rng(seed)
    A = None
    for _ in range(r):
        term = [np.outer(rng.standard_normal(n), rng.standard_normal(n)).reshape(1, n, n, 1)
                for _ in range(d)]
        A = term if A is None else o.mpo_add(A, term)
    return A


@pytest.mark.parametrize("q", [0, 1])
def test_exact_case_equals_closed_form(q):
    """rank(A) = K = 8: the computed subspace is range(A), so the pipeline's
    derivative is sum_j dsigma_j u_j v_j^T (the oracle's sigma_sum_grad, pinned
    to LAPACK's singular vectors).  With rank(A) < K the sketch Y = A Omega is
    rank deficient and the QR and eigen adjoints divide by its zero singular
    values, so that case is not differentiated here."""
    A = rank_r_mpo(6, 2, 8, 5)
    k, p = 3, 5
    om = omega_for(A, k + p, 21)
    w = np.array([1.0, 0.5, -2.0])
    ref = o.tnrsvd(A, k, p, q, omega=om)
    G_ref = o.sigma_sum_grad(A, ref, w)
    _, h = gpu_solve(A, k, p, q, omega=om)
    err = rel(gpu_grad(h, A, w), G_ref)
    print(f"exact case q={q}: pipeline gradient vs closed form rel err {err:.3e}")
    assert err <= 1e-8
    h.close()


def test_truncating_spectrum_f64_against_oracle():
    """Known spectrum with the FP64 rounding tolerance: the product roundings
    truncate (ranks 25 -> 5), so the frozen ranks matter."""
    W = wl.spectrum()
    om = omega_for(W.cores, W.K, W.omega_seed)
    eps = W.eps_by_precision["f64"]
    ref = o.tnrsvd(W.cores, W.k, W.p, W.q, omega=om, eps=eps, rmax=W.rmax)
    w = np.linspace(1.0, 2.0, W.k)
    G_ref = o.pipeline_grad(W.cores, W.k, W.p, W.q, omega=om, eps=eps, rmax=W.rmax, dsigma=w,
                            ranks=ref.ranks)
    _, h = gpu_solve(W.cores, W.k, W.p, W.q, eps=eps, rmax=W.rmax, omega=om)
    err = rel(gpu_grad(h, W.cores, w), G_ref)
    print(f"spectrum f64 pipeline gradient: rel err {err:.3e}")
    assert err <= 1e-8
    h.close()


def test_spectrum_f64_finite_differences():
    """Central differences of the FP64 GPU pipeline on three cores (step 1e-6
    on unit directions).  The step stays below the smallest kept singular
    values' scale (sigma_19 ~ 2e-5), where the h^2 term of the difference on
    the last core is ~2e-7; perturbing the first cores can lift a rounding's
    eps-rank by a direction of size ~h, which moves the sum by far less."""
    W = wl.spectrum()
    om = omega_for(W.cores, W.K, W.omega_seed)
    eps = W.eps_by_precision["f64"]
    _, h = gpu_solve(W.cores, W.k, W.p, W.q, eps=eps, rmax=W.rmax, omega=om)
    G = gpu_grad(h, W.cores)
    h.close()
    rng = np.random.default_rng(3)
    step = 1e-6
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
        assert abs(got - fd) <= 1e-6 * (abs(fd) + np.linalg.norm(G[i]))


def _grad_workload_f32():
    W = wl.grad()
    om = omega_for(W.cores, W.K, W.omega_seed)
    sig, h = gpu_solve(W.cores, W.k, W.p, W.q, precision="f32", eps=W.eps, rmax=W.rmax,
                       omega=om)
    G = gpu_grad(h, W.cores, dtype="f32")
    h.close()
    return W, om, sig, G


def test_grad_workload_f32_against_oracle():
    """d = 30, 4 x 4 cores, ranks 16, k = 16, p = 8, q = 1 (the last 3 cores
    merged); the FP32 inputs are exact FP64 numbers, so both sides
    differentiate the same pipeline on the same A."""
    import torch
    W, om, sig, G = _grad_workload_f32()
    A32 = [np.asarray(torch.as_tensor(c, dtype=torch.float32).double().numpy()) for c in W.cores]
    ref = o.tnrsvd(A32, W.k, W.p, W.q, omega=om, eps=W.eps, rmax=W.rmax)
    G_ref = o.pipeline_grad(A32, W.k, W.p, W.q, omega=om, eps=W.eps, rmax=W.rmax,
                            ranks=ref.ranks)
    err = rel(G, G_ref)
    print(f"grad workload f32: sigma rel err "
          f"{np.linalg.norm(sig - ref.sigma) / np.linalg.norm(ref.sigma):.3e}, pipeline "
          f"gradient rel err {err:.3e}")
    assert err <= 1e-4


def test_grad_workload_f32_finite_differences():
    """Central differences of the FP32 GPU pipeline (step h = 1e-3) along 8
    seeded directions E, N(0, 1) entries scaled to unit norm on every core and
    all cores moved at once: the directional derivative sum_i <dL/dA_i, D_i>
    must match (L(A+) - L(A-)) / 2h to 1e-2 relative.  A+ and A- are A +- hE
    rounded to FP32 and D = (A+ - A-) / 2h, so input rounding does not enter;
    FP32 rounding inside the solves moves L by ~1e2 against differences of
    1e5 - 1e6, and the h^2 term is ~1e-5 of the derivative at this step (each
    core moves by 6e-5 of its norm)."""
    W, om, _, G = _grad_workload_f32()
    rng = np.random.default_rng(12)
    h = 1e-3
    worst = 0.0
    for t in range(8):
        E = [rng.standard_normal(c.shape) for c in W.cores]
        E = [e / np.linalg.norm(e) for e in E]
        Ap = [(c + h * e).astype(np.float32).astype(np.float64) for c, e in zip(W.cores, E)]
        Am = [(c - h * e).astype(np.float32).astype(np.float64) for c, e in zip(W.cores, E)]
        sp, hp = gpu_solve(Ap, W.k, W.p, W.q, precision="f32", eps=W.eps, rmax=W.rmax, omega=om)
        sm, hm = gpu_solve(Am, W.k, W.p, W.q, precision="f32", eps=W.eps, rmax=W.rmax, omega=om)
        hp.close()
        hm.close()
        fd = (sp.sum() - sm.sum()) / (2 * h)
        got = float(sum(np.sum(g * (p - m)) for g, p, m in zip(G, Ap, Am))) / (2 * h)
        r = abs(got - fd) / abs(fd)
        worst = max(worst, r)
        print(f"  direction {t}: gradient {got:.6e}, pipeline FD {fd:.6e}, rel {r:.2e}")
        assert r <= 1e-2, (t, got, fd)
    print(f"grad workload f32 FD: worst rel {worst:.2e}")


def test_autograd_pipeline_spectrum_f32():
    import torch
    from paper_1707_07803_amd import TNrSVDFunction
    W = wl.spectrum()
    eps = W.eps_by_precision["f32"]
    A32 = [torch.as_tensor(c, dtype=torch.float32) for c in W.cores]
    A64 = [a.double().numpy() for a in A32]
    om = o.omega_from_seed(merged_cols(A64, W.K), W.K, W.omega_seed)
    ref = o.tnrsvd(A64, W.k, W.p, W.q, omega=om, eps=eps, rmax=W.rmax)
    wts = np.linspace(1.0, 2.0, W.k)
    G_ref = o.pipeline_grad(A64, W.k, W.p, W.q, omega=om, eps=eps, rmax=W.rmax, dsigma=wts,
                            ranks=ref.ranks)
    cores = [a.cuda().requires_grad_() for a in A32]
    opts = dict(k=W.k, p=W.p, q=W.q, seed=W.omega_seed, precision="f32", round_tol=eps,
                max_rank=W.rmax)
    sig = TNrSVDFunction.apply(opts, *cores)
    loss = (sig * torch.as_tensor(wts, device="cuda")).sum()
    loss.backward(retain_graph=True)
    G = [c.grad.double().cpu().numpy() for c in cores]
    assert all(c.grad.dtype == torch.float32 for c in cores)
    err = rel(G, G_ref)
    print(f"spectrum f32 autograd pipeline gradient: rel err {err:.3e}")
    assert err <= 1e-4
    # the handle is released by the first backward: a second one is refused
    with pytest.raises(RuntimeError):
        loss.backward()


def test_backward_after_refine_is_refused():
    import torch
    from paper_1707_07803_amd import TNrSVD, TNrSVDError
    W = wl.small()
    h = TNrSVD(to_device(W.cores), W.k, W.p, 0, seed=4)
    grads = [torch.empty(c.shape, dtype=torch.float64, device="cuda") for c in W.cores]
    h.run()
    h.backward(None, grads)                      # seeded Omega, all-ones weights
    G = [g.cpu().numpy() for g in grads]
    om = o.omega_from_seed(merged_cols(W.cores, W.K), W.K, 4)
    res = o.tnrsvd(W.cores, W.k, W.p, 0, omega=om)
    assert rel(G, o.pipeline_grad(W.cores, W.k, W.p, 0, omega=om, ranks=res.ranks)) <= 1e-8
    h.close()
    # a refined BF16 solve is no longer Algorithm 5.4's sequence
    hb = TNrSVD(to_device(W.cores, "f32"), W.k, W.p, 0, seed=4, precision="bf16")
    g32 = [torch.empty(c.shape, dtype=torch.float32, device="cuda") for c in W.cores]
    hb.run()
    hb.refine()
    with pytest.raises(TNrSVDError) as e:
        hb.backward(None, g32)
    assert e.value.status == -3
    hb.backward(None, g32, frozen=True)          # the frozen form still applies
    hb.close()
