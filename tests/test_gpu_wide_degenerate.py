"""Rank-deficient products on the multi-workgroup path and on the left-to-right
Jacobi that keeps no rotations: an MPO of true rank 3 stored with bond ranks 32
(the extra rank slots zero), so every product is wider than the one-workgroup
register path while almost all of its singular values are rounding noise.

The top three singular values have a closed form: A = sum_t c_t a_t b_t^T with
a_t, b_t Kronecker products of per-core vectors, so sigma(A) are the singular
values of Ga^(1/2) diag(c) Gb^(1/2), where Ga[s, t] = a_s . a_t is a product of
per-core inner products (likewise Gb)."""

import numpy as np
import pytest

from tests.gpu_helpers import to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1707_07803_amd import load_library
    load_library()
    yield


def padded_rank3(d, n, R, seed):
    rng = np.random.default_rng(seed)
    T = 3
    u = rng.standard_normal((T, d, n))
    v = rng.standard_normal((T, d, n))
    c = np.array([3.0, 1.0, 0.25])
    cores = []
    for i in range(d):
        rl = 1 if i == 0 else R
        rr = 1 if i == d - 1 else R
        G = np.zeros((rl, n, n, rr))
        for t in range(T):
            a = 0 if i == 0 else t
            b = 0 if i == d - 1 else t
            G[a, :, :, b] = np.outer(u[t, i], v[t, i]) * (c[t] if i == 0 else 1.0)
        cores.append(G)
    Ga = np.prod(np.einsum("sin,tin->sti", u, u), axis=2)
    Gb = np.prod(np.einsum("sin,tin->sti", v, v), axis=2)

    def sqrtm(S):
        w, Q = np.linalg.eigh(S)
        return (Q * np.sqrt(np.maximum(w, 0.0))) @ Q.T

    sig = np.linalg.svd(sqrtm(Ga) @ np.diag(c) @ sqrtm(Gb), compute_uv=False)
    return cores, sig


@pytest.mark.parametrize("precision,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_rank3_padded_to_32_on_the_wide_path(precision, tol):
    from paper_1707_07803_amd import TNrSVD
    cores, exact = padded_rank3(7, 4, 32, 11)
    h = TNrSVD(to_device(cores, precision), 16, 16, 1, seed=3, precision=precision, max_rank=32)
    sig = h.run()[0]
    P, _ = h.product_ranks()
    h.close()
    print(f"{precision}: top 3 {sig[:3]}, exact {exact}, largest product rank {max(P)}, "
          f"sigma_3 / sigma_0 {sig[3] / sig[0]:.2e}")
    assert max(P) > 128                               # the multi-workgroup path
    assert np.max(np.abs(sig[:3] - exact) / exact) <= tol
    assert sig[3] <= 1e-6 * sig[0] if precision == "f32" else sig[3] <= 1e-12 * sig[0]
    assert np.all(np.isfinite(sig)) and np.all(np.diff(sig) <= 1e-12 * sig[0])
