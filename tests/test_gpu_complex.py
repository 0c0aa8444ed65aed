"""GPU parity of the complex-MPO path: the real embedding (tnrsvd_complex_embed)
equals the oracle's bit for bit, and the solve of the real form (k' = 2k,
p' = 2p, every other value) matches the oracle's tnrsvd_complex with the same
seed and LAPACK's complex SVD of the dense matrix."""

import numpy as np
import pytest

from oracle import tnrsvd_oracle as o
from test_oracle_complex import complex_mpo, dense_complex

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1707_07803_amd import load_library
    load_library()
    yield


def dev(cores, dtype):
    import torch
    return [torch.as_tensor(c, dtype=dtype).cuda() for c in cores]


@pytest.mark.parametrize("shapes", [
    [(1, 2, 3, 3), (3, 3, 2, 4), (4, 2, 2, 1)],
    [(1, 3, 4, 1)],
    [(1, 4, 4, 3), (3, 4, 4, 1)],
])
def test_embedding_equals_the_oracle(shapes):
    import torch
    from paper_1707_07803_amd import complex_embed
    C = complex_mpo(shapes, 7)
    ref = o.complex_to_real_mpo(C)
    got = [t.cpu().numpy() for t in complex_embed(dev(C, torch.complex128))]
    assert [g.shape for g in got] == [r.shape for r in ref]
    for g, r in zip(got, ref):
        np.testing.assert_array_equal(g, r)
    C32 = [c.astype(np.complex64) for c in C]
    ref32 = o.complex_to_real_mpo(C32)
    got32 = [t.cpu().numpy() for t in complex_embed(dev(C32, torch.complex64))]
    for g, r in zip(got32, ref32):
        np.testing.assert_array_equal(g, r.astype(np.float32))


def test_solve_when_K_spans_the_space():
    import torch
    from paper_1707_07803_amd import solve_complex
    C = complex_mpo([(1, 4, 4, 3), (3, 4, 4, 1)], 3)
    ref = np.linalg.svd(dense_complex(C), compute_uv=False)[:4]
    s = solve_complex(dev(C, torch.complex128), 4, 12, 0, seed=4)
    np.testing.assert_allclose(s, ref, rtol=1e-11)


@pytest.mark.parametrize("precision,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_solve_against_oracle_and_lapack(precision, tol):
    import torch
    from paper_1707_07803_amd import solve_complex
    rng = np.random.default_rng(5)
    r = [1, 3, 3, 3, 3, 3, 1]
    C = [rng.standard_normal((r[k], 2, 2, r[k + 1])) + 1j * rng.standard_normal((r[k], 2, 2, r[k + 1]))
         for k in range(6)]
    ct = torch.complex128 if precision == "f64" else torch.complex64
    s = solve_complex(dev(C, ct), 3, 7, 4, seed=6, precision=precision)
    so = o.tnrsvd_complex(C, 3, 7, 4, seed=6)
    lap = np.linalg.svd(dense_complex(C), compute_uv=False)[:3]
    print(precision, "vs oracle", np.max(np.abs(s - so) / so), "vs lapack", np.max(np.abs(s - lap) / lap))
    np.testing.assert_allclose(s, so, rtol=tol)
    np.testing.assert_allclose(s, lap, rtol=1e-6 + tol)


def test_rejects_real_cores():
    import torch
    from paper_1707_07803_amd import TNrSVDError, complex_embed
    with pytest.raises(TNrSVDError):
        complex_embed([torch.zeros((1, 2, 2, 1), dtype=torch.float64, device="cuda")])
