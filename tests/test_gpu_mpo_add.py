"""GPU parity of MPO addition (tnrsvd_mpo_add, Sec. 3: ranks add) against the
oracle's mpo_add, whose pin densifies the sum against the sum of the dense
matrices.  The sum's cores are copies of the inputs' entries (and, for
d = 1, one addition), so the comparison is bit for bit."""

import numpy as np
import pytest

from oracle import tnrsvd_oracle as o
from tests.gpu_helpers import to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1707_07803_amd import load_library
    load_library()
    yield


def rand_mpo(I, J, R, seed):
    rng = np.random.default_rng(seed)
    r = [1] + list(R) + [1]
    return [rng.standard_normal((r[k], I[k], J[k], r[k + 1])) for k in range(len(I))]


CASES = {
    "d4_mixed": ([3, 1, 4, 2], [2, 5, 1, 3], [4, 6, 2], [1, 3, 5]),
    "d2_rank1": ([2, 3], [3, 2], [1], [1]),
    "d6_wide": ([2] * 6, [2] * 6, [8, 16, 32, 16, 8], [3, 3, 3, 3, 3]),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sum_cores_equal_the_oracle(case, dtype):
    from paper_1707_07803_amd import mpo_add
    I, J, Ra, Rb = CASES[case]
    A = rand_mpo(I, J, Ra, 1)
    B = rand_mpo(I, J, Rb, 2)
    if dtype == "f32":
        A = [a.astype(np.float32).astype(np.float64) for a in A]
        B = [b.astype(np.float32).astype(np.float64) for b in B]
    C = [c.double().cpu().numpy() for c in mpo_add(to_device(A, dtype), to_device(B, dtype))]
    ref = o.mpo_add(A, B)
    assert [c.shape for c in C] == [c.shape for c in ref]
    for c, r in zip(C, ref):
        np.testing.assert_array_equal(c, r)


def test_single_core_is_the_elementwise_sum():
    from paper_1707_07803_amd import mpo_add
    A = rand_mpo([7], [5], [], 3)
    B = rand_mpo([7], [5], [], 4)
    C = mpo_add(to_device(A), to_device(B))[0].cpu().numpy()
    np.testing.assert_array_equal(C, A[0] + B[0])


def test_rounding_the_sum_of_a_matrix_with_itself():
    """A + A is 2A: rounding it keeps A's rounded ranks (the doubled ranks are
    exactly rank deficient) and represents 2A within the rounding bound."""
    from paper_1707_07803_amd import mpo_add, round_mpo
    I, J, R = [2] * 5, [3] * 5, [4, 5, 5, 4]
    A = rand_mpo(I, J, R, 5)
    dA = to_device(A)
    S = mpo_add(dA, dA)
    assert [int(c.shape[3]) for c in S[:-1]] == [2 * r for r in R]
    Rd = [c.cpu().numpy() for c in round_mpo(S, 1e-12)]
    assert [c.shape[3] for c in Rd[:-1]] == [c.shape[3] for c in o.round_mpo(A, 1e-12)[:-1]]
    D = o.mpo_to_dense(A)
    assert np.linalg.norm(o.mpo_to_dense(Rd) - 2 * D) <= 1e-11 * np.linalg.norm(2 * D)


def test_errors():
    import torch
    from paper_1707_07803_amd import TNrSVDError, mpo_add
    A = to_device(rand_mpo([2, 2], [2, 2], [3], 6))
    with pytest.raises(TNrSVDError) as ei:
        mpo_add(A, to_device(rand_mpo([2, 3], [2, 2], [3], 7)))        # modes differ
    assert ei.value.status == -2
    with pytest.raises(TNrSVDError) as ei:
        mpo_add(A, [c.float() for c in A])                             # dtypes differ
    assert ei.value.status == -1
    with pytest.raises(TNrSVDError) as ei:
        mpo_add(A, A[:1])
    assert ei.value.status == -2
    bad = [torch.zeros((2, 2, 2, 3), dtype=torch.float64, device="cuda"), A[1]]
    with pytest.raises(TNrSVDError) as ei:                             # rank[0] != 1
        mpo_add(A, bad)
    assert ei.value.status == -2
