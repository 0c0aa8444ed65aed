"""The no-allocation sparse-to-MPO entry point (tnrsvd_sparse_to_mpo_noalloc)
against the allocating one (tnrsvd_sparse_to_mpo), both through the C ABI.

The two share every kernel; only the scratch differs (the library's static
device array instead of a hipMalloc'd buffer), so on inputs without duplicate
entries (no atomic sums in a free order) their cores must be bit-identical.
Two calls run back to back, the second with a smaller input, so leftovers of
the first call in the shared array would show.  Around the no-allocation calls
the device's free memory must not change.
"""

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1707_07803_amd import load_library
    load_library()
    yield


def random_coo(rows, cols, nnz, seed):
    M, N = int(np.prod(rows)), int(np.prod(cols))
    rng = np.random.default_rng(seed)
    pos = np.unique(rng.integers(0, M * N, size=nnz))    # no duplicate positions
    r, c = pos // N, pos % N
    v = rng.standard_normal(len(pos))
    v[v == 0.0] = 1.0
    return r, c, v


def abi_convert(fn, rows, cols, r, c, v):
    """Both calls of `fn` (count, then fill) on preallocated cores; returns the
    cores and the device's free memory before and after the two calls."""
    import torch
    dev = torch.device("cuda:0")
    R = torch.as_tensor(np.ascontiguousarray(r, dtype=np.int64), device=dev)
    C = torch.as_tensor(np.ascontiguousarray(c, dtype=np.int64), device=dev)
    V = torch.as_tensor(np.ascontiguousarray(v, dtype=np.float64), device=dev)
    d = len(rows)
    rr = (ctypes.c_int64 * d)(*rows)
    cc = (ctypes.c_int64 * d)(*cols)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    args = (ctypes.c_void_p(R.data_ptr()), ctypes.c_void_p(C.data_ptr()),
            ctypes.c_void_p(V.data_ptr()))
    # the rank is known beforehand (the number of nonzero blocks), so the cores
    # can be allocated before the measured calls
    nb_expect = len(np.unique((r // rows[0]) * (np.prod(cols) // cols[0]) + c // cols[0]))
    shapes = [(1 if k == 0 else nb_expect, rows[k], cols[k], 1 if k == d - 1 else nb_expect)
              for k in range(d)]
    cores = [torch.full(s, np.nan, dtype=torch.float64, device=dev) for s in shapes]
    ptrs = (ctypes.c_void_p * d)(*[t.data_ptr() for t in cores])
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(dev)[0]
    nb = ctypes.c_int64(0)
    st1 = fn(d, rr, cc, len(v), *args, ctypes.byref(nb), None, stream)
    n_count = nb.value
    st2 = fn(d, rr, cc, len(v), *args, ctypes.byref(nb), ptrs, stream)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info(dev)[0]
    return (st1, st2, n_count, nb_expect), [t.cpu().numpy() for t in cores], free0, free1


def test_noalloc_equals_allocating_entry():
    from paper_1707_07803_amd.tnrsvd import load_library
    L = load_library()
    cases = [
        ([64, 2, 2, 2, 2, 2, 2], [64, 2, 2, 2, 2, 2, 2], 6000, 11),   # 4096 x 4096, bitmap path
        ([16, 2, 2, 2, 2], [16, 2, 2, 2, 2], 500, 12),                 # 256 x 256, smaller
        ([2] * 16, [2] * 16, 300, 13),                                 # 2^30 positions: sort path
        ([5, 3, 2], [4, 3, 3], 60, 14),                                # mixed radix, smallest
    ]
    for rows, cols, nnz, seed in cases:
        print(f"no-alloc case rows={rows} cols={cols} nnz={nnz} seed={seed}", flush=True)
        r, c, v = random_coo(rows, cols, nnz, seed)
        sa, ref, _, _ = abi_convert(L.tnrsvd_sparse_to_mpo, rows, cols, r, c, v)
        sn, got, f0, f1 = abi_convert(L.tnrsvd_sparse_to_mpo_noalloc, rows, cols, r, c, v)
        assert sa == (0, 0, sa[3], sa[3]), sa
        assert sn == sa, (sn, sa)
        assert len(got) == len(ref)
        for g, x in zip(got, ref):
            assert g.shape == x.shape
            np.testing.assert_array_equal(g, x)
        assert f1 == f0, f"free device memory changed by {f0 - f1} bytes"


def test_noalloc_rejects_inputs_beyond_its_scratch():
    import torch
    from paper_1707_07803_amd.tnrsvd import load_library
    L = load_library()
    dev = torch.device("cuda:0")
    # 2^28 block positions: the bitmap path needs about 100 MB of scratch
    rows = cols = [2] * 15
    R = torch.zeros(1, dtype=torch.int64, device=dev)
    V = torch.ones(1, dtype=torch.float64, device=dev)
    d = len(rows)
    rr = (ctypes.c_int64 * d)(*rows)
    cc = (ctypes.c_int64 * d)(*cols)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    nb = ctypes.c_int64(0)
    st = L.tnrsvd_sparse_to_mpo_noalloc(d, rr, cc, 1, ctypes.c_void_p(R.data_ptr()),
                                        ctypes.c_void_p(R.data_ptr()),
                                        ctypes.c_void_p(V.data_ptr()), ctypes.byref(nb), None,
                                        stream)
    assert st == -2
    assert b"scratch" in L.tnrsvd_last_error()
    # the allocating entry point takes the same input
    st = L.tnrsvd_sparse_to_mpo(d, rr, cc, 1, ctypes.c_void_p(R.data_ptr()),
                                ctypes.c_void_p(R.data_ptr()), ctypes.c_void_p(V.data_ptr()),
                                ctypes.byref(nb), None, stream)
    assert st == 0 and nb.value == 1
    # more cores than the no-allocation call takes
    d = 65
    rr = (ctypes.c_int64 * d)(*([1] * d))
    st = L.tnrsvd_sparse_to_mpo_noalloc(d, rr, rr, 1, ctypes.c_void_p(R.data_ptr()),
                                        ctypes.c_void_p(R.data_ptr()),
                                        ctypes.c_void_p(V.data_ptr()), ctypes.byref(nb), None,
                                        stream)
    assert st == -2
