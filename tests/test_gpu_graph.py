"""Captured-graph solves (tnrsvd_run_graph) against eager solves (tnrsvd_run),
and the contraction autotuner (tnrsvd_autotune).

Every replay is checked against the eager result, with eager solves and
stream synchronisations between the replays; the kernels are deterministic,
so the comparison is exact.
"""

import numpy as np
import pytest

import workloads as wl
from tests.gpu_helpers import omega_for, cores_np, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1707_07803_amd import load_library
    load_library()
    yield


def test_graph_replays_equal_eager_spectrum_f32():
    import torch
    from paper_1707_07803_amd import TNrSVD, omega_flat
    W = wl.spectrum()
    h = TNrSVD(to_device(W.cores, "f32"), W.k, W.p, W.q, precision="f32",
               round_tol=W.eps_by_precision["f32"], max_rank=W.rmax)
    h.set_omega(omega_flat(*omega_for(W.cores, W.K, W.omega_seed)))
    ref = h.run()[0]
    qref = cores_np(h.factor(2))
    for rep in range(4):
        sig = h.run_graph()[0]
        np.testing.assert_array_equal(sig, ref, err_msg=f"replay {rep}")
        for a, b in zip(cores_np(h.factor(2)), qref):
            np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(h.run()[0], ref)     # eager work between replays
        torch.cuda.synchronize()
    # a new Omega written between replays is read by the graph
    h.set_omega(omega_flat(*omega_for(W.cores, W.K, 77)))
    sig2 = h.run_graph()[0]
    np.testing.assert_array_equal(sig2, h.run()[0])
    assert not np.array_equal(sig2, ref)
    h.close()


def test_graph_replays_equal_eager_uneven_batch_f64():
    import torch
    from paper_1707_07803_amd import TNrSVD
    rng = np.random.default_rng(21)
    mpos = []
    for d, n, r in [(6, 2, 3), (9, 2, 4), (5, 4, 2), (7, 2, 5)]:
        ranks = [1] + [r] * (d - 1) + [1]
        mpos.append([rng.standard_normal((ranks[i], n, n, ranks[i + 1])) for i in range(d)])
    h = TNrSVD([to_device(c) for c in mpos], 6, 4, 1, seed=3, max_rank=16)
    ref = h.run()
    for rep in range(3):
        np.testing.assert_array_equal(h.run_graph(), ref, err_msg=f"replay {rep}")
        torch.cuda.synchronize()
        np.testing.assert_array_equal(h.run(), ref)
    h.close()


def test_graph_refuses_profiling():
    from paper_1707_07803_amd import TNrSVD, TNrSVDError
    W = wl.small()
    h = TNrSVD(to_device(W.cores), W.k, W.p, 0, seed=1)
    h.profile(True)
    with pytest.raises(TNrSVDError) as e:
        h.run_graph()
    assert e.value.status == -3
    h.profile(False)
    ref = h.run()[0]
    np.testing.assert_array_equal(h.run_graph()[0], ref)
    h.close()


def test_autotune_keeps_results_and_recaptures_the_graph():
    from paper_1707_07803_amd import TNrSVD, TNrSVDError, omega_flat
    W = wl.spectrum()
    h = TNrSVD(to_device(W.cores, "f32"), W.k, W.p, W.q, precision="f32",
               round_tol=W.eps_by_precision["f32"], max_rank=W.rmax)
    h.set_omega(omega_flat(*omega_for(W.cores, W.K, W.omega_seed)))
    ref = h.run()[0]
    np.testing.assert_array_equal(h.run_graph()[0], ref)
    choice = h.autotune(3)
    for op in ("A_X", "At_X"):
        assert choice[op]["threads"] in (64, 128, 256, 512)
        assert choice[op]["blocks_per_core_cap"] in (64, 256, 1024, 4096)
    with pytest.raises(TNrSVDError) as e:     # results were invalidated
        h.solve()
    assert e.value.status == -3
    # every launch shape computes each output with the same arithmetic
    np.testing.assert_array_equal(h.run()[0], ref)
    np.testing.assert_array_equal(h.run_graph()[0], ref)
    h.close()


def test_graph_on_bf16_handle_then_refine():
    from paper_1707_07803_amd import TNrSVD, omega_flat
    W = wl.spectrum()
    h = TNrSVD(to_device(W.cores, "f32"), W.k, W.p, W.q, precision="bf16",
               round_tol=W.eps_by_precision["bf16"], max_rank=W.rmax)
    h.set_omega(omega_flat(*omega_for(W.cores, W.K, W.omega_seed)))
    ref = h.run()[0]
    ref_refined = h.refine(W.eps_by_precision["f32"])[0]
    # the graph restores BF16 after a refinement and replays the BF16 solve
    for _ in range(2):
        np.testing.assert_array_equal(h.run_graph()[0], ref)
        np.testing.assert_array_equal(h.refine(W.eps_by_precision["f32"])[0], ref_refined)
    h.close()
