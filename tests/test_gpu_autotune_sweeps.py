"""The sweep autotuner (tnrsvd_autotune_sweeps / tnrsvd_set_sweep_config):
every launch choice computes the same factorisations, so sigma agrees across
choices to the rounding of the FP64 sweeps; a choice kept in the cache is
applied without timing; graphs are recaptured under the new choice."""

import numpy as np
import pytest

import workloads as wl
from tests.gpu_helpers import to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1707_07803_amd import load_library
    load_library()
    yield


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def test_large_every_choice_agrees():
    """d = 50, ranks 10, q = 2, FP64: product panels of 640 x 320 take the
    multi-workgroup path at wmin 129 and 257 and the one-workgroup blocked
    path at 513 and 0."""
    from paper_1707_07803_amd import TNrSVD
    W = wl.large()
    h = TNrSVD(to_device(W.cores), W.k, W.p, W.q, seed=W.omega_seed, max_rank=W.rmax)
    ref = h.run()[0]
    for choice in ([257, 1], [513, 1], [0, 1], [129, 1]):
        h.set_sweep_config(choice)
        sig = h.run()[0]
        print(f"large, choice {choice}: sigma rel diff {rel(sig, ref):.3e}")
        assert rel(sig, ref) <= 1e-10
    h.close()


def test_autotune_batch_and_cache(tmp_path):
    from paper_1707_07803_amd import TNrSVD, TNrSVDError
    # the ten cheapest of the first 64 members of the uneven draw (d n^2 R^3)
    Ws = sorted(wl.batched(64), key=lambda w: len(w.cores) * w.cores[1].shape[1] ** 2
                * w.cores[1].shape[0] ** 3)[:10]
    mpos = [to_device(w.cores) for w in Ws]
    print(f"batch of {len(Ws)}: R = {[w.cores[1].shape[0] for w in Ws]}", flush=True)
    h = TNrSVD(mpos, 8, 8, 1, seed=9, max_rank=32)
    ref = h.run()
    path = str(tmp_path / "sweeps.json")
    got = h.autotune_sweeps(reps=1, cache=path)
    print(f"autotuned: {got}", flush=True)
    assert not got["cached"] and got["lpt"] in (0, 1)
    assert got["wmin"] in (0, 129, 257, 513)
    sig = h.run()
    assert max(rel(a, b) for a, b in zip(sig, ref)) <= 1e-10
    again = h.autotune_sweeps(reps=1, cache=path)
    assert again["cached"] and (again["wmin"], again["lpt"]) == (got["wmin"], got["lpt"])
    # the graph is recaptured under the applied choice and replays bit for bit
    h.set_sweep_config([0, 0])
    eager = h.run()
    g1 = h.run_graph()
    g2 = h.run_graph()
    for a, b, c in zip(eager, g1, g2):
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(a, c)
    for bad in ([64, 1], [-1, 1], [129, 2]):
        with pytest.raises(TNrSVDError) as e:
            h.set_sweep_config(bad)
        assert e.value.status == -1
    h.close()
