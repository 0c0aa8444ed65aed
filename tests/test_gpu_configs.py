"""GPU parity on the large and batched-uneven workloads at their full sizes.

* large: d = 50, 2 x 2 cores, ranks 10, k = 10, p = 10, q = 2, rank cap 32;
  product ranks reach 320, so these solves go through the blocked
  (GEMM-based) Householder path.  Whole sigma against the FP64 oracle.
* batched uneven: MPOs of the 512-member draw (d in [10, 40], I = J in {2, 4},
  ranks in [4, 32]; k = 8, p = 8, q = 1, FP32) solved together in one
  persistent launch; the oracle recomputes sampled members one by one (the
  cheapest of the draw, so the CPU side stays within seconds).
* the three costliest members of the draw (R = 32, 32, 29 with 4 x 4 cores,
  product ranks up to 1024, right-to-left panels up to 4096 x 1024, so the
  multi-workgroup path; one with d = 40) interleaved with three cheap ones in
  one handle, FP32 and FP64, against oracle singular values stored by
  tests/golden/make_batched_members.py; and the same batch replayed as a
  captured graph, bit-equal to the eager solve.
"""

import json
import os

import numpy as np
import pytest

from oracle import tnrsvd_oracle as o
import workloads as wl
from tests.gpu_helpers import omega_for, gpu_solve, rel_err, to_device

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5}
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batched_members.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1707_07803_amd import load_library
    load_library()
    yield


@pytest.fixture(scope="module")
def large_ref():
    W = wl.large()
    om = omega_for(W.cores, W.K, W.omega_seed)
    return W, om, o.tnrsvd(W.cores, W.k, W.p, W.q, omega=om, eps=W.eps, rmax=W.rmax)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_large_full_size(large_ref, precision):
    W, om, ref = large_ref
    sig, h = gpu_solve(W.cores, W.k, W.p, W.q, precision=precision, eps=W.eps, rmax=W.rmax,
                       omega=om)
    err = rel_err(sig, ref.sigma)
    print(f"large {precision}: sigma rel err {err:.3e}, ranks {h.ranks()}")
    assert err <= TOL[precision]
    assert h.ranks() == [1] + ref.ranks[-2][1:] + [W.K]
    h.close()


def test_batched_uneven_sampled_members():
    from paper_1707_07803_amd import TNrSVD
    Ws = wl.batched(512)
    cost = [len(w.cores) * w.cores[0].shape[1] ** 2 * w.cores[1].shape[0] ** 3 for w in Ws]
    order = sorted(range(len(Ws)), key=lambda b: cost[b])
    sel = order[:48]
    h = TNrSVD([to_device(Ws[b].cores, "f32") for b in sel], 8, 8, 1, seed=9, precision="f32",
               max_rank=32)
    sig = h.run()
    for j in (0, 7, 23, 47):
        w = Ws[sel[j]]
        ref = o.tnrsvd(w.cores, 8, 8, 1, seed=9 + j, eps=0.0, rmax=32)
        err = rel_err(sig[j], ref.sigma)
        print(f"batched member {sel[j]} (d={len(w.cores)}, I={w.cores[0].shape[1]}, "
              f"R={w.cores[1].shape[0]}): {err:.3e}")
        assert err <= TOL["f32"]
    h.close()


def _costly_batch(precision):
    from paper_1707_07803_amd import TNrSVD
    with open(GOLDEN) as f:
        gold = json.load(f)
    Ws = wl.batched(512)
    members = [m["member"] for m in gold["members"]]
    h = TNrSVD([to_device(Ws[b].cores, precision) for b in members], gold["k"], gold["p"],
               gold["q"], seed=gold["seed_base"], precision=precision, max_rank=gold["rmax"])
    return gold, h


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_batched_uneven_costliest_members(precision):
    gold, h = _costly_batch(precision)
    sig = h.run()
    for j, m in enumerate(gold["members"]):
        err = rel_err(sig[j], m["sigma"])
        print(f"batched member {m['member']} (d={m['d']}, I={m['I']}, R={m['R']}) {precision}: "
              f"sigma rel err {err:.3e}")
        assert err <= TOL[precision]
    h.close()


def test_batched_uneven_costliest_members_graph_replay():
    gold, h = _costly_batch("f32")
    eager = h.run()
    for _ in range(2):
        rep = h.run_graph()
        assert np.array_equal(rep, eager)
        again = h.run()
        assert np.array_equal(again, eager)
    h.close()
