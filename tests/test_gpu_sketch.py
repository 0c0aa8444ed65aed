"""GPU parity of the sketched product truncation (tnrsvd_opts.sketch_rank),
an opt-in step that is not in the paper, against the oracle's mode
(tnrsvd(..., sketch_rank=, sketch_seed=)), on the same Omega and the same
counter-based sketch.

Where ell is below the products' true ranks the result depends on the exact
sketch entries, so agreement there also checks that both sides draw the same
Gaussian chain.  Where ell reaches them the sketched solve equals the plain
one.
"""

import numpy as np
import pytest

from oracle import tnrsvd_oracle as o
import workloads as wl
from gpu_helpers import omega_for, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1707_07803_amd import load_library
    load_library()
    yield


def solve(cores, k, p, q, om, ell, seed, precision="f64", eps=0.0, rmax=0, orientation="k_last",
          profile=False):
    from paper_1707_07803_amd import TNrSVD, omega_flat
    h = TNrSVD(to_device(cores, "f64" if precision == "f64" else "f32"), k, p, q, seed=seed,
               precision=precision, round_tol=eps, max_rank=rmax, sketch_rank=ell,
               orientation=orientation)
    h.set_omega(omega_flat(*om))
    if profile:
        h.profile(True)
    return h.run()[0], h


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("ell,q", [(16, 1), (8, 1), (5, 0)])
def test_small_against_oracle(ell, q):
    W = wl.small()
    om = omega_for(W.cores, W.K, 3)
    s, h = solve(W.cores, W.k, W.p, q, om, ell, seed=11)
    ref = o.tnrsvd(W.cores, W.k, W.p, q, omega=om, sketch_rank=ell, sketch_seed=11).sigma
    plain = o.tnrsvd(W.cores, W.k, W.p, q, omega=om).sigma
    print(f"ell={ell} q={q}: vs sketched oracle {rel(s, ref):.2e}, vs plain {rel(s, plain):.2e}")
    assert rel(s, ref) < 1e-10
    if ell >= 16:                                   # the products' true ranks
        assert rel(s, plain) < 1e-10
    else:
        assert rel(ref, plain) > 1e-6               # the sketch does cut here


def test_fp32_contractions_follow_the_oracle():
    W = wl.small()
    om = omega_for(W.cores, W.K, 3)
    s, _ = solve(W.cores, W.k, W.p, 1, om, 8, seed=4, precision="f32")
    ref = o.tnrsvd(W.cores, W.k, W.p, 1, omega=om, sketch_rank=8, sketch_seed=4).sigma
    assert rel(s, ref) < 1e-5


def test_large_workload_against_oracle():
    W = wl.large()
    om = omega_for(W.cores, W.K, W.omega_seed)
    s, h = solve(W.cores, W.k, W.p, W.q, om, 48, seed=5, eps=W.eps, rmax=W.rmax, profile=True)
    ref = o.tnrsvd(W.cores, W.k, W.p, W.q, omega=om, eps=W.eps, rmax=W.rmax, sketch_rank=48,
                   sketch_seed=5).sigma
    print(f"large: vs sketched oracle {rel(s, ref):.2e}; sketch {h.profile_read('sketch')}, "
          f"rl sweeps {h.profile_read('rl_sweep')}, lr sweeps {h.profile_read('lr_sweep')}")
    assert rel(s, ref) < 1e-9


@pytest.mark.parametrize("N", [20, 30])
def test_hilbert_sketched_against_plain_oracle(N):
    """At ell = 64 the sketch keeps more than the ranks the 1e-9 rounding
    keeps (up to 35), so the singular values stay those of the plain solve."""
    from paper_1707_07803_amd import TNrSVD, omega_flat, round_mpo
    W = wl.hilbert(N)
    P = round_mpo(to_device(W.cores), wl.HILBERT_MPO_TOL)
    L_shapes = o.reverse_mpo([np.zeros(tuple(c.shape)) for c in P])
    om = omega_for(L_shapes, W.K, W.omega_seed)
    h = TNrSVD(P, W.k, W.p, W.q, seed=N, round_tol=W.eps, max_rank=W.rmax, sketch_rank=64,
               orientation="k_first")
    h.set_omega(omega_flat(*om))
    s = h.run()[0]
    Pn = o.round_mpo(W.cores, wl.HILBERT_MPO_TOL)
    L = o.reverse_mpo(Pn)
    m = o.merge_plan([c.shape[1] for c in L], [c.shape[2] for c in L], W.K)
    A1 = o.reverse_mpo(o.merge_tail(L, m))
    ref = o.tnrsvd_paper_orientation(A1, W.k, W.p, W.q, om[1], om[0][::-1], eps=W.eps,
                                     rmax=W.rmax)
    print(f"hilbert{N} sketched: rel err vs plain oracle {rel(s, ref):.2e}")
    assert rel(s, ref) < 1e-8


def test_invalid_sketch_rank():
    from paper_1707_07803_amd import TNrSVD, TNrSVDError
    W = wl.small()
    with pytest.raises(TNrSVDError) as ei:
        TNrSVD(to_device(W.cores), W.k, W.p, 0, sketch_rank=-1)
    assert ei.value.status == -1
    with pytest.raises(TNrSVDError) as ei:
        TNrSVD(to_device(W.cores), W.k, W.p, 0, sketch_rank=257)
    assert ei.value.status == -1


def test_graph_replay_and_batch_match_eager():
    """The sketch kernel under hipGraph capture (replayed several times, with
    eager work between) and in a batch of uneven MPOs gives the eager,
    one-MPO singular values: every launch reads its product index and the
    MPO's seed offset from its own arguments."""
    import torch
    from paper_1707_07803_amd import TNrSVD
    W = wl.small()
    V = wl.random_mpo(7, 2, 3, 4, 0.5, 17)
    dev = [to_device(W.cores), to_device(V)]
    eager = []
    for b, cores in enumerate(dev):
        h = TNrSVD(cores, 6, 4, 1, seed=30 + b, sketch_rank=6)
        eager.append(h.run()[0])
        h.close()
    hb = TNrSVD(dev, 6, 4, 1, seed=30, sketch_rank=6)
    for rep in range(3):
        s = hb.run_graph()
        for b in range(2):
            np.testing.assert_allclose(s[b], eager[b], rtol=1e-12)
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()    # eager work between replays
    np.testing.assert_allclose(hb.run()[1], eager[1], rtol=1e-12)
    hb.close()


def test_paper_orientation_with_sketch_matches_mirror():
    from paper_1707_07803_amd import TNrSVD, omega_flat
    W = wl.small()
    om = omega_flat(*omega_for(W.cores, W.K, 3))
    hl = TNrSVD(to_device(W.cores), W.k, W.p, 1, seed=2, sketch_rank=8)
    hf = TNrSVD(to_device(o.reverse_mpo(W.cores)), W.k, W.p, 1, seed=2, sketch_rank=8,
                orientation="k_first")
    hl.set_omega(om)
    hf.set_omega(om)
    np.testing.assert_array_equal(hf.run()[0], hl.run()[0])


def test_known_spectrum_fp64_and_bf16_against_oracle():
    """The known-spectrum workload (products of rank 125, rounding 1e-12): the
    sketched FP64 solve follows the oracle's sketched mode; with BF16 storage
    the compressed cores are written in BF16 and the result stays within the
    BF16 path's tolerance."""
    W = wl.spectrum()
    om = omega_for(W.cores, W.K, W.omega_seed)
    ref = o.tnrsvd(W.cores, W.k, W.p, W.q, omega=om, eps=W.eps_by_precision["f64"], rmax=W.rmax,
                   sketch_rank=16, sketch_seed=5).sigma
    s64, _ = solve(W.cores, W.k, W.p, W.q, om, 16, seed=5, eps=W.eps_by_precision["f64"],
                   rmax=W.rmax)
    print("spectrum sketched f64 vs oracle", rel(s64, ref))
    assert rel(s64, ref) < 1e-10
    from paper_1707_07803_amd import TNrSVD, omega_flat
    h = TNrSVD(to_device(W.cores, "f32"), W.k, W.p, W.q, seed=5, precision="bf16",
               round_tol=W.eps_by_precision["bf16"], max_rank=W.rmax, sketch_rank=16)
    h.set_omega(omega_flat(*om))
    sb = h.run()[0]
    print("spectrum sketched bf16 vs prescribed", rel(sb, W.sigma_exact[: W.k]))
    assert rel(sb, W.sigma_exact[: W.k]) < 1e-2
