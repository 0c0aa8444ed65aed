"""Writes batched_members.json: oracle singular values of members of the
512-MPO uneven draw (d in [10, 40], I = J in {2, 4}, ranks in [4, 32],
N(0, 1/R) cores; k = 8, p = 8, q = 1, rank cap 32), for the GPU test that
solves them inside one uneven batch.

The three costliest members of the draw by rounding work are taken (R >= 28
with 4 x 4 cores, product ranks up to 1024; one of them with d = 40, the
largest d of the draw), interleaved with three of the cheapest.  Member j of
that test batch draws its random test matrix from the counter generator with
seed 9 + j, as the library does for the j-th MPO of a handle created with
seed 9.  Only oracle/ and workloads.py are called: the values are the plain
FP64 oracle's (TNrSVD as in Sec. 5.4, rounding of Sec. 3).  Takes a few
minutes on the CPU.

    python tests/golden/make_batched_members.py
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import tnrsvd_oracle as o  # noqa: E402
import workloads as wl  # noqa: E402

EXPENSIVE = [289, 173, 469]   # R = 32, 32, 29; I = 4; d = 35, 34, 40
CHEAP = [344, 103, 362]       # among the cheapest: R = 4, 4, 6; I = 2; d = 21, 37, 11


def main():
    Ws = wl.batched(512)
    members = [EXPENSIVE[0], CHEAP[0], EXPENSIVE[1], CHEAP[1], EXPENSIVE[2], CHEAP[2]]
    out = {"citation": "oracle TNrSVD (Sec. 5.4 subspace iteration with the Sec. 3 rounding), "
                       "written by tests/golden/make_batched_members.py",
           "k": 8, "p": 8, "q": 1, "rmax": 32, "seed_base": 9, "members": []}
    for j, b in enumerate(members):
        w = Ws[b]
        t0 = time.perf_counter()
        res = o.tnrsvd(w.cores, 8, 8, 1, seed=9 + j, eps=0.0, rmax=32)
        dt = time.perf_counter() - t0
        out["members"].append({
            "member": b, "batch_index": j, "seed": 9 + j, "d": len(w.cores),
            "I": int(w.cores[0].shape[1]), "R": int(w.cores[0].shape[3]),
            "sigma": [float(x) for x in res.sigma], "ranks_last": [int(x) for x in res.ranks[-1]],
            "oracle_seconds": round(dt, 1)})
        print(f"member {b}: d={len(w.cores)} I={w.cores[0].shape[1]} R={w.cores[0].shape[3]} "
              f"{dt:.1f} s sigma[0]={res.sigma[0]:.6e}", flush=True)
    with open(os.path.join(HERE, "batched_members.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
