"""Seeded synthetic workloads for the TNrSVD hot path.

This module only draws inputs: MPO cores of A and the Gaussian factors of the
random test MPO.  It holds none of the method's arithmetic and imports neither
the oracle nor the GPU package; both of those receive its arrays as inputs.

Workloads (sizes follow the paper's experiments of Sec. 6.3, whose matrices
are 2^N x 2^N MPOs with 2 x 2 cores; no dataset is involved):

* ``small``      d=8, 2x2 cores (256 x 256), ranks 3, N(0,1) cores, K = 10+6, q=0
* ``spectrum``   d=20 equivalent (2^20 x 2^20) built as U diag(sigma) V^T from
                 left-orthonormal rank-5 MPOs in merged layout: 15 cores of
                 2 x 2 and a last core of 32 x 32; sigma_j = 10^(-j/4), j<50;
                 K = 20+10, q = 1 (stand-in for the prescribed-spectrum
                 experiment of Sec. 6.3)
* ``large``      d=50, 2x2 cores (2^50 x 2^50), ranks 10, N(0,1/10), K=10+10, q=2
* ``batched``    512 MPOs, d in [10,40], I=J in {2,4}, ranks in [4,32],
                 N(0,1/R), K = 8+8, q = 1
* ``grad``       d=30, 4x4 cores, ranks 16, N(0,1/16), K = 16+8, q = 1
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

__all__ = ["Workload", "random_mpo", "gaussian_omega", "orthonormal_mps",
           "known_spectrum_mpo", "small", "spectrum", "large", "batched",
           "grad", "get", "WORKLOADS"]


@dataclass
class Workload:
    name: str
    cores: List[np.ndarray]           # A's MPO cores (R, I, J, R'), float64
    k: int
    p: int
    q: int
    eps: float = 0.0                  # rounding tolerance (per precision below)
    rmax: int = 0                     # rounding rank cap (0 = none)
    eps_by_precision: dict = field(default_factory=dict)
    omega_seed: int = 0
    sigma_exact: Optional[np.ndarray] = None  # prescribed spectrum, if any

    @property
    def K(self) -> int:
        return self.k + self.p


def random_mpo(d: int, I: int, J: int, R: int, std: float, seed) -> List[np.ndarray]:
    """MPO with uniform inner rank R and i.i.d. N(0, std^2) entries (PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ranks = [1] + [R] * (d - 1) + [1]
    return [rng.standard_normal((ranks[i], I, J, ranks[i + 1])) * std for i in range(d)]


def gaussian_omega(cols: List[int], K: int, seed) -> Tuple[List[np.ndarray], np.ndarray]:
    """Gaussian factors of the rank-1 random MPO: vectors of length J_i for all
    but the last core, and a J_d x K matrix for the last (merged) core."""
    rng = np.random.Generator(np.random.PCG64(seed))
    vecs = [rng.standard_normal(J) for J in cols[:-1]]
    last = rng.standard_normal((cols[-1], K))
    return vecs, last


def orthonormal_mps(ranks: List[int], dims: List[int], ncols: int, seed) -> List[np.ndarray]:
    """Left-orthonormal MPS-like cores from the Q factor of N(0,1) draws.

    Core i has shape (ranks[i], dims[i], ranks[i+1]); the last core has shape
    (ranks[-1], dims[-1], ncols).  Every unfolding (r*n) x r' has orthonormal
    columns, so the whole chain has orthonormal columns.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    d = len(dims)
    for i in range(d):
        r, n = ranks[i], dims[i]
        r2 = ranks[i + 1] if i < d - 1 else ncols
        G = rng.standard_normal((r * n, r2))
        Q, _ = np.linalg.qr(G)
        out.append(Q.reshape(r, n, r2))
    return out


def known_spectrum_mpo(U: List[np.ndarray], V: List[np.ndarray],
                       sigma: np.ndarray) -> List[np.ndarray]:
    """MPO cores of U diag(sigma) V^T for MPS-like U, V (column leg on the last core).

    Inner cores are the outer products U_i[a,x,b] V_i[a',y,b'] with combined
    ranks (a, a') -> a * r_V + a'; the last core contracts the column leg
    with sigma.
    """
    out = []
    d = len(U)
    for i in range(d):
        u, v = U[i], V[i]
        ra, nx, rb = u.shape
        sa, ny, sb = v.shape
        if i < d - 1:
            c = np.einsum("axb,cye->acxybe", u, v).reshape(ra * sa, nx, ny, rb * sb)
        else:
            c = np.einsum("axj,j,cyj->acxy", u, sigma, v).reshape(ra * sa, nx, ny, 1)
        out.append(np.ascontiguousarray(c))
    return out


def small() -> Workload:
    return Workload("small", random_mpo(8, 2, 2, 3, 1.0, 1), k=10, p=6, q=0,
                    omega_seed=2)


def spectrum(d_inner: int = 15, last: int = 32, r: int = 5, n_sig: int = 50,
             k: int = 20, p: int = 10, q: int = 1) -> Workload:
    """Known-spectrum MPO in merged layout (d_inner cores of 2x2 plus one last x last)."""
    ranks = [1]
    for i in range(d_inner):
        ranks.append(min(r, ranks[-1] * 2))
    dims = [2] * d_inner + [last]
    U = orthonormal_mps(ranks, dims, n_sig, 3)
    V = orthonormal_mps(ranks, dims, n_sig, 4)
    sig = 10.0 ** (-np.arange(n_sig) / 4.0)
    cores = known_spectrum_mpo(U, V, sig)
    # FP32 product cores carry a relative error of a few 1e-7, so the FP32
    # rounding tolerance sits above that floor (the tail test compares squared
    # singular values against (eps |Y|)^2 / (d - 1)); with 1e-6 some draws of
    # Omega keep noise directions through the power step and inflate ranks.
    return Workload("spectrum", cores, k=k, p=p, q=q, eps=1e-12, rmax=32,
                    eps_by_precision={"f64": 1e-12, "f32": 1e-5, "bf16": 1e-2},
                    omega_seed=5, sigma_exact=sig)


def large() -> Workload:
    return Workload("large", random_mpo(50, 2, 2, 10, 10 ** -0.5, 6), k=10, p=10,
                    q=2, eps=0.0, rmax=32, omega_seed=7)


def batched(n: int = 512) -> List[Workload]:
    children = np.random.SeedSequence(8).spawn(n)
    out = []
    for b, ss in enumerate(children):
        rng = np.random.Generator(np.random.PCG64(ss))
        d = int(rng.integers(10, 41))
        I = int(rng.choice([2, 4]))
        R = int(rng.integers(4, 33))
        ranks = [1] + [R] * (d - 1) + [1]
        cores = [rng.standard_normal((ranks[i], I, I, ranks[i + 1])) / np.sqrt(R)
                 for i in range(d)]
        out.append(Workload(f"batched[{b}]", cores, k=8, p=8, q=1, eps=0.0,
                            rmax=32, omega_seed=1000 + b))
    return out


def grad() -> Workload:
    return Workload("grad", random_mpo(30, 4, 4, 16, 0.25, 10), k=16, p=8, q=1,
                    eps=0.0, rmax=32, omega_seed=11)


WORKLOADS = {"small": small, "spectrum": spectrum, "large": large, "grad": grad}


def get(name: str) -> Workload:
    return WORKLOADS[name]()
