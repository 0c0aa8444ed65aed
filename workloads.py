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

Sparse matrices for the conversion of Algorithm 4.1 (stand-ins for the
matrices of the collection used in Sec. 6.1 and 6.2, which are not shipped):
banded patterns with a full diagonal, band offsets ~ round(N(0, s^2)) clipped
to the bandwidth, a few far symmetric pairs, N(0,1) values (diagonal 4 + |N|),
duplicates merged (one entry per position, as a stored sparse matrix has):

* ``power16k``   16384 x 16384 (nonzeros in the leading 15838 x 15838, the
                 rest zero padding), I_1 = J_1 = 256 then six 2 x 2 modes
                 (d = 7), bandwidth 200, ~4 entries per row, 115 far pairs
* ``circuit150k`` 150102 x 150102, I = J = (1614, 31, 3) (d = 3), bandwidth
                 1962, s = 400, ~5 entries per row
* ``hilbert(N)``  the 2^N x 2^(N-1) submatrix H(:, 1:2^(N-1)) of the Hilbert
                 matrix (Sec. 6.3), 10 <= N <= 50: an MPO of N cores (2 x 2,
                 the last 2 x 1) from an exponential sum for 1/x; rank-16
                 approximation, K = 16+16, q = 2 (N <= 30), 3 (N <= 40), 4
* ``power16k_stencil``, ``circuit150k_stencil``  the same sizes and
                 partitions with a fixed stencil (every row has its entries at
                 the same offsets with the same values, cut at the matrix
                 edge): banded Toeplitz matrices, whose Algorithm 4.1 MPOs
                 round to small ranks as the paper's matrices do (Sec. 6.1)
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

__all__ = ["Workload", "random_mpo", "gaussian_omega", "orthonormal_mps",
           "known_spectrum_mpo", "small", "spectrum", "large", "batched",
           "grad", "get", "WORKLOADS", "SparseWorkload", "banded_sparse", "power16k",
           "circuit150k", "stencil_sparse", "power16k_stencil", "circuit150k_stencil",
           "SPARSE_WORKLOADS", "ROUND_WORKLOADS", "hilbert_mpo", "hilbert", "HILBERT_N"]


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


@dataclass
class SparseWorkload:
    name: str
    rows: List[int]                   # I_1..I_d (eq. (1) ordering, first fastest)
    cols: List[int]                   # J_1..J_d
    coo_row: np.ndarray               # int64
    coo_col: np.ndarray               # int64
    coo_val: np.ndarray               # float64


def banded_sparse(n: int, n_used: int, half_bw: int, spread: float, per_row: int,
                  n_far: int, seed) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """COO of an n x n banded sparse matrix whose nonzeros lie in the leading
    n_used x n_used part: the full diagonal, per_row - 1 band entries per row at
    offsets round(N(0, spread^2)) clipped to [-half_bw, half_bw], and n_far
    symmetric pairs at uniform positions; entries on one position are merged
    (the last drawn value is kept).  Sorted by (row, col)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    i = np.repeat(np.arange(n_used, dtype=np.int64), per_row - 1)
    off = np.clip(np.rint(rng.standard_normal(i.size) * spread), -half_bw, half_bw).astype(np.int64)
    j = i + off
    ok = (j >= 0) & (j < n_used)
    fi = rng.integers(0, n_used, n_far)
    fj = rng.integers(0, n_used, n_far)
    diag = np.arange(n_used, dtype=np.int64)
    r = np.concatenate([diag, i[ok], fi, fj])
    c = np.concatenate([diag, j[ok], fj, fi])
    fv = rng.standard_normal(n_far)
    v = np.concatenate([4.0 + np.abs(rng.standard_normal(n_used)),
                        rng.standard_normal(int(ok.sum())), fv, fv])
    key = r * n + c
    _, last = np.unique(key[::-1], return_index=True)
    keep = key.size - 1 - last                       # last occurrence of every position
    order = np.argsort(key[keep], kind="stable")
    keep = keep[order]
    return r[keep], c[keep], v[keep]


def power16k() -> SparseWorkload:
    r, c, v = banded_sparse(16384, 15838, 200, 80.0, 4, 115, 21)
    return SparseWorkload("power16k", [256] + [2] * 6, [256] + [2] * 6, r, c, v)


def circuit150k() -> SparseWorkload:
    r, c, v = banded_sparse(150102, 150102, 1962, 400.0, 5, 0, 22)
    return SparseWorkload("circuit150k", [1614, 31, 3], [1614, 31, 3], r, c, v)


SPARSE_WORKLOADS = {"power16k": power16k, "circuit150k": circuit150k}


def stencil_sparse(n: int, n_used: int, half_bw: int, n_off: int,
                   seed) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """COO of an n x n banded Toeplitz matrix supported on its leading
    n_used x n_used part: offset 0 (value 4 + |N(0,1)|) and n_off - 1 further
    distinct offsets drawn uniformly from [-half_bw, half_bw], each with one
    N(0,1) value shared by every row.  Sorted by (row, col)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    others = rng.choice(np.setdiff1d(np.arange(-half_bw, half_bw + 1), [0]), n_off - 1,
                        replace=False)
    offs = np.concatenate([[0], np.sort(others)]).astype(np.int64)
    vals = np.concatenate([[4.0 + abs(rng.standard_normal())], rng.standard_normal(n_off - 1)])
    i = np.repeat(np.arange(n_used, dtype=np.int64), n_off)
    j = i + np.tile(offs, n_used)
    v = np.tile(vals, n_used)
    ok = (j >= 0) & (j < n_used)
    return i[ok], j[ok], v[ok]


def power16k_stencil() -> SparseWorkload:
    r, c, v = stencil_sparse(16384, 15838, 200, 7, 23)
    return SparseWorkload("power16k_stencil", [256] + [2] * 6, [256] + [2] * 6, r, c, v)


def circuit150k_stencil() -> SparseWorkload:
    r, c, v = stencil_sparse(150102, 150102, 1962, 9, 24)
    return SparseWorkload("circuit150k_stencil", [1614, 31, 3], [1614, 31, 3], r, c, v)


ROUND_WORKLOADS = {"power16k_stencil": power16k_stencil,
                   "circuit150k_stencil": circuit150k_stencil, "power16k": power16k}


# ------------------------------------------------------------------ Hilbert

def hilbert_mpo(N: int, h: float = 0.3, tail: float = 1e-14) -> List[np.ndarray]:
    """MPO of the 2^N x 2^(N-1) matrix A(i, j) = 1 / (i + j + 1) (0-based i, j:
    the first 2^(N-1) columns of the Hilbert matrix), N cores with the
    little-endian index of eq. (1): core k carries bit k of i and of j, and the
    last core has J = 1 (bit N-1 of j is 0).

    Built from the integral 1/x = int_R exp(t - x e^t) dt (x > 0), taken by the
    trapezoidal rule with step h: 1/x ~ sum_l w_l exp(-a_l x), a_l = e^(t_l),
    w_l = h e^(t_l), over t_l in [ln(tail / X), ln(-ln tail)] with X the largest
    x.  The integrand is analytic in the strip |Im t| < pi/2, so the rule's
    relative error is about exp(-pi^2 / h) (5e-15 at h = 0.3); the cut tails add
    at most `tail` relative.  With x = 1 + sum_k 2^k (i_k + j_k) each term is a
    Kronecker product of 2 x 2 factors exp(-a_l 2^k (i_k + j_k)), so the sum is an
    MPO whose rank is the number of nodes (about 140 at N = 10, 240 at N = 50),
    with diagonal cores.  Rounding brings it to the small ranks the matrix has.
    """
    if N < 2:
        raise ValueError("N >= 2")
    X = 2.0 ** N + 2.0 ** (N - 1) - 1.0
    t0, t1 = np.log(tail / X), np.log(-np.log(tail))
    t = np.arange(np.floor(t0 / h), np.ceil(t1 / h) + 1) * h
    a, w = np.exp(t), h * np.exp(t)
    R = a.size
    cores = []
    for k in range(N):
        J = 1 if k == N - 1 else 2
        f = np.exp(-np.multiply.outer(a * 2.0 ** k, np.add.outer(np.arange(2), np.arange(J))))
        if k == 0:
            c = (f * (w * np.exp(-a))[:, None, None]).transpose(1, 2, 0)[None]
        elif k == N - 1:
            c = f[:, :, :, None]
        else:
            c = np.zeros((R, 2, J, R))
            c[np.arange(R), :, :, np.arange(R)] = f
        cores.append(np.ascontiguousarray(c))
    return cores


HILBERT_N = (10, 15, 20, 25, 30, 35, 40, 45, 50)
HILBERT_MPO_TOL = 1e-12   # rounding of the exponential-sum MPO (the paper's MPO: 1e-11)


def hilbert(N: int) -> Workload:
    """The Hilbert experiment of Sec. 6.3 at size N: rank 16 (K = 32), rounding
    tolerance 1e-9, q by N as in the paper.  ``cores`` is the unrounded
    exponential-sum MPO; it is rounded at HILBERT_MPO_TOL before the solve.
    The rank cap 64 only bounds the planned capacity: the rounded ranks stay
    below it (the paper caps nothing)."""
    q = 2 if N <= 30 else (3 if N <= 40 else 4)
    return Workload(f"hilbert{N}", hilbert_mpo(N), k=16, p=16, q=q, eps=1e-9, rmax=64,
                    omega_seed=70 + N)
