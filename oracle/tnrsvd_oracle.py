"""Plain FP64 CPU oracle of the Tensor Network randomized SVD (TNrSVD).

TEST INFRASTRUCTURE ONLY.  This module is imported by ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``; the
GPU library neither links nor calls it, and it imports nothing from the GPU
package.  Everything is numpy float64; LAPACK (through ``numpy.linalg.qr`` and
``numpy.linalg.svd``) is used only as a step where the paper itself calls for
a QR or an SVD.

Source: Batselier, Yu, Daniel, Wong, "Computing low-rank approximations of
large-scale matrices with the Tensor Network randomized SVD" (arXiv 1707.07803).

Orientation (a reading of the paper, recorded in the design notes): the paper
puts the K-column leg of the random MPO, of Y and of Q on the FIRST core and
sweeps right-to-left (lemma on random MPOs in Sec. 5.1, Algorithms 5.2 and
5.3).  This oracle uses the mirror image: the K leg sits on the LAST core and
the orthogonalisation sweeps run left-to-right.  Reversing the core order of
an MPO only permutes the rows and columns of the matrix it represents, so the
singular values are unchanged; ``tnrsvd_paper_orientation`` below implements
the paper's own orientation and the tests check that the two agree.

Layouts (C order, 0-based):
  * MPO core i of A:           (R_i, I_i, J_i, R_{i+1}),  R_1 = R_{d+1} = 1
  * MPS-like core (Y, Q, Z, B^T, U, V): (r_i, n_i, r_{i+1}); the last core is
    (r_d, n_d, K) -- its right leg is the K column leg.
  * Row/column multi-indices are little-endian as in eq. (1): the index of the
    first core varies fastest, [i_1 ... i_d] = i_1 + I_1 i_2 + I_1 I_2 i_3 + ...
  * Product cores of an MPO with an MPS combine ranks as p = a * r + c, where
    a is A's rank index and c the MPS rank index.

Parity status of each function is stated in its docstring; the pins live in
``tests/test_oracle_*.py``.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "multi_index", "mpo_to_dense", "mps_to_dense", "kron_chain",
    "rank_bounds", "merge_plan", "merge_tail",
    "splitmix64", "gaussian_counter", "omega_from_seed", "omega_as_mps",
    "mpo_times_mps", "mpo_t_times_mps", "mpo_add", "mps_gram", "mps_norm",
    "lq_nonneg", "qr_nonneg", "svd_signfix", "choose_rank",
    "round_sweep", "tnrsvd", "TNrSVDResult", "dense_rsvd",
    "tnrsvd_paper_orientation", "reverse_mpo",
    "gaussian_counter_array", "sketch_counter_base", "sketch_compress",
    "complex_to_real_mpo", "tnrsvd_complex",
    "merge_tail_adjoint", "sigma_sum_grad",
    "mpo_times_mps_adjoint", "mpo_t_times_mps_adjoint", "round_sweep_gram", "qr_adjoint",
    "round_sweep_gram_adjoint", "pipeline_grad",
    "sparse_to_mpo", "round_mpo",
]

# --------------------------------------------------------------------------
# Sec. 2: multi-indices, reshaping, Kronecker products
# --------------------------------------------------------------------------

def multi_index(idx: Sequence[int], dims: Sequence[int]) -> int:
    """Linear index of the multi-index [i_1 i_2 ... i_d], eq. (1), 0-based.

    The first index varies fastest (MATLAB column-major convention).
    Pinned by the 4x3x2 reshape and vectorisation examples of Sec. 2.
    """
    lin, stride = 0, 1
    for i, n in zip(idx, dims):
        if not 0 <= i < n:
            raise IndexError("index out of range")
        lin += i * stride
        stride *= n
    return lin


def kron_chain(mats: Sequence[np.ndarray]) -> np.ndarray:
    """A^(d) kron ... kron A^(1) for mats = [A^(1), ..., A^(d)] (Theorem 3.1).

    The first core is the LAST Kronecker factor.
    """
    out = np.ones((1, 1))
    for m in mats:
        out = np.kron(m, out)
    return out


def mpo_to_dense(cores: Sequence[np.ndarray]) -> np.ndarray:
    """Contract an MPO into the (prod I) x (prod J) matrix it represents (Sec. 3).

    Entry ([i_1..i_d], [j_1..j_d]) is A_1[:, i_1, j_1, :] A_2[:, i_2, j_2, :] ...
    with little-endian multi-indices (eq. 1).  Pinned by Theorem 3.1 (rank-1
    MPO equals the reversed Kronecker product) and by the 2 x 6 example of
    Sec. 4.2.
    """
    c0 = np.asarray(cores[0], dtype=np.float64)
    if c0.shape[0] != 1:
        raise ValueError("first MPO rank must be 1")
    rows, cols = c0.shape[1], c0.shape[2]
    T = c0.reshape(rows, cols, c0.shape[3])
    for c in cores[1:]:
        c = np.asarray(c, dtype=np.float64)
        r, I, J, r2 = c.shape
        if r != T.shape[2]:
            raise ValueError("rank mismatch")
        # new row = old_row + rows * x, new col = old_col + cols * y
        N = np.einsum("abr,rxys->xaybs", T, c)
        rows, cols = rows * I, cols * J
        T = N.reshape(rows, cols, r2)
    if T.shape[2] != 1:
        raise ValueError("last MPO rank must be 1")
    return T[:, :, 0]


def mps_to_dense(cores: Sequence[np.ndarray]) -> np.ndarray:
    """Contract an MPS-like chain (last core carries the K leg) to (prod n) x K."""
    c0 = np.asarray(cores[0], dtype=np.float64)
    if c0.shape[0] != 1:
        raise ValueError("first rank must be 1")
    rows = c0.shape[1]
    T = c0.reshape(rows, c0.shape[2])
    for c in cores[1:]:
        c = np.asarray(c, dtype=np.float64)
        r, n, r2 = c.shape
        if r != T.shape[1]:
            raise ValueError("rank mismatch")
        N = np.einsum("ar,rxs->xas", T, c)
        rows *= n
        T = N.reshape(rows, r2)
    return T


def rank_bounds(rows: Sequence[int], cols: Sequence[int]) -> List[int]:
    """Upper bounds on the canonical MPO ranks R_2..R_d (Theorem 3.2).

    R_k <= min(prod_{i<k} I_i J_i, prod_{i>=k} I_i J_i).
    """
    d = len(rows)
    s = [r * c for r, c in zip(rows, cols)]
    out = []
    for k in range(1, d):
        out.append(min(math.prod(s[:k]), math.prod(s[k:])))
    return out


# --------------------------------------------------------------------------
# Merging the cores at the K end (Sec. 6.3 contracts the first cores so that
# the K-core is at least K x K; mirrored here to the last cores)
# --------------------------------------------------------------------------

def merge_plan(rows: Sequence[int], cols: Sequence[int], K: int) -> int:
    """Smallest m such that the last m cores give prod I >= K and prod J >= K.

    The random-MPO lemma of Sec. 5.1 needs K <= J of the K-core, Algorithm 5.2
    needs I >= K on that core and Algorithm 5.3 needs J >= K.  Raises
    ValueError when even the whole MPO is too small.
    """
    d = len(rows)
    pi, pj = 1, 1
    for m in range(1, d + 1):
        pi *= rows[d - m]
        pj *= cols[d - m]
        if pi >= K and pj >= K:
            return m
    raise ValueError("prod(I) or prod(J) is smaller than K")


def merge_tail(cores: Sequence[np.ndarray], m: int) -> List[np.ndarray]:
    """Contract the last m MPO cores into one core (R, prod I, prod J, 1).

    The merged row index is little-endian within the group (first merged core
    fastest), which keeps the global multi-index of eq. (1) unchanged.
    """
    cores = [np.asarray(c, dtype=np.float64) for c in cores]
    d = len(cores)
    if not 1 <= m <= d:
        raise ValueError("bad merge count")
    head = cores[: d - m]
    T = cores[d - m]
    for c in cores[d - m + 1:]:
        a, I1, J1, _ = T.shape
        _, I2, J2, b = c.shape
        N = np.einsum("axyr,rXYb->aXxYyb", T, c)
        T = N.reshape(a, I2 * I1, J2 * J1, b)
    return head + [T]


# --------------------------------------------------------------------------
# Random test matrix in MPO form (lemma on random MPOs, Sec. 5.1)
# --------------------------------------------------------------------------

_MASK64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


def splitmix64(seed: int, n: int) -> int:
    """n-th output (0-based) of SplitMix64 (Steele, Lea, Flood 2014), counter form.

    state_n = seed + (n + 1) * 0x9E3779B97F4A7C15 (mod 2^64), then the
    published finaliser: xor-shift 30, multiply 0xBF58476D1CE4E5B9,
    xor-shift 27, multiply 0x94D049BB133111EB, xor-shift 31.
    """
    z = (seed + (n + 1) * _GOLDEN) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def gaussian_counter(seed: int, n: int) -> float:
    """n-th standard normal of the counter-based stream (Box and Muller 1958).

    Pair k = n // 2 uses u1 = (splitmix64(seed, 2k) >> 11 + 1) * 2^-53 in (0, 1]
    and u2 = (splitmix64(seed, 2k+1) >> 11) * 2^-53 in [0, 1); even n takes
    sqrt(-2 ln u1) cos(2 pi u2), odd n the sine.  Uses the platform libm
    through Python's math module.
    """
    k = n // 2
    u1 = ((splitmix64(seed, 2 * k) >> 11) + 1) * (2.0 ** -53)
    u2 = (splitmix64(seed, 2 * k + 1) >> 11) * (2.0 ** -53)
    rad = math.sqrt(-2.0 * math.log(u1))
    ang = 2.0 * math.pi * u2
    return rad * (math.cos(ang) if n % 2 == 0 else math.sin(ang))


def omega_from_seed(cols: Sequence[int], K: int, seed: int
                    ) -> Tuple[List[np.ndarray], np.ndarray]:
    """Rank-1 random MPO of the lemma in Sec. 5.1 (mirrored: matrix on the last core).

    Returns ([omega_1, ..., omega_{d-1}], Omega_d) with omega_i of length J_i
    and Omega_d of shape (J_d, K).  Draw order: omega_1 ... omega_{d-1}, then
    Omega_d in C order, one counter value per entry.
    """
    n = 0
    vecs = []
    for J in cols[:-1]:
        vecs.append(np.array([gaussian_counter(seed, n + t) for t in range(J)]))
        n += J
    Jd = cols[-1]
    last = np.array([gaussian_counter(seed, n + t) for t in range(Jd * K)])
    return vecs, last.reshape(Jd, K)


def omega_as_mps(vecs: Sequence[np.ndarray], last: np.ndarray) -> List[np.ndarray]:
    """Rank-1 MPS-like cores of Omega: (1, J_i, 1) and (1, J_d, K)."""
    cores = [np.asarray(v, dtype=np.float64).reshape(1, -1, 1) for v in vecs]
    cores.append(np.asarray(last, dtype=np.float64).reshape(1, *last.shape))
    return cores


# --------------------------------------------------------------------------
# Matrix multiplication in MPO form (Sec. 5.2)
# --------------------------------------------------------------------------

def mpo_times_mps(A: Sequence[np.ndarray], X: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Cores of A X: sum over the column index j_i of every core (Sec. 5.2).

    Y_i[(a,c), x, (b,e)] = sum_y A_i[a,x,y,b] X_i[c,y,e];
    on the last core e is the K leg and A's right rank is 1.
    Ranks multiply: R_i r_i.
    """
    if len(A) != len(X):
        raise ValueError("core count mismatch")
    out = []
    d = len(A)
    for i, (a, x) in enumerate(zip(A, X)):
        R, I, J, R2 = a.shape
        r, Jx, r2 = x.shape
        if Jx != J:
            raise ValueError("inner dimension mismatch")
        Y = np.einsum("axyb,cye->acxbe", a, x)
        if i == d - 1:
            if R2 != 1:
                raise ValueError("last MPO rank must be 1")
            out.append(Y.reshape(R * r, I, r2))
        else:
            out.append(Y.reshape(R * r, I, R2 * r2))
    return out


def mpo_t_times_mps(A: Sequence[np.ndarray], X: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Cores of A^T X: sum over the row index i_i of every core (Sec. 5.2).

    Z_i[(a,c), y, (b,e)] = sum_x A_i[a,x,y,b] X_i[c,x,e].
    """
    if len(A) != len(X):
        raise ValueError("core count mismatch")
    out = []
    d = len(A)
    for i, (a, x) in enumerate(zip(A, X)):
        R, I, J, R2 = a.shape
        r, Ix, r2 = x.shape
        if Ix != I:
            raise ValueError("inner dimension mismatch")
        Z = np.einsum("axyb,cxe->acybe", a, x)
        if i == d - 1:
            out.append(Z.reshape(R * r, J, r2))
        else:
            out.append(Z.reshape(R * r, J, R2 * r2))
    return out


def mpo_add(A: Sequence[np.ndarray], B: Sequence[np.ndarray]) -> List[np.ndarray]:
    """MPO addition: ranks add, cores are block diagonal (Sec. 3).

    The first core concatenates along its right rank, the last along its left
    rank, inner cores are block diagonal.  Works for MPO (4-way) cores.
    """
    d = len(A)
    out = []
    for i, (a, b) in enumerate(zip(A, B)):
        ra, I, J, ra2 = a.shape
        rb, _, _, rb2 = b.shape
        if d == 1:
            out.append(a + b)
        elif i == 0:
            out.append(np.concatenate([a, b], axis=3))
        elif i == d - 1:
            out.append(np.concatenate([a, b], axis=0))
        else:
            c = np.zeros((ra + rb, I, J, ra2 + rb2))
            c[:ra, :, :, :ra2] = a
            c[ra:, :, :, ra2:] = b
            out.append(c)
    return out


def mps_gram(X: Sequence[np.ndarray], Y: Sequence[np.ndarray]) -> np.ndarray:
    """X^T Y (K_x x K_y) of two MPS-like chains by transfer matrices, no densify."""
    E = np.ones((1, 1))
    for x, y in zip(X, Y):
        # E[c, e] with c rank of X, e rank of Y
        E = np.einsum("ce,cxa,exb->ab", E, x, y)
    return E


def mps_norm(X: Sequence[np.ndarray]) -> float:
    """Frobenius norm of an MPS-like chain (including its K leg)."""
    return float(math.sqrt(max(np.trace(mps_gram(X, X)), 0.0)))


# --------------------------------------------------------------------------
# Small dense factorisations with fixed gauges
# --------------------------------------------------------------------------

def qr_nonneg(M: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Economy Householder QR (LAPACK) with diag(R) >= 0 (reading AMB-4).

    Q is m x k, R is k x n, k = min(m, n).
    """
    Q, R = np.linalg.qr(M, mode="reduced")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :], R * s[:, None]


def lq_nonneg(M: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Economy LQ, M = L Q with orthonormal rows of Q and diag(L) >= 0."""
    Qt, Rt = qr_nonneg(M.T)
    return Rt.T, Qt.T


def svd_signfix(M: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Economy SVD M = U diag(S) Vt with a fixed sign per singular pair.

    The paper leaves singular-vector signs free; here each left singular
    vector is flipped (with its right partner) so that its entry of largest
    magnitude (the first one on exact ties) is positive.
    """
    U, S, Vt = np.linalg.svd(M, full_matrices=False)
    if U.shape[1]:
        piv = np.argmax(np.abs(U), axis=0)
        s = np.sign(U[piv, np.arange(U.shape[1])])
        s[s == 0] = 1.0
        U = U * s[None, :]
        Vt = Vt * s[:, None]
    return U, S, Vt


def choose_rank(S: np.ndarray, delta: float, rmax: int) -> int:
    """Rank kept at one bond of the rounding sweep (reading AMB-5).

    Smallest rho >= 1 whose discarded tail satisfies sum_{l >= rho} S_l^2 <=
    delta^2, then capped at rmax when rmax > 0.  With delta = 0 only exact
    zeros are dropped.
    """
    n = len(S)
    if n == 0:
        return 0
    sq = S.astype(np.float64) ** 2
    tail = np.concatenate([np.cumsum(sq[::-1])[::-1], [0.0]])  # tail[rho]
    rho = n
    for cand in range(1, n + 1):
        if tail[cand] <= delta * delta:
            rho = cand
            break
    if rmax > 0:
        rho = min(rho, rmax)
    return max(rho, 1)


# --------------------------------------------------------------------------
# Rounding fused with the orthogonalisation sweep (Sec. 3 rounding of
# Oseledets' TT-rounding; Algorithms 5.2/5.3 and the integration described in
# Sec. 5.4), mirrored to run left-to-right
# --------------------------------------------------------------------------

def round_sweep(cores: Sequence[np.ndarray], eps: float, rmax: int,
                last: str = "qr"):
    """ROUND followed by the orthogonalisation of an MPS-like chain.

    Step 1, right-to-left: LQ of every core (p_i x n_i p_{i+1}); the L factor
    is absorbed into the left neighbour, leaving cores 2..d with orthonormal
    rows.
    Step 2: delta = eps * ||Y||_F / sqrt(d - 1).
    Step 3, left-to-right: SVD of the (s_i n_i) x p_{i+1} panel of the carried
    factor times core i; the first rho columns of U become core i of the
    result and diag(S) Vt is carried right.  The K leg is never truncated.
    Step 4, last core: 'qr' -> economy QR with diag(R) >= 0 gives Q_d and the
    K x K R (Algorithm 5.2, mirrored); 'svd' -> SVD gives V_d, sigma and W
    (Algorithm 5.3, mirrored).

    Returns a dict with 'cores', 'ranks' (the bond ranks kept), 'norm', and
    'R' or ('sigma', 'W').
    """
    C = [np.array(c, dtype=np.float64, copy=True) for c in cores]
    d = len(C)
    if C[0].shape[0] != 1:
        raise ValueError("first rank must be 1")
    for i in range(d - 1, 0, -1):
        p, n, q = C[i].shape
        L, Qr = lq_nonneg(C[i].reshape(p, n * q))
        k = L.shape[1]
        C[i] = Qr.reshape(k, n, q)
        C[i - 1] = np.tensordot(C[i - 1], L, axes=(2, 0))
    nrm = float(np.linalg.norm(C[0]))
    delta = eps * nrm / math.sqrt(d - 1) if d > 1 else 0.0
    T = np.ones((1, 1))
    ranks = [1]
    for i in range(d - 1):
        M = np.tensordot(T, C[i], axes=(1, 0))
        s, n, q = M.shape
        U, S, Vt = svd_signfix(M.reshape(s * n, q))
        rho = choose_rank(S, delta, rmax)
        C[i] = U[:, :rho].reshape(s, n, rho)
        T = S[:rho, None] * Vt[:rho]
        ranks.append(rho)
    M = np.tensordot(T, C[d - 1], axes=(1, 0))
    s, n, K = M.shape
    out = {"norm": nrm, "ranks": ranks}
    if last == "qr":
        Q, R = qr_nonneg(M.reshape(s * n, K))
        C[d - 1] = Q.reshape(s, n, Q.shape[1])
        out["R"] = R
    elif last == "svd":
        X, S, Wt = svd_signfix(M.reshape(s * n, K))
        C[d - 1] = X.reshape(s, n, X.shape[1])
        out["sigma"] = S
        out["W"] = Wt.T
    else:
        raise ValueError("last must be 'qr' or 'svd'")
    out["cores"] = C
    return out


# --------------------------------------------------------------------------
# Sketched product truncation (not in the paper): an opt-in step before ROUND
# --------------------------------------------------------------------------

def gaussian_counter_array(seed: int, idx: np.ndarray) -> np.ndarray:
    """gaussian_counter(seed, n) for every n in idx (uint64 arithmetic wraps
    mod 2^64 as SplitMix64 requires); numpy's log/cos/sin may differ from the
    math module's in the last bit, which no consumer of this stream relies on."""
    idx = np.asarray(idx, dtype=np.uint64)
    k = idx // np.uint64(2)
    g = np.uint64(_GOLDEN)
    sd = np.uint64(seed & _MASK64)

    def mix(c):
        with np.errstate(over="ignore"):
            z = sd + (c + np.uint64(1)) * g
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))

    u1 = ((mix(np.uint64(2) * k) >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (mix(np.uint64(2) * k + np.uint64(1)) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return rad * np.where(idx % np.uint64(2) == 0, np.cos(ang), np.sin(ang))


def sketch_counter_base(t: int) -> int:
    """First counter of the sketch of the t-th product of a solve (t = 0 for
    Y = A Omega, then one per product): beyond Omega's counters."""
    return (t + 1) << 40


def sketch_compress(Y: Sequence[np.ndarray], ell: int, seed: int, t: int) -> List[np.ndarray]:
    """Compress a product chain Y (cores (P_i, n_i, P_{i+1}), the last
    (P, n, K)) to bond ranks <= ell before ROUND, by the randomize-then-
    orthogonalize rounding of Al Daas, Ballard et al. (SIAM J. Sci. Comput.
    2023): a Gaussian chain S with bond ranks l_k = min(ell, P_k) sketches the
    right parts, W_k = Y_{>=k} S_{>=k}^T (P_k x l_k), right to left; then, left
    to right, the panel (C Y_k) W_{k+1} ((s n) x l_{k+1}) is orthogonalised by
    QR with diag(R) >= 0, its Q becomes core k and Q^T (C Y_k) is carried
    right; the last core takes C Y_{d-1}.  The K leg is never cut.  Y is
    returned unchanged when no bond rank exceeds ell.

    Sketch entries: gaussian_counter(seed, sketch_counter_base(t) + o_k + j),
    with core k's block at o_k = sum over 1 <= j < k of ell n_j ell, entry
    (c, i, c') at j = (c n_k + i) ell + c' (cores 1 .. d-2), and on the last
    core (c, i, kappa) at j = c n K + i K + kappa (the leading l_k x l_{k+1}
    block of an ell x n x ell layout is used).

    Not in the paper; parity of the GPU mode is against this function.  Pinned
    by exactness when ell reaches the chain's true bond ranks, by the skip rule,
    and by the dense projection it amounts to on tiny inputs.
    """
    Y = [np.asarray(y, dtype=np.float64) for y in Y]
    d = len(Y)
    P = [Y[0].shape[0]] + [y.shape[2] for y in Y]
    if d == 1 or max(P[1:d]) <= ell:
        return [y.copy() for y in Y]
    n = [y.shape[1] for y in Y]
    K = P[d]
    l = [None] + [min(ell, P[k]) for k in range(1, d)]
    base = sketch_counter_base(t)
    off = [0] * (d + 1)
    for k in range(1, d - 1):
        off[k + 1] = off[k] + ell * n[k] * ell

    def sketch_core(k):
        if k == d - 1:
            c, j = np.meshgrid(np.arange(l[k]), np.arange(n[k] * K), indexing="ij")
            idx = base + off[k] + c * (n[k] * K) + j
            return gaussian_counter_array(seed, idx.astype(np.uint64))       # (l_k, n K)
        c, i, c2 = np.meshgrid(np.arange(l[k]), np.arange(n[k]), np.arange(l[k + 1]),
                               indexing="ij")
        idx = base + off[k] + (c * n[k] + i) * ell + c2
        return gaussian_counter_array(seed, idx.astype(np.uint64))           # (l_k, n, l_k+1)

    W = [None] * (d + 1)
    W[d - 1] = Y[d - 1].reshape(P[d - 1], n[d - 1] * K) @ sketch_core(d - 1).T
    for k in range(d - 2, 0, -1):
        Sk = sketch_core(k)
        T1 = np.tensordot(Y[k], W[k + 1], axes=(2, 0))          # (P_k, n, l_k+1)
        W[k] = np.tensordot(T1, Sk, axes=([1, 2], [1, 2]))       # (P_k, l_k)
    out = []
    C = np.ones((1, 1))
    for k in range(d - 1):
        Zt = np.tensordot(C, Y[k], axes=(1, 0))                  # (s, n, P_{k+1})
        s_ = Zt.shape[0]
        Zr = Zt.reshape(s_ * n[k], P[k + 1])
        Q, _ = qr_nonneg(Zr @ W[k + 1])
        out.append(Q.reshape(s_, n[k], Q.shape[1]))
        C = Q.T @ Zr
    out.append(np.tensordot(C, Y[d - 1], axes=(1, 0)))
    return out


# --------------------------------------------------------------------------
# TNrSVD: Algorithm 5.1 with the subspace iteration of Algorithm 5.4
# --------------------------------------------------------------------------

@dataclass
class TNrSVDResult:
    sigma: np.ndarray                 # top-k singular values, descending
    U: List[np.ndarray]               # MPS-like cores, last (r, I_d, k)
    V: List[np.ndarray]               # MPS-like cores, last (s, J_d, k)
    sigma_all: np.ndarray             # all K values of the last-core SVD
    W: np.ndarray                     # K x K
    Q: List[np.ndarray]               # final orthonormal basis cores
    merged: List[np.ndarray]          # A after merging
    ranks: List[List[int]] = field(default_factory=list)  # per rounding
    Y0: Optional[List[np.ndarray]] = None   # first product A Omega (gauge free)


def tnrsvd(A_cores: Sequence[np.ndarray], k: int, p: int, q: int,
           omega: Optional[Tuple[Sequence[np.ndarray], np.ndarray]] = None,
           seed: Optional[int] = None, eps: float = 0.0, rmax: int = 0,
           merge: bool = True, sketch_rank: int = 0, sketch_seed: int = 0) -> TNrSVDResult:
    """TNrSVD of an MPO matrix A (Algorithm 5.1 in MPO form, Sec. 5).

    1. merge the last cores so that the K-core has I, J >= K (Sec. 6.3);
    2. Omega: rank-1 random MPO (lemma of Sec. 5.1), given or from ``seed``;
    3. Y = A Omega (Sec. 5.2); Q = ORTH(ROUND(Y)) (Algorithm 5.2 fused with
       rounding, Sec. 5.4);
    4. q times: Y = A^T Q, Q = ORTH(ROUND(Y)); Y = A Q, Q = ORTH(ROUND(Y))
       (Algorithm 5.4);
    5. B^T = A^T Q; ROUND and sweep it; SVD of the last core gives sigma, V
       and W (Algorithm 5.3 mirrored); U = Q W on the last core (Sec. 5.4);
    6. keep the first k = K - p values and vectors (oversampling, Sec. 5.1).

    sketch_rank > 0 (not in the paper): every product t = 0, 1, ... (Y = A
    Omega first, B^T last) goes through sketch_compress(., sketch_rank,
    sketch_seed, t) before its ROUND.
    """
    K = k + p
    A = [np.asarray(c, dtype=np.float64) for c in A_cores]
    rows = [c.shape[1] for c in A]
    cols = [c.shape[2] for c in A]
    if merge:
        m = merge_plan(rows, cols, K)
        A = merge_tail(A, m)
    else:
        if A[-1].shape[1] < K or A[-1].shape[2] < K:
            raise ValueError("last core smaller than K")
    cols_m = [c.shape[2] for c in A]
    if omega is None:
        if seed is None:
            raise ValueError("need omega or seed")
        omega = omega_from_seed(cols_m, K, seed)
    Om = omega_as_mps(*omega)
    ranks = []
    nprod = [0]

    def cut(X):
        if sketch_rank <= 0:
            return X
        t = nprod[0]
        nprod[0] += 1
        return sketch_compress(X, sketch_rank, sketch_seed, t)

    Y = mpo_times_mps(A, Om)
    Y0 = [y.copy() for y in Y]
    r = round_sweep(cut(Y), eps, rmax, "qr")
    ranks.append(r["ranks"])
    Q = r["cores"]
    for _ in range(q):
        Z = mpo_t_times_mps(A, Q)
        r = round_sweep(cut(Z), eps, rmax, "qr")
        ranks.append(r["ranks"])
        Y = mpo_times_mps(A, r["cores"])
        r = round_sweep(cut(Y), eps, rmax, "qr")
        ranks.append(r["ranks"])
        Q = r["cores"]
    Bt = mpo_t_times_mps(A, Q)
    r = round_sweep(cut(Bt), eps, rmax, "svd")
    ranks.append(r["ranks"])
    sig = r["sigma"]
    W = r["W"]
    V = r["cores"]
    U = [c.copy() for c in Q[:-1]]
    U.append(np.einsum("cxk,kj->cxj", Q[-1], W))
    Uk = U[:-1] + [U[-1][:, :, :k]]
    Vk = V[:-1] + [V[-1][:, :, :k]]
    return TNrSVDResult(sigma=sig[:k].copy(), U=Uk, V=Vk, sigma_all=sig, W=W,
                        Q=Q, merged=A, ranks=ranks, Y0=Y0)


def dense_rsvd(A: np.ndarray, Omega: np.ndarray, q: int):
    """Algorithm 5.1 on dense matrices with re-orthogonalisation (Algorithm 5.4).

    Y = A Omega, Q = qr(Y); q times {Z = A^T Q, Q_z = qr(Z); Y = A Q_z,
    Q = qr(Y)}; B = Q^T A = W S V^T; U = Q W.  Used only to pin the MPO
    pipeline on small matrices.
    """
    Q, _ = qr_nonneg(A @ Omega)
    for _ in range(q):
        Qz, _ = qr_nonneg(A.T @ Q)
        Q, _ = qr_nonneg(A @ Qz)
    B = Q.T @ A
    W, S, Vt = np.linalg.svd(B, full_matrices=False)
    return Q @ W, S, Vt.T


# --------------------------------------------------------------------------
# The paper's own orientation (K leg on the first core, right-to-left sweeps)
# --------------------------------------------------------------------------

def reverse_mpo(cores: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Reverse the core order of an MPO (swapping each core's rank legs)."""
    return [np.ascontiguousarray(np.transpose(c, (3, 1, 2, 0))) for c in cores[::-1]]


def _paper_round_orth(C: List[np.ndarray], eps: float, rmax: int, last: str):
    """Rounding + Algorithm 5.2 / 5.3 in the paper's orientation.

    Cores are (r, n, r') with the K leg stored as the FIRST core's left leg,
    shape (K, n_1, r_2).  Left-to-right QR orthogonalisation, then a
    right-to-left truncated-SVD sweep whose last step (core 1) is the
    K x (n_1 r_2) RQ or SVD of Algorithms 5.2 / 5.3.
    """
    C = [c.copy() for c in C]
    d = len(C)
    for i in range(d - 1):
        p, n, r2 = C[i].shape
        Q, R = qr_nonneg(C[i].reshape(p * n, r2))
        C[i] = Q.reshape(p, n, Q.shape[1])
        C[i + 1] = np.tensordot(R, C[i + 1], axes=(1, 0))
    nrm = float(np.linalg.norm(C[d - 1]))
    delta = eps * nrm / math.sqrt(d - 1) if d > 1 else 0.0
    T = np.ones((1, 1))
    for i in range(d - 1, 0, -1):
        M = np.tensordot(C[i], T, axes=(2, 0))
        p, n, s = M.shape
        # SVD of the p x (n s) unfolding; keep rows of Vt as the new core
        U, S, Vt = np.linalg.svd(M.reshape(p, n * s), full_matrices=False)
        rho = choose_rank(S, delta, rmax)
        C[i] = Vt[:rho].reshape(rho, n, s)
        T = U[:, :rho] * S[None, :rho]
    M = np.tensordot(C[0], T, axes=(2, 0))   # (K, n_1, s)
    K, n, s = M.shape
    A1 = M.reshape(K, n * s)
    if last == "qr":
        # A1 = R Q1 with Q1 orthonormal rows (RQ factorisation)
        L, Qr = lq_nonneg(A1)
        C[0] = Qr.reshape(Qr.shape[0], n, s)
        return C, L
    X, S, Vt = np.linalg.svd(A1, full_matrices=False)
    C[0] = Vt.reshape(Vt.shape[0], n, s)
    return C, S


def tnrsvd_paper_orientation(A_cores: Sequence[np.ndarray], k: int, p: int,
                             q: int, omega_first: np.ndarray,
                             omega_vecs: Sequence[np.ndarray],
                             eps: float = 0.0, rmax: int = 0) -> np.ndarray:
    """Singular values of TNrSVD with the K leg on the FIRST core (as printed).

    A_cores must already have a first core with I_1, J_1 >= K.  omega_first
    is J_1 x K, omega_vecs are the vectors of cores 2..d.  Returns the top k
    singular values.  Used to pin the mirrored orientation of ``tnrsvd``.
    """
    K = k + p
    A = [np.asarray(c, dtype=np.float64) for c in A_cores]
    d = len(A)

    def times(X, transpose):
        out = []
        for i, (a, x) in enumerate(zip(A, X)):
            R, I, J, R2 = a.shape
            r, n, r2 = x.shape
            if transpose:
                Z = np.einsum("axyb,cxe->acybe", a, x)
                out.append(Z.reshape(R * r, J, R2 * r2))
            else:
                Z = np.einsum("axyb,cye->acxbe", a, x)
                out.append(Z.reshape(R * r, I, R2 * r2))
        return out

    # The K leg rides on the first core's left leg: shape (K, J_1, 1).
    Om = [np.ascontiguousarray(omega_first.T).reshape(K, -1, 1)]
    Om += [np.asarray(v, dtype=np.float64).reshape(1, -1, 1) for v in omega_vecs]
    assert len(Om) == d
    Q, _ = _paper_round_orth(times(Om, False), eps, rmax, "qr")
    for _ in range(q):
        Qz, _ = _paper_round_orth(times(Q, True), eps, rmax, "qr")
        Q, _ = _paper_round_orth(times(Qz, False), eps, rmax, "qr")
    _, S = _paper_round_orth(times(Q, True), eps, rmax, "svd")
    return S[:k]


# --------------------------------------------------------------------------
# Complex-valued MPOs through the real embedding (the paper allows complex
# tensors; the embedding is a standard identity, not the paper's)
# --------------------------------------------------------------------------

def complex_to_real_mpo(cores: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Real MPO of the real form B of a complex MPO A: every complex number z on
    a bond becomes the 2 x 2 block phi(z) = [[Re z, -Im z], [Im z, Re z]]
    (phi(xy) = phi(x) phi(y), so bond products carry over).  Inner ranks double;
    the first core's new left component becomes the most significant digit of
    its row mode (I_1 -> 2 I_1) and the last core's new right component the most
    significant digit of its column mode (J_d -> 2 J_d).  B(i', j') with those
    digits s, t is phi(A(i, j))[s, t]: a row and column permutation of
    [[Re A, -Im A], [Im A, Re A]], whose singular values are A's, each twice.
    Pinned by LAPACK's complex SVD of the dense A.
    """
    d = len(cores)
    out = []
    for k, G in enumerate(cores):
        G = np.asarray(G, dtype=np.complex128)
        R0, I, J, R1 = G.shape
        E = np.zeros((R0, 2, I, J, R1, 2))
        E[:, 0, :, :, :, 0] = G.real
        E[:, 0, :, :, :, 1] = -G.imag
        E[:, 1, :, :, :, 0] = G.imag
        E[:, 1, :, :, :, 1] = G.real
        # bond index (a, s) -> 2 a + s
        E = E.transpose(0, 1, 2, 3, 4, 5)                     # (a, s, i, j, b, t)
        if k == 0:
            # s joins the row mode as its most significant digit: i' = s I + i
            E = E.reshape(1, 2, I, J, R1, 2).reshape(1, 2 * I, J, R1, 2)
        else:
            E = E.reshape(2 * R0, I, J, R1, 2)
        a0, Ii, Jj = E.shape[0], E.shape[1], E.shape[2]
        if k == d - 1:
            # t joins the column mode: j' = t J + j
            E = E.reshape(a0, Ii, Jj, 1, 2).transpose(0, 1, 4, 2, 3).reshape(a0, Ii, 2 * Jj, 1)
        else:
            E = E.reshape(a0, Ii, Jj, 2 * R1)
        out.append(np.ascontiguousarray(E))
    return out


def tnrsvd_complex(A_cores: Sequence[np.ndarray], k: int, p: int, q: int, **kw) -> np.ndarray:
    """Top-k singular values of a complex MPO: TNrSVD of its real form with
    k' = 2k, p' = 2p, then every other value (each appears twice)."""
    res = tnrsvd(complex_to_real_mpo(A_cores), 2 * k, 2 * p, q, **kw)
    return res.sigma[0::2].copy()


# --------------------------------------------------------------------------
# Gradient of the sum of the computed singular values (not in the paper)
# --------------------------------------------------------------------------

def merge_tail_adjoint(tail: Sequence[np.ndarray], dM: np.ndarray) -> List[np.ndarray]:
    """Adjoint of ``merge_tail`` over the cores ``tail``: given dL/dM for the
    merged core M, return dL/d(each core of ``tail``) by the chain rule through
    the pairwise merges (the forward chain is recomputed)."""
    tail = [np.asarray(c, dtype=np.float64) for c in tail]
    chain = [tail[0]]
    for c in tail[1:]:
        T = chain[-1]
        a, I1, J1, _ = T.shape
        _, I2, J2, b = c.shape
        chain.append(np.einsum("axyr,rXYb->aXxYyb", T, c).reshape(a, I2 * I1, J2 * J1, b))
    grads = [None] * len(tail)
    dT = np.asarray(dM, dtype=np.float64)
    for j in range(len(tail) - 1, 0, -1):
        T, c = chain[j - 1], tail[j]
        a, I1, J1, _ = T.shape
        _, I2, J2, b = c.shape
        dN = dT.reshape(a, I2, I1, J2, J1, b)
        grads[j] = np.einsum("aXxYyb,axyr->rXYb", dN, T)
        dT = np.einsum("aXxYyb,rXYb->axyr", dN, c)
    grads[0] = dT
    return grads


def sigma_sum_grad(A_cores: Sequence[np.ndarray], res: "TNrSVDResult",
                   dsigma: Optional[np.ndarray] = None) -> List[np.ndarray]:
    """Gradient of L = sum_j dsigma_j sigma_j (dsigma = 1 by default) with
    respect to the original cores of A, with the computed singular subspaces
    held fixed: dL/dA = sum_j dsigma_j u_j v_j^T, written into each core by
    contracting U and V with A's other cores (left environments E_i and right
    environments F_i), then through the merge of the trailing cores.

    This is the derivative of sum_j dsigma_j u_j^T A v_j at fixed (u_j, v_j);
    it equals the derivative of the pipeline's output (and of the exact
    singular values) when the subspace is exact, e.g. rank(A) <= K with no
    truncation.  Parity: pinned by the dense bilinear form and, in the exact
    case, by finite differences of the whole pipeline and by LAPACK's
    singular vectors.
    """
    A = [np.asarray(c, dtype=np.float64) for c in A_cores]
    M = res.merged
    dm = len(M)
    U, V = res.U, res.V
    k = U[-1].shape[2]
    w = np.ones(k) if dsigma is None else np.asarray(dsigma, dtype=np.float64)
    # every environment update is three two-operand contractions
    E = [np.ones((1, 1, 1))]
    for i in range(dm - 1):
        t1 = np.einsum("ras,rxR->axsR", E[i], U[i])
        t2 = np.einsum("axsR,axyb->ysRb", t1, M[i])
        E.append(np.einsum("ysRb,syS->RbS", t2, V[i]))
    F = np.zeros((k, 1, k))
    F[np.arange(k), 0, np.arange(k)] = w
    gm = [None] * dm
    for i in range(dm - 1, -1, -1):
        s1 = np.einsum("syS,RbS->Rbsy", V[i], F)
        t1 = np.einsum("ras,rxR->axsR", E[i], U[i])
        gm[i] = np.einsum("axsR,Rbsy->axyb", t1, s1)
        s2 = np.einsum("axyb,Rbsy->Raxs", M[i], s1)
        F = np.einsum("rxR,Raxs->ras", U[i], s2)
    m = len(A) - dm + 1
    return gm[:-1] + merge_tail_adjoint(A[dm - 1:], gm[-1]) if m > 1 else gm


# --------------------------------------------------------------------------
# Derivative of the whole pipeline (not in the paper): reverse mode through
# the products, the rounding sweeps, the last-core factorisations and the
# merge, with Omega fixed and the truncation ranks frozen at their forward
# values.
#
# Each rounding is differentiated through its Gram (environment) form, which
# computes the same map as ``round_sweep``:
#   right Grams  G_d = I_K,  G_i = sum_x Y_i[:, x, :] G_{i+1} Y_i[:, x, :]^T;
#   left to right, with T_0 = 1 and M_i = (T_i Y_i) reshaped (s_i n_i) x P_{i+1},
#   the kept left singular vectors of the i-th panel of ``round_sweep`` are the
#   top rho eigenvectors of H_i = M_i G_{i+1} M_i^T (that panel is M_i L_{i+1}
#   with L_{i+1} L_{i+1}^T = G_{i+1}); core i is U_rho, T_{i+1} = U_rho^T M_i;
#   the last core is the QR or SVD of M_{d-1} (s n x K) as in ``round_sweep``.
# Unlike the LQ factors of the right-to-left pass, this form stays
# differentiable when a product is rank deficient, which products of
# structured MPOs often are.
# --------------------------------------------------------------------------

def mpo_times_mps_adjoint(A, X, dY):
    """Adjoint of ``mpo_times_mps`` (bilinear): returns (dA, dX) for the
    cotangent dY of the product cores.
    dA[a,x,y,b] = sum_{c,e} dY[(a,c),x,(b,e)] X[c,y,e];
    dX[c,y,e] = sum_{a,x,b} dY[(a,c),x,(b,e)] A[a,x,y,b]."""
    dA, dX = [], []
    for a, x, g in zip(A, X, dY):
        R, I, J, R2 = a.shape
        r, _, r2 = x.shape
        g5 = np.asarray(g, dtype=np.float64).reshape(R, r, I, R2, r2)
        dA.append(np.einsum("acxbe,cye->axyb", g5, x))
        dX.append(np.einsum("acxbe,axyb->cye", g5, a))
    return dA, dX


def mpo_t_times_mps_adjoint(A, X, dZ):
    """Adjoint of ``mpo_t_times_mps``: (dA, dX) for the cotangent dZ.
    dA[a,x,y,b] = sum_{c,e} dZ[(a,c),y,(b,e)] X[c,x,e];
    dX[c,x,e] = sum_{a,y,b} dZ[(a,c),y,(b,e)] A[a,x,y,b]."""
    dA, dX = [], []
    for a, x, g in zip(A, X, dZ):
        R, I, J, R2 = a.shape
        r, _, r2 = x.shape
        g5 = np.asarray(g, dtype=np.float64).reshape(R, r, J, R2, r2)
        dA.append(np.einsum("acybe,cxe->axyb", g5, x))
        dX.append(np.einsum("acybe,axyb->cxe", g5, a))
    return dA, dX


def _signfix_cols(U: np.ndarray) -> np.ndarray:
    """Flip each column so that its entry of largest magnitude (the first on
    ties) is positive, as ``svd_signfix`` does for left singular vectors."""
    if U.shape[1] == 0:
        return U
    piv = np.argmax(np.abs(U), axis=0)
    sg = np.sign(U[piv, np.arange(U.shape[1])])
    sg[sg == 0] = 1.0
    return U * sg[None, :]


def round_sweep_gram(cores: Sequence[np.ndarray], eps: float, rmax: int, last: str = "qr",
                     ranks: Optional[Sequence[int]] = None):
    """The map of ``round_sweep`` computed in the Gram form described above,
    keeping every intermediate for ``round_sweep_gram_adjoint``.

    ranks: the bond ranks [1, rho_1, ..., rho_{d-1}] to keep (frozen, e.g. the
    ones ``round_sweep`` chose); without them the tail rule runs on the square
    roots of the eigenvalues, limited to the min(s n, rho') values the
    factorised panel has (rho' = the economy rank of the right-to-left pass).
    Same gauges as ``round_sweep`` (largest-magnitude entry of each kept
    vector positive; diag(R) >= 0), so its cores equal ``round_sweep``'s up to
    rounding; eigenvalues below ~1e-16 of the largest are not resolved, which
    only matters for ranks decided without ``ranks``.
    """
    Y = [np.asarray(c, dtype=np.float64) for c in cores]
    d = len(Y)
    if Y[0].shape[0] != 1:
        raise ValueError("first rank must be 1")
    K = Y[-1].shape[2]
    G = [None] * (d + 1)
    G[d] = np.eye(K)
    for i in range(d - 1, -1, -1):
        P, n, P2 = Y[i].shape
        T1 = Y[i].reshape(P * n, P2) @ G[i + 1]
        G[i] = T1.reshape(P, n * P2) @ Y[i].reshape(P, n * P2).T
    nrm = float(math.sqrt(max(G[0][0, 0], 0.0)))
    delta = eps * nrm / math.sqrt(d - 1) if d > 1 else 0.0
    econ = [0] * (d + 1)                       # economy ranks of the right-to-left pass
    econ[d] = K
    for i in range(d - 1, 0, -1):
        econ[i] = min(Y[i].shape[0], Y[i].shape[1] * econ[i + 1])
    T = np.ones((1, 1))
    rec = {"G": G, "T": [], "M": [], "U": [], "lam": [], "rho": [1], "Y": Y, "last": last,
           "K": K}
    out = []
    for i in range(d - 1):
        P, n, P2 = Y[i].shape
        s_ = T.shape[0]
        M = (T @ Y[i].reshape(P, n * P2)).reshape(s_ * n, P2)
        H = M @ G[i + 1] @ M.T
        H = 0.5 * (H + H.T)
        lam, U = np.linalg.eigh(H)
        lam, U = lam[::-1].copy(), U[:, ::-1].copy()
        if ranks is not None:
            rho = int(ranks[i + 1])
        else:
            nv = min(s_ * n, econ[i + 1])
            rho = choose_rank(np.sqrt(np.maximum(lam[:nv], 0.0)), delta, rmax)
        Ur = _signfix_cols(U[:, :rho])
        U = U.copy()
        U[:, :rho] = Ur
        rec["T"].append(T)
        rec["M"].append(M)
        rec["U"].append(U)
        rec["lam"].append(lam)
        rec["rho"].append(rho)
        out.append(Ur.reshape(s_, n, rho))
        T = Ur.T @ M
    P, n, _ = Y[d - 1].shape
    s_ = T.shape[0]
    M = (T @ Y[d - 1].reshape(P, n * K)).reshape(s_ * n, K)
    rec["T"].append(T)
    rec["M"].append(M)
    res = {"norm": nrm, "ranks": rec["rho"][:], "rec": rec}
    if last == "qr":
        Q, R = qr_nonneg(M)
        out.append(Q.reshape(s_, n, Q.shape[1]))
        res["R"] = R
        rec["Q"], rec["R"] = Q, R
    elif last == "svd":
        X, S, Wt = svd_signfix(M)
        out.append(X.reshape(s_, n, X.shape[1]))
        res["sigma"] = S
        res["W"] = Wt.T
        rec["X"], rec["S"], rec["Wt"] = X, S, Wt
    else:
        raise ValueError("last must be 'qr' or 'svd'")
    res["cores"] = out
    return res


def qr_adjoint(Q: np.ndarray, R: np.ndarray, dQ: np.ndarray, dR: Optional[np.ndarray] = None
               ) -> np.ndarray:
    """Cotangent of M for the economy QR M = Q R (m >= n, R invertible, diag(R) > 0):
    dM = (dQ + Q copyltu(R dR^T - dQ^T Q)) R^{-T}, copyltu(X) = the symmetric
    matrix whose lower triangle is X's (the result of differentiating Q^T Q = I
    and the triangularity of R)."""
    n = R.shape[0]
    C = -dQ.T @ Q
    if dR is not None:
        C = C + R @ dR.T
    S = np.tril(C) + np.tril(C, -1).T
    B = dQ + Q @ S
    # B R^{-T}: solve R X^T = B^T
    return np.linalg.solve(R, B.T).T if n else B


def round_sweep_gram_adjoint(rec, dcores: Optional[Sequence[np.ndarray]] = None,
                             dlast: Optional[np.ndarray] = None,
                             dsigma: Optional[np.ndarray] = None) -> List[np.ndarray]:
    """Reverse pass of ``round_sweep_gram``: the cotangents of its input cores
    from those of its outputs.

    dcores: cotangents of the output cores 0..d-2 (shapes (s, n, rho)), or None;
    dlast: cotangent of the last core's Q (mode 'qr', shape (s, n, K));
    dsigma: cotangent of sigma (mode 'svd'; the singular vectors are not used).
    Steps, last core first: the QR (``qr_adjoint``) or sigma_j = x_j^T M w_j
    (dM = sum_j dsigma_j x_j w_j^T); then for each core i from d-2 down to 0:
    T_{i+1} = U^T M gives dM += U dT, dU += M dT^T; the kept eigenvectors of
    H = M G M^T give dH = V (F o (V^T dU)) U^T with V all eigenvectors,
    F_aj = 1/(lam_j - lam_a) (a != j, zero on the diagonal); then
    dM += (dH + dH^T) M G, dG_{i+1} += M^T dH M, and M = T_i Y_i gives dT_i and
    dY_i.  Last, the right Grams in reverse (left to right):
    dY_i[:, x, :] += (dG_i + dG_i^T) Y_i[:, x, :] G_{i+1},
    dG_{i+1} += sum_x Y_i[:, x, :]^T dG_i Y_i[:, x, :].  The norm (and so the
    tolerance) only decides ranks, which are frozen: it has no cotangent.
    Requires distinct kept eigenvalues, separated from the discarded ones, and
    a last panel of full column rank (mode 'qr').
    """
    Y, G = rec["Y"], rec["G"]
    d = len(Y)
    K = rec["K"]
    dY = [np.zeros_like(y) for y in Y]
    dG = [np.zeros_like(g) if g is not None else None for g in G]
    # last core
    M = rec["M"][d - 1]
    T = rec["T"][d - 1]
    if rec["last"] == "qr":
        dQ = np.zeros_like(rec["Q"]) if dlast is None else np.asarray(dlast).reshape(rec["Q"].shape)
        dM = qr_adjoint(rec["Q"], rec["R"], dQ)
    else:
        ws = np.zeros(len(rec["S"]))
        if dsigma is not None:
            ws[:len(dsigma)] = dsigma
        dM = (rec["X"] * ws[None, :]) @ rec["Wt"]
    P, n, _ = Y[d - 1].shape
    s_ = T.shape[0]
    dMr = dM.reshape(s_, n * K)
    dT = dMr @ Y[d - 1].reshape(P, n * K).T
    dY[d - 1] += (T.T @ dMr).reshape(Y[d - 1].shape)
    for i in range(d - 2, -1, -1):
        M, T, U, lam = rec["M"][i], rec["T"][i], rec["U"][i], rec["lam"][i]
        rho = rec["rho"][i + 1]
        P, n, P2 = Y[i].shape
        s_ = T.shape[0]
        Ur = U[:, :rho]
        dU = np.zeros_like(Ur) if dcores is None else np.asarray(dcores[i]).reshape(Ur.shape).copy()
        dM = Ur @ dT
        dU += M @ dT.T
        diff = lam[None, :rho] - lam[:, None]           # lam_j - lam_a
        with np.errstate(divide="ignore"):
            F = np.where(np.arange(len(lam))[:, None] == np.arange(rho)[None, :], 0.0,
                         1.0 / np.where(diff == 0.0, np.inf, diff))
        dH = U @ (F * (U.T @ dU)) @ Ur.T
        dM += (dH + dH.T) @ M @ G[i + 1]
        dG[i + 1] += M.T @ dH @ M
        dMr = dM.reshape(s_, n * P2)
        Yr = Y[i].reshape(P, n * P2)
        dT = dMr @ Yr.T
        dY[i] += (T.T @ dMr).reshape(Y[i].shape)
    for i in range(1, d):
        P, n, P2 = Y[i].shape
        Sd = dG[i] + dG[i].T
        YG = (Y[i].reshape(P * n, P2) @ G[i + 1]).reshape(P, n * P2)
        dY[i] += (Sd @ YG).reshape(P, n, P2)
        if i + 1 < d:
            DY = (dG[i] @ Y[i].reshape(P, n * P2)).reshape(P * n, P2)
            dG[i + 1] += Y[i].reshape(P * n, P2).T @ DY
    return dY


def pipeline_grad(A_cores: Sequence[np.ndarray], k: int, p: int, q: int,
                  omega: Tuple[Sequence[np.ndarray], np.ndarray], eps: float = 0.0,
                  rmax: int = 0, dsigma: Optional[np.ndarray] = None,
                  ranks: Optional[List[List[int]]] = None) -> List[np.ndarray]:
    """Gradient of L = sum_{j<k} dsigma_j sigma_j (dsigma = 1 by default) of the
    TNrSVD pipeline ``tnrsvd`` with respect to the original cores of A, with
    Omega fixed and every rounding's bond ranks frozen (``ranks``, one list per
    rounding in the order of ``TNrSVDResult.ranks``; taken from a run of
    ``tnrsvd`` when not given).

    Forward, recomputed: merge; Y = A Omega; each rounding in its Gram form
    (``round_sweep_gram``) with the frozen ranks; Algorithm 5.4's products
    and roundings; B^T = A^T Q and its rounding with the last-core SVD.
    Backward: the same steps in reverse (``round_sweep_gram_adjoint``, the
    product adjoints, both contributing to dA), then the merge adjoint.
    Parity: pinned by central finite differences of ``tnrsvd`` and, where the
    computed subspace is exact, by the closed form sum_j u_j v_j^T.
    """
    K = k + p
    A0 = [np.asarray(c, dtype=np.float64) for c in A_cores]
    rows = [c.shape[1] for c in A0]
    cols = [c.shape[2] for c in A0]
    m = merge_plan(rows, cols, K)
    A = merge_tail(A0, m)
    if ranks is None:
        ranks = tnrsvd(A0, k, p, q, omega=omega, eps=eps, rmax=rmax).ranks
    if len(ranks) != 2 * q + 2:
        raise ValueError("one rank list per rounding is needed")
    Om = omega_as_mps(*omega)
    stages = []          # (op, X, rounding record)
    Y = mpo_times_mps(A, Om)
    r = round_sweep_gram(Y, eps, rmax, "qr", ranks=ranks[0])
    stages.append((0, Om, r["rec"]))
    Q = r["cores"]
    t = 1
    for _ in range(q):
        Z = mpo_t_times_mps(A, Q)
        r = round_sweep_gram(Z, eps, rmax, "qr", ranks=ranks[t])
        stages.append((1, Q, r["rec"]))
        Qz = r["cores"]
        Y = mpo_times_mps(A, Qz)
        r = round_sweep_gram(Y, eps, rmax, "qr", ranks=ranks[t + 1])
        stages.append((0, Qz, r["rec"]))
        Q = r["cores"]
        t += 2
    Bt = mpo_t_times_mps(A, Q)
    r = round_sweep_gram(Bt, eps, rmax, "svd", ranks=ranks[t])
    stages.append((1, Q, r["rec"]))
    w = np.ones(k) if dsigma is None else np.asarray(dsigma, dtype=np.float64)
    dA = [np.zeros_like(a) for a in A]
    dX_out = None            # cotangent of the basis produced by the stage below
    for si in range(len(stages) - 1, -1, -1):
        op, X, rec = stages[si]
        if rec["last"] == "svd":
            dP = round_sweep_gram_adjoint(rec, dsigma=w)
        else:
            dP = round_sweep_gram_adjoint(rec, dcores=dX_out[:-1], dlast=dX_out[-1])
        adj = mpo_times_mps_adjoint if op == 0 else mpo_t_times_mps_adjoint
        gA, gX = adj(A, X, dP)
        for j in range(len(A)):
            dA[j] += gA[j]
        dX_out = gX
    return dA[:-1] + merge_tail_adjoint(A0[len(A) - 1:], dA[-1]) if m > 1 else dA


# --------------------------------------------------------------------------
# Sparse matrix to MPO (Algorithm 4.1, Sec. 4.1)
# --------------------------------------------------------------------------

def sparse_to_mpo(coo_row: np.ndarray, coo_col: np.ndarray, coo_val: np.ndarray,
                  rows: Sequence[int], cols: Sequence[int]) -> List[np.ndarray]:
    """Algorithm 4.1 on a matrix given by its nonzero entries (COO).

    The partition into I_1 x J_1 blocks follows the Kronecker ordering
    A^(d) x ... x A^(1) (eq. (1): the first core carries the fastest index), so
    the block of entry (i, j) is (i // I_1, j // J_1) and its position at level
    k >= 2 is the k-th mixed-radix digit of that block index.  Every nonzero
    block X becomes the rank-1 MPO (X, E^(2), ..., E^(d)) with E^(k) the unit
    matrix of that digit pair, and the terms are summed (MPO addition), so the
    rank is the number of nonzero blocks (a lemma of Sec. 4.2).  Blocks are
    taken in increasing order of block_row * (J / J_1) + block_col.
    """
    d = len(rows)
    I1, J1 = rows[0], cols[0]
    nbc = int(np.prod(cols[1:])) if d > 1 else 1
    r = np.asarray(coo_row, dtype=np.int64)
    c = np.asarray(coo_col, dtype=np.int64)
    v = np.asarray(coo_val, dtype=np.float64)
    keys = (r // I1) * nbc + (c // J1)
    blocks = sorted(set(int(k) for k in keys[v != 0.0])) if len(v) else []
    mpo = None
    for key in blocks:
        br, bc = divmod(key, nbc)
        X = np.zeros((I1, J1))
        sel = keys == key
        np.add.at(X, (r[sel] % I1, c[sel] % J1), v[sel])
        term = [X.reshape(1, I1, J1, 1)]
        for k in range(1, d):
            E = np.zeros((rows[k], cols[k]))
            E[br % rows[k], bc % cols[k]] = 1.0
            br //= rows[k]
            bc //= cols[k]
            term.append(E.reshape(1, rows[k], cols[k], 1))
        mpo = term if mpo is None else mpo_add(mpo, term)
    if mpo is None:   # the zero matrix: one zero rank-1 term
        mpo = [np.zeros((1, rows[k], cols[k], 1)) for k in range(d)]
    return mpo


def round_mpo(cores: Sequence[np.ndarray], eps: float, rmax: int = 0) -> List[np.ndarray]:
    """SVD-based rounding of an MPO (Sec. 3): the MPS rounding of the chain
    whose core k has its row and column indices grouped into one index of
    size I_k J_k (C order, row index slower), i.e. round_sweep with a K leg of
    size 1.  Right-to-left LQ, then left-to-right truncated SVDs with tail
    delta = eps |A|_F / sqrt(d - 1); the last core keeps the remaining factor
    (Q R of its final QR).  Returns cores (r, I, J, r'), cores 1..d-1
    left-orthonormal with sign-fixed singular vectors.  Reading taken for the
    zero matrix (the paper does not treat it): all-zero rank-1 cores, whether
    every core is zero or only their product (|A|_F = 0 after the first pass).
    """
    d = len(cores)
    dims = [(c.shape[1], c.shape[2]) for c in cores]
    if not any(np.any(c) for c in cores):
        return [np.zeros((1, I, J, 1)) for (I, J) in dims]
    C = [np.asarray(c, dtype=np.float64).reshape(c.shape[0], c.shape[1] * c.shape[2], c.shape[3])
         for c in cores]
    out = round_sweep(C, eps, rmax, last="qr")
    if out["norm"] == 0.0:
        # a zero product of nonzero cores (e.g. one zero core): the same reading
        return [np.zeros((1, I, J, 1)) for (I, J) in dims]
    res = out["cores"]
    res[-1] = np.tensordot(res[-1], out["R"], axes=(2, 0))
    return [c.reshape(c.shape[0], I, J, c.shape[2]) for c, (I, J) in zip(res, dims)]
