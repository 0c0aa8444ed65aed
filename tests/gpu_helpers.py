"""Helpers shared by the GPU tests: staging workloads and comparing results.

Only test infrastructure: it may call the oracle (to compute expected values)
and the GPU binding (to compute the values under test); neither of those
imports this file.
"""

from __future__ import annotations

import numpy as np

from oracle import tnrsvd_oracle as o
import workloads as wl


def merged_cols(cores, K):
    rows = [c.shape[1] for c in cores]
    cols = [c.shape[2] for c in cores]
    m = o.merge_plan(rows, cols, K)
    return cols[: len(cols) - m] + [int(np.prod(cols[len(cols) - m:]))]


def omega_for(cores, K, seed):
    """Seeded Gaussian Omega factors in the merged layout (drawn by workloads)."""
    return wl.gaussian_omega(merged_cols(cores, K), K, seed)


def to_device(cores, dtype="f64"):
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    return [torch.as_tensor(np.ascontiguousarray(c), dtype=td).cuda() for c in cores]


def gpu_solve(cores, k, p, q, *, precision="f64", eps=0.0, rmax=0, omega=None, seed=0,
              input_dtype=None):
    """Run the whole pipeline through the C ABI; return (sigma, handle)."""
    from paper_1707_07803_amd import TNrSVD, omega_flat
    if input_dtype is None:
        input_dtype = "f64" if precision == "f64" else "f32"
    h = TNrSVD(to_device(cores, input_dtype), k, p, q, seed=seed, precision=precision,
               round_tol=eps, max_rank=rmax)
    if omega is not None:
        h.set_omega(omega_flat(*omega))
    sig = h.run()[0]
    return sig, h


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def cores_np(tensors):
    return [t.double().cpu().numpy() for t in tensors]
