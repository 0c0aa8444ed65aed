"""MI355X (gfx950) Tensor Network randomized SVD (arXiv 1707.07803).

The hot path -- MPO x random-MPO contraction, FP64 rounding + Householder QR
sweeps, projection and the small SVD of the last core -- runs in the HIP
kernels of ``libtnrsvd.so`` behind the C ABI of ``include/tnrsvd.h``.  This
package holds the build script and a thin ctypes binding.
"""

from .tnrsvd import (TNrSVD, TNrSVDError, TNrSVDFunction, solve, sparse_to_mpo, sparse_round,  # noqa: F401
                     round_mpo, complex_embed, solve_complex, mpo_add,
                     load_library, omega_flat, LIB_PATH, EXPORTS, PRECISIONS, ORIENTATIONS)

__all__ = ["TNrSVD", "TNrSVDError", "TNrSVDFunction", "solve", "sparse_to_mpo", "sparse_round", "round_mpo", "complex_embed", "solve_complex", "mpo_add", "load_library", "omega_flat", "LIB_PATH",
           "EXPORTS", "PRECISIONS", "ORIENTATIONS"]
