"""Thin ctypes binding of libtnrsvd.so (the C ABI declared in include/tnrsvd.h).

Argument marshalling only: every step of TNrSVD runs in the HIP kernels of the
library.  PyTorch provides device memory (input cores, output copies) and the
stream.  Loading fails loudly when the library has not been built; there is no
CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtnrsvd.so")

F64, F32, BF16 = 0, 1, 2
PRECISIONS = {"f64": F64, "f32": F32, "bf16": BF16}

# the C function names exported by the library, in header order
EXPORTS = [
    "tnrsvd_create", "tnrsvd_mult", "tnrsvd_orthogonalize", "tnrsvd_project",
    "tnrsvd_solve", "tnrsvd_run", "tnrsvd_run_graph", "tnrsvd_refine", "tnrsvd_backward",
    "tnrsvd_backward_frozen", "tnrsvd_autotune", "tnrsvd_autotune_sweeps",
    "tnrsvd_set_sweep_config",
    "tnrsvd_get_factor", "tnrsvd_copy_factor",
    "tnrsvd_get_omega", "tnrsvd_set_omega", "tnrsvd_get_ranks", "tnrsvd_destroy",
    "tnrsvd_profile", "tnrsvd_profile_read", "tnrsvd_get_product_ranks",
    "tnrsvd_sparse_to_mpo", "tnrsvd_sparse_to_mpo_noalloc", "tnrsvd_sparse_round", "tnrsvd_round_mpo", "tnrsvd_complex_embed", "tnrsvd_solve_complex", "tnrsvd_mpo_add", "tnrsvd_rounded_ranks",
    "tnrsvd_rounded_copy", "tnrsvd_rounded_destroy", "tnrsvd_last_error", "tnrsvd_version",
]

# kernel kinds reported by tnrsvd_profile_read
KERNELS = {"contract": 0, "rl_sweep": 1, "lr_sweep": 2, "form_u": 3, "load_omega": 4,
           "copy_y0": 5, "sketch": 6}

STATUS = {0: "OK", -1: "E_INVALID", -2: "E_SHAPE", -3: "E_STATE", -4: "E_NOMEM",
          -5: "E_DEVICE", -6: "E_NONFINITE"}


def _bucket(x: int, edges) -> str:
    for e in edges:
        if x <= e:
            return f"<={e}"
    return f">{edges[-1]}"


def sweep_shape_class(shapes, k: int, p: int, q: int, round_tol: float, max_rank: int,
                      sketch_rank: int, orientation: str) -> str:
    """The shape class a sweep launch choice is cached under: the batch size and
    the largest core count, mode and bond of the MPOs (bucketed), and the solve
    options that set the ranks of the products."""
    d = max(len(s) for s in shapes)
    n = max(max(c[1], c[2]) for s in shapes for c in s)
    r = max(max(c[0], c[3]) for s in shapes for c in s)
    return (f"batch{_bucket(len(shapes), [1, 16, 256, 4096])}|d{_bucket(d, [8, 16, 32, 64])}"
            f"|n{n}|R{_bucket(r, [4, 8, 16, 32, 64])}|K{k + p}|q{q}|rmax{max_rank}"
            f"|tol{'>0' if round_tol > 0 else '0'}|sketch{sketch_rank}|{orientation}")


def sweep_cache_path() -> str:
    return os.environ.get("TNRSVD_SWEEP_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "tnrsvd", "sweeps.json"))


def read_sweep_cache(path: str) -> dict:
    import json
    try:
        with open(path) as f:
            table = json.load(f)
    except (OSError, ValueError):
        return {}
    return {k: [int(v[0]), int(v[1])] for k, v in table.items()
            if isinstance(v, list) and len(v) == 2}


def write_sweep_cache(path: str, key: str, choice) -> None:
    """Add one entry (read, update, write to a temporary file, rename)."""
    import json
    table = read_sweep_cache(path)
    table[key] = [int(choice[0]), int(choice[1])]
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


class TNrSVDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Mpo(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int),
                ("rank", ctypes.POINTER(ctypes.c_int64)),
                ("rows", ctypes.POINTER(ctypes.c_int64)),
                ("cols", ctypes.POINTER(ctypes.c_int64)),
                ("core", ctypes.POINTER(ctypes.c_void_p)),
                ("dtype", ctypes.c_int)]


class _Opts(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("p", ctypes.c_int), ("q", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("precision", ctypes.c_int),
                ("round_tol", ctypes.c_double), ("max_rank", ctypes.c_int64),
                ("check_finite", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("orientation", ctypes.c_int), ("sketch_rank", ctypes.c_int)]

# where the K leg of Omega, Y, Q, U and V sits: "k_last" is the library's own
# layout, "k_first" the paper's (Sec. 5), reached by reading the MPO reversed
ORIENTATIONS = {"k_last": 0, "k_first": 1}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libtnrsvd.so and declare the C signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_1707_07803_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(path)
    H = ctypes.c_void_p
    I = ctypes.c_int
    L.tnrsvd_create.argtypes = [ctypes.POINTER(H), I, ctypes.POINTER(_Mpo), ctypes.POINTER(_Opts)]
    L.tnrsvd_mult.argtypes = [H, I]
    L.tnrsvd_orthogonalize.argtypes = [H]
    L.tnrsvd_project.argtypes = [H]
    L.tnrsvd_solve.argtypes = [H, ctypes.POINTER(ctypes.c_double)]
    L.tnrsvd_run.argtypes = [H, ctypes.POINTER(ctypes.c_double)]
    L.tnrsvd_run_graph.argtypes = [H, ctypes.POINTER(ctypes.c_double)]
    L.tnrsvd_refine.argtypes = [H, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
    L.tnrsvd_backward.argtypes = [H, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_void_p)]
    L.tnrsvd_backward_frozen.argtypes = L.tnrsvd_backward.argtypes
    L.tnrsvd_autotune.argtypes = [H, I, ctypes.POINTER(I)]
    L.tnrsvd_autotune_sweeps.argtypes = [H, I, ctypes.POINTER(I)]
    L.tnrsvd_set_sweep_config.argtypes = [H, ctypes.POINTER(I)]
    L.tnrsvd_get_factor.argtypes = [H, I, I, I, ctypes.POINTER(ctypes.c_void_p),
                                    ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(I)]
    L.tnrsvd_copy_factor.argtypes = [H, I, I, I, ctypes.c_void_p]
    L.tnrsvd_get_omega.argtypes = [H, I, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int64)]
    L.tnrsvd_set_omega.argtypes = [H, I, ctypes.POINTER(ctypes.c_double)]
    L.tnrsvd_get_ranks.argtypes = [H, I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(I)]
    L.tnrsvd_destroy.argtypes = [H]
    L.tnrsvd_profile.argtypes = [H, I]
    L.tnrsvd_profile_read.argtypes = [H, I, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64)]
    L.tnrsvd_get_product_ranks.argtypes = [H, I, ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_int64)]
    P64 = ctypes.POINTER(ctypes.c_int64)
    L.tnrsvd_sparse_to_mpo.argtypes = [I, P64, P64, ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, P64,
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]
    L.tnrsvd_sparse_to_mpo_noalloc.argtypes = L.tnrsvd_sparse_to_mpo.argtypes
    L.tnrsvd_sparse_round.argtypes = [I, P64, P64, ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, I,
                                      ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    L.tnrsvd_round_mpo.argtypes = [ctypes.POINTER(_Mpo), ctypes.c_double, I, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_void_p)]
    L.tnrsvd_complex_embed.argtypes = [ctypes.POINTER(_Mpo), ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.c_void_p]
    L.tnrsvd_solve_complex.argtypes = [ctypes.POINTER(_Mpo), ctypes.POINTER(_Opts),
                                       ctypes.POINTER(ctypes.c_double)]
    L.tnrsvd_mpo_add.argtypes = [ctypes.POINTER(_Mpo), ctypes.POINTER(_Mpo),
                                 ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]
    L.tnrsvd_rounded_ranks.argtypes = [ctypes.c_void_p, P64]
    L.tnrsvd_rounded_copy.argtypes = [ctypes.c_void_p, I, ctypes.c_void_p]
    L.tnrsvd_rounded_destroy.argtypes = [ctypes.c_void_p]
    L.tnrsvd_last_error.restype = ctypes.c_char_p
    L.tnrsvd_last_error.argtypes = []
    L.tnrsvd_version.restype = ctypes.c_char_p
    L.tnrsvd_version.argtypes = []
    for name in EXPORTS:
        if name not in ("tnrsvd_last_error", "tnrsvd_version"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        msg = _lib.tnrsvd_last_error().decode(errors="replace")
        raise TNrSVDError(status, msg)


def _dptr(a, *, ntype) -> List[float]:
    return (ntype * len(a))(*a)


class TNrSVD:
    """One handle of the C ABI: a batch of MPOs staged on the current HIP device.

    mpos: list of MPOs, each a list of device tensors (R, I, J, R') in float64
    or float32 (C-contiguous).  The cores are copied (and the trailing ones
    merged) inside the library, so the tensors may be freed afterwards.
    orientation "k_first" returns factors in the paper's layout (K leg on
    core 0, leading cores merged); ranks() and factor() follow it.
    """

    def __init__(self, mpos, k: int, p: int = 0, q: int = 0, seed: int = 0,
                 precision: str = "f64", round_tol: float = 0.0, max_rank: int = 0,
                 check_finite: bool = False, stream=None, orientation: str = "k_last",
                 sketch_rank: int = 0):
        import torch
        L = load_library()
        if isinstance(mpos[0], torch.Tensor):
            mpos = [mpos]
        self.k, self.p, self.q = k, p, q
        self.K = k + p
        self.batch = len(mpos)
        self.precision = precision
        self._shape_class = sweep_shape_class(
            [[tuple(int(x) for x in c.shape) for c in cores] for cores in mpos], k, p, q,
            float(round_tol), int(max_rank), int(sketch_rank), orientation)
        keep = []
        structs = (_Mpo * self.batch)()
        for b, cores in enumerate(mpos):
            st, held = _mpo_struct(cores)
            structs[b] = st
            keep += held
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        opts = _Opts(k=k, p=p, q=q, seed=seed, precision=PRECISIONS[precision],
                     round_tol=float(round_tol), max_rank=int(max_rank),
                     check_finite=1 if check_finite else 0,
                     stream=ctypes.c_void_p(stream.cuda_stream),
                     orientation=ORIENTATIONS[orientation], sketch_rank=int(sketch_rank))
        self.orientation = orientation
        h = ctypes.c_void_p()
        _check(L.tnrsvd_create(ctypes.byref(h), self.batch, structs, ctypes.byref(opts)))
        self._h = h
        self._lib = L

    # -- Algorithm 5.4 / 5.1 steps ------------------------------------------
    def mult(self, op: int):
        _check(self._lib.tnrsvd_mult(self._h, op))

    def orthogonalize(self):
        _check(self._lib.tnrsvd_orthogonalize(self._h))

    def project(self):
        _check(self._lib.tnrsvd_project(self._h))

    def solve(self, want_sigma: bool = True) -> Optional[np.ndarray]:
        if not want_sigma:
            _check(self._lib.tnrsvd_solve(self._h, None))
            return None
        out = np.zeros(self.batch * self.k, dtype=np.float64)
        _check(self._lib.tnrsvd_solve(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out.reshape(self.batch, self.k)

    def run(self, want_sigma: bool = True) -> Optional[np.ndarray]:
        if not want_sigma:
            _check(self._lib.tnrsvd_run(self._h, None))
            return None
        out = np.zeros(self.batch * self.k, dtype=np.float64)
        _check(self._lib.tnrsvd_run(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out.reshape(self.batch, self.k)

    def refine(self, round_tol: float = 0.0, want_sigma: bool = True) -> Optional[np.ndarray]:
        """One FP32 power step + projection + solve from the basis of a BF16 solve."""
        if not want_sigma:
            _check(self._lib.tnrsvd_refine(self._h, float(round_tol), None))
            return None
        out = np.zeros(self.batch * self.k, dtype=np.float64)
        _check(self._lib.tnrsvd_refine(self._h, float(round_tol),
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out.reshape(self.batch, self.k)

    def backward(self, dsigma, grads, frozen: bool = False) -> None:
        """tnrsvd_backward: write d(sum_j dsigma_j sigma_j)/d(core) of the last solve
        (the whole pipeline, Omega and the rounding ranks fixed) into the device
        tensors ``grads`` (one per original core of every MPO, in order).
        frozen=True: tnrsvd_backward_frozen, the derivative at fixed singular
        vectors instead."""
        w = None
        if dsigma is not None:
            w = np.ascontiguousarray(np.asarray(dsigma, dtype=np.float64).reshape(-1))
            if w.size != self.batch * self.k:
                raise TNrSVDError(-1, "dsigma must hold batch * k values")
        for g in grads:
            if not g.is_cuda or not g.is_contiguous():
                raise TNrSVDError(-1, "gradients must be contiguous device tensors")
        ptrs = (ctypes.c_void_p * len(grads))(*[g.data_ptr() for g in grads])
        fn = self._lib.tnrsvd_backward_frozen if frozen else self._lib.tnrsvd_backward
        _check(fn(
            self._h, None if w is None else w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ptrs))

    def autotune(self, reps: int = 5) -> dict:
        """tnrsvd_autotune: pick the contraction launch shapes for this handle."""
        out = (ctypes.c_int * 4)()
        _check(self._lib.tnrsvd_autotune(self._h, int(reps), out))
        return {"A_X": {"threads": out[0], "blocks_per_core_cap": out[1]},
                "At_X": {"threads": out[2], "blocks_per_core_cap": out[3]}}

    def set_sweep_config(self, choice) -> None:
        """tnrsvd_set_sweep_config: apply a sweep launch choice {wmin, lpt}."""
        arr = (ctypes.c_int * 2)(int(choice[0]), int(choice[1]))
        _check(self._lib.tnrsvd_set_sweep_config(self._h, arr))

    def autotune_sweeps(self, reps: int = 1, cache: Optional[str] = "default") -> dict:
        """tnrsvd_autotune_sweeps, with a cache of choices keyed by the shape class,
        precision and device architecture (sweep_cache_key).  cache: a JSON file
        path, "default" (TNRSVD_SWEEP_CACHE or ~/.cache/tnrsvd/sweeps.json) or None
        (always time).  Returns {"wmin", "lpt", "key", "cached"}."""
        path = sweep_cache_path() if cache == "default" else cache
        key = self.sweep_cache_key()
        table = read_sweep_cache(path) if path else {}
        if key in table:
            choice = table[key]
            self.set_sweep_config(choice)
            return {"wmin": choice[0], "lpt": choice[1], "key": key, "cached": True}
        out = (ctypes.c_int * 2)()
        _check(self._lib.tnrsvd_autotune_sweeps(self._h, int(reps), out))
        choice = [int(out[0]), int(out[1])]
        if path:
            write_sweep_cache(path, key, choice)
        return {"wmin": choice[0], "lpt": choice[1], "key": key, "cached": False}

    def sweep_cache_key(self) -> str:
        import torch
        arch = getattr(torch.cuda.get_device_properties(torch.cuda.current_device()),
                       "gcnArchName", "unknown").split(":")[0]
        return f"{arch}|{self.precision}|{self._shape_class}"

    def run_graph(self, want_sigma: bool = True) -> Optional[np.ndarray]:
        """tnrsvd_run captured once into a HIP graph, replayed on later calls."""
        if not want_sigma:
            _check(self._lib.tnrsvd_run_graph(self._h, None))
            return None
        out = np.zeros(self.batch * self.k, dtype=np.float64)
        _check(self._lib.tnrsvd_run_graph(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out.reshape(self.batch, self.k)

    # -- getters --------------------------------------------------------------
    def ranks(self, b: int = 0) -> List[int]:
        dm = ctypes.c_int()
        _check(self._lib.tnrsvd_get_ranks(self._h, b, None, ctypes.byref(dm)))
        buf = (ctypes.c_int64 * (dm.value + 1))()
        _check(self._lib.tnrsvd_get_ranks(self._h, b, buf, ctypes.byref(dm)))
        return list(buf)

    def d_merged(self, b: int = 0) -> int:
        dm = ctypes.c_int()
        _check(self._lib.tnrsvd_get_ranks(self._h, b, None, ctypes.byref(dm)))
        return dm.value

    def factor(self, which: int, b: int = 0):
        """Copies of the cores of U (0), V (1), the current basis (2) or Y = A Omega (3)."""
        import torch
        out = []
        for core in range(self.d_merged(b)):
            ptr = ctypes.c_void_p()
            shape = (ctypes.c_int64 * 4)()
            dt = ctypes.c_int()
            _check(self._lib.tnrsvd_get_factor(self._h, b, which, core, ctypes.byref(ptr), shape,
                                               ctypes.byref(dt)))
            tdt = {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16}[dt.value]
            t = torch.empty((shape[0], shape[1], shape[2]), dtype=tdt, device="cuda")
            _check(self._lib.tnrsvd_copy_factor(self._h, b, which, core, ctypes.c_void_p(t.data_ptr())))
            out.append(t)
        return out

    def omega(self, b: int = 0) -> np.ndarray:
        n = ctypes.c_int64()
        _check(self._lib.tnrsvd_get_omega(self._h, b, None, ctypes.byref(n)))
        buf = np.zeros(n.value, dtype=np.float64)
        _check(self._lib.tnrsvd_get_omega(self._h, b, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          ctypes.byref(n)))
        return buf

    def set_omega(self, values, b: int = 0):
        buf = np.ascontiguousarray(values, dtype=np.float64)
        n = ctypes.c_int64()
        _check(self._lib.tnrsvd_get_omega(self._h, b, None, ctypes.byref(n)))
        if buf.size != n.value:
            raise TNrSVDError(-2, f"Omega needs {n.value} values, got {buf.size}")
        _check(self._lib.tnrsvd_set_omega(self._h, b, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def product_ranks(self, b: int = 0):
        """(P_0..P_d, rho_0..rho_d) of the last product and of its right-to-left sweep."""
        d = self.d_merged(b)
        P = (ctypes.c_int64 * (d + 1))()
        R = (ctypes.c_int64 * (d + 1))()
        _check(self._lib.tnrsvd_get_product_ranks(self._h, b, P, R))
        return list(P), list(R)

    def profile(self, enable: bool = True):
        _check(self._lib.tnrsvd_profile(self._h, 1 if enable else 0))

    def profile_read(self, kernel: str):
        """(total ms, launches) of one kernel kind since profiling was enabled."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(self._lib.tnrsvd_profile_read(self._h, KERNELS[kernel], ctypes.byref(ms),
                                             ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.tnrsvd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def omega_flat(vecs: Sequence[np.ndarray], last: np.ndarray) -> np.ndarray:
    """Concatenate Omega's factors in the order tnrsvd_set_omega expects."""
    return np.concatenate([np.ravel(v) for v in vecs] + [np.ravel(np.asarray(last))])


def solve(cores, k: int, p: int = 0, q: int = 0, seed: int = 0, precision: str = "f64",
          round_tol: float = 0.0, max_rank: int = 0, omega=None):
    """One TNrSVD solve: returns (sigma[k], U cores, V cores) with U, V in FP64."""
    with TNrSVD(cores, k, p, q, seed, precision, round_tol, max_rank) as h:
        if omega is not None:
            h.set_omega(omega)
        sig = h.run()[0]
        U = h.factor(0)
        V = h.factor(1)
    U[-1] = U[-1][:, :, :k].contiguous()
    V[-1] = V[-1][:, :, :k].contiguous()
    return sig, U, V


def sparse_to_mpo(rows, cols, coo_row, coo_col, coo_val, noalloc=False):
    """Algorithm 4.1: the MPO cores of a sparse matrix given in COO form.

    rows, cols: mode sizes I_1..I_d, J_1..J_d (eq. (1) ordering, first core
    fastest).  coo_row, coo_col: int64 device tensors; coo_val: float64 device
    tensor (same length).  Returns d float64 device tensors (R, I_k, J_k, R')
    of rank R = number of nonzero I_1 x J_1 blocks, computed by
    tnrsvd_sparse_to_mpo on the current stream (noalloc=True: by
    tnrsvd_sparse_to_mpo_noalloc, whose scratch is the library's static
    device array; the cores are still allocated here, by torch).
    """
    import torch

    L = load_library()
    d = len(rows)
    if len(cols) != d:
        raise ValueError("rows and cols differ in length")
    rr = _dptr([int(x) for x in rows], ntype=ctypes.c_int64)
    cc = _dptr([int(x) for x in cols], ntype=ctypes.c_int64)
    nnz = int(coo_val.numel())
    for t, dt in ((coo_row, torch.int64), (coo_col, torch.int64), (coo_val, torch.float64)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous() or t.numel() != nnz:
            raise ValueError("COO arrays must be contiguous device tensors of equal length "
                             "(int64 indices, float64 values)")
    dev = coo_val.device
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    args = (ctypes.c_void_p(coo_row.data_ptr()), ctypes.c_void_p(coo_col.data_ptr()),
            ctypes.c_void_p(coo_val.data_ptr()))
    fn = L.tnrsvd_sparse_to_mpo_noalloc if noalloc else L.tnrsvd_sparse_to_mpo
    nb = ctypes.c_int64(0)
    _check(fn(d, rr, cc, nnz, *args, ctypes.byref(nb), None, stream))
    R = nb.value
    shapes = [(1 if k == 0 else R, rows[k], cols[k], 1 if k == d - 1 else R) for k in range(d)]
    cores = [torch.empty(s, dtype=torch.float64, device=dev) for s in shapes]
    ptrs = (ctypes.c_void_p * d)(*[c.data_ptr() for c in cores])
    _check(fn(d, rr, cc, nnz, *args, ctypes.byref(nb), ptrs, stream))
    return cores


def _coo_args(rows, cols, coo_row, coo_col, coo_val):
    import torch
    d = len(rows)
    if len(cols) != d:
        raise ValueError("rows and cols differ in length")
    nnz = int(coo_val.numel())
    for t, dt in ((coo_row, torch.int64), (coo_col, torch.int64), (coo_val, torch.float64)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous() or t.numel() != nnz:
            raise ValueError("COO arrays must be contiguous device tensors of equal length "
                             "(int64 indices, float64 values)")
    rr = _dptr([int(x) for x in rows], ntype=ctypes.c_int64)
    cc = _dptr([int(x) for x in cols], ntype=ctypes.c_int64)
    ptrs = (ctypes.c_void_p(coo_row.data_ptr()), ctypes.c_void_p(coo_col.data_ptr()),
            ctypes.c_void_p(coo_val.data_ptr()))
    stream = ctypes.c_void_p(torch.cuda.current_stream(coo_val.device).cuda_stream)
    return d, rr, cc, nnz, ptrs, stream


def sparse_round(rows, cols, coo_row, coo_col, coo_val, round_tol: float, max_rank: int = 0):
    """SVD-based rounding (Sec. 3) of the MPO that Algorithm 4.1 builds from a
    COO matrix, computed by tnrsvd_sparse_round on the current stream.

    Returns the rounded cores as float64 device tensors (r_k, I_k, J_k, r_{k+1}),
    the first d - 1 left-orthonormal.
    """
    import torch

    L = load_library()
    d, rr, cc, nnz, ptrs, stream = _coo_args(rows, cols, coo_row, coo_col, coo_val)
    h = ctypes.c_void_p()
    _check(L.tnrsvd_sparse_round(d, rr, cc, nnz, *ptrs, float(round_tol), int(max_rank), stream,
                                 ctypes.byref(h)))
    return _take_rounded(L, h, rows, cols, coo_val.device)


def _take_rounded(L, h, rows, cols, device):
    """Copy the cores of a rounded-MPO handle into new device tensors, then free it."""
    import torch
    d = len(rows)
    try:
        ranks = (ctypes.c_int64 * (d + 1))()
        _check(L.tnrsvd_rounded_ranks(h, ranks))
        cores = []
        for k in range(d):
            t = torch.empty((ranks[k], rows[k], cols[k], ranks[k + 1]), dtype=torch.float64,
                            device=device)
            _check(L.tnrsvd_rounded_copy(h, k, ctypes.c_void_p(t.data_ptr())))
            cores.append(t)
    finally:
        L.tnrsvd_rounded_destroy(h)
    return cores


def round_mpo(cores, round_tol: float, max_rank: int = 0):
    """SVD-based rounding (Sec. 3) of an MPO given as device tensors (r, I, J, r')
    in float64 or float32, computed by tnrsvd_round_mpo on the current stream.

    Returns float64 device tensors, the first d - 1 cores left-orthonormal.
    """
    import torch
    L = load_library()
    st, keep = _mpo_struct(cores)
    h = ctypes.c_void_p()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _check(L.tnrsvd_round_mpo(ctypes.byref(st), float(round_tol), int(max_rank), stream,
                              ctypes.byref(h)))
    del keep
    return _take_rounded(L, h, [int(c.shape[1]) for c in cores], [int(c.shape[2]) for c in cores],
                         cores[0].device)


def complex_embed(cores):
    """Real form of a complex MPO (device tensors (R, I, J, R') of complex128 or
    complex64), computed by tnrsvd_complex_embed: float64 / float32 device
    tensors with the inner ranks doubled, 2 I on the first core and 2 J on the
    last.  Its singular values are the complex matrix's, each twice."""
    import torch
    L = load_library()
    if cores[0].dtype not in (torch.complex128, torch.complex64):
        raise TNrSVDError(-1, "cores must be complex128 or complex64")
    real = [torch.view_as_real(c.contiguous()) for c in cores]      # (..., 2) interleaved
    rdt = torch.float64 if cores[0].dtype == torch.complex128 else torch.float32
    d = len(cores)
    rank = [int(cores[0].shape[0])] + [int(c.shape[3]) for c in cores]
    rows = [int(c.shape[1]) for c in cores]
    cols = [int(c.shape[2]) for c in cores]
    st = _Mpo()
    ra = (ctypes.c_int64 * (d + 1))(*rank)
    ro = (ctypes.c_int64 * d)(*rows)
    co = (ctypes.c_int64 * d)(*cols)
    pt = (ctypes.c_void_p * d)(*[c.data_ptr() for c in real])
    st.d, st.rank, st.rows, st.cols, st.core = d, ra, ro, co, pt
    st.dtype = F64 if rdt == torch.float64 else F32
    outs = []
    for k in range(d):
        shape = (1 if k == 0 else 2 * rank[k], (2 if k == 0 else 1) * rows[k],
                 (2 if k == d - 1 else 1) * cols[k], 1 if k == d - 1 else 2 * rank[k + 1])
        outs.append(torch.empty(shape, dtype=rdt, device=cores[0].device))
    op = (ctypes.c_void_p * d)(*[t.data_ptr() for t in outs])
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _check(L.tnrsvd_complex_embed(ctypes.byref(st), op, stream))
    return outs


def _mpo_view(cores, dtype):
    """A tnrsvd_mpo describing device tensors `cores` (kept alive by the caller)."""
    d = len(cores)
    st = _Mpo()
    keep = ((ctypes.c_int64 * (d + 1))(*([int(cores[0].shape[0])] + [int(c.shape[3]) for c in cores])),
            (ctypes.c_int64 * d)(*[int(c.shape[1]) for c in cores]),
            (ctypes.c_int64 * d)(*[int(c.shape[2]) for c in cores]),
            (ctypes.c_void_p * d)(*[c.data_ptr() for c in cores]))
    st.d, st.rank, st.rows, st.cols, st.core = d, *keep
    st.dtype = dtype
    return st, keep


def mpo_add(a, b):
    """The MPO of A + B (device tensors (r, I, J, r'), both float64 or both
    float32, equal modes), computed by tnrsvd_mpo_add: ranks add, inner cores
    block diagonal.  Returns new device tensors; round them with round_mpo."""
    import torch
    L = load_library()
    if len(a) != len(b) or not a:
        raise TNrSVDError(-2, "both MPOs need the same number of cores")
    if a[0].dtype not in (torch.float64, torch.float32) or any(
            c.dtype != a[0].dtype for c in list(a) + list(b)):
        raise TNrSVDError(-1, "cores must all be float64 or all float32")
    a = [c.contiguous() for c in a]
    b = [c.contiguous() for c in b]
    dt = F64 if a[0].dtype == torch.float64 else F32
    sa, ka = _mpo_view(a, dt)
    sb, kb = _mpo_view(b, dt)
    d = len(a)
    outs = []
    for k in range(d):
        left = 1 if k == 0 else int(a[k].shape[0] + b[k].shape[0])
        right = 1 if k == d - 1 else int(a[k].shape[3] + b[k].shape[3])
        outs.append(torch.empty((left, int(a[k].shape[1]), int(a[k].shape[2]), right),
                                dtype=a[0].dtype, device=a[0].device))
    op = (ctypes.c_void_p * d)(*[t.data_ptr() for t in outs])
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _check(L.tnrsvd_mpo_add(ctypes.byref(sa), ctypes.byref(sb), op, stream))
    return outs


def solve_complex(cores, k: int, p: int = 0, q: int = 0, seed: int = 0, precision: str = "f64",
                  round_tol: float = 0.0, max_rank: int = 0, sketch_rank: int = 0):
    """Top-k singular values of a complex MPO (device tensors (R, I, J, R') of
    complex128 or complex64) by tnrsvd_solve_complex: the library embeds it in
    its real form, solves that with k' = 2k and p' = 2p and returns every other
    value."""
    import torch
    L = load_library()
    if cores[0].dtype not in (torch.complex128, torch.complex64):
        raise TNrSVDError(-1, "cores must be complex128 or complex64")
    real = [torch.view_as_real(c.contiguous()) for c in cores]      # (..., 2) interleaved
    d = len(cores)
    st = _Mpo()
    ra = (ctypes.c_int64 * (d + 1))(*([int(cores[0].shape[0])] + [int(c.shape[3]) for c in cores]))
    ro = (ctypes.c_int64 * d)(*[int(c.shape[1]) for c in cores])
    co = (ctypes.c_int64 * d)(*[int(c.shape[2]) for c in cores])
    pt = (ctypes.c_void_p * d)(*[c.data_ptr() for c in real])
    st.d, st.rank, st.rows, st.cols, st.core = d, ra, ro, co, pt
    st.dtype = F64 if cores[0].dtype == torch.complex128 else F32
    stream = torch.cuda.current_stream()
    opts = _Opts(k=k, p=p, q=q, seed=seed, precision=PRECISIONS[precision],
                 round_tol=float(round_tol), max_rank=int(max_rank), check_finite=0,
                 stream=ctypes.c_void_p(stream.cuda_stream), orientation=0,
                 sketch_rank=int(sketch_rank))
    out = np.zeros(k, dtype=np.float64)
    _check(L.tnrsvd_solve_complex(ctypes.byref(st), ctypes.byref(opts),
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def _mpo_struct(cores):
    """A tnrsvd_mpo describing the device tensors ``cores`` (checked for shape,
    dtype and layout); returns it with the arrays it points to."""
    import torch
    ds = {c.dtype for c in cores}
    if len(ds) != 1 or next(iter(ds)) not in (torch.float64, torch.float32):
        raise TNrSVDError(-1, "cores must all be float64 or all float32")
    for c in cores:
        if not c.is_cuda or not c.is_contiguous() or c.dim() != 4:
            raise TNrSVDError(-1, "cores must be contiguous 4-way device tensors")
    d = len(cores)
    rank = [int(cores[0].shape[0])] + [int(c.shape[3]) for c in cores]
    for i in range(1, d):
        if int(cores[i].shape[0]) != rank[i]:
            raise TNrSVDError(-2, f"rank mismatch between cores {i - 1} and {i}")
    ra = (ctypes.c_int64 * (d + 1))(*rank)
    ro = (ctypes.c_int64 * d)(*[int(c.shape[1]) for c in cores])
    co = (ctypes.c_int64 * d)(*[int(c.shape[2]) for c in cores])
    pt = (ctypes.c_void_p * d)(*[c.data_ptr() for c in cores])
    st = _Mpo()
    st.d = d
    st.rank = ra
    st.rows = ro
    st.cols = co
    st.core = pt
    st.dtype = F64 if cores[0].dtype == torch.float64 else F32
    return st, [ra, ro, co, pt, cores]


def _autograd_function():
    import torch

    from torch.autograd.function import once_differentiable

    class TNrSVDFunction(torch.autograd.Function):
        """sigma_top_k = TNrSVDFunction.apply(options, *cores) for one MPO.

        Forward: one solve in the library (contractions, FP64 sweeps, final SVD).
        Backward: tnrsvd_backward with the incoming gradient of sigma -- the
        derivative of the whole solve with Omega and the rounding ranks held
        fixed (see include/tnrsvd.h).  Differentiable once: the handle is
        released by the backward, or when the graph is dropped without one.
        ``options`` is a dict of TNrSVD keyword arguments (k, p, q, seed,
        precision, round_tol, max_rank).
        """

        @staticmethod
        def forward(ctx, options, *cores):
            import weakref
            h = TNrSVD([c.detach().contiguous() for c in cores], **options)
            sig = h.run()[0]
            ctx.h = h
            ctx.like = [(c.shape, c.dtype) for c in cores]
            weakref.finalize(ctx, h.close)
            return torch.as_tensor(sig, dtype=torch.float64, device=cores[0].device)

        @staticmethod
        @once_differentiable
        def backward(ctx, gsig):
            h = ctx.h
            if h is None or getattr(h, "_h", None) is None:
                raise RuntimeError("TNrSVDFunction can be differentiated once per forward "
                                   "(its solve handle has been released)")
            grads = [torch.empty(sh, dtype=dt, device="cuda") for sh, dt in ctx.like]
            h.backward(gsig.detach().to("cpu", torch.float64).numpy(), grads)
            h.close()
            ctx.h = None
            return (None, *grads)

    return TNrSVDFunction


class _Lazy:
    def __init__(self):
        self._f = None

    def apply(self, *args):
        if self._f is None:
            self._f = _autograd_function()
        return self._f.apply(*args)


TNrSVDFunction = _Lazy()
