"""The C-ABI library loads and exports every function include/tnrsvd.h declares.

CPU only: loading the shared library does not touch a GPU, and no entry point
is called except tnrsvd_version and tnrsvd_last_error, which do no device work.
"""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tnrsvd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tnrsvd_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1707_07803_amd import LIB_PATH
    if not os.path.exists(LIB_PATH):
        from paper_1707_07803_amd import build
        build.build()
    return ctypes.CDLL(LIB_PATH)


def test_header_declares_the_boundary():
    names = declared_functions()
    for core in ("tnrsvd_create", "tnrsvd_mult", "tnrsvd_orthogonalize", "tnrsvd_project",
                 "tnrsvd_solve", "tnrsvd_destroy"):
        assert core in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"declared in tnrsvd.h but not exported: {missing}"


def test_binding_declares_every_symbol():
    from paper_1707_07803_amd import EXPORTS
    assert sorted(EXPORTS) == declared_functions()


def test_version_and_error_string_without_gpu(lib):
    lib.tnrsvd_version.restype = ctypes.c_char_p
    lib.tnrsvd_last_error.restype = ctypes.c_char_p
    assert lib.tnrsvd_version().decode().startswith("tnrsvd")
    assert isinstance(lib.tnrsvd_last_error(), bytes)


def test_sparse_to_mpo_rejects_bad_arguments_on_the_host(lib):
    """Argument checks of tnrsvd_sparse_to_mpo run before any device call."""
    f = lib.tnrsvd_sparse_to_mpo
    P64 = ctypes.POINTER(ctypes.c_int64)
    f.argtypes = [ctypes.c_int, P64, P64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_void_p, P64, ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]
    f.restype = ctypes.c_int
    A2 = ctypes.c_int64 * 2
    nb = ctypes.c_int64(0)
    one = ctypes.c_void_p(8)      # never dereferenced: every case fails first
    cases = [
        ((0, A2(2, 2), A2(2, 2), 0, None, None, None, ctypes.byref(nb), None, None), -2),
        ((2, None, A2(2, 2), 0, None, None, None, ctypes.byref(nb), None, None), -1),
        ((2, A2(2, 2), A2(2, 2), -1, None, None, None, ctypes.byref(nb), None, None), -2),
        ((2, A2(2, 2), A2(2, 2), 1 << 31, one, one, one, ctypes.byref(nb), None, None), -2),
        ((2, A2(2, 2), A2(2, 2), 3, None, one, one, ctypes.byref(nb), None, None), -1),
        ((2, A2(2, 0), A2(2, 2), 0, None, None, None, ctypes.byref(nb), None, None), -2),
        ((2, A2(1 << 40, 1 << 30), A2(2, 2), 0, None, None, None, ctypes.byref(nb), None, None),
         -2),
        ((2, A2(2, 2), A2(2, 2), 0, None, None, None, None, None, None), -1),
        ((2, A2(2, 2), A2(2, 2), 0, None, None, None, ctypes.byref(nb),
          (ctypes.c_void_p * 2)(8, 8), None), -1),                   # *nblocks = 0 with cores
    ]
    nb5 = ctypes.c_int64(5)           # rank 5 from no entries: E_SHAPE before any device call
    cases.append(((2, A2(2, 2), A2(2, 2), 0, None, None, None, ctypes.byref(nb5),
                   (ctypes.c_void_p * 2)(8, 8), None), -2))
    for args, want in cases:
        assert f(*args) == want, args


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of tnrsvd_opts and tnrsvd_mpo have the C layout
    (size and every field offset), as a C compiler lays them out."""
    import shutil
    import subprocess
    from paper_1707_07803_amd import tnrsvd as binding
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"tnrsvd_opts": binding._Opts, "tnrsvd_mpo": binding._Mpo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tnrsvd.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py)
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_new_entry_points_reject_bad_arguments_on_the_host(lib):
    """tnrsvd_create (orientation, sketch_rank), tnrsvd_round_mpo,
    tnrsvd_complex_embed, tnrsvd_solve_complex and tnrsvd_mpo_add check their
    arguments before any device call."""
    from paper_1707_07803_amd import tnrsvd as binding
    P64 = ctypes.c_int64
    Mpo, Opts = binding._Mpo, binding._Opts
    core = ctypes.c_void_p(8)        # never dereferenced: every case fails first

    def mpo(rank, rows, cols, dtype=0, cores=None):
        d = len(rows)
        st = Mpo()
        st.d = d
        st.rank = (P64 * (d + 1))(*rank)
        st.rows = (P64 * d)(*rows)
        st.cols = (P64 * d)(*cols)
        st.core = (ctypes.c_void_p * d)(*([core] * d if cores is None else cores))
        st.dtype = dtype
        return st

    create = lib.tnrsvd_create
    create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.POINTER(Mpo),
                       ctypes.POINTER(Opts)]
    h = ctypes.c_void_p()
    good = mpo([1, 2, 1], [2, 2], [2, 2])
    for kw, want in [(dict(orientation=5), -1), (dict(sketch_rank=-1), -1),
                     (dict(sketch_rank=257), -1), (dict(orientation=1, sketch_rank=300), -1)]:
        o = Opts(k=2, p=2, q=0, seed=1, precision=0, round_tol=0.0, max_rank=0, check_finite=0,
                 stream=None, **kw)
        assert create(ctypes.byref(h), 1, ctypes.byref(good), ctypes.byref(o)) == want, kw
    bad = mpo([1, 2, 1], [2, 2], [2, 2])
    bad.d = 0
    o = Opts(k=2, p=2, q=0, seed=1, precision=0, round_tol=0.0, max_rank=0, check_finite=0,
             stream=None, orientation=1)
    assert create(ctypes.byref(h), 1, ctypes.byref(bad), ctypes.byref(o)) == -2
    edge = mpo([2, 2, 1], [2, 2], [2, 2])        # rank[0] != 1, refused before staging
    assert create(ctypes.byref(h), 1, ctypes.byref(edge), ctypes.byref(o)) == -2

    rnd = lib.tnrsvd_round_mpo
    rnd.argtypes = [ctypes.POINTER(Mpo), ctypes.c_double, ctypes.c_int, ctypes.c_void_p,
                    ctypes.POINTER(ctypes.c_void_p)]
    cases = [
        ((ctypes.byref(good), 1e-3, 0, None, None), -1),                       # null out
        ((None, 1e-3, 0, None, ctypes.byref(h)), -1),                          # null MPO
        ((ctypes.byref(good), -1.0, 0, None, ctypes.byref(h)), -1),            # round_tol < 0
        ((ctypes.byref(good), float("inf"), 0, None, ctypes.byref(h)), -1),
        ((ctypes.byref(good), 1e-3, -1, None, ctypes.byref(h)), -1),           # max_rank < 0
        ((ctypes.byref(mpo([2, 2, 1], [2, 2], [2, 2])), 1e-3, 0, None, ctypes.byref(h)), -2),
        ((ctypes.byref(mpo([1, 0, 1], [2, 2], [2, 2])), 1e-3, 0, None, ctypes.byref(h)), -2),
        ((ctypes.byref(mpo([1, 5000, 1], [2, 2], [2, 2])), 1e-3, 0, None, ctypes.byref(h)), -2),
        ((ctypes.byref(mpo([1, 2, 1], [2, 2], [2, 2], dtype=2)), 1e-3, 0, None,
          ctypes.byref(h)), -1),                                               # BF16 input
        ((ctypes.byref(mpo([1, 2, 1], [2, 2], [2, 2], cores=[core, None])), 1e-3, 0, None,
          ctypes.byref(h)), -2),                                               # null core
    ]
    for args, want in cases:
        assert rnd(*args) == want, args

    emb = lib.tnrsvd_complex_embed
    emb.argtypes = [ctypes.POINTER(Mpo), ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]
    outs = (ctypes.c_void_p * 2)(8, 8)
    assert emb(None, outs, None) == -1
    assert emb(ctypes.byref(good), None, None) == -1
    assert emb(ctypes.byref(mpo([1, 2, 2], [2, 2], [2, 2])), outs, None) == -2
    assert emb(ctypes.byref(mpo([1, 2, 1], [2, 2], [2, 2], dtype=2)), outs, None) == -1
    assert emb(ctypes.byref(good), (ctypes.c_void_p * 2)(8, None), None) == -2

    sc = lib.tnrsvd_solve_complex
    sc.argtypes = [ctypes.POINTER(Mpo), ctypes.POINTER(Opts), ctypes.POINTER(ctypes.c_double)]
    sig = (ctypes.c_double * 4)()
    oc = Opts(k=2, p=2, q=0, seed=1, precision=0, round_tol=0.0, max_rank=0, check_finite=0,
              stream=None)
    assert sc(None, ctypes.byref(oc), sig) == -1
    assert sc(ctypes.byref(good), None, sig) == -1
    assert sc(ctypes.byref(good), ctypes.byref(oc), None) == -1
    for kw in (dict(k=0, p=2), dict(k=2, p=-1)):
        ob = Opts(q=0, seed=1, precision=0, round_tol=0.0, max_rank=0, check_finite=0,
                  stream=None, **kw)
        assert sc(ctypes.byref(good), ctypes.byref(ob), sig) == -1, kw
    assert sc(ctypes.byref(mpo([1, 2, 1], [2, 2], [2, 2], dtype=2)), ctypes.byref(oc), sig) == -1
    assert sc(ctypes.byref(mpo([1, 2, 2], [2, 2], [2, 2])), ctypes.byref(oc), sig) == -2
    assert sc(ctypes.byref(mpo([1, 0, 1], [2, 2], [2, 2])), ctypes.byref(oc), sig) == -2
    assert sc(ctypes.byref(mpo([1, 2, 1], [2, 2], [2, 2], cores=[core, None])), ctypes.byref(oc),
              sig) == -2

    add = lib.tnrsvd_mpo_add
    add.argtypes = [ctypes.POINTER(Mpo), ctypes.POINTER(Mpo), ctypes.POINTER(ctypes.c_void_p),
                    ctypes.c_void_p]
    other = mpo([1, 3, 1], [2, 2], [2, 2])
    assert add(None, ctypes.byref(other), outs, None) == -1
    assert add(ctypes.byref(good), ctypes.byref(other), None, None) == -1
    assert add(ctypes.byref(good), ctypes.byref(mpo([1, 3, 1], [2, 2], [2, 2], dtype=1)), outs,
               None) == -1                                                     # dtypes differ
    assert add(ctypes.byref(good), ctypes.byref(mpo([1, 3, 1], [2, 3], [2, 2])), outs,
               None) == -2                                                     # modes differ
    assert add(ctypes.byref(good), ctypes.byref(mpo([1, 1], [4], [4])), outs, None) == -2
    assert add(ctypes.byref(good), ctypes.byref(mpo([1, 3, 2], [2, 2], [2, 2])), outs,
               None) == -2                                                     # rank[d] != 1
    assert add(ctypes.byref(good), ctypes.byref(mpo([1, 0, 1], [2, 2], [2, 2])), outs,
               None) == -2
    assert add(ctypes.byref(good), ctypes.byref(other), (ctypes.c_void_p * 2)(8, None),
               None) == -2                                                     # null out core

    # sizes whose products overflow 64 bits are refused, not wrapped
    huge = 2 ** 31 - 1
    assert rnd(ctypes.byref(mpo([1, 2, 1], [huge, 2], [huge, 2])), 1e-3, 0, None,
               ctypes.byref(h)) == -2
    big = mpo([1, 2, 1], [2 ** 40, 2], [2 ** 40, 2])
    assert add(ctypes.byref(big), ctypes.byref(mpo([1, 2, 1], [2 ** 40, 2], [2 ** 40, 2])),
               outs, None) == -2
    assert emb(ctypes.byref(mpo([1, 2, 1], [2 ** 31, 2], [2 ** 31, 2])), outs, None) == -2
