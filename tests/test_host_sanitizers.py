"""Host argument checks of the C ABI under AddressSanitizer and
UndefinedBehaviorSanitizer (no GPU): the library is rebuilt with both
sanitizers on its host code (device code is not instrumented), and a small
C++ driver (tests/host_rejects.cpp) calls every entry point with arguments it
must refuse before any device call.  The driver exits nonzero on a wrong
status, and the sanitizers abort it on a memory or undefined-behaviour error."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_host_rejections_under_asan_and_ubsan():
    from paper_1707_07803_amd import build
    out = os.path.join(ROOT, "paper_1707_07803_amd", "_build", "san")
    lib = build.build_sanitized(out)
    hipcc = build.hipcc()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    obj = os.path.join(out, "host_rejects.o")
    exe = os.path.join(out, "host_rejects")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-g", *san,
                        "-I" + os.path.join(ROOT, "include"), "-c",
                        os.path.join(HERE, "host_rejects.cpp"), "-o", obj],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([hipcc, "--offload-arch=gfx950", *san, obj, "-o", exe, "-L" + out,
                        "-l:" + os.path.basename(lib), "-Wl,-rpath," + out],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all host rejections as documented" in r.stdout
