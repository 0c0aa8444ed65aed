"""Host-side contracts that need no GPU: the binding refuses to run without
the built HIP library (there is no CPU fallback), and the benchmark refuses
more than one GPU with a message instead of running a partial job."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(code_or_args, timeout=120):
    return subprocess.run([sys.executable, *code_or_args], cwd=ROOT, capture_output=True,
                          text=True, timeout=timeout)


def test_missing_library_raises_instead_of_falling_back():
    r = run(["-c", "import paper_1707_07803_amd.tnrsvd as t\n"
                   "try:\n"
                   "    t.load_library('/nonexistent/libtnrsvd.so')\n"
                   "except RuntimeError as e:\n"
                   "    print('raised:', e)\n"])
    assert r.returncode == 0, r.stderr
    assert "raised:" in r.stdout and "no CPU fallback" in r.stdout


def test_bench_refuses_more_than_one_gpu():
    r = run(["bench.py", "--gpus", "2", "--steps", "1", "--warmup", "0"])
    assert r.returncode == 2
    line = [l for l in r.stdout.splitlines() if l.startswith("{")][-1]
    msg = json.loads(line)
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]
