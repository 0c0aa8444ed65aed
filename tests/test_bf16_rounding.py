"""BF16 storage rounding of the library (round to nearest, ties to even; NaN
stays NaN), pinned on the CPU against torch's own float32 -> bfloat16
conversion and against hand-worked ties.

The host side of the library's bf16 type is compiled with hipcc into a small
program that converts a file of float32 values; no GPU is involved.
"""

import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROGRAM = r'''
#include <cstdio>
#include <cstdint>
#include <vector>
#include "tnrsvd_internal.h"
int main(int argc, char** argv) {
  FILE* f = std::fopen(argv[1], "rb");
  std::vector<float> x;
  float v;
  while (std::fread(&v, sizeof v, 1, f) == 1) x.push_back(v);
  std::fclose(f);
  FILE* o = std::fopen(argv[2], "wb");
  for (float a : x) {
    const tnr::bf16 b(a);
    const float back = (float)b;
    std::fwrite(&b.u, sizeof b.u, 1, o);
    std::fwrite(&back, sizeof back, 1, o);
  }
  std::fclose(o);
  return 0;
}
'''


@pytest.fixture(scope="module")
def convert():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "bf16_conv.hip")
    exe = os.path.join(d, "bf16_conv")
    open(src, "w").write(PROGRAM)
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17",
                           "-I" + os.path.join(ROOT, "paper_1707_07803_amd", "csrc"),
                           "-I" + os.path.join(ROOT, "include"), src, "-o", exe],
                          stderr=subprocess.DEVNULL)

    def run(x):
        x = np.ascontiguousarray(x, dtype=np.float32)
        fin, fout = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
        x.tofile(fin)
        subprocess.check_call([exe, fin, fout])
        raw = np.fromfile(fout, dtype=np.uint8).reshape(-1, 6)
        bits = raw[:, :2].copy().view(np.uint16).ravel()
        back = raw[:, 2:].copy().view(np.float32).ravel()
        return bits, back

    yield run
    shutil.rmtree(d, ignore_errors=True)


def test_hand_worked_ties_and_specials(convert):
    one = 1.0
    cases = {
        one: 0x3F80,
        one + 2.0 ** -8: 0x3F80,          # halfway between 0x3F80 and 0x3F81: even wins
        one + 3 * 2.0 ** -8: 0x3F82,      # halfway between 0x3F81 and 0x3F82: even wins
        one + 2.0 ** -8 + 2.0 ** -20: 0x3F81,   # just above halfway: up
        -2.0: 0xC000,
        float(np.finfo(np.float32).max): 0x7F80,   # rounds up to +inf
        float("inf"): 0x7F80,
        0.0: 0x0000,
    }
    x = np.array(list(cases.keys()), dtype=np.float32)
    bits, back = convert(x)
    assert [int(b) for b in bits] == list(cases.values())
    nb, nback = convert(np.array([np.nan], dtype=np.float32))
    assert np.isnan(nback[0]) and (int(nb[0]) & 0x7F80) == 0x7F80 and (int(nb[0]) & 0x7F)


def test_matches_torch_round_to_nearest_even(convert):
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(20000).astype(np.float32) * 10.0 ** rng.integers(-30, 30, 20000),
        rng.integers(0, 2 ** 32, 20000, dtype=np.uint64).astype(np.uint32).view(np.float32),
    ])
    x = x[np.isfinite(x)]
    bits, back = convert(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(bits, ref)
    np.testing.assert_array_equal(back, torch.from_numpy(x).to(torch.bfloat16).float().numpy())
