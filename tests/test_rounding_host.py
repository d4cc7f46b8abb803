"""Host-side check of the FP32 -> BF16 / FP16 round-to-nearest-even
conversions the matrix-core stencil uses (csrc/rounding.h), compiled with the
host compiler and compared bit for bit with numpy's float16 and torch's
bfloat16 conversions on random bit patterns and edge cases."""

import os
import subprocess

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2211_13719_amd", "csrc", "rounding.h")

PROG = r"""
#include <cstdio>
#include "rounding.h"
int main(int argc, char** argv) {
  FILE* f = fopen(argv[1], "rb"); FILE* g = fopen(argv[2], "wb");
  unsigned u;
  while (fread(&u, 4, 1, f) == 1) {
    unsigned short h[2] = {mrhs::bf16_rne_bits(u), mrhs::f16_rne_bits(u)};
    fwrite(h, 2, 2, g);
  }
  fclose(f); fclose(g);
  return 0;
}
"""


@pytest.fixture(scope="module")
def conv(tmp_path_factory):
    d = tmp_path_factory.mktemp("rnd")
    src = d / "t.cpp"
    src.write_text(PROG)
    exe = d / "t"
    subprocess.check_call(["g++", "-O2", "-I", os.path.dirname(HDR), str(src), "-o", str(exe)])
    return d, exe


def test_rounding_matches_numpy_and_torch(conv):
    d, exe = conv
    rng = np.random.default_rng(7)
    a = rng.integers(0, 2**32, 400_000, dtype=np.uint64).astype(np.uint32)
    b = (rng.standard_normal(200_000) * 10.0 ** rng.integers(-9, 6, 200_000)).astype(np.float32).view(np.uint32)
    edge = np.array([0x38800000, 0x387FFFFF, 0x33000000, 0x33000001, 0x32FFFFFF, 0x33800000, 0x477FE000,
                     0x477FF000, 0x477FEFFF, 0x7F800000, 0x3F808000, 0x3F818000, 0x3F801000, 0x3F803000,
                     0x00000001, 0x38000000, 0x37800000, 0x7F7FFFFF], dtype=np.uint32)
    u = np.concatenate([a, b, edge, edge | 0x80000000])
    u.tofile(d / "in.bin")
    subprocess.check_call([str(exe), str(d / "in.bin"), str(d / "out.bin")])
    got = np.fromfile(d / "out.bin", dtype=np.uint16).reshape(-1, 2)
    f = u.view(np.float32)
    nan = np.isnan(f)
    with np.errstate(all="ignore"):
        want16 = f.astype(np.float16).view(np.uint16)
    want_bf = torch.from_numpy(f.copy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(got[~nan, 1], want16[~nan])
    assert np.array_equal(got[~nan, 0], want_bf[~nan])
    # NaN stays NaN in both formats
    assert np.all(np.isnan(got[nan, 1].view(np.float16)))
    assert np.all((got[nan, 0] & 0x7F80) == 0x7F80) and np.all((got[nan, 0] & 0x7F) != 0)
