"""Host-side test (no GPU) of the module-offset rules that SPV_OPT_DEBUG_CHECKS
checks on the device (paper_2305_09493_amd/csrc/spv_checks.h, constexpr
functions that the device kernel and this g++ shim share): a batch's offsets
start at 0, never decrease, end at the word count, and every module has
fewer than 2^32 words.  Checked against a plain statement of those rules on
hand-made and random offset arrays."""
import ctypes
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2305_09493_amd", "csrc")

SHIM = r"""
#include "spv_checks.h"
// the device kernel's verdict, computed on the host: 1 = offsets accepted
extern "C" int offsets_ok(const int64_t* mo, int64_t M, int64_t W) {
  bool ok = spv::offsets_ends_ok(mo[0], mo[M], W);
  for (int64_t i = 0; i < M; ++i) ok = ok && spv::offsets_pair_ok(mo[i], mo[i + 1]);
  return ok ? 1 : 0;
}
"""


@pytest.fixture(scope="module")
def lib():
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tempfile.mkdtemp()
    src, so = os.path.join(d, "shim.cpp"), os.path.join(d, "shim.so")
    with open(src, "w") as f:
        f.write(SHIM)
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, src, "-o", so], check=True)
    lib = ctypes.CDLL(so)
    lib.offsets_ok.restype = ctypes.c_int
    lib.offsets_ok.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64]
    yield lib
    shutil.rmtree(d, ignore_errors=True)


def _ok(lib, mo, W):
    mo = np.ascontiguousarray(mo, np.int64)
    return bool(lib.offsets_ok(mo.ctypes.data, mo.size - 1, W))


def _rule(mo, W):
    mo = [int(x) for x in mo]
    return (mo[0] == 0 and mo[-1] == W and all(a <= b for a, b in zip(mo, mo[1:]))
            and all(b - a < 2 ** 32 for a, b in zip(mo, mo[1:])))


@pytest.mark.parametrize("mo,W,ok", [
    ([0, 10, 20], 20, True),
    ([0, 0, 0], 0, True),            # empty modules
    ([0, 5, 5, 9], 9, True),
    ([1, 10, 20], 20, False),        # does not start at 0
    ([0, 10, 19], 20, False),        # does not end at W
    ([0, 10, 21], 20, False),
    ([0, 12, 10, 20], 20, False),    # decreasing
    ([0, -1, 20], 20, False),
    ([0, 2 ** 32, 2 ** 32 + 5], 2 ** 32 + 5, False),  # a module of 2^32 words
    ([0, 2 ** 32 - 1, 2 ** 32 + 5], 2 ** 32 + 5, True),
])
def test_hand_made_offsets(lib, mo, W, ok):
    assert _ok(lib, mo, W) == ok == _rule(mo, W)


def test_random_offsets(lib):
    rng = np.random.default_rng(3)
    for _ in range(3000):
        M = int(rng.integers(1, 12))
        sizes = rng.integers(0, 50, size=M)
        mo = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        W = int(mo[-1])
        kind = int(rng.integers(0, 4))
        if kind == 1:
            mo[int(rng.integers(0, M + 1))] += int(rng.integers(-3, 4))
        elif kind == 2:
            W += int(rng.integers(-2, 3))
        elif kind == 3:
            i = int(rng.integers(0, M))
            mo[i], mo[i + 1] = mo[i + 1], mo[i]
        assert _ok(lib, mo, W) == _rule(mo, W), (mo.tolist(), W)
