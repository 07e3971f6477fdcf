"""Host-side serving logic (no GPU): the server's admission rules and graph
size buckets (paper_2305_09493_amd/csrc/spv_admission.h), built with g++
through a small C shim and checked against the rules stated in the test."""
import ctypes
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2305_09493_amd", "csrc")
TAKE, REJECT = 1, 2

SHIM = r"""
#include "spv_admission.h"
extern "C" int64_t admit(int64_t n, const int64_t* sizes, int64_t max_batch, int64_t cap_modules,
                         int64_t cap_words, uint8_t* action) {
  return spv::admit_batch(n, [&](int64_t i) { return sizes[i]; }, max_batch, cap_modules, cap_words, action);
}
extern "C" int64_t bucket(int64_t x) { return spv::bucket_up(x); }
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
    lib.admit.restype = ctypes.c_int64
    lib.admit.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                          ctypes.c_void_p]
    lib.bucket.restype = ctypes.c_int64
    lib.bucket.argtypes = [ctypes.c_int64]
    yield lib
    shutil.rmtree(d, ignore_errors=True)


def _admit(lib, sizes, max_batch, cap_modules, cap_words):
    sizes = np.ascontiguousarray(sizes, dtype=np.int64)
    action = np.zeros(max(sizes.size, 1), np.uint8)
    n = lib.admit(sizes.size, sizes.ctypes.data, max_batch, cap_modules, cap_words, action.ctypes.data)
    return list(action[:n])


def _model(sizes, max_batch, cap_modules, cap_words):
    """The admission rules, one request at a time from the front."""
    out, m, w = [], 0, 0
    for n in sizes:
        if m >= max_batch or m + 2 > cap_modules:
            break
        if n > cap_words - 1:
            out.append(REJECT)
            continue
        if w + n > cap_words - 1:
            break
        out.append(TAKE)
        m, w = m + 1, w + n
    return out


def test_fifo_until_words_full(lib):
    assert _admit(lib, [10, 20, 30, 40], 100, 100, 62) == [TAKE, TAKE, TAKE]


def test_oversized_requests_rejected_in_place(lib):
    assert _admit(lib, [100, 5, 200, 6], 100, 100, 50) == [REJECT, TAKE, REJECT, TAKE]


def test_module_limits(lib):
    assert _admit(lib, [1] * 10, 3, 100, 1000) == [TAKE] * 3           # max_batch
    assert _admit(lib, [1] * 10, 100, 4, 1000) == [TAKE] * 3           # room for the padding module
    assert _admit(lib, [1] * 10, 1, 100, 1000) == [TAKE]               # one module per launch
    assert _admit(lib, [1, 1, 1000], 2, 100, 50) == [TAKE, TAKE]       # the oversized one waits its turn


def test_random_queues_follow_the_rules(lib):
    rng = np.random.default_rng(7)
    for _ in range(2000):
        sizes = rng.integers(1, 400, size=int(rng.integers(0, 40)))
        max_batch = int(rng.integers(1, 20))
        cap_modules = int(rng.integers(2, 25))
        cap_words = int(rng.integers(2, 800))
        got = _admit(lib, sizes, max_batch, cap_modules, cap_words)
        assert got == _model(sizes, max_batch, cap_modules, cap_words)
        taken = [int(s) for s, a in zip(sizes, got) if a == TAKE]
        assert sum(taken) <= cap_words - 1 and len(taken) <= min(max_batch, cap_modules - 1)


def test_graph_buckets_pad_little(lib):
    seen = set()
    for x in list(range(1, 5000)) + [int(v) for v in np.unique(np.logspace(3, 9, 4000).astype(np.int64))]:
        b = lib.bucket(x)
        assert b >= x and b >= 64
        if x > 64:
            assert b - x <= x // 8
        seen.add(b)
    # a few buckets per power of two
    assert all(lib.bucket(lib.bucket(x)) == lib.bucket(x) for x in range(1, 3000))
    assert len([b for b in seen if 1 << 20 <= b < 1 << 21]) <= 8
