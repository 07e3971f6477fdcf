"""Host-side serving logic (no GPU): the server's admission rules, graph
size buckets and batch completion records
(paper_2305_09493_amd/csrc/spv_admission.h), built with g++ through a small C
shim and checked against the rules stated in the test."""
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
struct R { int64_t id, t_arr_ns; };
// a batch of n requests whose launch failed (res == nullptr) or ran
extern "C" int64_t complete(int64_t n, const int64_t* ids, const int64_t* t_arr, const spv_result* res, int status,
                            int64_t t_done, spv_completion* out) {
  std::vector<R> batch;
  for (int64_t i = 0; i < n; ++i) batch.push_back(R{ids[i], t_arr[i]});
  std::vector<spv_completion> done;
  spv::complete_batch(n, [&](int64_t i) -> const R& { return batch[size_t(i)]; }, res, status, t_done, done);
  for (size_t i = 0; i < done.size(); ++i) out[i] = done[i];
  return int64_t(done.size());
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
    lib.admit.restype = ctypes.c_int64
    lib.admit.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                          ctypes.c_void_p]
    lib.bucket.restype = ctypes.c_int64
    lib.bucket.argtypes = [ctypes.c_int64]
    lib.complete.restype = ctypes.c_int64
    lib.complete.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                             ctypes.c_int64, ctypes.c_void_p]
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


COMPLETION = np.dtype([("id", "<i8"), ("code", "<u4"), ("sem_mask", "<u4"), ("err_word", "<u4"), ("n_inst", "<u4"),
                       ("status", "<i4"), ("pad", "<i4"), ("t_arrival_ns", "<i8"), ("t_done_ns", "<i8"),
                       ("batch_modules", "<i8")])


def _complete(lib, ids, t_arr, res, status, t_done):
    ids = np.ascontiguousarray(ids, np.int64)
    t_arr = np.ascontiguousarray(t_arr, np.int64)
    out = np.zeros(max(ids.size, 1), COMPLETION)
    rp = None if res is None else np.ascontiguousarray(res, np.uint32).ctypes.data
    n = lib.complete(ids.size, ids.ctypes.data, t_arr.ctypes.data, rp, status, t_done, out.ctypes.data)
    return out[:n]


def test_completion_layout_matches_the_header():
    """The record layout the test reads (spv_completion in include/spvgpu.h)."""
    import re
    hdr = open(os.path.join(ROOT, "include", "spvgpu.h")).read()
    body = hdr[hdr.index("typedef struct {", hdr.index("spv_completion") - 600):hdr.index("} spv_completion;")]
    fields = re.findall(r"(\w+)\s+(\w+)(?:\[\d+\])?;", body)
    assert [f for _, f in fields][:3] == ["id", "result", "status"]


def test_failed_launch_completes_every_request_with_the_error(lib):
    """A batch whose launch failed ends at once: every request gets the error
    status and a zero result (never a stale result of an earlier batch)."""
    ids, t_arr = [11, 12, 13], [100, 200, 300]
    out = _complete(lib, ids, t_arr, None, -4, 999)
    assert list(out["id"]) == ids and list(out["t_arrival_ns"]) == t_arr
    assert all(out["status"] == -4) and all(out["t_done_ns"] == 999) and all(out["batch_modules"] == 3)
    for k in ("code", "sem_mask", "err_word", "n_inst"):
        assert all(out[k] == 0)


def test_completed_batch_carries_its_results(lib):
    res = np.array([[0, 0, 0xFFFFFFFF, 7], [10, 4, 0xFFFFFFFF, 9]], np.uint32)
    out = _complete(lib, [5, 6], [1, 2], res, 0, 50)
    assert list(out["status"]) == [0, 0]
    assert list(out["code"]) == [0, 10] and list(out["n_inst"]) == [7, 9] and list(out["sem_mask"]) == [0, 4]
    # a completion that failed on the GPU keeps no result either
    out = _complete(lib, [5, 6], [1, 2], res, -4, 50)
    assert all(out["status"] == -4) and all(out["code"] == 0) and all(out["n_inst"] == 0)
