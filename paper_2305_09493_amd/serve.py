"""Continuous-batching validation server (binding of the spv_server_* C ABI).

The server itself - admission, batching, slots, streams, graphs, completion
polling - is native code in libspvgpu.so; this module marshals host arrays
and turns completions into numpy records.
"""
from __future__ import annotations

import ctypes
import time
from typing import List, Optional, Sequence

import numpy as np

from . import ERRORS, SPV_SUCCESS, SpvError, context, load_library


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("code", ctypes.c_uint32), ("sem_mask", ctypes.c_uint32),
                ("err_word", ctypes.c_uint32), ("n_inst", ctypes.c_uint32), ("status", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("t_arrival_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64),
                ("batch_modules", ctypes.c_int64)]


COMPLETION_DTYPE = np.dtype([("id", "<i8"), ("code", "<u4"), ("sem_mask", "<u4"), ("err_word", "<u4"),
                             ("n_inst", "<u4"), ("status", "<i4"), ("pad", "<i4"), ("t_arrival_ns", "<i8"),
                             ("t_done_ns", "<i8"), ("batch_modules", "<i8")])
assert ctypes.sizeof(Completion) == COMPLETION_DTYPE.itemsize == 56


def _bind(lib):
    if getattr(lib, "_spv_server_bound", False):
        return lib
    P, I64 = ctypes.c_void_p, ctypes.c_int64
    lib.spv_server_create.argtypes = [ctypes.POINTER(P), P, ctypes.c_int, ctypes.c_size_t, ctypes.c_int, I64, I64,
                                      ctypes.c_int]
    lib.spv_server_start.argtypes = [P]
    lib.spv_server_submit.argtypes = [P, I64, P, P, P, P]
    lib.spv_server_poll.argtypes = [P, P, I64, ctypes.POINTER(I64), ctypes.POINTER(I64)]
    lib.spv_server_stats.argtypes = [P] + [ctypes.POINTER(I64)] * 5
    lib.spv_server_destroy.argtypes = [P]
    lib.spv_server_cancel.argtypes = [P, I64, P]
    for n in ("spv_server_create", "spv_server_start", "spv_server_submit", "spv_server_poll",
              "spv_server_stats", "spv_server_destroy", "spv_server_cancel"):
        getattr(lib, n).restype = ctypes.c_int
    lib._spv_server_bound = True
    return lib


class Server:
    """Validation server on one device.

    device_budget_bytes bounds the device memory of all slots; max_batch_modules
    = 1 gives the one-module-per-launch baseline."""

    def __init__(self, device: int = 0, device_budget_bytes: int = 32 << 30, n_slots: int = 4,
                 max_batch_modules: int = 4096, slot_max_modules: int = 8192, use_graphs: bool = False):
        self.lib = _bind(load_library())
        self.ctx = context(device)
        h = ctypes.c_void_p()
        rc = self.lib.spv_server_create(ctypes.byref(h), self.ctx.h, device, device_budget_bytes, n_slots,
                                        max_batch_modules, slot_max_modules, int(use_graphs))
        if rc != SPV_SUCCESS:
            raise SpvError(f"spv_server_create failed: {ERRORS.get(rc, rc)}")
        self.h = h
        self._keep = []  # host buffers referenced by queued requests

    def start(self):
        rc = self.lib.spv_server_start(self.h)
        if rc != SPV_SUCCESS:
            raise SpvError(f"spv_server_start failed: {ERRORS.get(rc, rc)}")

    def submit(self, modules: Sequence[np.ndarray], ids: Optional[np.ndarray] = None,
               t_arrival_s: Optional[np.ndarray] = None):
        """Queue modules (uint32 arrays, kept alive here) in arrival order."""
        n = len(modules)
        arrs = [np.ascontiguousarray(m, dtype=np.uint32) for m in modules]
        self._keep.extend(arrs)
        ptrs = np.array([a.ctypes.data for a in arrs], dtype=np.uint64)
        sizes = np.array([a.size for a in arrs], dtype=np.int64)
        ids = np.arange(n, dtype=np.int64) if ids is None else np.ascontiguousarray(ids, dtype=np.int64)
        tarr = None if t_arrival_s is None else np.ascontiguousarray(np.round(np.asarray(t_arrival_s) * 1e9),
                                                                       dtype=np.int64)
        rc = self.lib.spv_server_submit(self.h, n, ids.ctypes.data, ptrs.ctypes.data, sizes.ctypes.data,
                                        None if tarr is None else tarr.ctypes.data)
        if rc != SPV_SUCCESS:
            raise SpvError(f"spv_server_submit failed: {ERRORS.get(rc, rc)}")
        self._keep.extend([ptrs, sizes, ids] + ([] if tarr is None else [tarr]))

    def cancel(self, ids):
        """Cancel queued requests (those no batch has taken yet complete with
        status SPV_ERR_CANCELED)."""
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        rc = self.lib.spv_server_cancel(self.h, ids.size, ids.ctypes.data)
        if rc != SPV_SUCCESS:
            raise SpvError(f"spv_server_cancel failed: {ERRORS.get(rc, rc)}")

    def poll(self, max_out: int = 65536):
        buf = np.zeros(max_out, dtype=COMPLETION_DTYPE)
        n = ctypes.c_int64()
        pending = ctypes.c_int64()
        rc = self.lib.spv_server_poll(self.h, buf.ctypes.data, max_out, ctypes.byref(n), ctypes.byref(pending))
        if rc != SPV_SUCCESS:
            raise SpvError(f"spv_server_poll failed: {ERRORS.get(rc, rc)}")
        return buf[:n.value].copy(), pending.value

    def drain(self, timeout_s: float = 120.0):
        """Poll until nothing is pending; returns all completions."""
        out = []
        t_end = time.time() + timeout_s
        while True:
            c, pending = self.poll()
            if c.size:
                out.append(c)
            if pending == 0:
                break
            if time.time() > t_end:
                raise SpvError(f"server drain timed out with {pending} requests pending")
            time.sleep(0.0005)
        return np.concatenate(out) if out else np.zeros(0, dtype=COMPLETION_DTYPE)

    def stats(self):
        v = [ctypes.c_int64() for _ in range(5)]
        self.lib.spv_server_stats(self.h, *[ctypes.byref(x) for x in v])
        return dict(batches=v[0].value, modules=v[1].value, words=v[2].value, max_batch=v[3].value,
                    slot_capacity_words=v[4].value)

    def close(self):
        if self.h is not None:
            self.lib.spv_server_destroy(self.h)
            self.h = None
            self._keep = []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def run_trace(modules: List[np.ndarray], arrivals_s: np.ndarray, pick: np.ndarray, warmup_s: float = 0.0,
              **server_kw):
    """Replay a Poisson trace: request i is modules[pick[i]] arriving at
    arrivals_s[i].  Requests arriving before warmup_s are served but left out
    of the summary (first graph captures, first touches of the staging
    buffers).  Returns (completions, summary dict)."""
    with Server(**server_kw) as srv:
        reqs = [modules[j] for j in pick]
        srv.submit(reqs, ids=np.arange(len(reqs)), t_arrival_s=arrivals_s)
        t0 = time.time()
        srv.start()
        comp = srv.drain(timeout_s=max(120.0, 4 * float(arrivals_s[-1]) if len(arrivals_s) else 120.0))
        wall = time.time() - t0
        st = srv.stats()
    all_comp = comp
    if warmup_s > 0 and comp.size:
        keep = arrivals_s[comp["id"]] >= warmup_s
        comp = comp[keep]
    lat_ms = (comp["t_done_ns"] - comp["t_arrival_ns"]) / 1e6
    words = int(sum(modules[pick[i]].size for i in comp["id"])) if comp.size else 0
    span_s = (comp["t_done_ns"].max() - comp["t_arrival_ns"].min()) / 1e9 if comp.size else 0.0
    summary = dict(requests=int(comp.size), words=words, span_s=float(span_s), wall_s=wall,
                   words_per_s=words / span_s if span_s > 0 else 0.0,
                   p50_ms=float(np.percentile(lat_ms, 50)) if comp.size else None,
                   p99_ms=float(np.percentile(lat_ms, 99)) if comp.size else None,
                   mean_batch=float(comp["batch_modules"].mean()) if comp.size else None,
                   warmup_s=warmup_s, **{"server_" + k: v for k, v in st.items()})
    return all_comp, summary
