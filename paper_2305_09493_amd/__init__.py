"""spvgpu: batched SPIR-V decode / validate / encode on MI355X (gfx950).

A thin ctypes binding of ``libspvgpu.so`` (C ABI declared in
``include/spvgpu.h``).  torch is used only for device memory and streams:
every step of decode, validate and encode runs in the library's HIP kernels.
The binding fails loudly when the library is missing; there is no CPU path.

The functions take CUDA (ROCm) tensors:
  words   : int32 or uint32 [W] (bit pattern of the SPIR-V words)
  mod_off : int64 [M+1]
and return CUDA tensors on the current stream (no host synchronisation).
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspvgpu.so")

SPV_SUCCESS = 0
ERRORS = {-1: "invalid argument", -2: "capacity", -3: "workspace", -4: "HIP error", -5: "limit", -6: "canceled"}

OK, E_TRUNCATED_HEADER, E_BAD_MAGIC, E_BAD_VERSION, E_BAD_SCHEMA = 0, 1, 2, 3, 4
E_BAD_WORD_COUNT, E_UNKNOWN_OPCODE, E_BAD_STRING = 5, 6, 7
E_ID_OUT_OF_BOUND, E_DUPLICATE_ID, E_UNDEFINED_ID = 8, 9, 10
E_MODULE_RULES = 11  # validate(module_rules=True): sem_mask = 8 no capability | 16 no memory model | 32 no function | 64 no entry point
OPT_NO_SEMANTIC, OPT_MODULE_RULES, OPT_DEBUG_CHECKS, OPT_SEM_OFFSETS, OPT_DEF_BEFORE_USE = 1, 2, 4, 8, 16  # spv_validate option bits
E_SPIN_LIMIT = 0xDEAD  # every result of a call whose inter-block wait gave up (repeat the call)
ENC_OK, ENC_UNKNOWN_OPCODE, ENC_OPERAND_COUNT, ENC_BAD_STRING, ENC_TOO_LONG, ENC_BAD_ID, ENC_CAPACITY = range(7)

_lib = None
_lock = threading.Lock()


class SpvError(RuntimeError):
    pass


def load_library():
    """Load libspvgpu.so (built by ``paper_2305_09493_amd.build``)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise SpvError(f"{LIB_PATH} is missing: build it with `python -m paper_2305_09493_amd.build` "
                           "(the library has no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        P, I64, U32, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
        lib.spv_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
        lib.spv_destroy.argtypes = [P]
        lib.spv_last_hip_error.argtypes = [P]
        lib.spv_last_hip_error.restype = ctypes.c_char_p
        lib.spv_set_tuning.argtypes = [P, ctypes.c_int, ctypes.c_int]
        lib.spv_workspace_size.argtypes = [P, I64, I64, ctypes.POINTER(SZ)]
        lib.spv_decode.argtypes = [P, P, P, I64, I64, P, P, I64, P, P, SZ, P]
        lib.spv_validate.argtypes = [P, P, P, I64, I64, P, P, I64, P, U32, P, SZ, P]
        lib.spv_validate_noalloc.argtypes = [P, P, P, I64, I64, P, P, I64, P, U32, P]
        lib.spv_encode_bound.argtypes = [I64, I64, I64, I64, I64, ctypes.POINTER(I64)]
        lib.spv_encode_workspace_size.argtypes = [P, I64, I64, ctypes.POINTER(SZ)]
        lib.spv_encode.argtypes = [P, P, P, P, P, P, P, I64, I64, U32, U32, P, P, I64, P, P, P, SZ, P]
        lib.spv_records_workspace_size.argtypes = [P, I64, I64, ctypes.POINTER(SZ)]
        lib.spv_decode_records.argtypes = [P, P, P, I64, I64, P, P, P, P, P, P, P, P, P, SZ, P]
        lib.spv_text_workspace_size.argtypes = [P, I64, I64, U32, ctypes.POINTER(SZ)]
        lib.spv_decode_text.argtypes = [P, P, P, I64, I64, P, P, U32, P, I64, P, P, SZ, P]
        lib.spv_set_timing.argtypes = [P, ctypes.c_int]
        lib.spv_get_tuning.argtypes = [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        lib.spv_set_grids.argtypes = [P, ctypes.c_int, ctypes.c_int]
        lib.spv_get_grids.argtypes = [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        lib.spv_read_timing.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64)]
        for name in ("spv_create", "spv_destroy", "spv_set_tuning", "spv_workspace_size", "spv_decode",
                     "spv_validate", "spv_validate_noalloc", "spv_encode_bound", "spv_encode_workspace_size", "spv_encode",
                     "spv_records_workspace_size", "spv_decode_records", "spv_text_workspace_size", "spv_decode_text",
                     "spv_set_timing", "spv_read_timing", "spv_get_tuning", "spv_set_grids", "spv_get_grids",
                     "spv_server_create", "spv_server_start", "spv_server_submit",
           "spv_server_poll", "spv_server_stats", "spv_server_destroy", "spv_server_cancel"):
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


EXPORTS = ("spv_create", "spv_destroy", "spv_last_hip_error", "spv_set_tuning", "spv_workspace_size",
           "spv_decode", "spv_validate", "spv_validate_noalloc", "spv_encode_bound", "spv_encode_workspace_size", "spv_encode",
           "spv_records_workspace_size", "spv_decode_records", "spv_text_workspace_size", "spv_decode_text",
           "spv_set_timing", "spv_read_timing", "spv_get_tuning", "spv_set_grids", "spv_get_grids",
           "spv_server_create", "spv_server_start", "spv_server_submit",
           "spv_server_poll", "spv_server_stats", "spv_server_destroy", "spv_server_cancel")


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Context:
    """One spv_ctx on a device plus a reusable workspace tensor."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        self.device = device
        h = ctypes.c_void_p()
        rc = self.lib.spv_create(ctypes.byref(h), device)
        if rc != SPV_SUCCESS:
            raise SpvError(f"spv_create failed ({ERRORS.get(rc, rc)})")
        self.h = h
        self._ws = None

    def close(self):
        if self.h is not None:
            self.lib.spv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc: int, what: str):
        if rc != SPV_SUCCESS:
            detail = self.lib.spv_last_hip_error(self.h).decode() if rc == -4 else ""
            raise SpvError(f"{what} failed: {ERRORS.get(rc, rc)} {detail}")

    def set_tuning(self, blocks_per_cu: int = 0, encode_block: int = 0):
        self.check(self.lib.spv_set_tuning(self.h, blocks_per_cu, encode_block), "spv_set_tuning")

    def set_grids(self, chain_blocks_per_cu: int = 0, walk_blocks_per_cu: int = 0):
        self.check(self.lib.spv_set_grids(self.h, chain_blocks_per_cu, walk_blocks_per_cu), "spv_set_grids")

    def get_grids(self):
        c, w = ctypes.c_int(), ctypes.c_int()
        self.check(self.lib.spv_get_grids(self.h, ctypes.byref(c), ctypes.byref(w)), "spv_get_grids")
        return c.value, w.value

    def get_tuning(self):
        """(blocks_per_cu, encode_block) currently in use."""
        a, b = ctypes.c_int(), ctypes.c_int()
        self.check(self.lib.spv_get_tuning(self.h, ctypes.byref(a), ctypes.byref(b)), "spv_get_tuning")
        return a.value, b.value

    def set_timing(self, enable: bool):
        self.check(self.lib.spv_set_timing(self.h, int(bool(enable))), "spv_set_timing")

    def read_timing(self):
        """(summed milliseconds of the instruction-walk kernel, launches) since the last read."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self.check(self.lib.spv_read_timing(self.h, ctypes.byref(ms), ctypes.byref(n)), "spv_read_timing")
        return ms.value, n.value

    def workspace(self, nbytes: int):
        torch = _torch()
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def workspace_size(self, n_modules: int, n_words: int) -> int:
        sz = ctypes.c_size_t()
        self.check(self.lib.spv_workspace_size(self.h, n_modules, n_words, ctypes.byref(sz)), "spv_workspace_size")
        return sz.value

    def encode_workspace_size(self, n_modules: int, n_records: int) -> int:
        sz = ctypes.c_size_t()
        self.check(self.lib.spv_encode_workspace_size(self.h, n_modules, n_records, ctypes.byref(sz)),
                   "spv_encode_workspace_size")
        return sz.value


_default = {}


def context(device: Optional[int] = None) -> Context:
    torch = _torch()
    if device is None:
        device = torch.cuda.current_device()
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _run(semantic: bool, words, mod_off, index: bool, ctx: Optional[Context], stream, out=None, workspace=None,
         flags: int = 0):
    torch = _torch()
    ctx = ctx or context(words.device.index)
    W = int(words.numel())
    M = int(mod_off.numel()) - 1
    if not (words.is_cuda and mod_off.is_cuda and mod_off.dtype == torch.int64 and mod_off.is_contiguous()):
        raise SpvError("words and mod_off must be CUDA tensors, mod_off contiguous int64")
    if words.dtype not in (torch.int32, torch.uint32) or not words.is_contiguous():
        raise SpvError("words must be a contiguous int32 / uint32 CUDA tensor")
    dev = words.device
    if out is None:
        results = torch.empty((M, 4), dtype=torch.int32, device=dev)
        idx_off = torch.empty(W if index else 0, dtype=torch.int32, device=dev) if index else None
        idx_op = torch.empty(W if index else 0, dtype=torch.int16, device=dev) if index else None
    else:
        results, idx_off, idx_op = out
        if (results.dtype not in (torch.int32, torch.uint32) or results.numel() < 4 * M
                or not results.is_contiguous() or not results.is_cuda):
            raise SpvError(f"results must be a contiguous int32 CUDA tensor of {M} rows of 4")
        if index:
            if idx_off is None or idx_op is None:
                raise SpvError("index=True needs both idx_off and idx_op in out")
            for t, dt in ((idx_off, (torch.int32, torch.uint32)), (idx_op, (torch.int16, torch.uint16))):
                if t.dtype not in dt or not t.is_contiguous() or not t.is_cuda:
                    raise SpvError("idx_off must be contiguous int32 and idx_op contiguous int16 CUDA tensors")
        else:
            idx_off = idx_op = None
    # the library checks the capacity of the index buffers the caller gave
    idx_cap = min(int(idx_off.numel()), int(idx_op.numel())) if index else 0
    ws_bytes = ctx.workspace_size(M, W)
    ws = workspace if workspace is not None else ctx.workspace(ws_bytes)
    args = [ctx.h, _ptr(words), _ptr(mod_off), M, W, _ptr(idx_off), _ptr(idx_op), idx_cap,
            _ptr(results)]
    if semantic:
        rc = ctx.lib.spv_validate(*args, flags, _ptr(ws), ws.numel(), _stream(stream))
        ctx.check(rc, "spv_validate")
    else:
        rc = ctx.lib.spv_decode(*args, _ptr(ws), ws.numel(), _stream(stream))
        ctx.check(rc, "spv_decode")
    return results, idx_off, idx_op


def validate(words, mod_off, index: bool = True, ctx: Optional[Context] = None, stream=None, out=None,
             workspace=None, module_rules: bool = False, debug_checks: bool = False, sem_offsets: bool = False,
             def_before_use: bool = False):
    """Per-module results int32[M, 4] (code, sem_mask, err_word, n_inst) and,
    if index, the gapped-CSR instruction index (idx_off int32[W], idx_op
    int16[W]).  module_rules adds the module-level rules as a last stage
    (E_MODULE_RULES); debug_checks first checks mod_off on the device (the
    call then synchronises its stream, and a bad mod_off raises SpvError);
    sem_offsets puts the offset of the first instruction of the primary
    semantic failure in err_word; def_before_use needs every used ID defined
    by an earlier instruction (both need the index)."""
    flags = ((OPT_MODULE_RULES if module_rules else 0) | (OPT_DEBUG_CHECKS if debug_checks else 0) |
             (OPT_SEM_OFFSETS if sem_offsets else 0) | (OPT_DEF_BEFORE_USE if def_before_use else 0))
    return _run(True, words, mod_off, index, ctx, stream, out, workspace, flags)


NOALLOC_SCRATCH_BYTES = 64 << 20  # SPV_NOALLOC_SCRATCH_BYTES


def validate_noalloc(words, mod_off, out, ctx: Optional[Context] = None, stream=None, module_rules: bool = False):
    """spv_validate_noalloc: validate into caller-given outputs (results
    int32[M, 4], and idx_off int32[>= W] / idx_op int16[>= W] or None) with
    the library's own scratch instead of a workspace; nothing is allocated.
    Calls that overlap on one GPU race on its scratch."""
    torch = _torch()
    ctx = ctx or context(words.device.index)
    W = int(words.numel())
    M = int(mod_off.numel()) - 1
    if not (words.is_cuda and mod_off.is_cuda and mod_off.dtype == torch.int64 and mod_off.is_contiguous()):
        raise SpvError("words and mod_off must be CUDA tensors, mod_off contiguous int64")
    if words.dtype not in (torch.int32, torch.uint32) or not words.is_contiguous():
        raise SpvError("words must be a contiguous int32 / uint32 CUDA tensor")
    results, idx_off, idx_op = out
    if results.numel() < 4 * M or not results.is_contiguous():
        raise SpvError(f"results must be a contiguous int32 CUDA tensor of {M} rows of 4")
    index = idx_off is not None
    if index != (idx_op is not None):
        raise SpvError("give both idx_off and idx_op, or neither")
    idx_cap = min(int(idx_off.numel()), int(idx_op.numel())) if index else 0
    rc = ctx.lib.spv_validate_noalloc(ctx.h, _ptr(words), _ptr(mod_off), M, W, _ptr(idx_off), _ptr(idx_op), idx_cap,
                                      _ptr(results), OPT_MODULE_RULES if module_rules else 0, _stream(stream))
    ctx.check(rc, "spv_validate_noalloc")
    return results, idx_off, idx_op


def decode(words, mod_off, index: bool = True, ctx: Optional[Context] = None, stream=None, out=None,
           workspace=None):
    return _run(False, words, mod_off, index, ctx, stream, out, workspace)


def encode_bound(n_modules: int, n_records: int, n_opnd: int, n_string_records: int, n_chars: int) -> int:
    lib = load_library()
    out = ctypes.c_int64()
    rc = lib.spv_encode_bound(n_modules, n_records, n_opnd, n_string_records, n_chars, ctypes.byref(out))
    if rc != SPV_SUCCESS:
        raise SpvError(f"spv_encode_bound failed: {ERRORS.get(rc, rc)}")
    return out.value


def encode(op, opnd_off, opnd, str_off, chars, rec_mod_off, version_word: int = 0x00010600,
           generator_word: int = 0, words_cap: Optional[int] = None, ctx: Optional[Context] = None, stream=None):
    """Encode CSR records (CUDA tensors: op int16/uint16 [N], opnd_off int32
    [N+1], opnd int32 [*], str_off int32 [N+1], chars uint8 [*], rec_mod_off
    int64 [M+1]).  Returns (words int32[cap], word_mod_off int64[M+1],
    enc_code int32[M], enc_bad_record int64[M])."""
    torch = _torch()
    ctx = ctx or context(op.device.index)
    dev = op.device
    M = int(rec_mod_off.numel()) - 1
    N = int(op.numel())
    if words_cap is None:
        words_cap = encode_bound(M, N, int(opnd.numel()), N, int(chars.numel()))
    words = torch.empty(max(words_cap, 1), dtype=torch.int32, device=dev)
    word_mod_off = torch.empty(M + 1, dtype=torch.int64, device=dev)
    code = torch.empty(M, dtype=torch.int32, device=dev)
    bad = torch.empty(M, dtype=torch.int64, device=dev)
    ws_bytes = ctx.encode_workspace_size(M, N)
    ws = ctx.workspace(ws_bytes)
    rc = ctx.lib.spv_encode(ctx.h, _ptr(op), _ptr(opnd_off), _ptr(opnd), _ptr(str_off), _ptr(chars),
                            _ptr(rec_mod_off), M, N, version_word, generator_word, _ptr(words), _ptr(word_mod_off),
                            words_cap, _ptr(code), _ptr(bad), _ptr(ws), ws.numel(), _stream(stream))
    ctx.check(rc, "spv_encode")
    return words, word_mod_off, code, bad


# options of decode_text: the disassembler's five switches, in its options listing's order
TEXT_HIGHLIGHT, TEXT_INLINE_NAMES, TEXT_NO_INDENT, TEXT_GROUP, TEXT_NO_HEADER = 1, 2, 4, 8, 16


def decode_text(words, mod_off, idx_off, results, options: int = 0, text=None, ctx: Optional[Context] = None,
                stream=None):
    """Decode's text mode: SPIR-V assembly text of every module's valid
    instruction prefix, from the index and results of a decode / validate
    call on the same batch.  With ``text`` (a 4-byte aligned CUDA uint8
    tensor), one asynchronous call fills it with the first min(total,
    text.numel()) bytes; without it, a sizing call and a host read of the
    total come first.  Returns (text, text_mod_off): module m's text is
    text[text_mod_off[m]:text_mod_off[m+1]]; text_mod_off[-1] is the total."""
    torch = _torch()
    ctx = ctx or context(words.device.index)
    dev = words.device
    W = int(words.numel())
    M = int(mod_off.numel()) - 1
    tmo = torch.empty(M + 1, dtype=torch.int64, device=dev)
    sz = ctypes.c_size_t()
    ctx.check(ctx.lib.spv_text_workspace_size(ctx.h, M, W, options, ctypes.byref(sz)), "spv_text_workspace_size")
    ws = ctx.workspace(sz.value)

    def call(buf, cap):
        rc = ctx.lib.spv_decode_text(ctx.h, _ptr(words), _ptr(mod_off), M, W, _ptr(idx_off), _ptr(results),
                                     options, _ptr(buf) if buf is not None else None, cap, _ptr(tmo), _ptr(ws),
                                     ws.numel(), _stream(stream))
        ctx.check(rc, "spv_decode_text")

    if text is None:
        call(None, 0)
        total = int(tmo[-1].item()) if M > 0 else 0
        if total < 0:
            raise SpvError("spv_decode_text: a kernel's wait exceeded its spin limit")
        text = torch.empty(max(total, 4), dtype=torch.uint8, device=dev)
    elif text.dtype != torch.uint8 or not text.is_cuda or text.data_ptr() % 4:
        raise SpvError("text must be a 4-byte aligned CUDA uint8 tensor")
    call(text, int(text.numel()))
    return text, tmo


def decode_records(words, mod_off, idx_off, results, ctx: Optional[Context] = None, stream=None):
    """Decode's records mode: the records of every module's valid instruction
    prefix, from the index (idx_off) and results of a decode / validate call
    on the same batch, in the layout encode takes.  Returns a dict of CUDA
    tensors sized for the batch's capacity (op, opnd_off, opnd, str_off,
    chars, rec_mod_off); the record count is rec_mod_off[-1], read without a
    host synchronisation here."""
    torch = _torch()
    ctx = ctx or context(words.device.index)
    dev = words.device
    W = int(words.numel())
    M = int(mod_off.numel()) - 1
    out = dict(op=torch.empty(max(W, 1), dtype=torch.int16, device=dev),
               opnd_off=torch.empty(W + 1, dtype=torch.int32, device=dev),
               opnd=torch.empty(max(W, 1), dtype=torch.int32, device=dev),
               str_off=torch.empty(W + 1, dtype=torch.int32, device=dev),
               chars=torch.empty(max(4 * W, 1), dtype=torch.uint8, device=dev),
               rec_mod_off=torch.empty(M + 1, dtype=torch.int64, device=dev))
    sz = ctypes.c_size_t()
    ctx.check(ctx.lib.spv_records_workspace_size(ctx.h, M, W, ctypes.byref(sz)), "spv_records_workspace_size")
    ws = ctx.workspace(sz.value)
    rc = ctx.lib.spv_decode_records(ctx.h, _ptr(words), _ptr(mod_off), M, W, _ptr(idx_off), _ptr(results),
                                    _ptr(out["op"]), _ptr(out["opnd_off"]), _ptr(out["opnd"]), _ptr(out["str_off"]),
                                    _ptr(out["chars"]), _ptr(out["rec_mod_off"]), _ptr(ws), ws.numel(),
                                    _stream(stream))
    ctx.check(rc, "spv_decode_records")
    return out
