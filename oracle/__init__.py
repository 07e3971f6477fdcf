"""CPU oracle for batched SPIR-V decode / validate / encode (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import this package.  It wraps ``oracle.c`` (plain sequential C, built with
gcc) through ctypes on numpy arrays; it never touches the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

OK, E_TRUNCATED_HEADER, E_BAD_MAGIC, E_BAD_VERSION, E_BAD_SCHEMA = 0, 1, 2, 3, 4
E_BAD_WORD_COUNT, E_UNKNOWN_OPCODE, E_BAD_STRING = 5, 6, 7
E_ID_OUT_OF_BOUND, E_DUPLICATE_ID, E_UNDEFINED_ID = 8, 9, 10
E_MODULE_RULES = 11  # with rules: sem_mask = 8 no OpCapability | 16 no OpMemoryModel | 32 no OpFunction | 64 no OpEntryPoint
# disassembly options, the options listing's five switches in its order
DIS_HIGHLIGHT, DIS_INLINE_NAMES, DIS_NO_INDENT, DIS_GROUP, DIS_NO_HEADER = 1, 2, 4, 8, 16
ENC_OK, ENC_UNKNOWN_OPCODE, ENC_OPERAND_COUNT, ENC_BAD_STRING, ENC_TOO_LONG, ENC_BAD_ID = range(6)

RESULT_DTYPE = np.dtype([("code", "<u4"), ("sem_mask", "<u4"), ("err_word", "<u4"), ("n_inst", "<u4")])


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no SIMD flags)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = f"{_LIB_PATH}.tmp{os.getpid()}"  # parallel test workers may build at once
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            P = ctypes.c_void_p
            lib.oracle_validate.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_int, P, P, P]
            lib.oracle_validate.restype = ctypes.c_int
            lib.oracle_records.argtypes = [P, P, ctypes.c_int64, P, P, P, P, P, P]
            lib.oracle_records.restype = ctypes.c_int
            lib.oracle_encode_bound.argtypes = [ctypes.c_int64] * 4
            lib.oracle_encode_bound.restype = ctypes.c_int64
            lib.oracle_encode.argtypes = [P, P, P, P, P, P, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32, P, P,
                                          ctypes.c_int64, P, P]
            lib.oracle_encode.restype = ctypes.c_int64
            lib.oracle_disassemble.argtypes = [P, P, ctypes.c_int64, ctypes.c_uint32, P, ctypes.c_int64, P]
            lib.oracle_disassemble.restype = ctypes.c_int64
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else ctypes.c_void_p(0)


def _contig(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def validate(words, mod_off, semantic: bool = True, index: bool = True, rules: bool = False, offsets: bool = False,
             before_use: bool = False):
    """Per-module results (structured array) and, if index, the gapped-CSR
    instruction index (idx_off uint32[W], idx_op uint16[W]; entries past each
    module's n_inst are left 0).  With semantic and rules, modules that pass
    every check are held to the module-level rules (section "Validation
    Rules"; code E_MODULE_RULES).  before_use counts an ID used before any
    instruction defines it as undefined (OpName targets and OpEntryPoint
    functions may name later definitions); offsets puts the word offset of
    the first instruction of the primary semantic class in err_word."""
    lib = _load()
    words = _contig(words, np.uint32)
    mod_off = _contig(mod_off, np.int64)
    m = mod_off.size - 1
    res = np.zeros(m, dtype=RESULT_DTYPE)
    idx_off = np.zeros(words.size, np.uint32) if index else None
    idx_op = np.zeros(words.size, np.uint16) if index else None
    opts = (1 if rules else 0) | (2 if offsets else 0) | (4 if before_use else 0)
    rc = lib.oracle_validate(_ptr(words), _ptr(mod_off), m, int(bool(semantic)), opts,
                             _ptr(idx_off) if index else None, _ptr(idx_op) if index else None, _ptr(res))
    if rc != 0:
        raise RuntimeError("oracle_validate failed")
    return (res, idx_off, idx_op) if index else res


def decode(words, mod_off, index: bool = True):
    return validate(words, mod_off, semantic=False, index=index)


def records(words, mod_off):
    """Records of every module's valid instruction prefix (dict of arrays)."""
    lib = _load()
    words = _contig(words, np.uint32)
    mod_off = _contig(mod_off, np.int64)
    m = mod_off.size - 1
    n = max(words.size, 1)
    op = np.zeros(n, np.uint16)
    opnd_off = np.zeros(n + 1, np.int32)
    opnd = np.zeros(n, np.uint32)
    str_off = np.zeros(n + 1, np.int32)
    chars = np.zeros(4 * n, np.uint8)
    rec_mod_off = np.zeros(m + 1, np.int64)
    rc = lib.oracle_records(_ptr(words), _ptr(mod_off), m, _ptr(op), _ptr(opnd_off), _ptr(opnd), _ptr(str_off),
                            _ptr(chars), _ptr(rec_mod_off))
    if rc != 0:
        raise RuntimeError("oracle_records failed")
    nr = int(rec_mod_off[-1])
    return dict(op=op[:nr].copy(), opnd_off=opnd_off[:nr + 1].copy(), opnd=opnd[:opnd_off[nr]].copy(),
                str_off=str_off[:nr + 1].copy(), chars=chars[:str_off[nr]].copy(), rec_mod_off=rec_mod_off)


def encode_bound(n_modules, n_records, n_opnd, n_chars) -> int:
    return int(_load().oracle_encode_bound(n_modules, n_records, n_opnd, n_chars))


def encode(op, opnd_off, opnd, str_off, chars, rec_mod_off, version_word: int = 0x00010600,
           generator_word: int = 0):
    """(words, word_mod_off, enc_code, enc_bad_record) for a batch of records."""
    lib = _load()
    op = _contig(op, np.uint16)
    opnd_off = _contig(opnd_off, np.int32)
    opnd = _contig(opnd, np.uint32)
    str_off = _contig(str_off, np.int32)
    chars = _contig(chars, np.uint8)
    rec_mod_off = _contig(rec_mod_off, np.int64)
    m = rec_mod_off.size - 1
    cap = encode_bound(m, op.size, opnd.size, chars.size)
    out = np.zeros(max(cap, 1), np.uint32)
    word_mod_off = np.zeros(m + 1, np.int64)
    code = np.zeros(m, np.uint32)
    bad = np.zeros(m, np.int64)
    n = lib.oracle_encode(_ptr(op), _ptr(opnd_off), _ptr(opnd), _ptr(str_off), _ptr(chars), _ptr(rec_mod_off), m,
                          version_word, generator_word, _ptr(out), _ptr(word_mod_off), cap, _ptr(code), _ptr(bad))
    if n < 0:
        raise RuntimeError("oracle_encode: output capacity exceeded")
    return out[:n].copy(), word_mod_off, code, bad


def disassemble(words, mod_off, options: int = 0, text_cap=None):
    """(text bytes, text_mod_off int64[M+1], total) for a batch: module m's text
    is text[text_mod_off[m] : text_mod_off[m+1]].  With text_cap, only the
    first min(total, text_cap) bytes are produced (total is always the full
    size)."""
    lib = _load()
    words = _contig(words, np.uint32)
    mod_off = _contig(mod_off, np.int64)
    m = mod_off.size - 1
    tmo = np.zeros(m + 1, np.int64)
    if text_cap is None:
        total = lib.oracle_disassemble(_ptr(words), _ptr(mod_off), m, options, None, 0, _ptr(tmo))
        if total < 0:
            raise RuntimeError("oracle_disassemble failed")
        text_cap = total
    buf = np.zeros(max(int(text_cap), 1), np.uint8)
    total = lib.oracle_disassemble(_ptr(words), _ptr(mod_off), m, options, _ptr(buf), int(text_cap), _ptr(tmo))
    if total < 0:
        raise RuntimeError("oracle_disassemble failed")
    return buf[:min(total, int(text_cap))].tobytes(), tmo, int(total)
