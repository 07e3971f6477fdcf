"""Oracle on real SPIR-V modules built here (hipcc, generic SPIR-V target).
Pins: the word-count chain from word 5, walked here independently, ends
exactly at the module's end; along that walk, the first instruction outside
the twelve-opcode contract (an opcode not in the table, or a table opcode
whose word count differs from the table's) is where the oracle reports its
parse failure, with the instructions before it as its index."""
import numpy as np
import pytest

import oracle
import realspv

pytestmark = pytest.mark.skipif(not realspv.available(), reason="hipcc / clang-offload-bundler not available")

# the contract's word counts (None: OpName, at least 3)
TABLE = {5: None, 14: 3, 17: 2, 21: 4, 43: 4, 54: 5, 56: 1, 61: 4, 62: 3, 128: 5, 248: 2, 253: 1}
E_BAD_WORD_COUNT, E_UNKNOWN_OPCODE = 5, 6


def _walk(w):
    p, starts = 5, []
    while p < w.size:
        wc = int(w[p]) >> 16
        assert wc > 0, p
        starts.append(p)
        p += wc
    return p, starts


@pytest.mark.parametrize("name", sorted(realspv.SOURCES))
def test_real_module_chain_and_first_failure(name):
    w = realspv.module(name)
    assert w.size > 100 and w[0] == 0x07230203 and w[4] == 0
    end, starts = _walk(w)
    assert end == w.size
    expect = None
    for k, p in enumerate(starts):
        wc, op = int(w[p]) >> 16, int(w[p]) & 0xFFFF
        if op not in TABLE:
            expect = (E_UNKNOWN_OPCODE, p, k)
            break
        want = TABLE[op]
        if (want is None and wc < 3) or (want is not None and wc != want):
            expect = (E_BAD_WORD_COUNT, p, k)
            break
    assert expect is not None  # real modules use opcodes beyond the twelve
    res, io, iop = oracle.decode(w, np.array([0, w.size], np.int64))
    r = res[0]
    assert (int(r["code"]), int(r["err_word"]), int(r["n_inst"])) == expect
    k = expect[2]
    assert np.array_equal(io[:k], np.array(starts[:k], np.uint32))
    assert np.array_equal(iop[:k], (w[starts[:k]] & 0xFFFF).astype(np.uint16))
