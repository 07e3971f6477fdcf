"""Oracle pins for the module-level rules (section "Validation Rules"): a
module must declare a capability, define its memory model, declare a
function and declare an entry point.  Hand-built modules whose answers follow
from the rules as stated; the rule stage runs only on modules that pass every
earlier check."""
import numpy as np
import pytest

import oracle

HDR = [0x07230203, 0x00010600, 0]
CAP = [2 << 16 | 17, 1]                  # OpCapability Shader
MEM = [3 << 16 | 14, 0, 1]               # OpMemoryModel Logical GLSL450
INT = [4 << 16 | 21, 1, 32, 0]           # %1 = OpTypeInt 32 0
FUN = [5 << 16 | 54, 1, 2, 0, 1]         # %2 = OpFunction %1 None %1
END = [1 << 16 | 56]                     # OpFunctionEnd
ENT = [5 << 16 | 15, 6, 2, 0x6E69616D, 0]  # OpEntryPoint Kernel %2 "main"


def _module(*parts, bound=3):
    body = [w for part in parts for w in part]
    return HDR + [bound, 0] + body


def _run(mods, rules=True):
    sizes = np.array([len(m) for m in mods], np.int64)
    mod_off = np.concatenate([[0], np.cumsum(sizes)])
    words = np.array([x for m in mods for x in m], np.uint32)
    res = oracle.validate(words, mod_off, semantic=True, index=False, rules=rules)
    return [(int(r["code"]), int(r["sem_mask"])) for r in res]


@pytest.mark.parametrize("parts, expect", [
    ((CAP, MEM, ENT, INT, FUN, END), (0, 0)),
    ((MEM, ENT, INT, FUN, END), (11, 8)),
    ((CAP, ENT, INT, FUN, END), (11, 16)),
    ((CAP, MEM, INT), (11, 32 | 64)),
    ((CAP, MEM, INT, FUN, END), (11, 64)),
    ((INT,), (11, 8 | 16 | 32 | 64)),
    ((), (11, 8 | 16 | 32 | 64)),              # header only
    ((INT, FUN, END, ENT, MEM, CAP), (0, 0)),  # order is not part of these rules
    ((CAP, CAP, MEM, ENT, ENT, INT, FUN, END), (0, 0)),
])
def test_rules_on_valid_modules(parts, expect):
    assert _run([_module(*parts)]) == [expect]
    assert _run([_module(*parts)], rules=False) == [(0, 0)]


def test_earlier_stages_win():
    dup = [4 << 16 | 21, 1, 32, 0]  # %1 defined a second time, and no capability
    bad_count = [3 << 16 | 17, 1, 0]
    assert _run([_module(MEM, INT, dup, FUN, END)]) == [(9, 2)]
    assert _run([_module(bad_count, MEM)])[0][0] == 5
    assert _run([HDR[:2]])[0][0] == 1
    # an entry point naming an undefined function is an undefined ID first
    assert _run([_module(CAP, MEM, ENT, INT)]) == [(10, 4)]
    # the rules apply per module in a batch
    assert _run([_module(CAP, MEM, ENT, INT, FUN, END), _module(MEM, ENT, INT, FUN, END), _module(CAP, MEM, INT),
                 _module(CAP, MEM, INT, FUN)]) == [(0, 0), (11, 8), (11, 96), (11, 64)]


@pytest.mark.parametrize("ent, expect", [
    ([4 << 16 | 15, 6, 2, 0x00000000], (0, 0)),                  # empty name
    ([6 << 16 | 15, 6, 2, 0x64636261, 0x00676665, 0], (7, 0)),   # NUL before the last word: interface IDs are not part of the grammar
    ([3 << 16 | 15, 6, 2], (5, 0)),                              # no string word
    ([5 << 16 | 15, 6, 2, 0x6E69616D, 0x00010000], (7, 0)),      # padding not zero
    ([5 << 16 | 15, 6, 9, 0x6E69616D, 0], (8, 0)),               # function ID out of bound
])
def test_entry_point_forms(ent, expect):
    """OpEntryPoint: execution model, function ID (an ID use), then a name
    that ends in the last word."""
    m = _module(CAP, MEM, ent, INT, FUN, END)
    got = _run([m])[0]
    assert got[0] == expect[0], got
    if expect[0] == 0:
        assert got == expect
