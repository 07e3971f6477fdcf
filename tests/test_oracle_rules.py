"""Oracle pins for the module-level rules (section "Validation Rules"): a
module must declare a capability, define its memory model and declare a
function.  Hand-built modules whose answers follow from the rule as stated;
the rule stage runs only on modules that pass every earlier check."""
import numpy as np
import pytest

import oracle

HDR = [0x07230203, 0x00010600, 0]
CAP = [2 << 16 | 17, 1]                  # OpCapability Shader
MEM = [3 << 16 | 14, 0, 1]               # OpMemoryModel Logical GLSL450
INT = [4 << 16 | 21, 1, 32, 0]           # %1 = OpTypeInt 32 0
FUN = [5 << 16 | 54, 1, 2, 0, 1]         # %2 = OpFunction %1 None %1
END = [1 << 16 | 56]                     # OpFunctionEnd


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
    ((CAP, MEM, INT, FUN, END), (0, 0)),
    ((MEM, INT, FUN, END), (11, 8)),
    ((CAP, INT, FUN, END), (11, 16)),
    ((CAP, MEM, INT), (11, 32)),
    ((INT,), (11, 8 | 16 | 32)),
    ((), (11, 8 | 16 | 32)),              # header only
    ((INT, FUN, END, MEM, CAP), (0, 0)),  # order is not part of these rules
    ((CAP, CAP, MEM, INT, FUN, END), (0, 0)),
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
    # the rules apply per module in a batch
    assert _run([_module(CAP, MEM, INT, FUN, END), _module(MEM, INT, FUN, END), _module(CAP, MEM, INT)]) == \
        [(0, 0), (11, 8), (11, 32)]
