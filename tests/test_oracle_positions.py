"""Pins of the oracle's semantic positions and defined-before-use mode:
hand-written modules with the offsets and codes worked out by hand (the ID
rules of section "Enabling Function Composition": each result ID defined
once, every used ID defined; the bound of section "SPIR-V Library"), and
agreement with the second statement in oracle/spec.py on random tiny modules
and on generated modules with random ID rewrites."""
import numpy as np
import pytest

import oracle
import spvgen
from oracle import spec

H = [0x07230203, 0x00010600, 0]


def _mod(bound, *insts):
    words = H + [bound, 0]
    for i in insts:
        words += list(i)
    return np.array(words, np.uint32)


def TYPEINT(r):
    return (0x00040015, r, 32, 0)


def CONST(t, r, v):
    return (0x0004002B, t, r, v)


def IADD(t, r, a, b):
    return (0x00050080, t, r, a, b)


# (name, module, expected (code, sem_mask, err_word) plain / with offsets /
# with before_use / with both)
CASES = [
    # %1 at 5, %2 at 9, %2 again at 13 (first duplicate), %3 at 17 and 21
    ("duplicate", _mod(4, TYPEINT(1), TYPEINT(2), CONST(1, 2, 7), TYPEINT(3), TYPEINT(3)),
     (9, 2, 0xFFFFFFFF), (9, 2, 13), (9, 2, 0xFFFFFFFF), (9, 2, 13)),
    # %5 is used at 13 and 18 and defined nowhere
    ("undefined", _mod(6, TYPEINT(1), CONST(1, 2, 7), IADD(1, 3, 2, 5), (0x0004003D, 1, 4, 5)),
     (10, 4, 0xFFFFFFFF), (10, 4, 13), (10, 4, 0xFFFFFFFF), (10, 4, 13)),
    # a duplicate at 9, then %3 out of bound (bound 3) at 17: the position of
    # the primary class, out of bound
    ("out of bound first", _mod(3, TYPEINT(1), TYPEINT(1), CONST(1, 2, 7), (0x0003003E, 1, 3)),
     (8, 3, 0xFFFFFFFF), (8, 3, 17), (8, 3, 0xFFFFFFFF), (8, 3, 17)),
    # result ID 0 at 9 (ID 0 is never valid), %5 out of bound (bound 3) at 13
    ("ID 0", _mod(3, TYPEINT(1), CONST(1, 0, 7), (0x0003003E, 1, 5)),
     (8, 1, 0xFFFFFFFF), (8, 1, 9), (8, 1, 0xFFFFFFFF), (8, 1, 9)),
    # OpName %2 "x" at 5 (a forward use, allowed), OpConstant at 8 uses %1
    # that OpTypeInt defines only at 12: valid, but not in defined-before-use
    ("use before definition", _mod(4, (0x00030005, 2, 0x78), CONST(1, 2, 7), TYPEINT(1), IADD(1, 3, 2, 2)),
     (0, 0, 0xFFFFFFFF), (0, 0, 0xFFFFFFFF), (10, 4, 0xFFFFFFFF), (10, 4, 8)),
    # OpIAdd at 9 reads its own result %2
    ("self use", _mod(3, TYPEINT(1), IADD(1, 2, 2, 1)),
     (0, 0, 0xFFFFFFFF), (0, 0, 0xFFFFFFFF), (10, 4, 0xFFFFFFFF), (10, 4, 9)),
    # OpEntryPoint Kernel %2 "m" names the function defined after it: allowed
    ("entry point forward", _mod(3, (0x0004000F, 6, 2, 0x6D), TYPEINT(1), (0x00050036, 1, 2, 0, 1)),
     (0, 0, 0xFFFFFFFF), (0, 0, 0xFFFFFFFF), (0, 0, 0xFFFFFFFF), (0, 0, 0xFFFFFFFF)),
    # a parse failure keeps its own offset whatever the options
    ("parse failure", _mod(3, TYPEINT(1), (0x00010063,)),
     (6, 0, 9), (6, 0, 9), (6, 0, 9), (6, 0, 9)),
]
OPTS = [dict(), dict(offsets=True), dict(before_use=True), dict(offsets=True, before_use=True)]


@pytest.mark.parametrize("name,words,plain,off,bu,both", CASES, ids=[c[0] for c in CASES])
def test_hand_written_positions(name, words, plain, off, bu, both):
    for kw, want in zip(OPTS, (plain, off, bu, both)):
        r = oracle.validate(words, [0, words.size], index=False, **kw)[0]
        assert (int(r["code"]), int(r["sem_mask"]), int(r["err_word"])) == want, (name, kw)
        assert spec.check(words, **kw)[:3] == want, (name, kw, "spec")


def test_rules_follow_the_before_use_stage():
    """The module-level rules apply only to a module that passes every other
    check, defined-before-use included."""
    w = [c for c in CASES if c[0] == "use before definition"][0][1]
    r = oracle.validate(w, [0, w.size], index=False, rules=True)[0]
    assert int(r["code"]) == 11  # no capability, memory model, function or entry point
    r = oracle.validate(w, [0, w.size], index=False, rules=True, before_use=True)[0]
    assert int(r["code"]) == 10


def _tiny(rng):
    ops = [TYPEINT, CONST, IADD]
    body = []
    for _ in range(int(rng.integers(1, 7))):
        ids = [int(x) for x in rng.integers(0, 6, size=4)]
        k = int(rng.integers(0, 6))
        if k == 0:
            body.append(TYPEINT(ids[0]))
        elif k == 1:
            body.append(CONST(ids[0], ids[1], 7))
        elif k == 2:
            body.append(IADD(*ids))
        elif k == 3:
            body.append((0x00030005, ids[0], 0x61))           # OpName
        elif k == 4:
            body.append((0x0004000F, 6, ids[0], 0x61))        # OpEntryPoint
        else:
            body.append((0x0004003D, ids[0], ids[1], ids[2]))  # OpLoad
    return _mod(int(rng.integers(1, 7)), *body)


def test_random_tiny_modules_agree_with_second_statement():
    rng = np.random.default_rng(21)
    for _ in range(3000):
        w = _tiny(rng)
        for kw in OPTS + [dict(offsets=True, before_use=True, rules=True)]:
            r = oracle.validate(w, [0, w.size], index=False, **kw)[0]
            got = (int(r["code"]), int(r["sem_mask"]), int(r["err_word"]))
            assert got == spec.check(w, **kw)[:3], (w.tolist(), kw)


def test_generated_modules_with_rewritten_ids():
    rng = np.random.default_rng(22)
    for seed in range(60):
        m = spvgen.gen_module([50, seed], int(rng.integers(5, 400)))
        w = m.words.copy()
        for _ in range(int(rng.integers(0, 4))):
            i = int(rng.integers(5, w.size))
            w[i] = int(rng.integers(0, 12))
        for kw in OPTS:
            r = oracle.validate(w, [0, w.size], index=False, **kw)[0]
            assert (int(r["code"]), int(r["sem_mask"]), int(r["err_word"])) == spec.check(w, **kw)[:3], (seed, kw)


def test_generated_modules_pass_defined_before_use():
    """The generator draws every use from earlier results (its entry point
    names the function that follows it): valid in the stricter mode too."""
    b = spvgen.config3(n_modules=40, n_faults=0, median=300.0, hi=3000)
    r = oracle.validate(b.words, b.mod_off, index=False, before_use=True, offsets=True)
    assert np.all(r["code"] == 0)
