"""Brute force: every opcode sequence of up to three instructions (with ID
assignments from {0..4} and bounds from {0..5}) and every single-field
mutation of small modules, oracle.c against the independent checker in
oracle/spec.py, including the instruction index."""
import itertools

import numpy as np

import oracle
from oracle import spec

OPCODES = sorted(spec.KINDS)
NAMES = [b"", b"a", b"abc", b"abcd", b"abcdefgh"]


def _inst_words(opcode, ids, name):
    kinds = spec.KINDS[opcode]
    out, k = [], 0
    body = []
    for kind in kinds:
        if kind in ("id", "result"):
            body.append(ids[k])
            k += 1
        elif kind == "lit":
            body.append(32)
        else:  # string
            padded = name + b"\x00"
            padded += b"\x00" * (-len(padded) % 4)
            body.extend(int.from_bytes(padded[i:i + 4], "little") for i in range(0, len(padded), 4))
    out.append((1 + len(body)) << 16 | opcode)
    return out + body


def _n_ids(opcode):
    return sum(k in ("id", "result") for k in spec.KINDS[opcode])


def _modules():
    rng = np.random.default_rng(2305)
    mods = []
    for length in range(4):
        for seq in itertools.product(OPCODES, repeat=length):
            s = sum(_n_ids(o) for o in seq)
            if 5 ** s <= 25:
                assigns = list(itertools.product(range(5), repeat=s))
            else:
                assigns = [tuple(rng.integers(0, 5, size=s)) for _ in range(12)]
            for a_i, a in enumerate(assigns):
                words, k = [], 0
                for j, o in enumerate(seq):
                    n = _n_ids(o)
                    words += _inst_words(o, a[k:k + n], NAMES[(a_i + j) % len(NAMES)])
                    k += n
                bound = a_i % 6
                mods.append([0x07230203, 0x00010600, 0, bound, 0] + words)
    return mods


def _mutations(base, rng):
    out = []
    for p in range(len(base)):
        w = base[p]
        vals = {w ^ 0xFF, 0, 0xFFFFFFFF}
        if p >= 5:
            wc, op = w >> 16, w & 0xFFFF
            vals |= {(wc + 1) << 16 | op, max(wc - 1, 0) << 16 | op, 0xFFFF << 16 | op, wc << 16 | 999,
                     wc << 16, w & 0xFFFF00FF}
        else:
            vals |= {0x03022307, 0x00010700, 0x00010000, 0x00020000, 1, w + 1}
        for v in vals:
            m = list(base)
            m[p] = v & 0xFFFFFFFF
            out.append(m)
    out.append(base[:-1])
    out.append(base + [0])
    return out


def _compare(mods, semantic, rules=False):
    sizes = np.array([len(m) for m in mods], np.int64)
    mod_off = np.concatenate([[0], np.cumsum(sizes)])
    words = np.array([x for m in mods for x in m], np.uint32)
    res, io, iop = oracle.validate(words, mod_off, semantic=semantic, rules=rules)
    for i, m in enumerate(mods):
        code, mask, err, n_inst, insts = spec.check(m, semantic=semantic, rules=rules)
        got = tuple(int(res[i][k]) for k in ("code", "sem_mask", "err_word", "n_inst"))
        assert got == (code, mask, err, n_inst), (m, got)
        b = mod_off[i]
        assert [(int(io[b + j]), int(iop[b + j])) for j in range(n_inst)] == insts
    return res


def test_bruteforce_small_modules():
    mods = _modules()
    assert len(mods) > 10_000
    _compare(mods, True)


def test_bruteforce_single_field_mutations():
    rng = np.random.default_rng(9493)
    bases = _modules()
    pick = rng.choice(len(bases), size=150, replace=False)
    mods = []
    for i in pick:
        mods += _mutations(bases[i], rng)
    _compare(mods, True)
    _compare(mods[::7], False)


def test_bruteforce_encode():
    """Encoding records with the same enumeration agrees with spec.encode_module."""
    rng = np.random.default_rng(55)
    recs_all = []
    for length in range(3):
        for seq in itertools.product(OPCODES + [99], repeat=length):
            for t in range(3):
                recs = []
                for j, o in enumerate(seq):
                    kinds = spec.KINDS.get(o, ("id",))
                    n = 1 if "str" in kinds else len(kinds)
                    n += int(rng.integers(-1, 2)) if rng.random() < 0.15 else 0
                    ops = [int(rng.choice([1, 2, 3, 0xFFFFFFFF] if rng.random() < 0.1 else [1, 2, 3]))
                           for _ in range(max(n, 0))]
                    name = NAMES[(t + j) % len(NAMES)]
                    if rng.random() < 0.1:
                        name = b"x\x00y" if "str" in kinds else b"z"
                    recs.append((o, ops, name if ("str" in kinds or rng.random() < 0.1) else b""))
                recs_all.append(recs)
    op = np.array([r[0] for recs in recs_all for r in recs], np.uint16)
    opnd = np.array([v for recs in recs_all for r in recs for v in r[1]], np.uint32)
    opnd_off = np.concatenate([[0], np.cumsum([len(r[1]) for recs in recs_all for r in recs])]).astype(np.int32)
    chars = np.frombuffer(b"".join(r[2] for recs in recs_all for r in recs), np.uint8)
    str_off = np.concatenate([[0], np.cumsum([len(r[2]) for recs in recs_all for r in recs])]).astype(np.int32)
    rec_mod_off = np.concatenate([[0], np.cumsum([len(recs) for recs in recs_all])]).astype(np.int64)
    w, wmo, code, bad = oracle.encode(op, opnd_off, opnd, str_off, chars, rec_mod_off)
    for i, recs in enumerate(recs_all):
        exp = spec.encode_module(recs)
        if isinstance(exp, tuple):
            assert (int(code[i]), int(bad[i])) == exp and wmo[i + 1] == wmo[i], (recs, code[i], bad[i])
        else:
            assert code[i] == 0 and [int(x) for x in w[wmo[i]:wmo[i + 1]]] == exp, recs


def _rule_subset_modules():
    """Every subset of the four rule opcodes (capability, memory model,
    function, entry point) in several orders, around an OpTypeInt %1; the
    function is %2 = OpFunction %1 None %1 and the entry point names %2 when
    the function is present, else %1 (the rules do not look at its type)."""
    rng = np.random.default_rng(674)
    mods = []
    for bits in range(16):
        has = [bool(bits >> k & 1) for k in range(4)]
        parts = [[4 << 16 | 21, 1, 32, 0]]
        if has[0]:
            parts.append([2 << 16 | 17, 6])
        if has[1]:
            parts.append([3 << 16 | 14, 2, 2])
        if has[2]:
            parts.append([5 << 16 | 54, 1, 2, 0, 1])
        if has[3]:
            parts.append([5 << 16 | 15, 6, 2 if has[2] else 1, 0x6E69616D, 0])
        for _ in range(4):
            order = rng.permutation(len(parts))
            body = [w for i in order for w in parts[i]]
            mods.append([0x07230203, 0x00010600, 0, 3 if has[2] else 2, 0] + body)
    return mods


def test_bruteforce_module_rules():
    """With the module-level rules: every presence pattern of the four rule
    opcodes, against the independent checker."""
    mods = _modules() + _rule_subset_modules()
    res = _compare(mods, True, rules=True)
    rules = res["code"] == oracle.E_MODULE_RULES
    assert set(int(x) for x in np.unique(res["sem_mask"][rules])) == set(range(8, 128, 8))
    assert int(np.sum(res["code"] == 0)) > 0
    # without the rules the same modules keep their codes, except that rule
    # failures read as valid
    plain = _compare(mods, True)
    assert np.array_equal(plain["code"][~rules], res["code"][~rules])
    assert np.all(plain["code"][rules] == 0)
