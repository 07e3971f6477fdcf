"""Pins of the CPU oracle against facts fixed outside the oracle itself:
the paper's worked examples (tests/golden), the generator's by-construction
layout and faults, numpy set definitions, round-trip identity and the header
rules of the binary format."""
import numpy as np
import pytest

import oracle
import spvgen


def _recs_to_arrays(recs):
    op = np.array([r[0] for r in recs], np.uint16)
    opnd = np.array([v for r in recs for v in r[1]], np.uint32)
    opnd_off = np.concatenate([[0], np.cumsum([len(r[1]) for r in recs])]).astype(np.int32)
    chars = np.frombuffer(b"".join(r[2] for r in recs), np.uint8)
    str_off = np.concatenate([[0], np.cumsum([len(r[2]) for r in recs])]).astype(np.int32)
    return op, opnd_off, opnd, str_off, chars


def test_paper_examples_encode(golden_cases):
    """Section "Examples" / header listing: records -> the hand-derived words."""
    for case in golden_cases:
        op, opnd_off, opnd, str_off, chars = _recs_to_arrays(case["recs"])
        words, wmo, code, bad = oracle.encode(op, opnd_off, opnd, str_off, chars,
                                              np.array([0, len(case["recs"])], np.int64),
                                              case["version"], case["generator"])
        assert code[0] == 0 and bad[0] == -1, case["name"]
        assert [int(x) for x in words] == case["words"], case["name"]
        assert list(wmo) == [0, len(case["words"])]


def test_paper_examples_decode(golden_cases):
    """The disassembler view of the same words: one instruction per record,
    each at 5 + the sum of the earlier word counts, and the records back."""
    for case in golden_cases:
        w = np.array(case["words"], np.uint32)
        res, io, iop = oracle.validate(w, [0, w.size])
        assert res[0]["code"] == 0 and res[0]["n_inst"] == len(case["recs"]), case["name"]
        assert [int(x) for x in iop[:len(case["recs"])]] == [r[0] for r in case["recs"]]
        pos = 5
        for j, r in enumerate(case["recs"]):
            assert io[j] == pos
            pos += 1 + len(r[1]) + ((len(r[2]) // 4 + 1) if r[0] in (5, 15) else 0)
        rec = oracle.records(w, [0, w.size])
        assert [int(x) for x in rec["opnd"]] == [v for r in case["recs"] for v in r[1]]
        assert bytes(rec["chars"]) == b"".join(r[2] for r in case["recs"])


def test_generator_layout_pins_index():
    """starts == 5 + exclusive cumsum of the generator's own word counts."""
    for seed, n in [(1, 10_000), (5, 777), (9, 5)]:
        m = spvgen.gen_module(seed, n)
        res, io, iop = oracle.validate(m.words, [0, m.words.size])
        assert res[0]["code"] == 0 and res[0]["sem_mask"] == 0 and res[0]["n_inst"] == n
        expect = 5 + np.concatenate([[0], np.cumsum(m.wc)[:-1]])
        assert np.array_equal(io[:n], expect)
        assert np.array_equal(iop[:n], m.opcodes)


def test_injected_faults_known_by_construction():
    b = spvgen.config3(n_modules=240, n_faults=60)
    res = oracle.validate(b.words, b.mod_off, index=False)
    n_checked = 0
    for i, m in enumerate(b.modules):
        got = tuple(int(res[i][k]) for k in ("code", "sem_mask", "err_word", "n_inst"))
        if m.expect is None:
            assert got == (0, 0, 0xFFFFFFFF, m.n_inst)
        else:
            e = m.expect
            assert got == (e["code"], e["sem_mask"], e["err_word"], e["n_inst"]), (i, e, got)
            n_checked += 1
    assert n_checked == 60


def _id_slots(m):
    d, u = [], []
    for i in range(m.n_inst):
        for s, role in enumerate(spvgen.ROLES[m.kind[i]]):
            if role == "D":
                d.append(m.starts[i] + 1 + s)
            elif role == "U":
                u.append(m.starts[i] + 1 + s)
    return np.array(d, np.int64), np.array(u, np.int64)


def test_semantic_against_numpy_sets():
    """OOB / DUP / UNDEF from np.unique and np.setdiff1d over the generator's
    own slot positions, after random rewrites of ID words and of the bound."""
    rng = np.random.default_rng(123)
    seen = set()
    for trial in range(120):
        m = spvgen.gen_module([77, trial], int(rng.integers(5, 400)))
        dpos, upos = _id_slots(m)
        w = m.words.copy()
        allpos = np.concatenate([dpos, upos])
        for _ in range(int(rng.integers(0, 4))):
            p = allpos[rng.integers(0, allpos.size)]
            w[p] = rng.integers(0, m.bound + 2)
        if rng.integers(0, 4) == 0:
            w[3] = rng.integers(0, m.bound + 3)
        bound = int(w[3])
        dv, uv = w[dpos].astype(np.int64), w[upos].astype(np.int64)
        oob = bool(np.any((dv == 0) | (dv >= bound)) or np.any((uv == 0) | (uv >= bound)))
        dv_in = dv[(dv > 0) & (dv < bound)]
        uv_in = uv[(uv > 0) & (uv < bound)]
        _, counts = np.unique(dv_in, return_counts=True)
        dup = bool(np.any(counts > 1))
        undef = np.setdiff1d(uv_in, dv_in).size > 0
        mask = int(oob) | 2 * int(dup) | 4 * int(undef)
        code = 8 if oob else 9 if dup else 10 if undef else 0
        res = oracle.validate(w, [0, w.size], index=False)
        assert (int(res[0]["code"]), int(res[0]["sem_mask"])) == (code, mask), trial
        seen.add(mask)
    assert len(seen) >= 5


def test_round_trip_identity():
    """encode(records(decode(w))) == w and decode(encode(r)) == r."""
    mods = [spvgen.gen_module([8, i], n) for i, n in enumerate([5, 10, 100, 2_500])]
    b = spvgen.pack(mods)
    rec = oracle.records(b.words, b.mod_off)
    w, wmo, code, bad = oracle.encode(rec["op"], rec["opnd_off"], rec["opnd"], rec["str_off"], rec["chars"],
                                      rec["rec_mod_off"])
    assert np.array_equal(w, b.words) and np.array_equal(wmo, b.mod_off)
    assert np.all(code == 0) and np.all(bad == -1)
    r2 = spvgen.pack_records(mods)
    for k in ("op", "opnd_off", "opnd", "str_off", "chars", "rec_mod_off"):
        assert np.array_equal(rec[k], r2[k]), k


def test_encode_sizes():
    """sum(wc) + 5 == module words; OpName string takes floor(L/4)+1 words."""
    mods = [spvgen.gen_module([9, i], 500) for i in range(3)]
    r = spvgen.pack_records(mods)
    w, wmo, code, bad = oracle.encode(**r)
    for i, m in enumerate(mods):
        assert wmo[i + 1] - wmo[i] == 5 + int(m.wc.sum())


HDR = [0x07230203, 0x00010600, 0, 10, 0]


@pytest.mark.parametrize("words,expect", [
    ([], (1, 0, 0, 0)),
    ([0x07230203], (1, 0, 1, 0)),
    ([0x07230203, 0x00010600, 0, 10], (1, 0, 4, 0)),
    ([0x03022307, 0x00010600, 0, 10, 0], (2, 0, 0, 0)),       # byte-swapped magic
    ([0x07230203, 0x00010700, 0, 10, 0], (3, 0, 1, 0)),       # minor 7
    ([0x07230203, 0x00020000, 0, 10, 0], (3, 0, 1, 0)),       # major 2
    ([0x07230203, 0x00010601, 0, 10, 0], (3, 0, 1, 0)),       # reserved low byte
    ([0x07230203, 0x01010600, 0, 10, 0], (3, 0, 1, 0)),       # reserved high byte
    ([0x07230203, 0x00010000, 0, 10, 0], (0, 0, 0xFFFFFFFF, 0)),  # 1.0, empty module
    ([0x07230203, 0x00010600, 0, 10, 1], (4, 0, 4, 0)),       # schema 1
    (HDR + [0x00000011], (5, 0, 5, 0)),                       # wc 0
    (HDR + [0x00030011, 6], (5, 0, 5, 0)),                    # overrun
    (HDR + [0x00020011, 6, 0x00020063, 1], (6, 0, 7, 1)),     # unknown opcode 99
    (HDR + [0x00030011, 6, 7], (5, 0, 5, 0)),                 # OpCapability with 3 words
    (HDR + [0x00020005, 1], (5, 0, 5, 0)),                    # OpName with 2 words
    (HDR + [0x00030005, 1, 0x64636261], (7, 0, 5, 0)),        # no terminator
    (HDR + [0x00040005, 1, 0x00636261, 0], (7, 0, 5, 0)),     # NUL before the last word
    (HDR + [0x00030005, 1, 0x61000062], (7, 0, 5, 0)),        # byte after NUL
    (HDR + [0x00030005, 1, 0x00000000], (10, 4, 0xFFFFFFFF, 1)),  # empty name; %1 undefined
    (HDR + [0x000200F8, 0], (8, 1, 0xFFFFFFFF, 1)),           # ID 0
    (HDR + [0x000200F8, 10], (8, 1, 0xFFFFFFFF, 1)),          # ID == bound
    (HDR + [0x000200F8, 3, 0x000200F8, 3], (9, 2, 0xFFFFFFFF, 2)),
    (HDR + [0x00030005, 3, 0x00006162, 0x000200F8, 3], (0, 0, 0xFFFFFFFF, 2)),  # forward reference
])
def test_rules(words, expect):
    res = oracle.validate(np.array(words, np.uint32), [0, len(words)], index=False)
    assert tuple(int(res[0][k]) for k in ("code", "sem_mask", "err_word", "n_inst")) == expect


def test_records_of_failing_modules():
    """Records mode keeps each module's valid instruction prefix: none when
    the header check fails, the instructions before the failing one when the
    parse stage fails, every instruction when only the semantic stage fails.
    Hand-written words; the expected records are read off them."""
    LBL = [0x000200F8, 1]                              # %1 = OpLabel
    ENT = [0x0005000F, 6, 1, 0x6E69616D, 0]            # OpEntryPoint Kernel %1 "main"
    mods = [
        [0x07230203, 0x00010700, 0, 5, 0] + LBL,       # minor 7: header fails
        [0x07230203, 0x00010600, 0],                   # truncated header
        HDR + LBL + [0x00020063, 1] + LBL,             # unknown opcode 99 second
        HDR + [0x00020011, 6, 0x00030011, 6, 7] + LBL,  # OpCapability with 3 words second
        HDR + LBL + [0x00030005, 1, 0x64636261] + LBL,  # OpName without terminator second
        HDR + [0x00030011, 6] + LBL,                   # first instruction overruns into the next one
        HDR + LBL + LBL,                               # %1 defined twice: semantic only
        HDR + ENT + LBL,                               # valid, with an entry point
    ]
    sizes = np.array([len(m) for m in mods], np.int64)
    mod_off = np.concatenate([[0], np.cumsum(sizes)])
    words = np.array([x for m in mods for x in m], np.uint32)
    expect = [[], [], [(248, [1], b"")], [(17, [6], b"")], [(248, [1], b"")],
              [(17, [6, 0x000200F8], b"")][:0], [(248, [1], b""), (248, [1], b"")],
              [(15, [6, 1], b"main"), (248, [1], b"")]]
    rec = oracle.records(words, mod_off)
    got = []
    for m in range(len(mods)):
        out = []
        for r in range(int(rec["rec_mod_off"][m]), int(rec["rec_mod_off"][m + 1])):
            a, b = int(rec["opnd_off"][r]), int(rec["opnd_off"][r + 1])
            c, d = int(rec["str_off"][r]), int(rec["str_off"][r + 1])
            out.append((int(rec["op"][r]), [int(x) for x in rec["opnd"][a:b]], bytes(rec["chars"][c:d])))
        got.append(out)
    assert got == expect
    res = oracle.validate(words, mod_off, index=False)
    assert [int(x) for x in res["code"]] == [3, 1, 6, 5, 7, 5, 9, 0]
    assert [int(x) for x in res["n_inst"]] == [len(e) for e in expect]


def test_decode_has_no_semantic_stage():
    w = np.array(HDR + [0x000200F8, 3, 0x000200F8, 3], np.uint32)
    res = oracle.decode(w, [0, w.size], index=False)
    assert (res[0]["code"], res[0]["sem_mask"], res[0]["n_inst"]) == (0, 0, 2)


@pytest.mark.parametrize("rec,code", [
    ((99, [1], b""), oracle.ENC_UNKNOWN_OPCODE),
    ((17, [1, 2], b""), oracle.ENC_OPERAND_COUNT),
    ((5, [], b"ab"), oracle.ENC_OPERAND_COUNT),
    ((17, [6], b"x"), oracle.ENC_BAD_STRING),
    ((5, [1], b"a\x00b"), oracle.ENC_BAD_STRING),
    ((5, [1], b"a" * 4 * 65533), oracle.ENC_TOO_LONG),
    ((248, [0xFFFFFFFF], b""), oracle.ENC_BAD_ID),
])
def test_encode_failures(rec, code):
    recs = [(248, [1], b""), rec, (253, [], b"")]
    op, opnd_off, opnd, str_off, chars = _recs_to_arrays(recs)
    # a good module after the bad one keeps its words; the bad one has none
    op = np.concatenate([op, [248]]).astype(np.uint16)
    opnd_off = np.concatenate([opnd_off, [opnd_off[-1] + 1]]).astype(np.int32)
    opnd = np.concatenate([opnd, [7]]).astype(np.uint32)
    str_off = np.concatenate([str_off, [str_off[-1]]]).astype(np.int32)
    w, wmo, c, bad = oracle.encode(op, opnd_off, opnd, str_off, chars, np.array([0, 3, 4], np.int64))
    assert list(c) == [code, 0] and list(bad) == [1, -1]
    assert list(wmo) == [0, 0, 7]
    assert [int(x) for x in w] == [0x07230203, 0x00010600, 0, 8, 0, 0x000200F8, 7]


def test_encode_longest_name_fits():
    # 2 + floor(L/4) + 1 == 65535 is the largest encodable OpName
    L = 4 * 65532
    recs = [(5, [1], b"a" * L)]
    op, opnd_off, opnd, str_off, chars = _recs_to_arrays(recs)
    w, wmo, c, bad = oracle.encode(op, opnd_off, opnd, str_off, chars, np.array([0, 1], np.int64))
    assert c[0] == 0 and w[5] >> 16 == 65535
