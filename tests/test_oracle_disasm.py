"""Pins of the oracle's disassembly to text (section "Dis/Assembler"): the
paper's printed disassembly of its capabilities example and hand-written
texts for every option (tests/golden/disassembly.txt), agreement with the
second statement of the format in oracle/spec.py on generated and random tiny
modules under all 32 option sets, batch layout and truncation."""
import os

import numpy as np
import pytest

import oracle
import spvgen
from conftest import ROOT
from oracle import spec

GOLDEN = os.path.join(ROOT, "tests", "golden", "disassembly.txt")


def parse_disasm_golden(path=GOLDEN):
    cases, cur, in_text = [], None, False
    with open(path) as f:
        for raw in f:
            line = raw.rstrip("\n")
            if in_text:
                if line == "endtext":
                    in_text = False
                    cases.append(cur)
                else:
                    cur["text"] += line.replace("<ESC>", "\x1b") + "\n"
                continue
            if not line or line.startswith("#"):
                continue
            tag, *rest = line.split()
            if tag == "case":
                cur = {"name": rest[0], "options": int(rest[1]), "words": [], "text": ""}
            elif tag == "words":
                cur["words"] += [int(x, 16) for x in rest]
            elif tag == "text":
                in_text = True
    return cases


CASES = parse_disasm_golden()


def test_golden_file_has_every_option():
    assert len(CASES) >= 10
    seen = 0
    for c in CASES:
        seen |= c["options"]
    assert seen == 31


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_golden_disassembly(case):
    w = np.array(case["words"], np.uint32)
    text, tmo, total = oracle.disassemble(w, [0, w.size], case["options"])
    assert text.decode("latin-1") == case["text"]
    assert list(tmo) == [0, total] and total == len(case["text"])


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_golden_second_statement(case):
    assert spec.disassemble_module(case["words"], case["options"]).decode("latin-1") == case["text"]


def test_paper_listing_is_the_capabilities_text():
    """The capabilities example: with no header and no indentation the text is
    exactly the paper's five lines."""
    c = [c for c in CASES if c["name"] == "capabilities_paper"][0]
    lines = ["OpCapability " + n for n in ("Addresses", "Linkage", "Kernel", "Int64", "Int8")]
    w = np.array(c["words"], np.uint32)
    assert oracle.disassemble(w, [0, w.size], 20)[0].decode().splitlines() == lines


@pytest.mark.parametrize("options", range(32))
def test_generated_modules_agree_with_second_statement(options):
    for seed in range(6):
        m = spvgen.gen_module([seed, options], 300)
        t, tmo, total = oracle.disassemble(m.words, [0, m.words.size], options)
        assert t == spec.disassemble_module(m.words, options), (seed, options)


def _tiny_module(rng):
    """A short module of random instructions of the grammar (decode-only:
    IDs are random small numbers, literals are drawn near the enumerant
    tables' edges, names from a small alphabet that includes the escaped
    characters), sometimes ending in a malformed instruction."""
    body = []
    for _ in range(int(rng.integers(0, 8))):
        op = int(rng.choice([5, 14, 15, 17, 21, 43, 54, 56, 61, 62, 128, 248, 253]))
        small = lambda: int(rng.choice([0, 1, 2, 3, 5, 6, 7, 9, 11, 12, 13, 16, 22, 39, 100, 0xFFFFFFFF]))
        if op in (5, 15):
            n = int(rng.integers(0, 7))
            name = bytes(rng.choice(list(b'ab9_Z"\\-'), size=n).astype(np.uint8))
            sw = name + b"\x00" * (4 - len(name) % 4)
            fixed = [small()] if op == 5 else [small(), small()]
            words = fixed + list(np.frombuffer(sw, "<u4").astype(np.int64))
        else:
            n = {14: 2, 17: 1, 21: 3, 43: 3, 54: 4, 56: 0, 61: 3, 62: 2, 128: 4, 248: 1, 253: 0}[op]
            words = [small() for _ in range(n)]
        body += [((1 + len(words)) << 16) | op] + words
    if rng.random() < 0.2:
        body += [int(rng.choice([0x00010063, 0x00090011, 0x00030005]))]
    hdr = [0x07230203, int(rng.choice([0x00010000, 0x00010600, 0x00010300])), int(rng.integers(0, 40)),
           int(rng.integers(0, 30)), 0]
    return np.array(hdr + body, np.uint32)


def test_random_tiny_modules_agree_with_second_statement():
    rng = np.random.default_rng(12)
    for _ in range(1500):
        w = _tiny_module(rng)
        options = int(rng.integers(0, 32))
        t, _, _ = oracle.disassemble(w, [0, w.size], options)
        assert t == spec.disassemble_module(w, options), (w.tolist(), options)


def test_batch_offsets_and_truncation():
    mods = [spvgen.gen_module(s, n).words for s, n in [(1, 50), (2, 5), (3, 200)]]
    bad = np.array([0x07230203, 0x00020000, 0, 1, 0], np.uint32)  # bad version: no text
    mods.insert(1, bad)
    words = np.concatenate(mods)
    mod_off = np.concatenate([[0], np.cumsum([m.size for m in mods])]).astype(np.int64)
    for options in (0, 2, 31):
        text, tmo, total = oracle.disassemble(words, mod_off, options)
        parts = [spec.disassemble_module(m, options) for m in mods]
        assert text == b"".join(parts)
        assert list(np.diff(tmo)) == [len(p) for p in parts]
        assert tmo[2] == tmo[1]
        for cap in (0, 1, total // 3, total - 1, total, total + 7):
            t2, tmo2, total2 = oracle.disassemble(words, mod_off, options, text_cap=cap)
            assert total2 == total and t2 == text[:min(cap, total)] and np.array_equal(tmo2, tmo)
