"""GPU parity: decode's text mode (spv_decode_text, disassembly to text)
against the oracle's disassembly, byte for byte, with text_mod_off compared
element by element: the hand-written golden texts, one 10,000-instruction
module under all 32 option sets, lognormal faulted batches, many tiny modules
(header gaps inside every slice of lines), header failures and empty
modules, long instructions (slices wider than the LDS stage), results from
validate with the module rules, and a clipped text buffer."""
import numpy as np
import pytest

import oracle
import spvgen
from gpu_util import to_dev
from test_oracle_disasm import CASES

pytestmark = pytest.mark.gpu


def _gpu_text(words, mod_off, options, semantic=False, rules=False, cap=None):
    import torch

    import paper_2305_09493_amd as spv
    w, mo = to_dev(words, mod_off)
    if semantic:
        res, io, _ = spv.validate(w, mo, module_rules=rules)
    else:
        res, io, _ = spv.decode(w, mo)
    if cap is None:
        text, tmo = spv.decode_text(w, mo, io, res, options)
    else:
        buf = torch.full((cap + 64,), 0xAA, dtype=torch.uint8, device=w.device)
        text, tmo = spv.decode_text(w, mo, io, res, options, text=buf[:cap])
        torch.cuda.synchronize()
        assert bool((buf[cap:] == 0xAA).all()), "bytes past text_cap were written"
    torch.cuda.synchronize()
    tmo = tmo.cpu().numpy()
    return text.cpu().numpy().tobytes()[:min(int(tmo[-1]), text.numel())], tmo


def _check(words, mod_off, options, label, **kw):
    print(f"[text parity] {label} M={len(mod_off) - 1} W={len(words)} options={options}", flush=True)
    g, gtmo = _gpu_text(words, mod_off, options, **kw)
    o, otmo, total = oracle.disassemble(words, mod_off, options)
    assert np.array_equal(gtmo, otmo), (label, options, np.nonzero(gtmo != otmo)[0][:10])
    if g != o:
        k = next(i for i in range(min(len(g), len(o))) if g[i] != o[i]) if min(len(g), len(o)) else 0
        raise AssertionError(f"{label} options={options}: text differs at byte {k}: "
                             f"gpu {g[max(0, k - 60):k + 60]!r} oracle {o[max(0, k - 60):k + 60]!r}")


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_golden_texts(case):
    w = np.array(case["words"], np.uint32)
    g, tmo = _gpu_text(w, np.array([0, w.size], np.int64), case["options"])
    assert g.decode("latin-1") == case["text"]
    assert list(tmo) == [0, len(case["text"])]


def test_golden_texts_as_one_batch():
    for options in (0, 11, 26, 31):
        mods = [np.array(c["words"], np.uint32) for c in CASES]
        mod_off = np.concatenate([[0], np.cumsum([m.size for m in mods])]).astype(np.int64)
        _check(np.concatenate(mods), mod_off, options, "golden batch")


def test_one_module_all_options():
    b = spvgen.config1()
    for options in range(32):
        _check(b.words, b.mod_off, options, "10k instructions")


@pytest.mark.parametrize("options", [0, 11, 2, 31])
def test_lognormal_faulted_batch(options):
    b = spvgen.config3(n_modules=256, n_faults=12, median=1000.0, hi=20_000)
    w = b.words.copy()
    w[b.mod_off[7]] = 0x03022307  # byte-swapped magic: no text
    w[b.mod_off[11] + 4] = 1      # schema: no text
    _check(w, b.mod_off, options, "faulted lognormal batch")


def test_many_tiny_modules():
    """Modules of 5 to 12 instructions: every slice of 256 lines spans dozens
    of modules, so header text lies between its lines."""
    rng = np.random.default_rng(5)
    mods = [spvgen.gen_module([40, i], int(rng.integers(5, 13))) for i in range(3000)]
    b = spvgen.pack(mods)
    for options in (0, 3, 16, 27):
        _check(b.words, b.mod_off, options, "tiny modules")


def test_header_failures_and_empty_modules():
    mods = [spvgen.gen_module([41, i], 60).words for i in range(4)]
    hdr = np.array([0x07230203, 0x00010600, 7, 1, 0], np.uint32)  # a header, no instructions
    short = np.array([0x07230203, 0x00010600], np.uint32)        # truncated header
    bad = np.array([0x07230203, 0x00010700, 0, 1, 0], np.uint32)  # minor version 7
    parts = [hdr, mods[0], short, bad, hdr, hdr, mods[1], np.zeros(0, np.uint32), mods[2], hdr, short,
             mods[3], hdr, bad]
    words = np.concatenate(parts)
    mod_off = np.concatenate([[0], np.cumsum([p.size for p in parts])]).astype(np.int64)
    for options in (0, 2, 16, 31):
        _check(words, mod_off, options, "header failures and empty modules")
    _check(hdr, np.array([0, 5], np.int64), 0, "one header-only module")
    _check(short, np.array([0, 2], np.int64), 0, "one truncated module")


def test_long_instructions():
    """Names of thousands of words: a slice of lines wider than the LDS stage
    is written straight to memory; with inline names each use of a named ID
    repeats the name."""
    from test_gpu_long import _batch
    plans = [[("name", 20000, ("start", 17), None), ("name", 4097, ("next", 0), None)],
             [("entry", 65535, ("end", 0), None)],
             [("name", 4096, ("start", 0), None), ("name", 8200, ("start", 5), "tail")]]
    words, mod_off = _batch(plans, 21)
    for options in (0, 1, 2, 31):
        _check(words, mod_off, options, "long instructions")


def test_text_after_validate_with_rules():
    """Results of validate with the module rules (code 11 for modules that
    lack one) describe the same instructions as decode's."""
    mods = [spvgen.gen_module([42, i], 200) for i in range(6)]
    b = spvgen.pack(mods)
    w = b.words.copy()
    _, io, iop = oracle.validate(w, b.mod_off)
    base = int(b.mod_off[2])
    for j in range(200):  # every OpCapability of module 2 becomes two OpReturns
        if iop[base + j] == 17:
            p = base + int(io[base + j])
            w[p], w[p + 1] = 0x000100FD, 0x000100FD
    res = oracle.validate(w, b.mod_off, semantic=True, index=False, rules=True)
    assert res["code"][2] == oracle.E_MODULE_RULES
    _check(w, b.mod_off, 11, "validate with rules", semantic=True, rules=True)


def test_clipped_text_buffer():
    b = spvgen.config3(n_modules=64, n_faults=3, median=500.0, hi=5_000)
    o, otmo, total = oracle.disassemble(b.words, b.mod_off, 11)
    for cap in (4, 1000, total // 2 + 4 - (total // 2) % 4, total - 4):
        print(f"[text parity] clipped at {cap} of {total}", flush=True)
        g, gtmo = _gpu_text(b.words, b.mod_off, 11, cap=cap)
        assert np.array_equal(gtmo, otmo)
        assert g == o[:cap]
