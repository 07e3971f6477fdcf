"""GPU parity on valid instructions that span one or more whole tiles:
OpName and OpEntryPoint of 4095 to 65535 words placed at chosen offsets
within the kernels' 4096-word tiles (at a tile start, just after one, in the
middle, and ending exactly on a tile boundary), two long ones back to back,
and long names with a malformed terminator.  Decode, validate and records
mode are each compared with the oracle element by element.  Such batches
take the single-pass walk; the second pass (undefined-ID search) is checked
there and in a batch without a long instruction."""
import numpy as np
import pytest

import oracle
import spvgen
from gpu_util import compare, to_dev

pytestmark = pytest.mark.gpu

T = 4096  # words per tile of the kernels
RET = 0x000100FD  # OpReturn, one word: filler that moves the next start by one word


def _string_words(n_words, rng, bad=None):
    """n_words string words of a valid name (its first NUL in the last word),
    or, with `bad`, a malformed one: "nonul" (no NUL at all), "early" (a NUL
    in the first word), "tail" (a non-zero byte after the NUL)."""
    r = int(rng.integers(0, 4))
    L = 4 * n_words - 1 - r
    b = bytearray(rng.integers(97, 123, size=4 * n_words).astype(np.uint8).tobytes())
    for k in range(L, 4 * n_words):
        b[k] = 0
    if bad == "nonul":
        b[-1] = 0x61
        for k in range(L, 4 * n_words):
            b[k] = 0x62
    elif bad == "early":
        b[1] = 0
    elif bad == "tail":
        b[L] = 0
        b[4 * n_words - 1] = 0x63
        if L == 4 * n_words - 1:  # the NUL is the last byte: move it one back
            b[L - 1] = 0
    return [int.from_bytes(bytes(b[k:k + 4]), "little") for k in range(0, 4 * n_words, 4)]


def _long_inst(wc, rng, entry=False, bad=None):
    if entry:  # OpEntryPoint Kernel %1 "..." (the use of %1 is defined: OpTypeInt %1)
        return [(wc << 16) | 15, 6, 1] + _string_words(wc - 3, rng, bad)
    return [(wc << 16) | 5, 1] + _string_words(wc - 2, rng, bad)


def _module(base, seed, plan, rng):
    """A generated module whose words are placed at global offset `base`;
    plan: list of (kind, wc, where, bad) long instructions, where = ("start",
    r) puts its first word at tile offset r, ("end", 0) makes it end exactly
    on a tile boundary, ("next", 0) places it right after the previous one."""
    m = spvgen.gen_module(seed, 3000)
    starts = [int(s) for s in m.starts] + [m.words.size]
    cut = [starts[spvgen.N_PROLOGUE + 400 * k] for k in range(len(plan) + 1)]
    out = [int(x) for x in m.words[:cut[0]]]
    pending = []  # body pieces held back until a run of back-to-back instructions ends
    for k, (kind, wc, where, bad) in enumerate(plan):
        if where[0] != "next":
            pos = base + len(out)
            if where[0] == "start":
                want = where[1]
            else:  # end on a tile boundary
                want = (-wc) % T
            out += [RET] * ((want - pos) % T)
        out += _long_inst(wc, rng, entry=(kind == "entry"), bad=bad)
        pending.append(k)
        if k + 1 < len(plan) and plan[k + 1][2][0] == "next":
            continue
        for j in pending:
            out += [int(x) for x in m.words[cut[j]:cut[j + 1]]]
        pending = []
    out += [int(x) for x in m.words[cut[len(plan)]:]]
    return np.array(out, np.uint32)


def _batch(plans, seed):
    rng = np.random.default_rng(seed)
    mods, base = [], 0
    for i, plan in enumerate(plans):
        w = _module(base, [seed, i], plan, rng)
        mods.append(w)
        base += w.size
    mod_off = np.concatenate([[0], np.cumsum([w.size for w in mods])]).astype(np.int64)
    return np.concatenate(mods), mod_off


WCS = [4095, 4096, 4097, 8200, 20000, 65535]


def _check_all(words, mod_off, label):
    compare(words, mod_off, label=label + " validate")
    compare(words, mod_off, semantic=False, label=label + " decode")
    compare(words, mod_off, index=False, label=label + " validate, no index")
    _records(words, mod_off, label)


def _records(words, mod_off, label):
    import torch

    import paper_2305_09493_amd as spv
    print(f"[records parity] {label}", flush=True)
    w, mo = to_dev(words, mod_off)
    res, io, _ = spv.decode(w, mo)
    rec = spv.decode_records(w, mo, io, res)
    torch.cuda.synchronize()
    o = oracle.records(words, mod_off)
    rmo = rec["rec_mod_off"].cpu().numpy()
    n = int(rmo[-1])
    assert np.array_equal(rmo, o["rec_mod_off"]), label
    assert np.array_equal(rec["op"].cpu().numpy().view(np.uint16)[:n], o["op"]), label
    oo = rec["opnd_off"].cpu().numpy()[:n + 1]
    so = rec["str_off"].cpu().numpy()[:n + 1]
    assert np.array_equal(oo, o["opnd_off"]) and np.array_equal(so, o["str_off"]), label
    assert np.array_equal(rec["opnd"].cpu().numpy().view(np.uint32)[:oo[-1]], o["opnd"]), label
    assert np.array_equal(rec["chars"].cpu().numpy()[:so[-1]], o["chars"]), label


@pytest.mark.parametrize("wc", WCS)
def test_long_opname_at_tile_offsets(wc):
    plans = [[("name", wc, ("start", 0), None)],
             [("name", wc, ("start", 1), None)],
             [("name", wc, ("start", 2047), None)],
             [("name", wc, ("end", 0), None)],
             [("name", wc, ("start", 4090), None)]]
    words, mod_off = _batch(plans, 100 + wc % 1000)
    _check_all(words, mod_off, f"OpName wc={wc}")


def test_long_instructions_back_to_back_and_entry_points():
    plans = [[("name", 4097, ("start", 3), None), ("name", 8200, ("next", 0), None)],
             [("entry", 65535, ("end", 0), None), ("name", 4095, ("next", 0), None)],
             [("entry", 4096, ("start", 0), None), ("entry", 20000, ("next", 0), None),
              ("name", 4096, ("next", 0), None)],
             [("name", 20000, ("start", 17), None), ("name", 65535, ("start", 5), None)]]
    words, mod_off = _batch(plans, 7)
    _check_all(words, mod_off, "back to back")


@pytest.mark.parametrize("bad", ["nonul", "early", "tail"])
def test_long_name_with_bad_terminator(bad):
    plans = [[("name", 8200, ("start", 9), bad)],
             [("name", 4096, ("end", 0), None), ("name", 20000, ("next", 0), bad)],
             [("entry", 4097, ("start", 0), bad)],
             [("name", 4095, ("start", 1), None)]]
    words, mod_off = _batch(plans, 11)
    o = oracle.validate(words, mod_off, semantic=True, index=False)
    assert int(np.sum(o["code"] == oracle.E_BAD_STRING)) == 3, o["code"]
    _check_all(words, mod_off, f"bad terminator {bad}")


def _pass2_modules(seed):
    """Generated modules whose result IDs do not cover [1, bound), so the
    second pass tests their uses: a raised bound with every use defined, a
    raised bound with a use of an undefined ID below it, and a duplicate
    result ID (the ID it replaces is left undefined)."""
    mods, want = [], []
    for i in range(6):
        m = spvgen.gen_module([seed, i], 2500)
        w = m.words.copy()
        upos, dpos = [], []
        for k in range(spvgen.N_PROLOGUE, m.n_inst):
            for s, r in enumerate(spvgen.ROLES[m.kind[k]]):
                if r == "U":
                    upos.append(int(m.starts[k]) + 1 + s)
                elif r == "D":
                    dpos.append(int(m.starts[k]) + 1 + s)
        w[3] += 7
        if i % 3 == 0:
            want.append(0)
        elif i % 3 == 1:
            w[upos[len(upos) // 2]] = w[3] - 2  # below the bound, never defined
            want.append(oracle.E_UNDEFINED_ID)
        else:
            w[dpos[len(dpos) // 3]] = w[dpos[len(dpos) // 3 - 1]]
            want.append(oracle.E_DUPLICATE_ID)
        mods.append(w)
    return mods, want


@pytest.mark.parametrize("fallback", [True, False])
def test_second_pass_with_and_without_the_single_pass_walk(fallback):
    """Modules that need the second pass (undefined-ID search), in a batch
    that takes the single-pass walk (a name spanning whole tiles: the second
    pass recovers instruction starts with lane transfer functions) and in
    one without it (the second pass reads the chain pass's lane starts)."""
    mods, want = _pass2_modules(31)
    if fallback:
        words, mod_off = _batch([[("name", 8200, ("start", 9), None)]], 29)
        mods = [words] + mods
        want = [0] + want
    mod_off = np.concatenate([[0], np.cumsum([w.size for w in mods])]).astype(np.int64)
    words = np.concatenate(mods)
    o = oracle.validate(words, mod_off, semantic=True, index=False)
    assert [int(c) for c in o["code"]] == want, o["code"]
    compare(words, mod_off, label=f"second pass, fallback={fallback}")
    compare(words, mod_off, index=False, label=f"second pass, no index, fallback={fallback}")
