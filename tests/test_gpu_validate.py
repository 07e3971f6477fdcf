"""GPU parity: spv_validate / spv_decode through the C ABI against the CPU
oracle, element by element (results and the instruction index), on seeded
inputs that span many tiles, ragged tails, module boundaries inside tiles and
lanes, crowded tiles, long instructions, corrupted counts and hash-mode IDs."""
import numpy as np
import pytest

import spvgen
from gpu_util import compare, gpu_run

pytestmark = pytest.mark.gpu

T = 4096  # words per tile of the kernels


def test_config1_single_module():
    b = spvgen.config1()
    compare(b.words, b.mod_off, label="config1 validate")
    compare(b.words, b.mod_off, semantic=False, label="config1 decode")
    compare(b.words, b.mod_off, index=False, label="config1 validate, no index")


def test_lognormal_batch_with_faults():
    b = spvgen.config3(n_modules=256, n_faults=24, median=600.0, hi=20_000)
    res = compare(b.words, b.mod_off, label="lognormal 256")
    for m, mod in enumerate(b.modules):
        if mod.expect:
            e = mod.expect
            assert tuple(int(x) for x in res[m]) == (e["code"], e["sem_mask"], e["err_word"], e["n_inst"])


def test_large_single_module_ids_above_64k():
    # IDs above 65535 make operand words look like instructions with wc > 0
    m = spvgen.gen_module(42, 300_000)
    compare(m.words, [0, m.words.size], label="300k instructions")


@pytest.mark.parametrize("n_words", [5, 6, 15, 16, 17, 31, 32, 33, T - 1, T, T + 1, 2 * T + 5])
def test_module_sizes_around_lane_and_tile_edges(n_words):
    # a valid module of exactly n_words: prologue then OpReturn filler
    w = [0x07230203, 0x00010600, 0, 2, 0]
    body = [0x00020011, 6, 0x0003000E, 2, 2, 0x00040015, 1, 32, 0]
    while len(w) + len(body) < n_words:
        body.append(0x000100FD)
    w = (w + body)[:n_words]
    mods = [np.array(w, np.uint32)] * 3
    words = np.concatenate(mods)
    mod_off = np.array([0, n_words, 2 * n_words, 3 * n_words], np.int64)
    compare(words, mod_off, label=f"edges {n_words}")


def test_boundaries_at_every_lane_offset():
    rng = np.random.default_rng(5)
    mods = [spvgen.gen_module([6, i], int(rng.integers(5, 40))) for i in range(600)]
    b = spvgen.pack(mods)
    compare(b.words, b.mod_off, label="small modules, boundaries everywhere")


def test_crowded_tiles_serial_path():
    # thousands of tiny modules: > 256 module starts per tile
    rng = np.random.default_rng(7)
    words, offs = [], [0]
    for i in range(6000):
        kind = i % 7
        if kind == 0:
            w = []                                       # empty
        elif kind == 1:
            w = [0x07230203, 0x00010600]                 # truncated
        elif kind == 2:
            w = [0x07230203, 0x00010600, 0, 5, 0]        # header only
        elif kind == 3:
            w = [0x07230203, 0x00010600, 0, 5, 0, 0x000200F8, 1, 0x000200F8, 1]  # dup
        elif kind == 4:
            w = [0x07230203, 0x00010600, 0, 5, 0, 0x00030005, 1, 0x00636261, 0x000200F8, 1]
        elif kind == 5:
            w = [0x03022307, 1, 2, 3, 4, 5]              # bad magic
        else:
            w = [0x07230203, 0x00010600, 0, 9, 0] + [int(x) for x in rng.integers(0, 1 << 32, size=int(rng.integers(0, 12)))]
        words += w
        offs.append(len(words))
    compare(np.array(words, np.uint32), np.array(offs, np.int64), label="crowded")


def test_long_opname_and_corrupted_counts():
    rng = np.random.default_rng(11)
    mods = []
    for i in range(60):
        m = spvgen.gen_module([9, i], 2000)
        w = list(int(x) for x in m.words)
        # insert long OpNames (wc 15..120) at random instruction boundaries
        starts = list(m.starts)
        for _ in range(3):
            j = int(rng.integers(3, len(starts)))
            L = int(rng.integers(48, 470))
            s = bytes(rng.integers(97, 123, size=L).astype(np.uint8)) + b"\0"
            s += b"\0" * (-len(s) % 4)
            sw = [int.from_bytes(s[k:k + 4], "little") for k in range(0, len(s), 4)]
            ins = [((2 + len(sw)) << 16) | 5, 1] + sw
            p = int(starts[j])
            w = w[:p] + ins + w[p:]
            starts = [x if x < p else x + len(ins) for x in starts]
        if i % 3 == 1:
            p = int(starts[int(rng.integers(3, len(starts)))])
            w[p] = (int(rng.integers(0, 65536)) << 16) | (w[p] & 0xFFFF)    # corrupted count
        if i % 3 == 2:
            p = int(starts[int(rng.integers(3, len(starts)))])
            s = [0x61616161] * 4                                              # bad string (no NUL)
            w = w[:p] + [((2 + len(s)) << 16) | 5, 1] + s + w[p:]
        mods.append(np.array(w, np.uint32))
    offs = np.concatenate([[0], np.cumsum([x.size for x in mods])]).astype(np.int64)
    compare(np.concatenate(mods), offs, label="long names / corruption")


def test_random_mutations():
    rng = np.random.default_rng(13)
    mods = []
    for i in range(200):
        m = spvgen.gen_module([10, i], int(rng.integers(5, 3000)))
        w = m.words.copy()
        for _ in range(int(rng.integers(0, 3))):
            p = int(rng.integers(0, w.size))
            w[p] = rng.integers(0, 1 << 32, dtype=np.uint64)
        mods.append(w)
    offs = np.concatenate([[0], np.cumsum([x.size for x in mods])]).astype(np.int64)
    words = np.concatenate(mods)
    compare(words, offs, label="mutations validate")
    compare(words, offs, semantic=False, label="mutations decode")


def test_hash_mode_sparse_bounds():
    mods = []
    for i in range(40):
        m = spvgen.gen_module([12, i], 500)
        w = m.words.copy()
        # scale every result and use by a large stride: bound >> 64 * words
        dpos, upos = [], []
        for k in range(m.n_inst):
            for s, r in enumerate(spvgen.ROLES[m.kind[k]]):
                if r in "UD":
                    (dpos if r == "D" else upos).append(m.starts[k] + 1 + s)
        pos = np.array(dpos + upos, np.int64)
        w[pos] = (w[pos].astype(np.uint64) * 1_000_003 % (1 << 31)).astype(np.uint32) | 1
        w[3] = 0xFFFFFFF0
        if i % 4 == 1:
            w[dpos[5]] = w[dpos[4]]          # duplicate
        if i % 4 == 2:
            w[upos[7]] = 0x7FFFFFF1          # undefined
        mods.append(w)
    offs = np.concatenate([[0], np.cumsum([x.size for x in mods])]).astype(np.int64)
    compare(np.concatenate(mods), offs, label="hash mode")


def test_repeat_runs_identical():
    b = spvgen.config3(n_modules=64, n_faults=6, median=1500.0, hi=30_000)
    r1 = compare(b.words, b.mod_off, label="repeat 1")
    r2 = compare(b.words, b.mod_off, label="repeat 2")
    assert np.array_equal(r1, r2)


def test_real_modules_mixed_with_generated():
    """Real SPIR-V modules built here (hipcc, generic SPIR-V target) between
    generated ones: the chain pass analyses every tile of the real binaries;
    results and index prefixes must equal the oracle's."""
    import realspv
    if not realspv.available():
        pytest.skip("hipcc / clang-offload-bundler not available")
    real = [realspv.module(n) for n in sorted(realspv.SOURCES)]
    gen = [spvgen.gen_module([33, i], n).words for i, n in enumerate([3000, 700])]
    mods = [real[0], gen[0], real[1], gen[1], real[0]]
    words = np.concatenate(mods).astype(np.uint32)
    mod_off = np.concatenate([[0], np.cumsum([m.size for m in mods])]).astype(np.int64)
    compare(words, mod_off, label="real + generated")
    compare(words, mod_off, semantic=False, label="real + generated, decode")
    for m in real:
        compare(m, [0, m.size], label=f"real module alone ({m.size} words)")


def _name_words(wc):
    """An OpName of %1 with wc words (its string: wc - 2 words, NUL in the last)."""
    n = 4 * (wc - 2) - 1
    b = (b"n" * n + b"\0").ljust(4 * (wc - 2), b"\0")
    return [(wc << 16) | 5, 1] + [int.from_bytes(b[k:k + 4], "little") for k in range(0, len(b), 4)]


@pytest.mark.parametrize("semantic", [True, False])
def test_invalid_start_in_first_lane_after_tile_entry(semantic):
    # The chain enters a tile at offset e (an OpName crossing the tile start
    # ends there), walks one-word instructions, and meets an invalid
    # instruction (OpLabel with word count 1) at offset q of the tile's first
    # lane: the parse error must be found at q.
    mods = []
    for e in (0, 1, 2, 5, 11):
        for q in range(e + 1, 16):
            m = spvgen.gen_module([14, q, e], 400)
            w = [int(x) for x in m.words[:int(m.starts[spvgen.N_PROLOGUE])]]
            base = sum(x.size for x in mods)
            if e == 0:
                w += [0x000100FD] * ((-(base + len(w))) % T)
            else:
                w += [0x000100FD] * ((-3 - (base + len(w))) % T)
                w += _name_words(3 + e)
            assert (base + len(w)) % T == e
            w += [0x000100FD] * (q - e)
            w += [0x000100F8, 0x000000FF]
            w += [int(x) for x in m.words[int(m.starts[spvgen.N_PROLOGUE]):]]
            mods.append(np.array(w, np.uint32))
    offs = np.concatenate([[0], np.cumsum([x.size for x in mods])]).astype(np.int64)
    words = np.concatenate(mods)
    res = compare(words, offs, semantic=semantic, label="invalid start in a tile's first lane")
    assert np.all(res[:, 0] == 5)
