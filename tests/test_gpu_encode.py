"""GPU parity: spv_encode through the C ABI against the CPU oracle (words,
module offsets, status codes), plus the decode round trip."""
import numpy as np
import pytest

import oracle
import spvgen

pytestmark = pytest.mark.gpu


def _dev(r):
    import torch
    return dict(op=torch.from_numpy(r["op"].view(np.int16)).cuda(),
                opnd_off=torch.from_numpy(r["opnd_off"]).cuda(),
                opnd=torch.from_numpy(r["opnd"].view(np.int32)).cuda(),
                str_off=torch.from_numpy(r["str_off"]).cuda(),
                chars=torch.from_numpy(r["chars"]).cuda(),
                rec_mod_off=torch.from_numpy(r["rec_mod_off"]).cuda())


def _gpu_encode(r, **kw):
    import torch
    import paper_2305_09493_amd as spv
    words, wmo, code, bad = spv.encode(**_dev(r), **kw)
    torch.cuda.synchronize()
    wmo = wmo.cpu().numpy()
    return words.cpu().numpy().view(np.uint32)[:wmo[-1]], wmo, code.cpu().numpy(), bad.cpu().numpy()


def _check(r, label, **kw):
    print(f"[encode parity] {label} M={r['rec_mod_off'].size - 1} N={r['op'].size}", flush=True)
    gw, gmo, gc, gb = _gpu_encode(r, **kw)
    ow, omo, oc, ob = oracle.encode(**r, **kw)
    assert np.array_equal(gc.astype(np.uint32), oc), label
    assert np.array_equal(gb, ob), label
    assert np.array_equal(gmo, omo), label
    assert np.array_equal(gw, ow), label
    return gw, gmo


def test_encode_generated_modules_and_round_trip():
    mods = [spvgen.gen_module([20, i], n) for i, n in enumerate([5, 50, 1000, 4000, 20000, 7])]
    r = spvgen.pack_records(mods)
    gw, gmo = _check(r, "generated")
    b = spvgen.pack(mods)
    assert np.array_equal(gw, b.words) and np.array_equal(gmo, b.mod_off)


def test_encode_block_sizes():
    import paper_2305_09493_amd as spv
    mods = [spvgen.gen_module([21, i], 3000) for i in range(8)]
    r = spvgen.pack_records(mods)
    for blk in (256, 1024, 2048):
        spv.context().set_tuning(encode_block=blk)
        _check(r, f"block {blk}")
    spv.context().set_tuning(encode_block=4096)


def test_encode_failures_compacted():
    rng = np.random.default_rng(3)
    mods = [spvgen.gen_module([22, i], int(rng.integers(5, 800))) for i in range(120)]
    r = spvgen.pack_records(mods)
    op = r["op"].copy()
    opnd = r["opnd"].copy()
    chars = r["chars"].copy()
    n = op.size
    for k in range(12):
        j = int(rng.integers(0, n))
        kind = k % 4
        if kind == 0:
            op[j] = 999
        elif kind == 1 and op[j] != 5:
            op[j] = 17 if op[j] != 17 else 14
        elif kind == 2 and chars.size:
            chars[int(rng.integers(0, chars.size))] = 0
        else:
            lo, hi = r["opnd_off"][j], r["opnd_off"][j + 1]
            if hi > lo and op[j] in (43, 54, 61, 62, 128, 248, 21, 5):
                opnd[lo] = 0xFFFFFFFF
    r2 = dict(r, op=op, opnd=opnd, chars=chars)
    _check(r2, "failures")


def test_encode_empty_modules_and_versions():
    mods = [spvgen.gen_module([23, i], 5) for i in range(3)]
    r = spvgen.pack_records(mods)
    # add empty modules at the front, middle and end
    rmo = r["rec_mod_off"]
    r["rec_mod_off"] = np.concatenate([[0, 0], rmo[1:2], rmo[1:2], rmo[2:], rmo[-1:]]).astype(np.int64)
    _check(r, "empty modules", version_word=0x00010200, generator_word=32)


def _records(mods):
    """CSR records from modules given as lists of (opcode, operands, name bytes)."""
    op, oo, od, so, ch, rmo = [], [0], [], [0], [], [0]
    for recs in mods:
        for opcode, operands, name in recs:
            op.append(opcode)
            od.extend(operands)
            oo.append(len(od))
            ch.append(name)
            so.append(so[-1] + len(name))
        rmo.append(len(op))
    chars = np.frombuffer(b"".join(ch), dtype=np.uint8).copy()
    return dict(op=np.array(op, np.uint16), opnd_off=np.array(oo, np.int32), opnd=np.array(od, np.uint32),
                str_off=np.array(so, np.int32), chars=chars, rec_mod_off=np.array(rmo, np.int64))


def _plain_module(rng, n):
    recs = [(17, [6], b""), (14, [2, 2], b""), (21, [1, 32, 0], b"")]
    nid = 2
    for _ in range(n - 3):
        k = int(rng.integers(0, 3))
        if k == 0:
            recs.append((5, [int(rng.integers(1, nid))], rng.integers(97, 123, size=int(rng.integers(0, 30))).astype(np.uint8).tobytes()))
        elif k == 1:
            recs.append((43, [1, nid, int(rng.integers(0, 1 << 32))], b""))
            nid += 1
        else:
            recs.append((62, [int(rng.integers(1, nid)), int(rng.integers(1, nid))], b""))
    return recs


def test_encode_runs_beyond_lds_staging():
    """Slices whose operand, character or output runs exceed what one step
    stages in LDS: long names, operand-count errors with many operands, a
    record over 65535 words, and blocks that hold hundreds of module starts."""
    rng = np.random.default_rng(24)
    mods = [_plain_module(rng, 700) for _ in range(3)]
    mods[0][100] = (5, [1], b"n" * 3000)             # 751 string words in one record
    mods[0][400] = (5, [1], b"a" * 1500)
    mods[0][401] = (5, [1], b"b" * 1501)
    mods[1][200] = (62, list(range(1, 2001)), b"")   # operand count error, 2000 operands
    mods[1][300] = (15, [6, 1], b"e" * 2001)          # an entry point with a 501-word name
    mods[0][500] = (15, [6, 1], b"main")
    mods[2][300] = (5, [1], b"x" * 270000)           # 1 + 1 + 67501 words: too long
    tiny = [_plain_module(rng, 3) for _ in range(700)]
    tiny[10] = []                                     # empty modules among tiny ones
    tiny[11] = []
    r = _records(mods + tiny + [_plain_module(rng, 900)])
    _check(r, "beyond staging")
    r = _records([mods[0], mods[2]] + tiny)
    _check(r, "beyond staging 2", version_word=0x00010500)


def test_encode_capacity_short_output():
    """words_cap below the batch's total: the modules that fit are written as
    the oracle writes them; every module that ends past words_cap reports
    code 6 and writes nothing (the rest are compacted over it)."""
    import torch
    import paper_2305_09493_amd as spv
    mods = [spvgen.gen_module([25, i], n) for i, n in enumerate([900, 1500, 700, 1200])]
    r = spvgen.pack_records(mods)
    ow, omo, oc, ob = oracle.encode(**r)
    cap = int(omo[2]) + 3  # modules 0 and 1 fit; module 2 would end past the capacity
    words, wmo, code, bad = spv.encode(**_dev(r), words_cap=cap)
    torch.cuda.synchronize()
    code = code.cpu().numpy()
    wmo = wmo.cpu().numpy()
    assert list(code) == [0, 0, 6, 6]
    assert list(bad.cpu().numpy()) == [-1, -1, -1, -1]
    assert np.array_equal(wmo[:3], omo[:3]) and wmo[3] == omo[2] and wmo[4] == omo[2]
    assert np.array_equal(words.cpu().numpy().view(np.uint32)[:omo[2]], ow[:omo[2]])
