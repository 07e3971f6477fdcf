"""GPU parity: decode's records mode (spv_decode_records) against the
oracle's records, element by element, and the GPU round trip
encode(records(decode(words))) == words for valid modules."""
import numpy as np
import pytest

import oracle
import spvgen
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _gpu_records(words, mod_off, semantic=False):
    import torch

    import paper_2305_09493_amd as spv
    w, mo = to_dev(words, mod_off)
    fn = spv.validate if semantic else spv.decode
    res, io, _ = fn(w, mo)
    rec = spv.decode_records(w, mo, io, res)
    torch.cuda.synchronize()
    rmo = rec["rec_mod_off"].cpu().numpy()
    n = int(rmo[-1])
    oo = rec["opnd_off"].cpu().numpy()[:n + 1]
    so = rec["str_off"].cpu().numpy()[:n + 1]
    return dict(op=rec["op"].cpu().numpy().view(np.uint16)[:n], opnd_off=oo,
                opnd=rec["opnd"].cpu().numpy().view(np.uint32)[:oo[-1]], str_off=so,
                chars=rec["chars"].cpu().numpy()[:so[-1]], rec_mod_off=rmo), (w, mo)


def _check(words, mod_off, label, semantic=False):
    print(f"[records parity] {label} M={len(mod_off) - 1} W={len(words)} semantic={semantic}", flush=True)
    g, dev = _gpu_records(words, mod_off, semantic)
    o = oracle.records(words, mod_off)
    for k in ("rec_mod_off", "op", "opnd_off", "opnd", "str_off", "chars"):
        assert np.array_equal(np.asarray(g[k]), np.asarray(o[k]).astype(np.asarray(g[k]).dtype)), (label, k)
    return g, dev


def test_records_of_generated_and_faulted_modules():
    mods = [spvgen.gen_module([30, i], n) for i, n in enumerate([5, 40, 1000, 5000, 17, 20000])]
    b = spvgen.pack(mods)
    _check(b.words, b.mod_off, "generated")
    _check(b.words, b.mod_off, "generated, from validate", semantic=True)
    # parse failures keep the valid prefix; header failures give no records
    b3 = spvgen.config3(n_modules=300, n_faults=30, median=500.0, hi=10_000)
    w = b3.words.copy()
    w[b3.mod_off[7]] = 0x03022307          # byte-swapped magic
    w[b3.mod_off[11] + 4] = 1               # schema
    _check(w, b3.mod_off, "faulted batch")
    _check(w, b3.mod_off, "faulted batch, from validate", semantic=True)


def test_records_empty_and_header_only_modules():
    mods = [spvgen.gen_module([31, i], 50) for i in range(3)]
    b = spvgen.pack(mods)
    hdr = np.array([0x07230203, 0x00010600, 0, 1, 0], np.uint32)
    words = np.concatenate([hdr, b.words, hdr, np.array([1, 2], np.uint32)])
    n0 = hdr.size
    mo = np.concatenate([[0], n0 + b.mod_off, [n0 + b.words.size + hdr.size, n0 + b.words.size + hdr.size,
                                             words.size]]).astype(np.int64)
    _check(words, mo, "empty, header-only and truncated modules")


def test_records_long_names_and_round_trip():
    import torch

    import paper_2305_09493_amd as spv
    rng = np.random.default_rng(32)
    mods = [spvgen.gen_module([32, i], n) for i, n in enumerate([4000, 9000, 1500])]
    b = spvgen.pack(mods)
    # long OpName strings (word counts up to 120) through the records path
    r0 = spvgen.pack_records(mods)
    names = np.nonzero(r0["op"] == 5)[0][:40]
    chars = [bytes(r0["chars"][r0["str_off"][j]:r0["str_off"][j + 1]]) for j in range(r0["op"].size)]
    for j in names:
        chars[j] = rng.integers(97, 123, size=int(rng.integers(1, 470))).astype(np.uint8).tobytes()
    lens = np.array([len(c) for c in chars], np.int64)
    r = dict(r0, chars=np.frombuffer(b"".join(chars), np.uint8).copy(),
             str_off=np.concatenate([[0], np.cumsum(lens)]).astype(np.int32))
    ow, omo, oc, ob = oracle.encode(**r)
    assert not oc.any()
    g, (w, mo) = _check(ow, omo, "long names")
    # GPU round trip: the records encode back to the same words
    d = dict(op=torch.from_numpy(g["op"].view(np.int16)).cuda(),
             opnd_off=torch.from_numpy(g["opnd_off"]).cuda(),
             opnd=torch.from_numpy(g["opnd"].view(np.int32)).cuda(),
             str_off=torch.from_numpy(g["str_off"]).cuda(),
             chars=torch.from_numpy(g["chars"]).cuda(),
             rec_mod_off=torch.from_numpy(g["rec_mod_off"]).cuda())
    words, wmo, code, _ = spv.encode(**d)
    torch.cuda.synchronize()
    wmo = wmo.cpu().numpy()
    assert not code.cpu().numpy().any()
    assert np.array_equal(wmo, omo)
    assert np.array_equal(words.cpu().numpy().view(np.uint32)[:wmo[-1]], ow)
    # and the generated batch round-trips too
    g2, _ = _check(b.words, b.mod_off, "generated for round trip")
    ow2, omo2, oc2, _ = oracle.encode(**g2)
    assert not oc2.any() and np.array_equal(ow2, b.words) and np.array_equal(omo2, b.mod_off)


def test_records_after_validate_with_rules():
    """A module that fails only the module rules (code 11) was decoded in full:
    its records are all of its instructions."""
    import torch

    import paper_2305_09493_amd as spv
    mods = [spvgen.gen_module([43, i], 200) for i in range(5)]
    b = spvgen.pack(mods)
    w = b.words.copy()
    _, io, iop = oracle.validate(w, b.mod_off)
    base = int(b.mod_off[1])
    for j in range(200):  # module 1 loses every OpCapability (each becomes two OpReturns)
        if iop[base + j] == 17:
            p = base + int(io[base + j])
            w[p], w[p + 1] = 0x000100FD, 0x000100FD
    print("[records parity] after validate with the module rules", flush=True)
    dw, dmo = to_dev(w, b.mod_off)
    res, dio, _ = spv.validate(dw, dmo, module_rules=True)
    rec = spv.decode_records(dw, dmo, dio, res)
    torch.cuda.synchronize()
    assert int(res[1, 0].item()) == oracle.E_MODULE_RULES
    o = oracle.records(w, b.mod_off)
    assert np.array_equal(rec["rec_mod_off"].cpu().numpy(), o["rec_mod_off"])
    n = int(o["rec_mod_off"][-1])
    assert np.array_equal(rec["op"].cpu().numpy().view(np.uint16)[:n], o["op"])
