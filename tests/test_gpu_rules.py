"""GPU parity of the module-level rules (spv_validate with
SPV_OPT_MODULE_RULES) against the oracle's rules stage: mixed batches with
modules lacking each rule (capability, memory model, function, entry point) (rewritten so that every ID check still passes),
modules failing earlier stages, header-only, short and empty modules, a
multi-tile module without functions, the full lognormal batch, and graph
replays of the captured call on changing inputs."""
import numpy as np
import pytest

import oracle
import spvgen
from spvgen import K_CAP, K_ENTRY, K_FUNC, K_MEM, K_TYPEINT

pytestmark = pytest.mark.gpu


def _type_id(mod):
    """Result ID of the module's first OpTypeInt (defined in every generated module)."""
    s = int(mod.starts[np.nonzero(mod.kind == K_TYPEINT)[0][0]])
    return int(mod.words[s + 1])


def drop_capability(mod):
    """Every OpCapability becomes an OpLabel defining a fresh ID (bound raised)."""
    w = mod.words.copy()
    bound = int(w[3])
    for s in mod.starts[mod.kind == K_CAP]:
        w[s] = (2 << 16) | 248
        w[s + 1] = bound
        bound += 1
    w[3] = bound
    return w


def drop_memory_model(mod):
    """Every OpMemoryModel becomes OpStore %t %t (t: the module's int type)."""
    w = mod.words.copy()
    t = _type_id(mod)
    for s in mod.starts[mod.kind == K_MEM]:
        w[s] = (3 << 16) | 62
        w[s + 1] = t
        w[s + 2] = t
    return w


def drop_functions(mod):
    """Every OpFunction becomes an OpIAdd with the same result (its control
    literal becomes a use of the int type)."""
    w = mod.words.copy()
    t = _type_id(mod)
    for s in mod.starts[mod.kind == K_FUNC]:
        w[s] = (5 << 16) | 128
        w[s + 3] = t
    return w


def drop_entry_point(mod):
    """The prologue's OpEntryPoint (5 words) becomes an OpName of its function
    with a 9-character name (5 words too)."""
    w = mod.words.copy()
    for s in mod.starts[mod.kind == K_ENTRY]:
        fn = int(w[s + 2])
        name = b"mainmain\0\0\0\0"
        w[s:s + 5] = [(5 << 16) | 5, fn] + [int.from_bytes(name[k:k + 4], "little") for k in (0, 4, 8)]
    return w


def _run(words_list, label):
    import torch

    import paper_2305_09493_amd as spv
    from gpu_util import to_dev
    sizes = np.array([w.size for w in words_list], np.int64)
    mod_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    words = np.concatenate(words_list).astype(np.uint32) if words_list else np.zeros(0, np.uint32)
    print(f"[rules parity] {label}: M={len(words_list)} W={words.size}", flush=True)
    w, mo = to_dev(words, mod_off)
    res, io, iop = spv.validate(w, mo, module_rules=True)
    torch.cuda.synchronize()
    g = res.cpu().numpy().view(np.uint32)
    o, oio, oiop = oracle.validate(words, mod_off, semantic=True, rules=True)
    o_arr = np.stack([o[k] for k in ("code", "sem_mask", "err_word", "n_inst")], axis=1).astype(np.uint32)
    bad = np.nonzero(np.any(g != o_arr, axis=1))[0]
    assert bad.size == 0, [(int(m), g[m].tolist(), o_arr[m].tolist()) for m in bad[:8]]
    # the index is the plain validate call's
    gio = io.cpu().numpy().view(np.uint32)
    giop = iop.cpu().numpy().view(np.uint16)
    for m in range(len(words_list)):
        b, n = int(mod_off[m]), int(o_arr[m, 3])
        assert np.array_equal(gio[b:b + n], oio[b:b + n]) and np.array_equal(giop[b:b + n], oiop[b:b + n]), m
    return o_arr


def test_rules_mixed_batch():
    mods = [spvgen.gen_module([11, i], n) for i, n in enumerate([5, 6, 9, 40, 200, 3000, 60_000, 20_000, 700])]
    words = [m.words for m in mods]
    words += [drop_capability(mods[5]), drop_memory_model(mods[4]), drop_functions(mods[6]),
              drop_functions(mods[7]), drop_capability(mods[3]), drop_entry_point(mods[0]),
              drop_entry_point(mods[6]), drop_entry_point(mods[8])]
    ne = spvgen.gen_module([11, 98], 4000)
    ne.words = drop_entry_point(ne)
    words.append(drop_functions(ne))
    both = spvgen.gen_module([11, 99], 5000)
    w = drop_memory_model(both)
    both.words = w
    words.append(drop_capability(both))
    words.append(drop_functions(both))
    # earlier stages win: a duplicate ID in a module without functions
    dup = spvgen.inject_dup(spvgen.gen_module([11, 77], 900), np.random.default_rng(5))
    dup.words = drop_functions(dup)
    words.append(dup.words)
    words += [np.array([0x07230203, 0x00010600, 0, 1, 0], np.uint32), np.zeros(0, np.uint32),
              np.array([0x07230203, 0x00010600, 0], np.uint32)]
    o = _run(words, "mixed")
    codes = set(int(c) for c in o[:, 0])
    masks = set(int(s) for c, s in zip(o[:, 0], o[:, 1]) if c == oracle.E_MODULE_RULES)
    assert {0, 1, 9, oracle.E_MODULE_RULES} <= codes
    assert {8, 16, 32, 64, 96, 120} <= masks


def test_rules_single_module_without_functions():
    mod = spvgen.gen_module([12, 1], 400_000)
    o = _run([drop_functions(mod)], "one module, 400k instructions, no OpFunction")
    assert (int(o[0, 0]), int(o[0, 1])) == (oracle.E_MODULE_RULES, 32)
    o = _run([mod.words], "the same module as generated")
    assert int(o[0, 0]) == 0


def test_rules_full_batched_workload():
    b = spvgen.config3()
    words = [b.words[b.mod_off[m]:b.mod_off[m + 1]] for m in range(b.n_modules)]
    o = _run(words, "lognormal batch, full size")
    assert int(np.sum(o[:, 0] == 0)) > 3000


def test_rules_graph_replays():
    """The validate call with the rules, captured once and replayed on new
    inputs of the same shape (modules with and without each rule swapped in
    place), eager work between replays; every replay against the oracle."""
    import torch

    import paper_2305_09493_amd as spv
    base = [spvgen.gen_module([13, i], 2000) for i in range(12)]
    variants = [lambda m: m.words, drop_capability, drop_memory_model, drop_functions, drop_entry_point]

    def batch(seed):
        return [variants[(i + seed) % 5](m) for i, m in enumerate(base)]

    w0 = batch(0)
    sizes = np.array([w.size for w in w0], np.int64)
    mod_off_h = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    W, M = int(mod_off_h[-1]), len(w0)
    words = torch.zeros(W, dtype=torch.int32, device="cuda")
    mod_off = torch.from_numpy(mod_off_h).cuda()
    res = torch.empty((M, 4), dtype=torch.int32, device="cuda")
    io = torch.empty(W, dtype=torch.int32, device="cuda")
    iop = torch.empty(W, dtype=torch.int16, device="cuda")
    ctx = spv.context()
    ws = torch.empty(ctx.workspace_size(M, W), dtype=torch.uint8, device="cuda")
    words.copy_(torch.from_numpy(np.concatenate(w0).view(np.int32)))
    spv.validate(words, mod_off, out=(res, io, iop), workspace=ws, module_rules=True)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            spv.validate(words, mod_off, out=(res, io, iop), workspace=ws, stream=s, module_rules=True)
    torch.cuda.synchronize()
    seen = set()
    for seed in [1, 2, 3, 0, 1]:
        wl = batch(seed)
        assert [w.size for w in wl] == sizes.tolist()
        host = np.concatenate(wl).astype(np.uint32)
        words.copy_(torch.from_numpy(host.view(np.int32)))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = res.cpu().numpy().view(np.uint32)
        o = oracle.validate(host, mod_off_h, semantic=True, index=False, rules=True)
        want = np.stack([o[k] for k in ("code", "sem_mask", "err_word", "n_inst")], axis=1).astype(np.uint32)
        assert np.array_equal(got, want), (seed, got[:, :2].tolist(), want[:, :2].tolist())
        seen |= set(int(x) for x in want[:, 1])
        # eager work between replays
        spv.validate(words, mod_off, out=(res, io, iop), workspace=ws)
        torch.cuda.synchronize()
    assert {8, 16, 32, 64} <= seen


def test_rules_without_the_index():
    """The rules come from the walk itself: the call without the index gives
    the same results."""
    import torch

    import paper_2305_09493_amd as spv
    from gpu_util import to_dev
    mods = [spvgen.gen_module([14, i], n) for i, n in enumerate([5, 300, 4000, 9000])]
    words = [m.words for m in mods] + [drop_capability(mods[1]), drop_entry_point(mods[2]),
                                       drop_functions(mods[3]), drop_memory_model(mods[0])]
    sizes = np.array([w.size for w in words], np.int64)
    mod_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    flat = np.concatenate(words).astype(np.uint32)
    w, mo = to_dev(flat, mod_off)
    res, _, _ = spv.validate(w, mo, index=False, module_rules=True)
    torch.cuda.synchronize()
    o = oracle.validate(flat, mod_off, semantic=True, index=False, rules=True)
    want = np.stack([o[k] for k in ("code", "sem_mask", "err_word", "n_inst")], axis=1).astype(np.uint32)
    assert np.array_equal(res.cpu().numpy().view(np.uint32), want)
    assert {8, 16, 32, 64} <= set(int(x) for x in want[:, 1])
