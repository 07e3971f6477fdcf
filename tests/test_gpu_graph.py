"""The library's calls are stream-ordered, allocation-free and host-sync-free,
so they can be captured in a HIP graph: capture spv_validate once, replay it
several times on new inputs of the same shape (with eager work and
synchronisations between replays) and check every replay against the eager
result and the oracle; the same for spv_encode.  Also: parity does not
depend on the persistent grid size."""
import numpy as np
import pytest

import oracle
import spvgen
from gpu_util import compare

pytestmark = pytest.mark.gpu


_BASE = None


def _batch(seed):
    """The same 24 modules for every seed (same sizes); each seed injects
    faults (which keep the word count) into a different subset."""
    global _BASE
    if _BASE is None:
        _BASE = [spvgen.gen_module([40, i], 3000) for i in range(24)]
    rng = np.random.default_rng(seed)
    mods = []
    for i, m in enumerate(_BASE):
        if seed and i % 5 == seed % 5:
            m = spvgen.FAULTS[(i + seed) % 3](m, rng)
        mods.append(m)
    return spvgen.pack(mods)


def test_graph_capture_replays_match_eager():
    import torch

    import paper_2305_09493_amd as spv
    b0 = _batch(0)
    W, M = b0.words.size, b0.n_modules
    words = torch.zeros(W, dtype=torch.int32, device="cuda")
    mod_off = torch.from_numpy(b0.mod_off).cuda()
    res = torch.empty((M, 4), dtype=torch.int32, device="cuda")
    io = torch.empty(W, dtype=torch.int32, device="cuda")
    iop = torch.empty(W, dtype=torch.int16, device="cuda")
    ctx = spv.context()
    ws = torch.empty(ctx.workspace_size(M, W), dtype=torch.uint8, device="cuda")
    words.copy_(torch.from_numpy(b0.words.view(np.int32)))
    spv.validate(words, mod_off, out=(res, io, iop), workspace=ws)  # warm-up outside capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            spv.validate(words, mod_off, out=(res, io, iop), workspace=ws, stream=s)
    torch.cuda.synchronize()
    for seed in range(1, 5):
        b = _batch(seed)
        assert b.words.size == W and np.array_equal(b.mod_off, b0.mod_off)
        words.copy_(torch.from_numpy(b.words.view(np.int32)))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = res.cpu().numpy().view(np.uint32).copy()
        # eager on the same input, then the oracle
        r2, _, _ = spv.validate(words, mod_off)
        torch.cuda.synchronize()
        o = oracle.validate(b.words, b.mod_off, index=False)
        exp = np.stack([o[k] for k in ("code", "sem_mask", "err_word", "n_inst")], axis=1)
        assert np.array_equal(got, r2.cpu().numpy().view(np.uint32)), seed
        assert np.array_equal(got, exp), seed
        _ = torch.ones(1 << 20, device="cuda").sum().item()  # unrelated eager work between replays


def _records_variant(r0, seed):
    """Records of the same shape as r0 (same counts and lengths) with new
    name characters; odd seeds also put an ID operand of 0xFFFFFFFF into one
    record (a failing module, so the replay also compacts)."""
    r = {k: v.copy() for k, v in r0.items()}
    if seed:
        rng = np.random.default_rng([41, seed])
        r["chars"] = rng.integers(97, 123, size=r["chars"].size).astype(np.uint8)
        if seed % 2:
            stores = np.nonzero(r["op"] == 62)[0]
            j = int(stores[(37 * seed) % stores.size])
            r["opnd"][r["opnd_off"][j]] = 0xFFFFFFFF
    return r


def test_encode_graph_capture_replays_match_eager():
    import torch

    import paper_2305_09493_amd as spv
    r0 = spvgen.pack_records([spvgen.gen_module([41, i], 2000) for i in range(6)])
    d = {k: torch.from_numpy(r0[k].view(np.int16) if k == "op" else
                             r0[k].view(np.int32) if k == "opnd" else r0[k]).cuda() for k in r0}
    spv.encode(**d)  # warm-up outside capture (sizes the context's workspace)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            gout = spv.encode(**d, stream=s)
    torch.cuda.synchronize()
    for seed in range(1, 5):
        r = _records_variant(r0, seed)
        d["chars"].copy_(torch.from_numpy(r["chars"]))
        d["opnd"].copy_(torch.from_numpy(r["opnd"].view(np.int32)))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        gw, gmo, gc, gb = [t.cpu().numpy() for t in gout]
        ew, emo, ec, eb = [t.cpu().numpy() for t in spv.encode(**d)]
        torch.cuda.synchronize()
        ow, omo, oc, ob = oracle.encode(**r)
        n = int(gmo[-1])
        assert np.array_equal(gmo, emo) and np.array_equal(gmo, omo), seed
        assert np.array_equal(gc, ec) and np.array_equal(gc.astype(np.uint32), oc), seed
        assert np.array_equal(gb, eb) and np.array_equal(gb, ob), seed
        assert np.array_equal(gw.view(np.uint32)[:n], ow) and np.array_equal(ew.view(np.uint32)[:n], ow), seed
        if seed % 2:
            assert (oc != 0).sum() == 1, seed
        _ = torch.ones(1 << 20, device="cuda").sum().item()  # unrelated eager work between replays


@pytest.mark.parametrize("grids", [(1, 1), (3, 12), (6, 6), (12, 3), (64, 64)])
def test_parity_independent_of_chain_and_walk_grids(grids):
    """The chain pass and the resolved walk take tiles in a static order: any
    grid gives the same results and index."""
    import paper_2305_09493_amd as spv
    ctx = spv.context()
    old = ctx.get_grids()
    try:
        ctx.set_grids(*grids)
        assert ctx.get_grids() == grids
        b = spvgen.config3(n_modules=96, n_faults=9, median=1200.0, hi=40_000)
        compare(b.words, b.mod_off, label=f"chain, walk grids {grids}")
        m = spvgen.gen_module(78, 300_000)
        compare(m.words, [0, m.words.size], label=f"one module, chain, walk grids {grids}")
    finally:
        ctx.set_grids(*old)


def test_grid_autotuner_picks_a_candidate_and_keeps_parity(tmp_path, monkeypatch):
    import torch

    import paper_2305_09493_amd as spv
    from paper_2305_09493_amd import tune
    monkeypatch.setenv("SPVGPU_TUNE_CACHE", str(tmp_path / "tune.json"))
    ctx = spv.context()
    old = ctx.get_grids()
    try:
        m = spvgen.gen_module(79, 200_000)
        w = torch.from_numpy(m.words.view(np.int32)).cuda()
        mo = torch.tensor([0, m.words.size], dtype=torch.int64, device="cuda")
        r = tune.autotune_grids(w, mo, chain=(2, 6), walk=(3, 6))
        assert (r["chain_blocks_per_cu"], r["walk_blocks_per_cu"]) in [(2, 3), (2, 6), (6, 3), (6, 6)]
        ctx.set_grids(*old)
        assert tune.apply("validate_grids", m.words.size)["walk_blocks_per_cu"] == r["walk_blocks_per_cu"]
        assert ctx.get_grids() == (r["chain_blocks_per_cu"], r["walk_blocks_per_cu"])
        compare(m.words, [0, m.words.size], label="after the grid autotuner")
    finally:
        ctx.set_grids(*old)


@pytest.mark.parametrize("bpc", [1, 2, 8])
def test_parity_independent_of_fallback_grid(bpc):
    """blocks_per_cu sizes the single-pass fallback walk, which returns at
    once on these inputs (every tile settles); crowded tiles below force it."""
    import paper_2305_09493_amd as spv
    ctx = spv.context()
    old = ctx.get_tuning()[0]
    try:
        ctx.set_tuning(blocks_per_cu=bpc)
        b = spvgen.config3(n_modules=96, n_faults=9, median=1200.0, hi=40_000)
        compare(b.words, b.mod_off, label=f"blocks_per_cu={bpc}")
        m = spvgen.gen_module(77, 120_000)
        compare(m.words, [0, m.words.size], label=f"one module, blocks_per_cu={bpc}")
        # 6000 tiny modules: more than 63 modules overlap a tile, so the
        # batch takes the single-pass walk with this grid
        tiny = spvgen.pack([spvgen.gen_module([80, i], 5) for i in range(6000)])
        compare(tiny.words, tiny.mod_off, label=f"crowded tiles, blocks_per_cu={bpc}")
    finally:
        ctx.set_tuning(blocks_per_cu=old)


def test_autotuner_picks_a_candidate_and_keeps_parity(tmp_path, monkeypatch):
    import torch

    import paper_2305_09493_amd as spv
    from paper_2305_09493_amd import tune
    monkeypatch.setenv("SPVGPU_TUNE_CACHE", str(tmp_path / "tune.json"))
    ctx = spv.context()
    old = ctx.get_tuning()
    try:
        b = spvgen.config3(n_modules=64, n_faults=6, median=1500.0, hi=30_000)
        w = torch.from_numpy(b.words.view(np.int32)).cuda()
        mo = torch.from_numpy(b.mod_off).cuda()
        r = tune.autotune_validate(w, mo, candidates=(1, 2, 4))
        assert r["blocks_per_cu"] in (1, 2, 4)
        ctx.set_tuning(blocks_per_cu=old[0])
        assert tune.apply("validate", b.words.size)["blocks_per_cu"] == r["blocks_per_cu"]
        compare(b.words, b.mod_off, label="after autotune")
        recs = spvgen.pack_records([spvgen.gen_module([41, i], 2000) for i in range(4)])
        d = dict(op=torch.from_numpy(recs["op"].view(np.int16)).cuda(),
                 opnd_off=torch.from_numpy(recs["opnd_off"]).cuda(),
                 opnd=torch.from_numpy(recs["opnd"].view(np.int32)).cuda(),
                 str_off=torch.from_numpy(recs["str_off"]).cuda(),
                 chars=torch.from_numpy(recs["chars"]).cuda(),
                 rec_mod_off=torch.from_numpy(recs["rec_mod_off"]).cuda())
        e = tune.autotune_encode(d, candidates=(256, 1024))
        assert e["encode_block"] in (256, 1024)
    finally:
        ctx.set_tuning(blocks_per_cu=old[0], encode_block=old[1])


def _id_word(m, want_role, tile_min, lane_pos=None, last_lane=False):
    """Position of an ID word of role want_role ('U' or 'D') in tile >= tile_min
    (optionally at lane position lane_pos, or in the tile's last lane)."""
    for k in range(spvgen.N_PROLOGUE, m.n_inst):
        for s, r in enumerate(spvgen.ROLES[m.kind[k]]):
            if r != want_role:
                continue
            pos = int(m.starts[k]) + 1 + s
            if pos // 4096 < tile_min:
                continue
            if lane_pos is not None and pos % 16 != lane_pos:
                continue
            if last_lane and pos % 4096 < 4080:
                continue
            return pos
    raise AssertionError("no such ID word")


@pytest.mark.parametrize("case", ["use", "def", "use at lane start", "use in last lane", "zero"])
def test_load_time_bound_test_on_later_tiles(case):
    """With one walk block per CU, a block's later tiles lie inside the module
    of its previous tile, where the walk tests the ID words' bound as they
    load: an out-of-bound use or result ID (or ID 0) placed there, also at a
    lane's first words (IDs of the previous lane's last instruction) and in
    a tile's last lane, is found as on the oracle."""
    import paper_2305_09493_amd as spv
    m = spvgen.gen_module(80, 400_000)
    w = m.words.copy()
    bound = int(w[3])
    if case == "use":
        w[_id_word(m, "U", 300)] = bound + 5
    elif case == "def":
        w[_id_word(m, "D", 300)] = bound
    elif case == "use at lane start":
        w[_id_word(m, "U", 300, lane_pos=1)] = 0xFFFFFFF0
    elif case == "use in last lane":
        w[_id_word(m, "U", 300, last_lane=True)] = bound + 1
    else:
        w[_id_word(m, "U", 300)] = 0
    o = oracle.validate(w, np.array([0, w.size], np.int64), semantic=True, index=False)
    assert int(o["code"][0]) == oracle.E_ID_OUT_OF_BOUND, o["code"]
    ctx = spv.context()
    old = ctx.get_grids()
    try:
        ctx.set_grids(1, 1)
        compare(w, [0, w.size], label=f"load-time bound test, {case}")
    finally:
        ctx.set_grids(*old)
