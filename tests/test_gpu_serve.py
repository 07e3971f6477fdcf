"""GPU serving: every request's result equals the oracle's and is the same
alone (one module per launch) and mixed into continuous batches (with and
without graph replay); oversized requests are rejected, not lost."""
import numpy as np
import pytest

import oracle
import spvgen

pytestmark = pytest.mark.gpu


def _pool():
    rng = np.random.default_rng(31)
    mods = []
    for i in range(160):
        m = spvgen.gen_module([31, i], int(rng.integers(3, 6000)))
        if i % 9 == 3:
            m = spvgen.FAULTS[i % 3](m, rng)
        mods.append(m.words)
    return mods


def _expected(mods):
    b = spvgen.pack([spvgen.Module(words=w, kind=None, wc=None, starts=None, n_results=0, bound=0, rec_op=None,
                                   rec_opnd_off=None, rec_opnd=None, rec_str_off=None, rec_chars=None)
                     for w in mods])
    res = oracle.validate(b.words, b.mod_off, index=False)
    return np.stack([res[k] for k in ("code", "sem_mask", "err_word", "n_inst")], axis=1)


def _run(mods, pick, arrivals, **kw):
    from paper_2305_09493_amd.serve import run_trace
    comp, summary = run_trace(mods, arrivals, pick, **kw)
    print(f"[serve] {kw} -> {summary}", flush=True)
    assert comp.size == pick.size and np.all(comp["status"] == 0)
    order = np.argsort(comp["id"])
    comp = comp[order]
    got = np.stack([comp[k] for k in ("code", "sem_mask", "err_word", "n_inst")], axis=1).astype(np.uint32)
    return got, comp


def test_alone_and_mixed_results_identical():
    mods = _pool()
    exp = _expected(mods)
    rng = np.random.default_rng(5)
    n = 600
    pick = rng.integers(0, len(mods), size=n)
    arrivals = np.sort(rng.uniform(0.0, 0.05, size=n))
    alone, c_alone = _run(mods, pick, arrivals, max_batch_modules=1, n_slots=1)
    mixed, c_mixed = _run(mods, pick, arrivals, max_batch_modules=4096, n_slots=4)
    graph, c_graph = _run(mods, pick, arrivals, max_batch_modules=4096, n_slots=3, use_graphs=True)
    assert np.array_equal(alone, exp[pick])
    assert np.array_equal(mixed, exp[pick])
    assert np.array_equal(graph, exp[pick])
    assert c_alone["batch_modules"].max() == 1
    assert c_mixed["batch_modules"].max() > 1  # requests really were mixed


def test_oversized_request_rejected():
    from paper_2305_09493_amd.serve import Server
    small = spvgen.gen_module(1, 50).words
    big = spvgen.gen_module(2, 200_000).words
    with Server(device_budget_bytes=12 << 20, n_slots=1, slot_max_modules=64) as srv:
        cap = srv.stats()["slot_capacity_words"]
        assert small.size < cap < big.size
        srv.submit([small, big, small])
        srv.start()
        comp = srv.drain()
    comp = comp[np.argsort(comp["id"])]
    assert list(comp["status"]) == [0, -2, 0]
    assert comp["code"][0] == 0 and comp["n_inst"][0] == 50
