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
        m = spvgen.gen_module([31, i], int(rng.integers(5, 6000)))
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


def test_cancelled_requests_complete_with_their_status():
    """Requests cancelled before a batch takes them complete with
    SPV_ERR_CANCELED and a zero result; the others are validated as usual."""
    from paper_2305_09493_amd.serve import Server
    mods = _pool()[:60]
    exp = _expected(mods)
    n = len(mods)
    with Server(max_batch_modules=4096, n_slots=2) as srv:
        srv.submit(mods, ids=np.arange(n), t_arrival_s=np.full(n, 0.3))  # arrive after the cancel
        cancel = np.arange(0, n, 3)
        srv.cancel(np.concatenate([cancel, [10_000]]))  # an unknown id is ignored
        srv.start()
        comp = srv.drain(timeout_s=60)
    comp = comp[np.argsort(comp["id"])]
    assert comp.size == n and np.array_equal(comp["id"], np.arange(n))
    is_c = np.isin(comp["id"], cancel)
    assert np.all(comp["status"][is_c] == -6) and np.all(comp["code"][is_c] == 0)
    assert np.all(comp["status"][~is_c] == 0)
    got = np.stack([comp[k] for k in ("code", "sem_mask", "err_word", "n_inst")], axis=1).astype(np.uint32)
    assert np.array_equal(got[~is_c], exp[~is_c])
