"""GPU parity of spv_validate's semantic positions (SPV_OPT_SEM_OFFSETS) and
defined-before-use mode (SPV_OPT_DEF_BEFORE_USE) against the oracle, every
result field of every module: the hand-worked modules of the oracle's pins
in one batch, faulted lognormal batches with random ID rewrites, a sparse
(hash-mode) module, a large module, and with the module-level rules."""
import numpy as np
import pytest

import oracle
import spvgen
from gpu_util import to_dev
from test_oracle_positions import CASES

pytestmark = pytest.mark.gpu

OPTS = [dict(sem_offsets=True), dict(def_before_use=True), dict(sem_offsets=True, def_before_use=True),
        dict(sem_offsets=True, def_before_use=True, module_rules=True)]


def _oracle_kw(kw):
    return dict(offsets=kw.get("sem_offsets", False), before_use=kw.get("def_before_use", False),
                rules=kw.get("module_rules", False))


def _check(words, mod_off, kw, label):
    import torch

    import paper_2305_09493_amd as spv
    print(f"[positions parity] {label} M={len(mod_off) - 1} W={len(words)} {kw}", flush=True)
    w, mo = to_dev(words, mod_off)
    res, _, _ = spv.validate(w, mo, **kw)
    torch.cuda.synchronize()
    g = res.cpu().numpy().view(np.uint32)
    o = oracle.validate(words, mod_off, index=False, **_oracle_kw(kw))
    oa = np.stack([o[k] for k in ("code", "sem_mask", "err_word", "n_inst")], axis=1).astype(np.uint32)
    bad = np.nonzero(np.any(g != oa, axis=1))[0]
    assert bad.size == 0, (label, kw, [(int(m), g[m].tolist(), oa[m].tolist()) for m in bad[:5]])
    return g


def _pack(mods):
    mods = [np.asarray(m, np.uint32) for m in mods]
    return np.concatenate(mods), np.concatenate([[0], np.cumsum([m.size for m in mods])]).astype(np.int64)


def test_hand_worked_modules_as_one_batch():
    words, mod_off = _pack([c[1] for c in CASES] + [spvgen.gen_module(60, 50).words])
    for kw in OPTS:
        _check(words, mod_off, kw, "hand-worked")


def _rewritten(seed, n_modules, max_rewrites=3):
    b = spvgen.config3(n_modules=n_modules, n_faults=max(1, n_modules // 20), median=400.0, hi=6000)
    w = b.words.copy()
    rng = np.random.default_rng(seed)
    for m in range(n_modules):
        if rng.random() < 0.5:
            continue
        lo, hi = int(b.mod_off[m]) + 5, int(b.mod_off[m + 1])
        for _ in range(int(rng.integers(1, max_rewrites + 1))):
            i = int(rng.integers(lo, hi))
            if (w[i] >> 16) == 0:  # leave first words (word counts) alone: rewrite operand-like words only
                bound = int(w[lo - 2])
                w[i] = int(rng.integers(1, 40)) if rng.random() < 0.4 else int(rng.integers(0, bound + 3))
    return w, b.mod_off


@pytest.mark.parametrize("kw", OPTS, ids=["offsets", "before_use", "both", "both+rules"])
def test_faulted_batch_with_rewritten_ids(kw):
    w, mo = _rewritten(61, 300)
    g = _check(w, mo, kw, "rewritten batch")
    assert np.sum((g[:, 0] >= 8) & (g[:, 0] <= 10)) > 20  # many semantic failures to place


def test_sparse_module_and_large_module():
    # hash mode: the bound far above the module size
    m = spvgen.gen_module(62, 3000).words.copy()
    m[3] = 0xFFFFFFF0
    big = spvgen.gen_module(63, 400_000).words.copy()
    # a duplicate and a use before definition deep in the large module
    _, io, iop = oracle.validate(big, [0, big.size])
    adds = np.nonzero(iop[:400_000] == 128)[0]
    p1 = int(io[adds[1000]])        # OpIAdd: type, result, a, b
    p2 = int(io[adds[80_000]])
    big[p2 + 2] = big[p1 + 2]       # result of the later OpIAdd duplicates the earlier one
    p3 = int(io[adds[30_000]])
    big[p3 + 3] = big[int(io[adds[100_000]]) + 2]  # operand a: a result defined much later
    words, mod_off = _pack([m, big])
    for kw in OPTS:
        _check(words, mod_off, kw, "sparse + large")


def test_positions_need_the_index():
    import paper_2305_09493_amd as spv
    m = spvgen.gen_module(64, 100).words
    w, mo = to_dev(m, np.array([0, m.size], np.int64))
    with pytest.raises(spv.SpvError):
        spv.validate(w, mo, index=False, sem_offsets=True)
