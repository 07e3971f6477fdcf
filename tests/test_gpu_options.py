"""GPU checks of spv_validate's option bits: SPV_OPT_NO_SEMANTIC gives
spv_decode's results, SPV_OPT_DEBUG_CHECKS leaves valid batches' results
unchanged and turns bad module offsets into SPV_ERR_INVALID_ARG before any
other kernel runs (the results buffer keeps its contents), and unknown or
contradictory bits are refused."""
import numpy as np
import pytest

import oracle
import spvgen
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _batch():
    return spvgen.config3(n_modules=40, n_faults=3, median=400.0, hi=4_000)


def test_no_semantic_is_decode():
    import torch

    import paper_2305_09493_amd as spv
    b = _batch()
    w, mo = to_dev(b.words, b.mod_off)
    print("[options] NO_SEMANTIC vs decode", flush=True)
    r1, i1, p1 = spv._run(True, w, mo, True, None, None, flags=spv.OPT_NO_SEMANTIC)
    r2, i2, p2 = spv.decode(w, mo)
    torch.cuda.synchronize()
    assert torch.equal(r1, r2)
    o = oracle.decode(b.words, b.mod_off, index=False)
    assert np.array_equal(r1.cpu().numpy().view(np.uint32)[:, 0], o["code"])


def test_debug_checks_pass_valid_offsets():
    import torch

    import paper_2305_09493_amd as spv
    b = _batch()
    w, mo = to_dev(b.words, b.mod_off)
    print("[options] DEBUG_CHECKS on a valid batch", flush=True)
    r1, i1, p1 = spv.validate(w, mo, debug_checks=True, module_rules=True)
    r2, i2, p2 = spv.validate(w, mo, module_rules=True)
    torch.cuda.synchronize()
    assert torch.equal(r1, r2)


@pytest.mark.parametrize("kind", ["first", "last", "decreasing"])
def test_debug_checks_refuse_bad_offsets(kind):
    import torch

    import paper_2305_09493_amd as spv
    b = _batch()
    mo_h = b.mod_off.copy()
    if kind == "first":
        mo_h[0] = 1
    elif kind == "last":
        mo_h[-1] -= 1
    else:  # module 5 ends before it starts
        mo_h[5], mo_h[6] = mo_h[6], mo_h[5]
    w, mo = to_dev(b.words, mo_h)
    M = mo_h.size - 1
    results = torch.full((M, 4), 77, dtype=torch.int32, device=w.device)
    idx_off = torch.empty(w.numel(), dtype=torch.int32, device=w.device)
    idx_op = torch.empty(w.numel(), dtype=torch.int16, device=w.device)
    print(f"[options] DEBUG_CHECKS refuse {kind}", flush=True)
    with pytest.raises(spv.SpvError, match="invalid argument"):
        spv.validate(w, mo, out=(results, idx_off, idx_op), debug_checks=True)
    torch.cuda.synchronize()
    assert bool((results == 77).all()), "a refused call wrote results"


def test_refused_option_bits():
    import paper_2305_09493_amd as spv
    b = _batch()
    w, mo = to_dev(b.words, b.mod_off)
    for flags in (32, 64, 1 << 31, spv.OPT_NO_SEMANTIC | spv.OPT_MODULE_RULES,
                  spv.OPT_NO_SEMANTIC | spv.OPT_SEM_OFFSETS, spv.OPT_NO_SEMANTIC | spv.OPT_DEF_BEFORE_USE):
        with pytest.raises(spv.SpvError):
            spv._run(True, w, mo, True, None, None, flags=flags)
