"""GPU parity at the benchmark's full sizes, in the launch configuration the
benchmark times (the context's default tuning):
  * the batched workload: 4096 lognormal modules (about 56M words) with 41
    injected faults; every result field and every module's index prefix
    against the oracle, each faulted module against the code its fault was
    built to produce, and decode's records of the whole batch;
  * the encode workload: 10M records in 1024 modules; every output word,
    offset and status against the oracle.
(The single 16M-instruction module is checked against the oracle by
bench.py on every run.)"""
import numpy as np
import pytest

import oracle
import spvgen
from gpu_util import compare

pytestmark = pytest.mark.gpu


def test_full_batched_workload_parity():
    b = spvgen.config3()
    assert b.n_modules == 4096
    res = compare(b.words, b.mod_off, label="batched workload, full size")
    faulted = [m for m, mod in enumerate(b.modules) if mod.expect]
    assert len(faulted) == 41
    for m in faulted:
        e = b.modules[m].expect
        assert tuple(int(x) for x in res[m]) == (e["code"], e["sem_mask"], e["err_word"], e["n_inst"]), m
    assert int(np.sum(res[:, 0] != 0)) == 41
    # decode's records mode on the same batch (faulted modules keep their
    # valid prefix)
    import torch

    import paper_2305_09493_amd as spv
    from gpu_util import to_dev
    w, mo = to_dev(b.words, b.mod_off)
    gres, gio, _ = spv.validate(w, mo)
    rec = spv.decode_records(w, mo, gio, gres)
    torch.cuda.synchronize()
    o = oracle.records(b.words, b.mod_off)
    rmo = rec["rec_mod_off"].cpu().numpy()
    n = int(rmo[-1])
    assert np.array_equal(rmo, o["rec_mod_off"])
    assert np.array_equal(rec["op"].cpu().numpy().view(np.uint16)[:n], o["op"])
    oo = rec["opnd_off"].cpu().numpy()[:n + 1]
    so = rec["str_off"].cpu().numpy()[:n + 1]
    assert np.array_equal(oo, o["opnd_off"]) and np.array_equal(so, o["str_off"])
    assert np.array_equal(rec["opnd"].cpu().numpy().view(np.uint32)[:oo[-1]], o["opnd"])
    assert np.array_equal(rec["chars"].cpu().numpy()[:so[-1]], o["chars"])


def test_full_encode_workload_parity():
    import torch

    import paper_2305_09493_amd as spv
    mods, r = spvgen.config4()
    print(f"[encode parity] full size: N={r['op'].size} M={r['rec_mod_off'].size - 1}", flush=True)
    d = dict(op=torch.from_numpy(r["op"].view(np.int16)).cuda(),
             opnd_off=torch.from_numpy(r["opnd_off"]).cuda(),
             opnd=torch.from_numpy(r["opnd"].view(np.int32)).cuda(),
             str_off=torch.from_numpy(r["str_off"]).cuda(),
             chars=torch.from_numpy(r["chars"]).cuda(),
             rec_mod_off=torch.from_numpy(r["rec_mod_off"]).cuda())
    words, wmo, code, bad = spv.encode(**d)
    torch.cuda.synchronize()
    wmo = wmo.cpu().numpy()
    ow, omo, oc, ob = oracle.encode(**r)
    assert np.array_equal(code.cpu().numpy().astype(np.uint32), oc)
    assert np.array_equal(bad.cpu().numpy(), ob)
    assert np.array_equal(wmo, omo)
    assert np.array_equal(words.cpu().numpy().view(np.uint32)[:omo[-1]], ow)
    assert int(omo[-1]) == sum(m.words.size for m in mods)
