"""Helpers for the GPU parity tests: run the HIP library and the CPU oracle
on the same seeded inputs and compare exactly."""
import sys

import numpy as np

import oracle


def to_dev(words, mod_off):
    import torch
    w = torch.from_numpy(np.ascontiguousarray(words, dtype=np.uint32).view(np.int32)).cuda()
    mo = torch.from_numpy(np.ascontiguousarray(mod_off, dtype=np.int64)).cuda()
    return w, mo


def gpu_run(words, mod_off, semantic=True, index=True):
    import torch
    import paper_2305_09493_amd as spv
    w, mo = to_dev(words, mod_off)
    fn = spv.validate if semantic else spv.decode
    res, io, iop = fn(w, mo, index=index)
    torch.cuda.synchronize()
    res = res.cpu().numpy().view(np.uint32)
    if index:
        io = io.cpu().numpy().view(np.uint32)
        iop = iop.cpu().numpy().view(np.uint16)
    return res, io, iop


def compare(words, mod_off, semantic=True, index=True, label=""):
    """Assert GPU == oracle: every result field and the valid index prefix."""
    print(f"[parity] {label} M={len(mod_off) - 1} W={len(words)} semantic={semantic} index={index}",
          flush=True)
    mod_off = np.asarray(mod_off, dtype=np.int64)
    g_res, g_io, g_iop = gpu_run(words, mod_off, semantic, index)
    o = oracle.validate(words, mod_off, semantic=semantic, index=index)
    o_res = o[0] if index else o
    o_arr = np.stack([o_res[k] for k in ("code", "sem_mask", "err_word", "n_inst")], axis=1).astype(np.uint32)
    bad = np.nonzero(np.any(g_res != o_arr, axis=1))[0]
    if bad.size:
        for m in bad[:10]:
            print(f"  module {m} [{mod_off[m]}, {mod_off[m + 1]}): gpu {g_res[m]} oracle {o_arr[m]}", file=sys.stderr)
    assert bad.size == 0, f"{bad.size} modules differ ({label})"
    if index:
        o_io, o_iop = o[1], o[2]
        n_inst = o_arr[:, 3].astype(np.int64)
        valid = np.zeros(len(words), dtype=bool)
        # entries [mod_off[m], mod_off[m] + n_inst[m]) are defined for every module
        starts = mod_off[:-1]
        for s, n in zip(starts[n_inst > 0], n_inst[n_inst > 0]):
            valid[s:s + n] = True
        d_off = np.nonzero(valid & (g_io != o_io))[0]
        d_op = np.nonzero(valid & (g_iop != o_iop))[0]
        assert d_off.size == 0, f"index offsets differ at {d_off[:10]} ({label})"
        assert d_op.size == 0, f"index opcodes differ at {d_op[:10]} ({label})"
    return g_res
