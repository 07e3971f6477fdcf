"""Autotuner for the library's launch knobs.

Knobs: the grids (blocks per CU) of the two kernels that run on every
decode/validate call whose tiles settle, the chain pass and the resolved
walk; blocks per CU of the single-pass fallback walk; and records per block
of the encoder.  (Tile shape, waves per tile, is a build-time constant:
2, 4 and 8 waves measured 0.83, 0.24 and 0.30 ms on the 16M-instruction
module, so the build uses 4.)  Each candidate is timed on the caller's own batch (HIP
events on the current stream, median of several calls) and the fastest is
kept in a JSON cache keyed by device, operation and a power-of-two size
bucket, so later processes reuse it (`apply`).  Cache path: $SPVGPU_TUNE_CACHE
or ~/.cache/spvgpu/tune.json.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Optional, Sequence

from . import context

VALIDATE_BPC = (1, 2, 3, 4, 6, 8)
CHAIN_BPC = (3, 4, 5, 6, 8, 12)
WALK_BPC = (3, 4, 5, 6, 8, 12)
ENCODE_BLOCKS = (256, 512, 1024, 2048, 4096)


def cache_path() -> str:
    return os.environ.get("SPVGPU_TUNE_CACHE", os.path.expanduser("~/.cache/spvgpu/tune.json"))


def _load() -> Dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(d: Dict):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def _key(op: str, size: int, device: int) -> str:
    import torch
    name = torch.cuda.get_device_properties(device).name
    return f"{name}|{op}|2^{int(math.log2(max(size, 1)))}"


def _time(fn, reps: int = 7) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def autotune_validate(words, mod_off, index: bool = True, candidates: Sequence[int] = VALIDATE_BPC,
                      device: Optional[int] = None, save: bool = True) -> Dict:
    """Time spv_validate for each blocks-per-CU candidate; keep the fastest."""
    import torch

    from . import validate
    ctx = context(device)
    W, M = int(words.numel()), int(mod_off.numel()) - 1
    res = torch.empty((M, 4), dtype=torch.int32, device=words.device)
    io = torch.empty(W, dtype=torch.int32, device=words.device) if index else None
    iop = torch.empty(W, dtype=torch.int16, device=words.device) if index else None
    ws = torch.empty(ctx.workspace_size(M, W), dtype=torch.uint8, device=words.device)
    times = {}
    for bpc in candidates:
        ctx.set_tuning(blocks_per_cu=bpc)
        times[bpc] = _time(lambda: validate(words, mod_off, index=index, ctx=ctx, out=(res, io, iop),
                                            workspace=ws))
    best = min(times, key=times.get)
    ctx.set_tuning(blocks_per_cu=best)
    out = {"blocks_per_cu": best, "ms": times[best], "all_ms": {str(k): v for k, v in times.items()}}
    if save:
        d = _load()
        d[_key("validate", W, ctx.device)] = out
        _save(d)
    return out


def autotune_grids(words, mod_off, index: bool = True, chain: Sequence[int] = CHAIN_BPC,
                   walk: Sequence[int] = WALK_BPC, device: Optional[int] = None, save: bool = True) -> Dict:
    """Time spv_validate for every (chain pass, resolved walk) grid pair and
    keep the fastest (median of several calls each)."""
    import torch

    from . import validate
    ctx = context(device)
    W, M = int(words.numel()), int(mod_off.numel()) - 1
    res = torch.empty((M, 4), dtype=torch.int32, device=words.device)
    io = torch.empty(W, dtype=torch.int32, device=words.device) if index else None
    iop = torch.empty(W, dtype=torch.int16, device=words.device) if index else None
    ws = torch.empty(ctx.workspace_size(M, W), dtype=torch.uint8, device=words.device)
    default = ctx.get_grids()
    times = {}
    for c in chain:
        for w in walk:
            ctx.set_grids(c, w)
            times[(c, w)] = _time(lambda: validate(words, mod_off, index=index, ctx=ctx, out=(res, io, iop),
                                                   workspace=ws))
    best = min(times, key=times.get)
    ctx.set_grids(*best)
    out = {"chain_blocks_per_cu": best[0], "walk_blocks_per_cu": best[1], "ms": times[best],
           "default": list(default), "default_ms": times.get(tuple(default)),
           "all_ms": {f"{c},{w}": v for (c, w), v in times.items()}}
    if save:
        d = _load()
        d[_key("validate_grids", W, ctx.device)] = out
        _save(d)
    return out


def autotune_encode(records: Dict, candidates: Sequence[int] = ENCODE_BLOCKS, device: Optional[int] = None,
                    save: bool = True) -> Dict:
    """Time spv_encode for each records-per-block candidate; keep the fastest.
    records: dict of CUDA tensors as taken by paper_2305_09493_amd.encode."""
    from . import encode
    ctx = context(device)
    N = int(records["op"].numel())
    times = {}
    for blk in candidates:
        ctx.set_tuning(encode_block=blk)
        times[blk] = _time(lambda: encode(**records, ctx=ctx))
    best = min(times, key=times.get)
    ctx.set_tuning(encode_block=best)
    out = {"encode_block": best, "ms": times[best], "all_ms": {str(k): v for k, v in times.items()}}
    if save:
        d = _load()
        d[_key("encode", N, ctx.device)] = out
        _save(d)
    return out


def apply(op: str, size: int, device: Optional[int] = None) -> Optional[Dict]:
    """Set the context's knobs from the cache for this operation and size."""
    ctx = context(device)
    d = _load().get(_key(op, size, ctx.device))
    if not d:
        return None
    if op == "validate":
        ctx.set_tuning(blocks_per_cu=int(d["blocks_per_cu"]))
    elif op == "validate_grids":
        ctx.set_grids(int(d["chain_blocks_per_cu"]), int(d["walk_blocks_per_cu"]))
    elif op == "encode":
        ctx.set_tuning(encode_block=int(d["encode_block"]))
    return d
