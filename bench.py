#!/usr/bin/env python
"""Benchmark: SPIR-V words/s decoded + validated on one MI355X.

Workload (timed): one synthetic module of 16M instructions (about 65M uint32
words, 260 MB) from the seeded generator (seed 2), decoded and validated with
the instruction index written - one step is one spv_validate call over the
whole module (header, boundary recovery, parse checks, index, result-ID
checks), replayed from a HIP graph captured once (every kernel runs in every
step; --eager launches each call instead).  Inputs are resident in HBM
before timing starts.

Also reported on the same JSON line:
  roofline      the decode/validate path's algorithmic bytes per call (4 B
                per word read + 6 B per index entry written) over the
                average duration of a whole validate call, timed with two
                HIP events around the K replays of the captured call on its
                stream (--eager: eager calls, the library's events around
                the chain pass, resolve pass, resolved walk and single-pass
                walk), against 8 TB/s; traffic: HBM bytes per call from the
                committed rocprofv3 counter summary, when it was taken on
                the current kernel code;
  cpu_baseline  the CPU oracle on the same module (one module is one
                sequential walk: one core), with the host CPU model;
  copy_ceiling  what a plain device copy reaches (read + write GB/s);
  batched       4096 lognormal modules with 41 injected faults per launch
                (graph replays of one captured call): words/s, p50 / p99
                per-launch latency, its roofline, and the oracle on the same
                batch module-parallel on every host thread (at most 16);
  records       decode's records mode on the timed module;
  text          decode's text mode (disassembly) of the timed module, with
                the paper's listing options (11) and with none (0);
  module_rules  the validate call with the module-level rules;
  encode        10M records in 1024 modules;
  serving       Poisson stream at 20k modules/s, batched vs one module per
                launch.
Each leg after the first has a --no-<leg> switch; --only-main keeps only the
timed call.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "validate_path_16M_counters.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2305_09493_amd", "csrc", "spv_validate.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_sha():
    """Fingerprint of the kernel code: sha256 of the source with // comments,
    trailing blanks and empty lines removed (comment edits keep it)."""
    import re
    with open(KERNEL_SRC) as f:
        lines = [re.sub(r"\s*//.*$", "", ln).rstrip() for ln in f]
    code = "\n".join(ln for ln in lines if ln)
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def traffic_from_counters(n_words, n_inst):
    """HBM bytes per call of the decode/validate path's kernels from the
    committed counter summary (FETCH_SIZE / WRITE_SIZE scaled by a
    copy-kernel calibration), or None when missing or taken on another
    kernel source or workload."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("source_sha") != kernel_source_sha() or c.get("n_words") != n_words:
        return None
    fetch = c["fetch_kib"] * 1024.0 * c["fetch_scale"]
    write = c["write_kib"] * 1024.0 * c["write_scale"]
    return fetch + write


def copy_calibration():
    """A plain device copy of known size, for the counter calibration."""
    import torch
    n = 1 << 28  # 1 GiB of int32
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy calibration: {n * 4} bytes per copy, 3 copies")


def encode_leg(ctx, dev, steps=10, cpu=True):
    """Encode 10M records split into 1024 modules; records/s and output words/s
    (graph replays of one captured call; the eager time per call too)."""
    import torch

    import paper_2305_09493_amd as spv
    import spvgen
    log("encode leg: generating 10M records in 1024 modules")
    mods, r = spvgen.config4()
    N = int(r["op"].size)
    M = int(r["rec_mod_off"].size - 1)
    d = dict(op=torch.from_numpy(r["op"].view(np.int16)).to(dev),
             opnd_off=torch.from_numpy(r["opnd_off"]).to(dev),
             opnd=torch.from_numpy(r["opnd"].view(np.int32)).to(dev),
             str_off=torch.from_numpy(r["str_off"]).to(dev),
             chars=torch.from_numpy(r["chars"]).to(dev),
             rec_mod_off=torch.from_numpy(r["rec_mod_off"]).to(dev))
    for _ in range(2):
        out = spv.encode(**d, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = spv.encode(**d, ctx=ctx)
    torch.cuda.synchronize()
    dt_eager = (time.perf_counter() - t0) / steps
    # the same call captured once and replayed (every kernel runs each time)
    graph, gs = torch.cuda.CUDAGraph(), torch.cuda.Stream()
    with torch.cuda.stream(gs):
        with torch.cuda.graph(graph, stream=gs):
            out = spv.encode(**d, ctx=ctx, stream=gs)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    words_out = int(out[1][-1].item())
    expect = int(sum(m.words.size for m in mods))
    bytes_moved = (2 * N + 4 * (N + 1) + 4 * r["opnd"].size + 4 * (N + 1) + r["chars"].size) + 4 * words_out
    leg = {"records": N, "modules": M, "ms_per_call": 1e3 * dt, "ms_per_call_eager": 1e3 * dt_eager,
           "records_per_s": N / dt,
           "words_out_per_s": words_out / dt, "algorithmic_GBps": bytes_moved / dt / 1e9,
           "hbm_frac": bytes_moved / dt / 1e9 / HBM_PEAK_GBS, "output_matches_generator": words_out == expect}
    if cpu:
        thr = host_threads()
        log(f"CPU oracle encode of the same records, module-parallel on {thr} threads")
        t_par, n_par = oracle_encode_parallel(r, thr)
        leg["cpu_oracle"] = {"value": N / t_par, "unit": "records/s", "cores": thr, "kind": "oracle",
                             "cpu_model": cpu_model(), "seconds": t_par,
                             "sample": f"all {N} records in {M} modules, module-parallel",
                             "words_match_gpu": n_par == words_out}
    return leg


def records_leg(ctx, words, mod_off, idx_off, res, W, steps=10):
    """Decode's records mode on the timed module: records of its 16M
    instructions from the index of the timed call; records/s and the
    algorithmic bytes (words and index read, records written) per second."""
    import torch

    import paper_2305_09493_amd as spv
    rec = spv.decode_records(words, mod_off, idx_off, res, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rec = spv.decode_records(words, mod_off, idx_off, res, ctx=ctx)
    torch.cuda.synchronize()
    dt_eager = (time.perf_counter() - t0) / steps
    graph, gs = torch.cuda.CUDAGraph(), torch.cuda.Stream()
    with torch.cuda.stream(gs):
        with torch.cuda.graph(graph, stream=gs):
            rec = spv.decode_records(words, mod_off, idx_off, res, ctx=ctx, stream=gs)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    n = int(rec["rec_mod_off"][-1].item())
    n_opnd = int(rec["opnd_off"][n].item())
    n_chars = int(rec["str_off"][n].item())
    bytes_moved = 4 * W + 4 * n + (2 * n + 8 * (n + 1) + 4 * n_opnd + n_chars)
    return {"records": n, "operand_words": n_opnd, "string_bytes": n_chars, "ms_per_call": 1e3 * dt,
            "ms_per_call_eager": 1e3 * dt_eager,
            "records_per_s": n / dt, "algorithmic_GBps": bytes_moved / dt / 1e9,
            "hbm_frac": bytes_moved / dt / 1e9 / HBM_PEAK_GBS}


def text_leg(ctx, words, mod_off, idx_off, res, W, n_inst, options_list=(11, 0), steps=10):
    """Decode's text mode (disassembly to text) on the timed module, from the
    index of the timed call: per option set, the text bytes, the time of one
    call (graph replays of the captured call between two HIP events on the
    replay stream) and the algorithmic bytes (words and index read, text
    written) per second.  Options 11 are the paper's options listing
    (highlight, inline names, indentation, grouping, header)."""
    import torch

    import paper_2305_09493_amd as spv
    out = []
    for options in options_list:
        text, tmo = spv.decode_text(words, mod_off, idx_off, res, options, ctx=ctx)  # sizing call + fill
        torch.cuda.synchronize()
        total = int(tmo[-1].item())
        graph, gs = torch.cuda.CUDAGraph(), torch.cuda.Stream()
        with torch.cuda.stream(gs):
            with torch.cuda.graph(graph, stream=gs):
                spv.decode_text(words, mod_off, idx_off, res, options, text=text, ctx=ctx, stream=gs)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        rs = torch.cuda.current_stream()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(rs)
        for _ in range(steps):
            graph.replay()
        ev1.record(rs)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        algo = 4.0 * W + 4.0 * n_inst + total
        out.append({"options": options, "text_bytes": total, "ms_per_call": ms,
                    "words_per_s": W / (ms / 1e3), "lines_per_s": n_inst / (ms / 1e3),
                    "algorithmic_bytes": algo, "algorithmic_GBps": algo / (ms / 1e3) / 1e9,
                    "hbm_frac": algo / (ms / 1e3) / 1e9 / HBM_PEAK_GBS})
        del graph, text
        torch.cuda.empty_cache()
    return out


def oracle_encode_parallel(r, threads):
    """The oracle's encoder over a record batch, module-parallel (contiguous
    groups of modules of about equal records, one per host thread).  Returns
    (seconds, words written)."""
    import concurrent.futures as cf

    import oracle
    rmo = r["rec_mod_off"]
    M = rmo.size - 1
    cuts = np.unique(np.searchsorted(rmo, np.linspace(0, rmo[-1], threads + 1)).clip(0, M))
    cuts[0], cuts[-1] = 0, M

    def run(a, b):
        r0, r1 = int(rmo[a]), int(rmo[b])
        oo = r["opnd_off"][r0:r1 + 1]
        so = r["str_off"][r0:r1 + 1]
        w, _, _, _ = oracle.encode(r["op"][r0:r1], oo - oo[0], r["opnd"][oo[0]:oo[-1]], so - so[0],
                                   r["chars"][so[0]:so[-1]], rmo[a:b + 1] - r0)
        return w.size

    oracle.encode_bound(1, 1, 1, 1)  # build / load outside the timing
    t = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        n = sum(ex.map(lambda ab: run(*ab), zip(cuts[:-1], cuts[1:])))
    return time.perf_counter() - t, n


def copy_ceiling(dev, n_bytes=1 << 30, steps=10):
    """What a plain device-to-device copy (torch's copy kernel) reaches on this
    GPU: read + write bytes per second, timed with HIP events."""
    import torch
    src = torch.ones(n_bytes // 4, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * n_bytes / (ms / 1e3) / 1e9


def host_threads():
    """Host threads this process may use (the CPU share, at most 16)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_parallel(words, mod_off, threads):
    """The oracle's validate over a batch, module-parallel: contiguous groups
    of modules of about equal words, one group per host thread (the oracle's
    C code runs without the GIL).  Returns (seconds, results)."""
    import concurrent.futures as cf

    import oracle
    M = mod_off.size - 1
    cuts = np.searchsorted(mod_off, np.linspace(0, mod_off[-1], threads + 1)).clip(0, M)
    cuts[0], cuts[-1] = 0, M
    cuts = np.unique(cuts)

    def run(a, b):
        lo, hi = int(mod_off[a]), int(mod_off[b])
        return oracle.validate(words[lo:hi], mod_off[a:b + 1] - lo, index=False)

    oracle.validate(words[:int(mod_off[1])], mod_off[:2], index=False)  # build / load outside the timing
    t = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(lambda ab: run(*ab), zip(cuts[:-1], cuts[1:])))
    dt = time.perf_counter() - t
    return dt, np.concatenate(parts)


def rules_leg(ctx, words, mod_off, plain_ms, steps=10):
    """The validate call with the module-level rules (a capability, the
    memory model, a function, an entry point) as a last stage, on the timed
    module: graph replays of the captured call, and the time the rules add to
    the plain call's step."""
    import torch

    import paper_2305_09493_amd as spv
    out = spv.validate(words, mod_off, ctx=ctx, module_rules=True)
    torch.cuda.synchronize()
    graph, gs = torch.cuda.CUDAGraph(), torch.cuda.Stream()
    with torch.cuda.stream(gs):
        with torch.cuda.graph(graph, stream=gs):
            out = spv.validate(words, mod_off, ctx=ctx, stream=gs, module_rules=True)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        graph.replay()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    res = out[0].cpu().numpy()
    return {"ms_per_call": ms, "extra_ms_over_plain_step": ms - plain_ms,
            "module_code": int(res[0, 0]), "module_sem_mask": int(res[0, 1])}


def serve_leg(args):
    """Poisson stream of validate requests: continuous batching vs one module
    per launch, same streams, kernels and arrival trace."""
    import spvgen
    from paper_2305_09493_amd.serve import run_trace
    log(f"serving leg: pool of {args.serve_pool} modules (lognormal median 5000 instructions, max 1M)")
    pool = [m.words for m in spvgen.serving_pool(n_pool=args.serve_pool)]
    out = []
    warm = args.serve_warmup
    for rate in [float(x) for x in args.serve_rates.split(",")]:
        arr = spvgen.poisson_arrivals(rate, warm + args.serve_seconds)
        pick = np.random.default_rng([5, int(rate)]).integers(0, len(pool), size=arr.size)
        row = {"rate_per_s": rate, "seconds": args.serve_seconds, "warmup_s": warm}
        for mode, kw in (("batched", dict(max_batch_modules=4096, n_slots=4)),
                         ("batched_graphs", dict(max_batch_modules=4096, n_slots=4, use_graphs=True)),
                         ("one_per_launch", dict(max_batch_modules=1, n_slots=4))):
            log(f"  rate {rate:.0f}/s {mode}")
            _, summ = run_trace(pool, arr, pick, warmup_s=warm, **kw)
            row[mode] = {k: summ[k] for k in ("requests", "words_per_s", "p50_ms", "p99_ms", "mean_batch",
                                             "server_batches")}
        out.append(row)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n-inst", type=int, default=16_000_000)
    ap.add_argument("--eager", action="store_true",
                    help="time eager calls (library events around the walk kernels) instead of graph replays")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched latency leg")
    ap.add_argument("--no-check", action="store_true", help="skip the full-size parity check")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--cache", default=None, help="npy file to keep the generated module between runs")
    ap.add_argument("--no-encode", action="store_true", help="skip the encode leg (10M records, 1024 modules)")
    ap.add_argument("--no-records", action="store_true", help="skip the records-mode leg")
    ap.add_argument("--no-text", action="store_true", help="skip the text-mode (disassembly) leg")
    ap.add_argument("--no-module-rules", action="store_true",
                    help="skip the leg of the validate call with the module-level rules")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg (Poisson stream, batched vs "
                                                            "one module per launch)")
    ap.add_argument("--only-main", action="store_true",
                    help="only the timed validate call with the default grids (no other leg, no autotuning)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default grids instead of autotuning the chain-pass and walk grids first")
    ap.add_argument("--serve-rates", default="20000", help="comma-separated arrival rates for --serve")
    ap.add_argument("--serve-seconds", type=float, default=3.0, help="measured seconds per rate")
    ap.add_argument("--serve-warmup", type=float, default=1.0,
                    help="seconds of arrivals served before the measured ones and left out of p50/p99")
    ap.add_argument("--serve-pool", type=int, default=8192)
    args = ap.parse_args()
    if args.only_main:
        args.no_cpu = args.no_batched = args.no_encode = args.no_records = args.no_text = True
        args.no_module_rules = args.no_serve = args.no_tune = True

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (batches would shard by a "
              "word-balanced cut of the module CSR, one large module by word ranges with one exchange of tile "
              "states)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2305_09493_amd as spv
    import spvgen

    if args.copy_calibration:
        copy_calibration()
        return

    dev = torch.device("cuda:0")
    t = time.time()
    if args.cache and os.path.exists(args.cache):
        cw = np.load(args.cache)
        batch = spvgen.Batch(words=cw, mod_off=np.array([0, cw.size], np.int64), modules=[])
        log(f"loaded cached module {args.cache}")
    else:
        log(f"generating module: {args.n_inst} instructions")
        batch = spvgen.config2(args.n_inst)
        if args.cache:
            np.save(args.cache, batch.words)
    W = int(batch.words.size)
    n_inst = args.n_inst
    log(f"generated {W} words in {time.time() - t:.1f}s")

    words = torch.from_numpy(batch.words.view(np.int32)).to(dev)
    mod_off = torch.from_numpy(batch.mod_off).to(dev)
    ctx = spv.context(0)
    res = torch.empty((1, 4), dtype=torch.int32, device=dev)
    idx_off = torch.empty(W, dtype=torch.int32, device=dev)
    idx_op = torch.empty(W, dtype=torch.int16, device=dev)
    ws = torch.empty(ctx.workspace_size(1, W), dtype=torch.uint8, device=dev)
    out = (res, idx_off, idx_op)

    def step(stream=None):
        spv.validate(words, mod_off, ctx=ctx, out=out, workspace=ws, stream=stream)

    # autotuner: the grids of the chain pass and the resolved walk, timed on
    # this module before the warm-up (the timed region uses the choice)
    lib_grids = ctx.get_grids()  # the library's default: each kernel's resident blocks per CU
    tuning = {"chain_blocks_per_cu": lib_grids[0], "walk_blocks_per_cu": lib_grids[1],
              "source": "default (resident blocks per CU)"}
    if not args.no_tune:
        from paper_2305_09493_amd import tune
        log("autotuning the chain-pass and walk grids on the timed module")
        tr = tune.autotune_grids(words, mod_off, save=False)
        tuning = {"chain_blocks_per_cu": tr["chain_blocks_per_cu"], "walk_blocks_per_cu": tr["walk_blocks_per_cu"],
                  "source": "autotuned on this module", "ms": tr["ms"], "default": tr["default"],
                  "default_ms": tr["default_ms"]}
        log(f"grids {tr['chain_blocks_per_cu']}, {tr['walk_blocks_per_cu']} blocks per CU: {tr['ms']:.3f} ms "
            f"(default {tr['default']}: {tr['default_ms']})")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    algo_bytes = 4.0 * W + 6.0 * n_inst
    if args.eager:
        # timed region: K whole-path calls; the library's events time its
        # boundary-recovery and walk kernels in each call
        ctx.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        k_ms, k_n = ctx.read_timing()
        ctx.set_timing(False)
        k_avg_s = (k_ms / k_n) / 1e3
        timed_kernels = "k_chain + k_resolve + k_walk (+ k_main, returns at once)"
    else:
        # timed region: K replays of one captured validate call (every kernel
        # of the call runs in every replay), between two HIP events on the
        # stream the replays run on
        graph = torch.cuda.CUDAGraph()
        gs = torch.cuda.Stream()
        with torch.cuda.stream(gs):
            with torch.cuda.graph(graph, stream=gs):
                step(gs)
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            graph.replay()
        torch.cuda.synchronize()
        # (replay() launches the graph on the current stream: the events go there)
        rs = torch.cuda.current_stream()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(rs)
        for _ in range(args.steps):
            graph.replay()
        ev1.record(rs)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        k_avg_s = ev0.elapsed_time(ev1) / 1e3 / args.steps
        timed_kernels = ("the whole validate call, graph replay: k_plan, k_chain, k_resolve, k_walk, k_main, "
                         "k_pass2" + (", k_finalize" if batch.mod_off.size - 1 > 256 else " (which writes the results: at most 256 modules)"))
    elapsed = t1 - t0
    value = W * args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    achieved = algo_bytes / k_avg_s / 1e9
    log(f"step {ms_per_step:.3f} ms, timed kernels {1e3 * k_avg_s:.3f} ms, {achieved:.0f} GB/s algorithmic")

    g = res.cpu().numpy().view(np.uint32)[0]
    checked = None
    cpu = None
    if not args.no_cpu or not args.no_check:
        import oracle
        log("CPU oracle on the same module (1 thread)")
        t = time.perf_counter()
        o, o_io, o_iop = oracle.validate(batch.words, batch.mod_off)
        t_cpu = time.perf_counter() - t
        exp = np.array([o[0][k] for k in ("code", "sem_mask", "err_word", "n_inst")], dtype=np.uint32)
        if not args.no_check:
            gi = idx_off.cpu().numpy().view(np.uint32)[:n_inst]
            gop = idx_op.cpu().numpy().view(np.uint16)[:n_inst]
            ok = (np.array_equal(g, exp) and np.array_equal(gi, o_io[:n_inst]) and
                  np.array_equal(gop, o_iop[:n_inst]))
            checked = bool(ok)
            if not ok:
                log(f"PARITY FAILURE: gpu {g} oracle {exp}")
        if not args.no_cpu:
            cpu = {"value": W / t_cpu, "unit": "words/s", "cores": 1, "kind": "oracle", "cpu_model": cpu_model(),
                   "host_threads": host_threads(),
                   "sample": f"the full timed module ({W} words), validate with index, one pass "
                             f"({t_cpu:.2f} s); one module is one sequential walk, so one core (the "
                             f"batched leg runs the oracle module-parallel on every host thread)"}

    batched = None
    if not args.no_batched:
        log("batched leg: 4096 lognormal modules")
        b3 = spvgen.config3()
        w3 = torch.from_numpy(b3.words.view(np.int32)).to(dev)
        m3 = torch.from_numpy(b3.mod_off).to(dev)
        M3, W3 = b3.n_modules, int(b3.words.size)
        r3 = torch.empty((M3, 4), dtype=torch.int32, device=dev)
        i3 = torch.empty(W3, dtype=torch.int32, device=dev)
        p3 = torch.empty(W3, dtype=torch.int16, device=dev)
        ws3 = torch.empty(ctx.workspace_size(M3, W3), dtype=torch.uint8, device=dev)
        tuning3 = {"chain_blocks_per_cu": tuning["chain_blocks_per_cu"],
                   "walk_blocks_per_cu": tuning["walk_blocks_per_cu"], "source": tuning["source"]}
        if not args.no_tune:
            from paper_2305_09493_amd import tune
            ctx.set_grids(*lib_grids)  # (the sweep reports the library default as its baseline)
            tr = tune.autotune_grids(w3, m3, save=False)
            tuning3 = {"chain_blocks_per_cu": tr["chain_blocks_per_cu"],
                       "walk_blocks_per_cu": tr["walk_blocks_per_cu"], "source": "autotuned on this batch",
                       "ms": tr["ms"], "default": tr["default"], "default_ms": tr["default_ms"]}
        for _ in range(3):
            spv.validate(w3, m3, ctx=ctx, out=(r3, i3, p3), workspace=ws3)
        torch.cuda.synchronize()
        # one launch = one replay of the captured call (as in the timed region)
        g3, s3 = torch.cuda.CUDAGraph(), torch.cuda.Stream()
        with torch.cuda.stream(s3):
            with torch.cuda.graph(g3, stream=s3):
                spv.validate(w3, m3, ctx=ctx, out=(r3, i3, p3), workspace=ws3, stream=s3)
        torch.cuda.synchronize()
        for _ in range(3):
            g3.replay()
        torch.cuda.synchronize()
        n_rep = 100
        rs = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_rep)]
        tb0 = time.perf_counter()
        for a, b in ev:
            a.record(rs)
            g3.replay()
            b.record(rs)
        torch.cuda.synchronize()
        tb1 = time.perf_counter()
        lat = np.array([a.elapsed_time(b) for a, b in ev])
        g3res = r3.cpu().numpy().view(np.uint32)
        faults = int(np.sum(g3res[:, 0] != 0))
        n3 = int(np.sum(g3res[:, 3]))
        algo3 = 4.0 * W3 + 6.0 * n3
        mean_ms = float(np.mean(lat))
        batched = {"modules": M3, "words": W3, "instructions": n3, "words_per_s": W3 * n_rep / (tb1 - tb0),
                   "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                   "modules_flagged": faults, "launches": n_rep, "tuning": tuning3,
                   "roofline": {"bound": "hbm", "achieved": algo3 / (mean_ms / 1e3) / 1e9, "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": algo3 / (mean_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                                "algorithmic_bytes": algo3,
                                "kernel": "one launch = one replay of the captured validate call (mean of "
                                          f"{n_rep} replays, HIP events on the replay stream)"}}
        if not args.no_cpu:
            thr = host_threads()
            log(f"CPU oracle on the 4096-module batch, module-parallel on {thr} threads")
            t_par, o3 = oracle_parallel(b3.words, b3.mod_off, thr)
            o3a = np.stack([o3[k] for k in ("code", "sem_mask", "err_word", "n_inst")], axis=1).astype(np.uint32)
            batched["cpu_oracle"] = {"value": W3 / t_par, "unit": "words/s", "cores": thr, "kind": "oracle",
                                     "cpu_model": cpu_model(), "seconds": t_par,
                                     "sample": f"the whole batch ({M3} modules, {W3} words), validate without "
                                               f"index, module-parallel",
                                     "results_match_gpu": bool(np.array_equal(o3a, g3res))}

    ctx.set_grids(tuning["chain_blocks_per_cu"], tuning["walk_blocks_per_cu"])  # the timed module's grids again
    records = records_leg(ctx, words, mod_off, idx_off, res, W) if not args.no_records else None
    text = None
    if not args.no_text:
        log("text leg: disassembly of the timed module, options 11 and 0")
        text = text_leg(ctx, words, mod_off, idx_off, res, W, n_inst)
    rules = rules_leg(ctx, words, mod_off, ms_per_step) if not args.no_module_rules else None
    encode = encode_leg(ctx, dev, cpu=not args.no_cpu) if not args.no_encode else None
    serving = serve_leg(args) if not args.no_serve else None
    copy_gbps = copy_ceiling(dev)
    log(f"plain device copy: {copy_gbps:.0f} GB/s")

    traffic = traffic_from_counters(W, n_inst)
    line = {
        "metric": "SPIR-V words/s decoded+validated (% HBM peak); p50/p99 module latency batched",
        "value": value,
        "unit": "words/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded generator: 12-opcode mix, sequential result IDs, uniform backward uses)",
        "config": {"workload": "one SPIR-V module, 16M instructions (~65M uint32 words), decode + validate "
                               "with the instruction index", "n_inst": n_inst, "n_words": W, "modules": 1,
                   "parallelism": "1 GPU", "tuning": tuning},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": timed_kernels,
                     "kernel_ms": 1e3 * k_avg_s,
                     "algorithmic_bytes": algo_bytes,
                     "copy_ceiling_GBps": copy_gbps,
                     "frac_of_copy_ceiling": achieved / copy_gbps},
        "cpu_baseline": cpu,
        "hbm_fraction_whole_call": (value * (algo_bytes / W) / 1e9) / HBM_PEAK_GBS,
        "batched": batched,
        "parity_checked": checked,
    }
    if records is not None:
        line["records"] = records
    if text is not None:
        line["text"] = text
    if rules is not None:
        line["module_rules"] = rules
    if encode is not None:
        line["encode"] = encode
    if serving is not None:
        line["serving"] = serving
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
