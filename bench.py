#!/usr/bin/env python3
"""Benchmark: single-buffer compression of the 256 MiB float32 field.

One step = one gpulz_compress call over the whole input already resident in
HBM (chunk encode with the longest-match search, global prefix sum + header,
record compaction). Prints one JSON line.

Workload: float32 field 512 x 512 x 256 (sum of 8 random plane waves plus
N(0, 1e-3) noise, quantised to 1e-4), 4-byte symbols, chunk 4096 symbols,
window 256, minimum match 2 (seed 1).

Other workloads (--workload), each printing its own JSON lines:
  small   1 MiB of uint16 Laplace codes (launch-latency bound): median of
          single launches and of graph replays;
  dense   256 MiB each of Zipf bytes and uint16 Laplace codes (match-dense:
          the exact search runs at almost every token);
  scan    match policy 1 (the paper's single window pass) beside policy 0
          on the field and on the 1 MiB codes;
  adaptive  the adaptive symbol width / window rule and its levels on each
          content kind, against the element-width default;
  host    a 1 GiB host-resident input streamed through the GPU in blocks
          (PCIe included);
  entropy 256 MiB of uint16 codes through LZSS then the Huffman stage, and
          back;
  sweep   1 GiB per symbol width (Zipf bytes, Laplace uint16 codes, sorted
          uint32 indices, float64 field), parameters from the autotuner;
  batch   4096 buffers, log-uniform 4 KiB..64 MiB, mixed widths, one
          graph-captured batch call against one gpulz_compress per buffer;
  serve   Poisson stream of compress/decompress requests with continuous
          batching under an HBM admission budget.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0

# HBM bytes per encode launch on this workload from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the
# same counter reads for a device copy of the 256 MiB input (FETCH_SIZE reads
# half the copied bytes: factor 2.0; WRITE_SIZE reads them exactly: 1.0).
# Valid only for the encoder sources they were taken on (sha256 below; the
# generated dense-parse assembly is left out: only 1- and 2-byte encoders
# instantiate it, and this workload has 4-byte symbols).
# "prep" is the compress call's preparation kernel (look-back descriptors
# and tickets zeroed); the step is prep + encode.
ENCODE_COUNTERS = {
    "sources_sha256": "2d96b58d2cec28f720430b5cc2d49e536ba57dc09fd90b1ae079cd0f15622aab",
    "fetch_kib": 140127.6, "write_kib": 277144.8,
    "prep_fetch_kib": 16.0, "prep_write_kib": 128.3,
    "fetch_scale": 2.0, "write_scale": 1.0,
}
ENCODE_SOURCES = ("paper_2304_07342_amd/csrc/lz_encode.hip", "paper_2304_07342_amd/csrc/encode_device.h",
                  "paper_2304_07342_amd/csrc/stream_device.h", "paper_2304_07342_amd/csrc/wave.h",
                  "paper_2304_07342_amd/csrc/gpulz_internal.h")


def encoder_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ENCODE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def encode_traffic_bytes():
    """Counter-derived HBM bytes per encode launch and per whole step (prep +
    encode), or (None, None) if the encoder has changed since the counters
    were taken."""
    c = ENCODE_COUNTERS
    if c["sources_sha256"] is None or encoder_sources_sha256() != c["sources_sha256"]:
        return None, None
    enc = (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]) * 1024
    prep = (c["prep_fetch_kib"] * c["fetch_scale"] + c["prep_write_kib"] * c["write_scale"]) * 1024
    return int(enc), int(enc + prep)
# 256 CUs x 64 lanes x 2.4 GHz: one 32-bit compare per lane per clock.
ALU_PEAK_TCMP = 256 * 64 * 2.4e9 / 1e12


def window_compares(m: int, C: int, W: int) -> int:
    """Symbol comparisons of an exhaustive window search: every position j of
    a chunk is compared with each of the min(j, W) symbols before it."""
    def per_chunk(c):
        if c <= W + 1:
            return c * (c - 1) // 2
        return W * (W + 1) // 2 + (c - 1 - W) * W
    full, last = divmod(m, C)
    return full * per_chunk(C) + (per_chunk(last) if last else 0)


def executed_hit_compares(m: int, C: int, W: int, S: int, MIN: int) -> int:
    """Symbol compares the encoder's hit phase executes: each lane owns V =
    16 / S positions of a 64 V block and compares every tested position
    (even ones when MIN >= 2) with W window offsets, masked or not. The
    exact searches at candidate positions come on top (data-dependent, rare
    on the field)."""
    V = 16 // S
    step = 2 if MIN >= 2 else 1

    def per_chunk(c):
        blocks = -(-c // (64 * V))
        return blocks * 64 * (V // step) * W
    full, last = divmod(m, C)
    return full * per_chunk(C) + (per_chunk(last) if last else 0)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_threads() -> int:
    """Host threads for the all-cores oracle run: the cores this process may
    use, at most 16 (one GPU's share of a shared host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(x: np.ndarray, S: int, C: int, W: int, MIN: int, sample_bytes: int,
                 threads: int = 1):
    """The C oracle on the first `sample_bytes` of the input; with threads > 1
    its chunks are spread over a thread pool (chunks are independent)."""
    import oracle
    oracle.build(force=False)
    sample = x[:sample_bytes]
    t0 = time.perf_counter()
    oracle.compress(sample, S, C, W, MIN, threads=threads)
    dt = time.perf_counter() - t0
    kind = "single-threaded C oracle" if threads == 1 else f"C oracle over {threads} threads"
    return {"value": round(sample.size / dt / 1e9, 6), "unit": "GB/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"first {sample.size >> 20} MiB ({sample.size // (C * S)} chunks) of the same "
                      f"input, {kind}, {dt:.1f} s"}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def pools_on_device(kinds, pool_bytes, seed0=100):
    """Generate each content kind's pool once and keep it on the device."""
    import torch
    from paper_2304_07342_amd import synth
    out = {}
    for i, kind in enumerate(kinds):
        S, gen = synth.POOL_KINDS[kind]
        log(f"pool {kind} {pool_bytes >> 20} MiB")
        host = gen(pool_bytes, seed0 + i)
        out[kind] = torch.from_numpy(host[:pool_bytes]).to("cuda")
        del host
    return out


def autotune_widths(pools, sample_bytes, log_fn=None):
    from paper_2304_07342_amd import autotune, synth
    samples = {}
    for S, kinds in synth.WIDTH_KINDS.items():
        samples[S] = pools[kinds[0]][:sample_bytes]
    return autotune.tune(samples, log=log_fn)


def run_sweep(args):
    import torch
    from paper_2304_07342_amd import autotune, gpulz, synth
    size = args.sweep_bytes
    kinds = {1: "zipf-u8", 2: "laplace-u16", 4: "sorted-u32", 8: "field-f64"}
    for S, kind in kinds.items():
        log(f"sweep {kind} {size >> 20} MiB")
        x = torch.from_numpy(synth.POOL_KINDS[kind][1](size, 200 + S)[:size]).to("cuda")
        tuned = autotune.tune_width(x[: min(size, 64 << 20)], S, log=log)
        autotune.apply({S: tuned})
        C, W, MIN, waves = tuned["chunk_symbols"], tuned["window"], tuned["min_match"], \
            tuned["waves_per_chunk"]
        comp = gpulz.Compressor(size, S, C, W, MIN)
        comp.compress_async(x)
        nbytes, status = comp.result()
        assert status == gpulz.GPULZ_OK
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            comp.compress_async(x)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        # decompression into preallocated buffers, same stream
        s_in = comp.out[:nbytes]
        d = torch.empty(size, dtype=torch.uint8, device="cuda")
        ws_bytes = gpulz.gpulz_decompress_workspace_size(nbytes)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        meta = torch.zeros(2, dtype=torch.int64, device="cuda")

        def dec():
            gpulz._check(gpulz.gpulz_decompress(s_in.data_ptr(), nbytes, d.data_ptr(), size,
                                                meta.data_ptr(), meta.data_ptr() + 8, ws.data_ptr(),
                                                ws_bytes, stream.cuda_stream), "gpulz_decompress")
        dec()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            dec()
        e1.record(stream)
        torch.cuda.synchronize()
        dms = e0.elapsed_time(e1) / args.steps
        if int(meta[1]) != 0 or not torch.equal(d, x):
            raise SystemExit(f"round trip mismatch for {kind}")
        print(json.dumps({"metric": "compress GB/s (input) + ratio", "workload": f"sweep-{kind}",
                          "symbol_bytes": S, "input_bytes": size, "value": round(size / ms / 1e6, 3),
                          "unit": "GB/s", "ms_per_step": round(ms, 4),
                          "ratio": round(size / nbytes, 4), "chunk_symbols": C, "window": W,
                          "min_match": MIN, "waves_per_chunk": waves,
                          "decompress_GBps": round(size / dms / 1e6, 3),
                          "autotune_candidates": len(tuned["measurements"])}), flush=True)
        del x, comp, d, ws
        torch.cuda.empty_cache()


def small_leg(args):
    """1 MiB of uint16 codes: launch-latency bound, so report the median of
    single launches and of graph replays of the same call."""
    import torch
    from paper_2304_07342_amd import gpulz, synth
    cfg = synth.WORKLOADS[synth.CODES_1MIB]
    S, C, W, MIN = cfg["S"], cfg["C"], cfg["W"], cfg["MIN"]
    x = torch.from_numpy(cfg["make"]().view(np.uint8).reshape(-1)).to("cuda")
    n = x.numel()
    comp = gpulz.Compressor(n, S, C, W, MIN)
    stream = torch.cuda.current_stream()
    reps = max(200, args.steps)

    def median_ms(launch):
        for _ in range(max(3, args.warmup)):
            launch()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            launch()
            b.record(stream)
        torch.cuda.synchronize()
        t = sorted(a.elapsed_time(b) for a, b in ev)
        return t[len(t) // 2]

    single = median_ms(lambda: comp.compress_async(x))
    size, status = comp.result()
    assert status == gpulz.GPULZ_OK
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        comp.compress_async(x)  # warm the launch path on the capture stream
        side.synchronize()
        with torch.cuda.graph(g, stream=side):
            comp.compress_async(x)
    stream.wait_stream(side)
    graph = median_ms(g.replay)
    size2, status2 = comp.result()
    assert status2 == gpulz.GPULZ_OK and size2 == size
    d = gpulz.decompress(comp.out[:size])
    if not torch.equal(d, x):
        raise SystemExit("round trip mismatch")
    return {"metric": "compress GB/s (input) + ratio", "workload": cfg["name"],
            "input_bytes": n, "ratio": round(n / size, 4), "symbol_bytes": S,
            "chunk_symbols": C, "window": W, "min_match": MIN, "runs": reps,
            "single_launch_ms_p50": round(single, 4),
            "single_launch_GBps": round(n / single / 1e6, 3),
            "graph_replay_ms_p50": round(graph, 4),
            "graph_replay_GBps": round(n / graph / 1e6, 3)}


def run_small(args):
    print(json.dumps(small_leg(args)), flush=True)


# Match-dense inputs: (kind, seed, S, MIN). Chunk size, window and waves per
# chunk are the autotuner's choice on the first 64 MiB of the same input.
DENSE_INPUTS = (("zipf-u8", 201, 1, 2), ("laplace-u16", 202, 2, 2))


def dense_leg(args, kind, seed, S, MIN, size, params=None):
    """One match-dense input: compress GB/s, ratio, the encode kernel's
    average time (HIP events on the call's stream) and its algorithmic
    compare rate against the ALU compare peak. `params` = (C, W, waves) skips
    the autotuner."""
    import torch
    from paper_2304_07342_amd import autotune, gpulz, synth
    log(f"dense {kind} {size >> 20} MiB")
    x = torch.from_numpy(synth.POOL_KINDS[kind][1](size, seed)[:size]).to("cuda")
    tuned = None
    if params is None:
        tuned = autotune.tune_width(x[: min(size, 64 << 20)], S, MIN)
        params = (tuned["chunk_symbols"], tuned["window"], tuned["waves_per_chunk"])
    C, W, waves = params
    saved = gpulz.gpulz_default_params(S)
    gpulz.gpulz_set_default_params(S, saved[0], saved[1], saved[2], waves)
    try:
        comp = gpulz.Compressor(size, S, C, W, MIN)
        for _ in range(max(1, args.warmup)):
            comp.compress_async(x)
        nbytes, status = comp.result()
        assert status == gpulz.GPULZ_OK
        stream = torch.cuda.current_stream()
        gpulz.gpulz_profile_enable(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        steps = max(1, min(args.steps, 10))
        e0.record(stream)
        for _ in range(steps):
            comp.compress_async(x)
        e1.record(stream)
        torch.cuda.synchronize()
        prof = gpulz.gpulz_profile_read()
        gpulz.gpulz_profile_enable(False)
    finally:
        gpulz.gpulz_set_default_params(S, *saved)
    ms = e0.elapsed_time(e1) / steps
    d = gpulz.decompress(comp.out[:nbytes])
    if not torch.equal(d, x):
        raise SystemExit(f"round trip mismatch for {kind}")
    kernel_ms = {k: round(v[0] / max(1, v[1]), 4) for k, v in prof.items() if v[1]}
    enc_ms = kernel_ms.get("encode", ms)
    cmp = window_compares(size // S, C, W)
    out = {"workload": f"dense-{kind}-{size >> 20}MiB", "symbol_bytes": S, "input_bytes": size,
           "value": round(size / ms / 1e6, 3), "unit": "GB/s", "ms_per_step": round(ms, 4),
           "ratio": round(size / nbytes, 4), "chunk_symbols": C, "window": W, "min_match": MIN,
           "waves_per_chunk": waves, "kernel_avg_ms": kernel_ms,
           "compare_peak_frac": round(cmp / (enc_ms / 1e3) / 1e12 / ALU_PEAK_TCMP, 4),
           "params_from": "autotuner" if tuned else "given"}
    if tuned:
        out["autotune_candidates"] = len(tuned["measurements"])
    del x, comp, d
    torch.cuda.empty_cache()
    return out


def run_dense(args):
    """256 MiB each of Zipf bytes and uint16 Laplace codes, the match-dense
    inputs where the exact search runs at almost every token."""
    for kind, seed, S, MIN in DENSE_INPUTS:
        params = tuple(args.dense_params) if args.dense_params else None
        leg = dense_leg(args, kind, seed, S, MIN, args.dense_mib << 20, params)
        leg["metric"] = "compress GB/s (input) + ratio"
        print(json.dumps(leg), flush=True)


def run_scan(args):
    """Match policy 1 (the paper's single window pass) against policy 0 (exact
    longest match) on the 256 MiB field and the 1 MiB uint16 codes: GB/s and
    ratio of each."""
    import torch
    from paper_2304_07342_amd import gpulz, synth
    for key in (synth.FIELD_256MIB, synth.CODES_1MIB):
        cfg = synth.WORKLOADS[key]
        S, C, W, MIN = cfg["S"], cfg["C"], cfg["W"], cfg["MIN"]
        x = torch.from_numpy(cfg["make"]().view(np.uint8).reshape(-1)).to("cuda")
        n = x.numel()
        res = {}
        for policy in (1, 0):
            comp = gpulz.Compressor(n, S, C, W, MIN, policy=policy)
            for _ in range(max(1, args.warmup)):
                comp.compress_async(x)
            size, status = comp.result()
            assert status == gpulz.GPULZ_OK
            stream = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                comp.compress_async(x)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            if policy == 1 and not torch.equal(gpulz.decompress(comp.out[:size]), x):
                raise SystemExit("round trip mismatch")
            res[policy] = (ms, size)
            del comp
        print(json.dumps({
            "metric": "compress GB/s (input) + ratio", "workload": f"{cfg['name']}-scan-policy",
            "input_bytes": n, "symbol_bytes": S, "chunk_symbols": C, "window": W,
            "min_match": MIN, "steps": args.steps,
            "scan_GBps": round(n / res[1][0] / 1e6, 3), "scan_ms": round(res[1][0], 4),
            "scan_ratio": round(n / res[1][1], 4),
            "exact_GBps": round(n / res[0][0] / 1e6, 3), "exact_ms": round(res[0][0], 4),
            "exact_ratio": round(n / res[0][1], 4)}), flush=True)
        del x
        torch.cuda.empty_cache()


def run_adaptive(args):
    """Section 3.2.3's adaptive width / window rule on each content kind
    (256 MiB, four 64 MiB fields): the element-width default against the
    adaptive plan at each level; GB/s and ratio of each."""
    import torch
    from paper_2304_07342_amd import adaptive, gpulz, synth
    kinds = {"zipf-u8": 1, "laplace-u16": 2, "sorted-u32": 4, "field-f32": 4, "field-f64": 8}
    size = args.pool_mib << 20
    for i, (kind, E) in enumerate(kinds.items()):
        x = torch.from_numpy(synth.POOL_KINDS[kind][1](size, 300 + i)[:size]).to("cuda")
        fields = list(x.split(size // 4))
        out = {"metric": "compress GB/s (input) + ratio", "workload": f"adaptive-{kind}",
               "input_bytes": size, "element_bytes": E, "runs": []}

        def timed(S, C, W, MIN):
            comp = gpulz.Compressor(size, S, C, W, MIN)
            comp.compress_async(x)
            nbytes, st = comp.result()
            assert st == gpulz.GPULZ_OK
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            stream = torch.cuda.current_stream()
            e0.record(stream)
            for _ in range(3):
                comp.compress_async(x)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 3
            return round(size / ms / 1e6, 3), round(size / nbytes, 4)

        C, W, MIN, _ = gpulz.gpulz_default_params(E)
        gbps, ratio = timed(E, C, W, MIN)
        out["runs"].append({"plan": "element width, default window", "S": E, "C": C, "W": W,
                            "GBps": gbps, "ratio": ratio})
        for level in (1, 2, 3, 4):
            p = adaptive.plan(fields, E, level)
            gbps, ratio = timed(p.symbol_bytes, p.chunk_symbols, p.window, p.min_match)
            out["runs"].append({"plan": f"adaptive level {level}", "S": p.symbol_bytes,
                                "C": p.chunk_symbols, "W": p.window,
                                "multi_byte_ratio": None if p.multi_byte_ratio is None
                                else round(p.multi_byte_ratio, 4),
                                "GBps": gbps, "ratio": ratio})
            log(f"adaptive {kind} level {level}: S={p.symbol_bytes} W={p.window} {gbps} GB/s r{ratio}")
        print(json.dumps(out), flush=True)
        del x, fields
        torch.cuda.empty_cache()


def run_host(args):
    """Host-resident input streamed in blocks (section 3.3.1): the 256 MiB
    field tiled 4x (1 GiB in pageable host memory, and again in pinned
    memory). Wall-clock rates include the host staging copies and PCIe both
    ways; the device-resident rate of the same input is printed beside
    them."""
    import torch
    from paper_2304_07342_amd import gpulz, stream_host, synth
    cfg = synth.WORKLOADS[synth.FIELD_256MIB]
    S, C, W, MIN = cfg["S"], cfg["C"], cfg["W"], cfg["MIN"]
    x = np.tile(cfg["make"]().view(np.uint8).reshape(-1), 4)
    n = x.size
    d = torch.from_numpy(x).to("cuda")
    comp = gpulz.Compressor(n, S, C, W, MIN)
    comp.compress_async(d)
    size, st = comp.result()
    ref = comp.out[:size].cpu().numpy()
    t0 = time.perf_counter()
    for _ in range(3):
        comp.compress_async(d)
    comp.result()
    dev_s = (time.perf_counter() - t0) / 3
    del comp, d
    torch.cuda.empty_cache()
    pinned = torch.from_numpy(x).pin_memory()
    threads = stream_host.default_threads()
    runs = []
    cases = [("pageable", x, b) for b in (64 << 20, 128 << 20, 256 << 20)]
    cases += [("pageable", x, None), ("pinned", pinned, 128 << 20)]
    for kind, src, block in cases:
        stream_host.compress_host(src, S, C, W, MIN, block_bytes=block)   # warm-up (pinned caches)
        t0 = time.perf_counter()
        s = stream_host.compress_host(src, S, C, W, MIN, block_bytes=block)
        ct = time.perf_counter() - t0
        if not np.array_equal(s, ref):
            raise SystemExit("block-streamed stream differs from the whole-input stream")
        stream_host.decompress_host(s, block_bytes=block)
        t0 = time.perf_counter()
        y = stream_host.decompress_host(s, block_bytes=block)
        dt = time.perf_counter() - t0
        if not np.array_equal(y, x):
            raise SystemExit("block-streamed round trip mismatch")
        runs.append({"input": kind, "block_bytes": block or stream_host.default_block_bytes(),
                     "compress_GBps": round(n / ct / 1e9, 3),
                     "decompress_GBps": round(n / dt / 1e9, 3)})
        log(f"host {runs[-1]}")
    print(json.dumps({"metric": "compress GB/s (input), host-resident, PCIe included",
                      "workload": "field-f32-1GiB-host", "input_bytes": n, "ratio": round(n / size, 4),
                      "threads": threads, "device_resident_wall_GBps": round(n / dev_s / 1e9, 3),
                      "runs": runs}), flush=True)


def run_entropy(args):
    """The entropy stage after LZSS (section 4.5 pairs gpuLZ with a Huffman
    coder): 256 MiB of uint16 quantization codes (the cuSZ stand-in) through
    LZSS (S=2, C=2048, W=128, MIN=2), Huffman on the LZSS stream, the two
    chained on one stream, Huffman on the raw codes, and the decoders; GB/s
    of each (over its own input bytes) and ratios."""
    import torch
    from paper_2304_07342_amd import gpulz, synth
    x = torch.from_numpy(synth.laplace_codes_pool(1 << 27, seed=7).view(np.uint8)).to("cuda")
    n = x.numel()
    stream = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(max(1, args.warmup)):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    def huff_decoder(s, cap):
        out = torch.empty(max(cap, 1), dtype=torch.uint8, device="cuda")
        ws_bytes = gpulz.gpulz_huff_decompress_workspace_size(s.numel())
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        meta = torch.zeros(2, dtype=torch.int64, device="cuda")

        def run():
            gpulz._check(gpulz.gpulz_huff_decompress(
                s.data_ptr(), s.numel(), out.data_ptr(), cap, meta.data_ptr(),
                meta.data_ptr() + 8, ws.data_ptr(), ws_bytes, stream.cuda_stream), "huff decode")
        return run, out, meta

    lz = gpulz.Compressor(n, 2, 2048, 128, 2)
    lz_ms = timed(lambda: lz.compress_async(x))
    lz_size, st = lz.result()
    assert st == gpulz.GPULZ_OK
    lz_stream = lz.out[:lz_size].clone()
    hc = gpulz.HuffCompressor(lz.capacity)
    huff_ms = timed(lambda: hc.compress_async(lz_stream))
    h_size, st = hc.result()
    assert st == gpulz.GPULZ_OK

    def chain():
        lz.compress_async(x)
        hc.compress_async(lz.out.data_ptr(), lz.capacity, d_nbytes=lz.meta.data_ptr())
    chain_ms = timed(chain)
    c_size, st = hc.result()
    assert st == gpulz.GPULZ_OK and c_size == h_size
    chain_stream = hc.out[:c_size].clone()
    raw = gpulz.HuffCompressor(n)
    raw_ms = timed(lambda: raw.compress_async(x))
    raw_size, st = raw.result()
    assert st == gpulz.GPULZ_OK

    hdec, hout, hmeta = huff_decoder(chain_stream, lz_size)
    hdec_ms = timed(hdec)
    if int(hmeta[1]) != 0 or not torch.equal(hout[:lz_size], lz_stream):
        raise SystemExit("Huffman decode mismatch")
    lz_out = torch.empty(n, dtype=torch.uint8, device="cuda")
    lz_ws_bytes = gpulz.gpulz_decompress_workspace_size(lz_size)
    lz_ws = torch.empty(lz_ws_bytes, dtype=torch.uint8, device="cuda")
    lz_meta = torch.zeros(2, dtype=torch.int64, device="cuda")

    def lz_dec():
        gpulz._check(gpulz.gpulz_decompress(hout.data_ptr(), lz_size, lz_out.data_ptr(), n,
                                            lz_meta.data_ptr(), lz_meta.data_ptr() + 8,
                                            lz_ws.data_ptr(), lz_ws_bytes, stream.cuda_stream),
                     "lz decode")
    lzdec_ms = timed(lz_dec)

    def chain_dec():
        hdec()
        lz_dec()
    chain_dec_ms = timed(chain_dec)
    if not torch.equal(lz_out, x):
        raise SystemExit("chain round trip mismatch")
    # the oracles on a sample of the same codes: LZSS over the host threads,
    # then the (single-threaded) Huffman oracle on its stream
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        threads = cpu_threads()
        sample = x[: 32 << 20].cpu().numpy()
        t0 = time.perf_counter()
        lz_s = oracle.compress(sample, 2, 2048, 128, 2, threads=threads)
        oracle.huff_compress(lz_s)
        dt = time.perf_counter() - t0
        cpu = {"value": round(sample.size / dt / 1e9, 6), "unit": "GB/s", "cores": threads,
               "kind": "oracle",
               "sample": f"first 32 MiB of the same codes: C oracle LZSS over {threads} threads, then "
                         f"the single-threaded Huffman oracle, {dt:.1f} s"}
    print(json.dumps({
        "metric": "compress GB/s (input) + ratio", "workload": "codes-u16-256MiB-lz-huffman",
        "input_bytes": n, "lz_bytes": lz_size, "chain_bytes": c_size, "raw_huffman_bytes": raw_size,
        "steps": args.steps,
        "lz_ratio": round(n / lz_size, 4), "chain_ratio": round(n / c_size, 4),
        "raw_huffman_ratio": round(n / raw_size, 4),
        "lz_GBps": round(n / lz_ms / 1e6, 3),
        "huffman_on_lz_GBps": round(lz_size / huff_ms / 1e6, 3), "huffman_on_lz_ms": round(huff_ms, 4),
        "chain_GBps": round(n / chain_ms / 1e6, 3), "chain_ms": round(chain_ms, 4),
        "huffman_on_codes_GBps": round(n / raw_ms / 1e6, 3),
        "huffman_decode_GBps": round(lz_size / hdec_ms / 1e6, 3), "huffman_decode_ms": round(hdec_ms, 4),
        "lz_decode_GBps": round(n / lzdec_ms / 1e6, 3),
        "chain_decode_GBps": round(n / chain_dec_ms / 1e6, 3),
        # Huffman stage: algorithmic HBM bytes (its input once + its stream once)
        # per call over the call's time, against the 8 TB/s peak
        "huffman_hbm_frac": {"compress": round((lz_size + h_size) / huff_ms / 1e6 / HBM_PEAK_GBPS, 4),
                             "decode": round((lz_size + c_size) / hdec_ms / 1e6 / HBM_PEAK_GBPS, 4)},
        "cpu_baseline": cpu}), flush=True)


def batch_leg(args):
    """4096 buffers (log-uniform sizes, mixed widths): one graph-captured
    gpulz_compress_batch replay against one gpulz_compress per buffer."""
    import torch
    from paper_2304_07342_amd import gpulz, synth
    pool_bytes = args.pool_mib << 20
    spec = synth.batch_spec(args.nbufs, seed=3, pool_bytes=pool_bytes)
    pools = pools_on_device(list(synth.POOL_KINDS), pool_bytes)
    tuned = autotune_widths(pools, 64 << 20, log)
    inputs = [pools[kind][off:off + n] for kind, S, off, n in spec]
    widths = [S for _, S, _, _ in spec]
    total = sum(n for _, _, _, n in spec)
    log(f"batch of {len(spec)} buffers, {total / 2**30:.2f} GiB")
    bc = gpulz.BatchCompressor(inputs, widths, None)
    bc.capture()
    stream = torch.cuda.current_stream()
    bc.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        bc.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    batched_ms = e0.elapsed_time(e1) / args.steps
    res = bc.results()
    assert all(st == gpulz.GPULZ_OK for st, _ in res)
    z = sum(int(s.numel()) for _, s in res)

    # plain: one gpulz_compress per buffer, same parameters, same stream
    log("plain path")
    params = {S: gpulz.gpulz_default_params(S) for S in (1, 2, 4, 8)}
    max_ws = max(gpulz.gpulz_compress_workspace_size(n, S, params[S][0]) for _, S, _, n in spec)
    ws = torch.empty(max_ws, dtype=torch.uint8, device="cuda")
    meta = torch.zeros(2 * len(spec), dtype=torch.int64, device="cuda")
    outs = [torch.empty_like(o) for o in bc.outputs]

    def plain(record=None):
        for i, (x, S) in enumerate(zip(inputs, widths)):
            C, W, MIN, _ = params[S]
            st = gpulz.gpulz_compress(x.data_ptr(), x.numel(), S, C, W, MIN, outs[i].data_ptr(),
                                      bc.caps[i], meta[2 * i:].data_ptr(), meta[2 * i + 1:].data_ptr(),
                                      ws.data_ptr(), max_ws, stream.cuda_stream)
            assert st == gpulz.GPULZ_OK
            if record is not None:
                record[i].record(stream)
    plain()
    torch.cuda.synchronize()
    ends = [torch.cuda.Event(enable_timing=True) for _ in spec]
    p0 = torch.cuda.Event(enable_timing=True)
    p0.record(stream)
    plain(ends)
    torch.cuda.synchronize()
    done = sorted(p0.elapsed_time(e) for e in ends)
    plain_ms = done[-1]
    # the two paths must produce the same streams
    sizes = meta.view(-1, 2)[:, 0].cpu().tolist()
    for i, (st, s) in enumerate(res):
        if sizes[i] != s.numel() or not torch.equal(outs[i][:sizes[i]], s):
            raise SystemExit(f"batched and plain streams differ for buffer {i}")
    pct = lambda v, q: v[min(len(v) - 1, int(q * len(v)))]
    out = {
        "metric": "batched GB/s and p99 latency vs plain", "workload": f"batch-{len(spec)}",
        "nbufs": len(spec), "input_bytes": total, "stream_bytes": z, "ratio": round(total / z, 4),
        "batched_GBps": round(total / batched_ms / 1e6, 3), "batched_ms": round(batched_ms, 3),
        "plain_GBps": round(total / plain_ms / 1e6, 3), "plain_ms": round(plain_ms, 3),
        "speedup": round(plain_ms / batched_ms, 3),
        "batched_completion_ms": {"p50": round(batched_ms, 3), "p99": round(batched_ms, 3)},
        "plain_completion_ms": {"p50": round(pct(done, 0.5), 3), "p99": round(pct(done, 0.99), 3)},
        "params": {str(S): list(p) for S, p in params.items()},
        "autotune_GBps": {str(S): round(v["GBps"], 2) for S, v in tuned.items()}}
    del bc, outs, ws, pools, inputs
    torch.cuda.empty_cache()
    return out


def run_batch(args):
    print(json.dumps(batch_leg(args)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="field",
                    choices=["field", "small", "dense", "scan", "sweep", "adaptive", "host",
                             "entropy", "batch", "serve"])
    ap.add_argument("--sweep-bytes", type=int, default=1 << 30)
    ap.add_argument("--dense-mib", type=int, default=256)
    ap.add_argument("--dense-params", type=int, nargs=3, metavar=("C", "W", "WAVES"),
                    help="dense workload at these parameters instead of the autotuner's")
    ap.add_argument("--nbufs", type=int, default=4096)
    ap.add_argument("--pool-mib", type=int, default=256)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--sweep-rates", type=float, nargs="*", default=[250.0, 500.0, 1000.0])
    ap.add_argument("--sweep-seconds", type=float, default=10.0)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-slots", type=int, default=3)
    ap.add_argument("--serve-streams", type=int, default=128)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-mib", type=int, default=128)
    ap.add_argument("--skip-decompress", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the field compression (no config 0, dense uint16 or batch keys)")
    ap.add_argument("--no-batch", action="store_true", help="no batch key")
    ap.add_argument("--profile-copy", action="store_true",
                    help="end with one untimed device copy of the input (a known-size "
                         "reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only; multi-GPU runs are not supported",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "small":
        return run_small(args)
    if args.workload == "dense":
        return run_dense(args)
    if args.workload == "scan":
        return run_scan(args)
    if args.workload == "adaptive":
        return run_adaptive(args)
    if args.workload == "host":
        return run_host(args)
    if args.workload == "entropy":
        return run_entropy(args)
    if args.workload == "sweep":
        return run_sweep(args)
    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "serve":
        from paper_2304_07342_amd import serve
        return serve.main_bench(args)

    import torch
    from paper_2304_07342_amd import gpulz, synth

    cfg = synth.WORKLOADS[synth.FIELD_256MIB]
    S, C, W, MIN = cfg["S"], cfg["C"], cfg["W"], cfg["MIN"]
    print(f"[bench] generating {cfg['name']}", file=sys.stderr, flush=True)
    x = cfg["make"]().view(np.uint8).reshape(-1)
    n = x.size
    d_in = torch.from_numpy(x).to("cuda")
    comp = gpulz.Compressor(n, S, C, W, MIN)
    torch.cuda.synchronize()

    print("[bench] warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        comp.compress_async(d_in)
    size, status = comp.result()
    if status != gpulz.GPULZ_OK:
        raise SystemExit(f"compress failed: {gpulz.status_string(status)}")

    print("[bench] timed steps", file=sys.stderr, flush=True)
    gpulz.gpulz_profile_enable(True)
    stream = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(args.steps):
        comp.compress_async(d_in)
    stop.record(stream)
    torch.cuda.synchronize()
    prof = gpulz.gpulz_profile_read()
    gpulz.gpulz_profile_enable(False)
    ms_step = start.elapsed_time(stop) / args.steps
    size, status = comp.result()
    assert status == gpulz.GPULZ_OK

    # exact round trip of the produced stream (outside the timed region)
    print("[bench] verify + decompress", file=sys.stderr, flush=True)
    dec_gbps = None
    if not args.skip_decompress:
        st_t = comp.out[:size]
        d = gpulz.decompress(st_t)
        if not torch.equal(d, d_in):
            raise SystemExit("round trip mismatch")
        ws_bytes = gpulz.gpulz_decompress_workspace_size(size)
        out = torch.empty(n, dtype=torch.uint8, device="cuda")
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        meta = torch.zeros(2, dtype=torch.int64, device="cuda")
        for _ in range(2):
            gpulz.gpulz_decompress(st_t.data_ptr(), size, out.data_ptr(), n, meta.data_ptr(),
                                   meta.data_ptr() + 8, ws.data_ptr(), ws_bytes, stream.cuda_stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        reps = max(3, args.steps // 2)
        for _ in range(reps):
            gpulz.gpulz_decompress(st_t.data_ptr(), size, out.data_ptr(), n, meta.data_ptr(),
                                   meta.data_ptr() + 8, ws.data_ptr(), ws_bytes, stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        dec_gbps = n / (e0.elapsed_time(e1) / reps / 1e3) / 1e9

    enc_ms, enc_launches = prof["encode"]
    enc_avg_ms = enc_ms / max(1, enc_launches)
    m = n // S
    compares = window_compares(m, C, W)
    executed = executed_hit_compares(m, C, W, S, MIN)
    achieved = compares / (enc_avg_ms / 1e3) / 1e12
    kernel_ms = {k: round(v[0] / max(1, v[1]), 4) for k, v in prof.items() if v[1]}
    value = n / (ms_step / 1e3) / 1e9
    traffic, step_traffic = encode_traffic_bytes()

    result = {
        "metric": "compress GB/s (input) + ratio at 1 GPU; batched GB/s and p99 latency vs plain",
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "field-f32-256MiB: float32 512x512x256, 8 plane waves + N(0,1e-3) "
                               "noise quantised to 1e-4, seed 1",
                   "symbol_bytes": S, "chunk_symbols": C, "window": W, "min_match": MIN,
                   "input_bytes": n},
        "ratio": round(n / size, 4),
        "stream_bytes": size,
        "decompress_GBps": round(dec_gbps, 3) if dec_gbps else None,
        "kernel_avg_ms": kernel_ms,
        "hbm_frac_whole_step": round((n + size) / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
        "roofline": {"bound": "alu",
                     "kernel": "encode_kernel<4,4> (match search, parse, look-back, record write-out)",
                     "achieved": round(achieved, 4), "peak": round(ALU_PEAK_TCMP, 3),
                     "unit": "Tcmp/s", "frac": round(achieved / ALU_PEAK_TCMP, 4),
                     "achieved_counts": "algorithmic compares: every position against each of "
                                        "its min(j, W) window offsets",
                     "compares_per_launch": compares,
                     "executed_hit_compares_per_launch": executed,
                     "executed_frac": round(executed / (enc_avg_ms / 1e3) / 1e12 / ALU_PEAK_TCMP, 4),
                     "traffic": traffic,
                     "hbm_algorithmic_bytes_per_launch": n + size,
                     "hbm_frac_encode": round((n + size) / (enc_avg_ms / 1e3) / 1e9 / HBM_PEAK_GBPS, 4)},
        "step_traffic": step_traffic,
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(x, S, C, W, MIN, args.cpu_sample_mib << 20)
        th = cpu_threads()
        if th > 1:
            result["cpu_baseline_all_cores"] = cpu_baseline(x, S, C, W, MIN, n, threads=th)
    if args.profile_copy:
        ref = torch.empty_like(d_in)
        ref.copy_(d_in)
        torch.cuda.synchronize()
    if not args.no_extras:
        # the other workloads the metric names, each as one key of this line
        del comp, d_in
        torch.cuda.empty_cache()
        print("[bench] config 0: 1 MiB uint16 codes", file=sys.stderr, flush=True)
        result["small"] = small_leg(args)
        kind, seed, S2, MIN2 = DENSE_INPUTS[1]
        result["dense_u16"] = dense_leg(args, kind, seed, S2, MIN2, 256 << 20)
        if not args.no_batch:
            print("[bench] config 3: batch of 4096 buffers", file=sys.stderr, flush=True)
            bargs = argparse.Namespace(**vars(args))
            bargs.steps = 1
            result["batch"] = batch_leg(bargs)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
