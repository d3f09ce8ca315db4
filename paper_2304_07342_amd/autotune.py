"""Autotuner for the per-width parameters (chunk size, window, waves per chunk).

The paper studies how chunk size C, window W and symbol width S trade
compression ratio against throughput (section 4.2, Tables 1 and 2) and lets
the user pick a window level (section 3.2.3). This tuner measures, for each
symbol width, every candidate (C, W, waves per chunk) on a sample of the
caller's data already on the device, and picks the fastest candidate whose
ratio is within `ratio_tol` of the best ratio among the candidates. The
choice is installed with gpulz_set_default_params (so the batch entry points
use it for zero parameters) and can be cached as JSON.

Timing uses HIP events around gpulz_compress on the current stream.
"""
from __future__ import annotations

import json
import os

from . import gpulz

CHUNKS = (1024, 2048, 4096, 8192)
WINDOWS = (32, 64, 128, 256)
WAVES = (1, 4)
MAX_CHUNK_BYTES = 48 * 1024


def default_cache_path() -> str:
    return os.environ.get("GPULZ_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "gpulz", "autotune.json"))


def candidates(S: int, chunks=CHUNKS, windows=WINDOWS, waves=WAVES):
    return [(C, W, w) for C in chunks if C * S <= MAX_CHUNK_BYTES for W in windows for w in waves]


def measure(sample, S: int, C: int, W: int, min_match: int, waves: int, reps: int = 3):
    """(median ms, ratio) of gpulz_compress on `sample` with these parameters."""
    import torch
    saved = gpulz.gpulz_default_params(S)
    try:
        gpulz.gpulz_set_default_params(S, saved[0], saved[1], saved[2], waves)
        comp = gpulz.Compressor(sample.numel(), S, C, W, min_match, device=sample.device)
        comp.compress_async(sample)  # warm-up
        size, status = comp.result()
        if status != gpulz.GPULZ_OK:
            raise gpulz.GpulzError(status, "autotune measurement")
        times = []
        stream = torch.cuda.current_stream()
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            comp.compress_async(sample)
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        times.sort()
        return times[len(times) // 2], sample.numel() / size
    finally:
        gpulz.gpulz_set_default_params(S, *saved)


def choose(results, ratio_tol: float):
    """results: [(C, W, waves, ms, ratio)] -> the fastest within ratio_tol of
    the best ratio."""
    best = max(r[4] for r in results)
    ok = [r for r in results if r[4] >= best * (1.0 - ratio_tol)]
    return min(ok, key=lambda r: r[3])


def tune_width(sample, S: int, min_match: int = 2, ratio_tol: float = 0.02, reps: int = 3,
               cands=None, log=None):
    results = []
    for C, W, w in (cands or candidates(S)):
        ms, ratio = measure(sample, S, C, W, min_match, w, reps)
        results.append((C, W, w, ms, ratio))
        if log:
            log(f"[autotune] S={S} C={C} W={W} waves={w}: {ms:.3f} ms, ratio {ratio:.4f}")
    C, W, w, ms, ratio = choose(results, ratio_tol)
    return {"chunk_symbols": C, "window": W, "min_match": min_match, "waves_per_chunk": w,
            "ms": ms, "ratio": ratio, "GBps": sample.numel() / (ms / 1e3) / 1e9,
            "measurements": [list(r) for r in results]}


def tune(samples, min_match: int = 2, ratio_tol: float = 0.02, reps: int = 3, cache_path=None,
         log=None):
    """samples: {S: uint8 device tensor}. Returns {S: choice}; installs the
    choices as defaults and, if cache_path is given, writes them as JSON."""
    import torch
    out = {}
    for S, sample in sorted(samples.items()):
        out[S] = tune_width(sample, S, min_match, ratio_tol, reps, log=log)
    apply(out)
    if cache_path:
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump({"device": torch.cuda.get_device_name(), "ratio_tol": ratio_tol,
                       "widths": {str(S): v for S, v in out.items()}}, f, indent=1)
    return out


def apply(choices) -> None:
    for S, c in choices.items():
        gpulz.gpulz_set_default_params(int(S), c["chunk_symbols"], c["window"], c["min_match"],
                                       c["waves_per_chunk"])


def load(cache_path=None):
    """Install cached choices (if the cache exists); returns them or None."""
    path = cache_path or default_cache_path()
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    choices = {int(S): v for S, v in data["widths"].items()}
    apply(choices)
    return choices
