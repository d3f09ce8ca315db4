"""Adaptive symbol width and window (gpuLZ section 3.2.3).

The paper picks the matching granularity per dataset:
  * matching starts with multi-byte symbols (S = the element width of the
    data) and a window enlarged S times, since multi-byte matching runs
    about S times faster than single-byte matching;
  * if the average compression ratio over the dataset's fields stays below
    1.5, it switches back to single-byte matching (S = 1), because byte-level
    repeats are then lost by multi-byte matching;
  * the user picks a level 1-4, the base window 32 / 64 / 128 / 255 symbols:
    higher levels compress more and run slower.
The enlarged window is capped at 256, the largest window the stream allows.
Chunk sizes and waves per chunk come from the per-width defaults (which the
autotuner may have set).
"""
from __future__ import annotations

from dataclasses import dataclass

from . import gpulz

LEVEL_WINDOWS = {1: 32, 2: 64, 3: 128, 4: 255}
RATIO_THRESHOLD = 1.5
MAX_WINDOW = 256


@dataclass
class Plan:
    symbol_bytes: int
    chunk_symbols: int
    window: int
    min_match: int
    multi_byte_ratio: float | None   # average ratio measured with S = element width


def multi_byte_window(element_bytes: int, level: int) -> int:
    return min(MAX_WINDOW, element_bytes * LEVEL_WINDOWS[level])


def decide(element_bytes: int, level: int, multi_byte_ratio: float | None, min_match: int = 2,
           chunk_for=None, threshold: float = RATIO_THRESHOLD) -> Plan:
    """The rule alone: `multi_byte_ratio` is the average ratio of the fields
    compressed with S = element_bytes and the enlarged window (None when the
    elements are single bytes)."""
    if level not in LEVEL_WINDOWS:
        raise ValueError("level must be 1, 2, 3 or 4")
    chunk_for = chunk_for or (lambda S: gpulz.gpulz_default_params(S)[0])
    if element_bytes == 1 or (multi_byte_ratio is not None and multi_byte_ratio < threshold):
        return Plan(1, chunk_for(1), LEVEL_WINDOWS[level], min_match, multi_byte_ratio)
    return Plan(element_bytes, chunk_for(element_bytes), multi_byte_window(element_bytes, level),
                min_match, multi_byte_ratio)


def _plan_with_streams(fields, element_bytes: int, level: int, min_match: int,
                       threshold: float):
    """The plan, and the multi-byte streams measured for it (None for
    single-byte elements)."""
    if element_bytes not in (1, 2, 4, 8):
        raise ValueError("element_bytes must be 1, 2, 4 or 8")
    if element_bytes == 1:
        return decide(1, level, None, min_match), None
    S = element_bytes
    C = gpulz.gpulz_default_params(S)[0]
    W = multi_byte_window(S, level)
    ratios, streams = [], []
    for f in fields:
        n = f.numel()
        s = gpulz.compress(f, S, C, W, min_match)
        streams.append(s)
        if n:
            ratios.append(n / s.numel())
    avg = sum(ratios) / len(ratios) if ratios else None
    return decide(S, level, avg, min_match, threshold=threshold), streams


def plan(fields, element_bytes: int, level: int = 3, min_match: int = 2,
         threshold: float = RATIO_THRESHOLD) -> Plan:
    """Measure the average multi-byte ratio over `fields` (uint8 device
    tensors of one dataset) and apply the rule."""
    return _plan_with_streams(fields, element_bytes, level, min_match, threshold)[0]


def compress(fields, element_bytes: int, level: int = 3, min_match: int = 2):
    """Compress every field with the plan chosen for the dataset; returns
    (plan, [streams]). When the plan keeps the multi-byte width, the streams
    measured for the decision are the result (same parameters)."""
    p, measured = _plan_with_streams(fields, element_bytes, level, min_match, RATIO_THRESHOLD)
    if measured is not None and p.symbol_bytes == element_bytes:
        return p, measured
    return p, [gpulz.compress(f, p.symbol_bytes, p.chunk_symbols, p.window, p.min_match)
               for f in fields]
