"""Independent pure-Python reference used to pin the C oracle.

Written separately from the oracle, in a different style: matches are found
by enumerating every (offset, length) pair and comparing list slices, and
the stream is assembled with ``struct``. It is slow (only for tiny inputs)
and shares nothing with the oracle or the GPU path.

Definitions it follows (gpuLZ, Zhang et al., ICS'23):
  * section 2.2, basic LZSS steps: greedy longest match from the coding
    position, pointer or literal, flag array;
  * section 3.2.3: symbols of S bytes;
  * section 3.3.1: independent chunks, no match across chunk boundaries;
  * section 3.3.2: a match is encoded iff its length reaches the minimum
    encode length, and its length never exceeds its offset;
  * one-byte pointer fields, so lengths are at most 255.
"""
from __future__ import annotations

import struct

HEADER = 64


def symbols(data: bytes, S: int):
    m = len(data) // S
    return [data[j * S:(j + 1) * S] for j in range(m)]


def brute_best(chunk, p: int, W: int):
    """Every (d, L) with the slice chunk[p:p+L] equal to chunk[p-d:p-d+L]
    is enumerated; the admissible ones (L <= d, L <= 255, inside the chunk,
    d within the window and the chunk) are kept; the longest wins and ties
    go to the largest d."""
    best = (0, 0)
    for d in range(1, W + 1):
        if p - d < 0:
            break
        for L in range(1, min(d, 255, len(chunk) - p) + 1):
            if chunk[p:p + L] == chunk[p - d:p - d + L]:
                if (L, d) > best:
                    best = (L, d)
    return best


def scan_best(chunk, p: int, W: int):
    """Match policy 1, the paper's single pass over the window (section
    3.3.2, matching steps 1-4): walk the window once from its oldest slot;
    a run of equal symbols (window slot vs. look-ahead) is a candidate that
    wins only if strictly longer; after a failed symbol the look-ahead starts
    over at p and the walk continues at the next slot. The run still open
    when the walk stops counts too; runs stop at 255 symbols."""
    best = (0, 0)
    run, run_from = 0, 0
    for w in range(max(0, p - W), p):
        if p + run >= len(chunk):
            break
        if run < 255 and chunk[p + run] == chunk[w]:
            if run == 0:
                run_from = w
            run += 1
            continue
        if run > best[0]:
            best = (run, p - run_from)
        run = 0
    if run > best[0]:
        best = (run, p - run_from)
    return best


def parse(chunk, W: int, MIN: int, policy: int = 0):
    """Greedy parse: list of (L, d) with L = 0 meaning a literal."""
    toks = []
    p = 0
    while p < len(chunk):
        L, d = brute_best(chunk, p, W) if policy == 0 else scan_best(chunk, p, W)
        if L >= MIN:
            toks.append((L, d))
            p += L
        else:
            toks.append((0, 0))
            p += 1
    return toks


def record(chunk, toks, S: int) -> tuple[bytes, int, int]:
    T = len(toks)
    flags = bytearray((T + 7) // 8)
    payload = bytearray()
    p = 0
    for t, (L, d) in enumerate(toks):
        if L:
            flags[t // 8] |= 1 << (t % 8)
            payload += bytes([L, d % 256])
            p += L
        else:
            payload += chunk[p]
            p += 1
    return bytes(flags) + bytes(payload), len(flags), len(payload)


def header(n: int, S: int, C: int, W: int, MIN: int, N: int, total: int, tail: bytes,
           policy: int = 0) -> bytes:
    h = b"GLZ1" + struct.pack("<HBBIHBBQQQB", 1, S, policy, C, W, MIN, 255, n, N, total,
                              len(tail))
    h += bytes(7) + tail + bytes(8 - len(tail)) + bytes(8)
    assert len(h) == HEADER
    return h


def compress(data: bytes, S: int, C: int, W: int, MIN: int, policy: int = 0) -> bytes:
    syms = symbols(data, S)
    m = len(syms)
    chunks = [syms[i:i + C] for i in range(0, m, C)]
    table = b""
    recs = b""
    for ch in chunks:
        rec, F, P = record(ch, parse(ch, W, MIN, policy), S)
        table += struct.pack("<II", F, P)
        recs += rec
    total = HEADER + len(table) + len(recs)
    tail = data[m * S:]
    return header(len(data), S, C, W, MIN, len(chunks), total, tail, policy) + table + recs


class Corrupt(Exception):
    pass


def tokens(stream: bytes):
    """Decode a stream into (params, per-chunk token lists); raise Corrupt on
    any rule violation. Tokens are (L, d) with L = 0 for a literal whose
    payload bytes are returned as d."""
    if len(stream) < HEADER or stream[:4] != b"GLZ1":
        raise Corrupt("magic")
    ver, S, pol, C, W, MIN, mx, n, N, total, r = struct.unpack_from("<HBBIHBBQQQB", stream, 4)
    if ver != 1 or pol not in (0, 1) or mx != 255 or S not in (1, 2, 4, 8):
        raise Corrupt("header field")
    if not (1 <= C <= 1 << 24 and 1 <= W <= 256 and 1 <= MIN <= 255):
        raise Corrupt("params")
    m = n // S
    if r != n % S or N != -(-m // C) or total != len(stream):
        raise Corrupt("sizes")
    if any(stream[41:48]) or any(stream[48 + r:64]):
        raise Corrupt("reserved")
    if HEADER + 8 * N > len(stream):
        raise Corrupt("table")
    table = [struct.unpack_from("<II", stream, HEADER + 8 * i) for i in range(N)]
    if HEADER + 8 * N + sum(F + P for F, P in table) != len(stream):
        raise Corrupt("table sum")
    pos = HEADER + 8 * N
    out_chunks = []
    for i, (F, P) in enumerate(table):
        c = min(C, m - i * C)
        flags = stream[pos:pos + F]
        pay = stream[pos + F:pos + F + P]
        q = 0
        u = 0
        t = 0
        toks = []
        while q < c:
            if t >= 8 * F:
                raise Corrupt("flags exhausted")
            if flags[t // 8] >> (t % 8) & 1:
                if u + 2 > P:
                    raise Corrupt("payload exhausted")
                L, O = pay[u], pay[u + 1] or 256
                u += 2
                if not (MIN <= L <= O <= W and O <= q and q + L <= c):
                    raise Corrupt("pointer range")
                toks.append((L, O))
                q += L
            else:
                if u + S > P:
                    raise Corrupt("payload exhausted")
                toks.append((0, bytes(pay[u:u + S])))
                u += S
                q += 1
            t += 1
        if -(-t // 8) != F or u != P:
            raise Corrupt("chunk sizes")
        for tt in range(t, 8 * F):
            if flags[tt // 8] >> (tt % 8) & 1:
                raise Corrupt("padding bit")
        out_chunks.append(toks)
        pos += F + P
    params = dict(n=n, S=S, C=C, W=W, MIN=MIN, N=N, tail=bytes(stream[48:48 + r]))
    return params, out_chunks


def decompress(stream: bytes) -> bytes:
    params, chunks = tokens(stream)
    S = params["S"]
    out = bytearray()
    for toks in chunks:
        syms = []
        for L, d in toks:
            if L == 0:
                syms.append(d)
            else:
                for _ in range(L):
                    syms.append(syms[len(syms) - d])
        out += b"".join(syms)
    return bytes(out) + params["tail"]
