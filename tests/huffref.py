"""Independent pure-Python reference for the Huffman stage, used to pin the
C oracle. Written separately and in another style: the tree is built with a
binary heap, codes are assigned by walking symbols in (length, symbol) order
(the sequential form of canonical coding), and bits are handled as strings
of '0'/'1'. Slow; small inputs only.

Definitions: Huffman's algorithm (Huffman, 1952) with ties broken by
(weight, node index), leaves indexed by symbol before internal nodes in
creation order; lengths limited to 15 by halving weights (rounding up) and
rebuilding; canonical codes (RFC 1951 section 3.2.2); the chunked stream
layout described in the oracle's header.
"""
from __future__ import annotations

import heapq
import struct

CHUNK, SUB, LIMIT, PRE = 4096, 128, 15, 192


def lengths(freq, limit: int = LIMIT):
    freq = list(freq) + [0] * (256 - len(freq))
    w = {s: f for s, f in enumerate(freq) if f}
    if not w:
        return [0] * 256
    if len(w) == 1:
        return [1 if f else 0 for f in freq]
    while True:
        heap = [(f, s) for s, f in w.items()]
        heapq.heapify(heap)
        children = {}
        nxt = 256
        while len(heap) > 1:
            wa, a = heapq.heappop(heap)
            wb, b = heapq.heappop(heap)
            children[nxt] = (a, b)
            heapq.heappush(heap, (wa + wb, nxt))
            nxt += 1
        depth = {}
        stack = [(heap[0][1], 0)]
        while stack:
            node, d = stack.pop()
            if node in children:
                stack += [(c, d + 1) for c in children[node]]
            else:
                depth[node] = d
        if max(depth.values()) <= limit:
            return [depth.get(s, 0) for s in range(256)]
        w = {s: (f + 1) // 2 for s, f in w.items()}


def codes(lens):
    """{symbol: bit string}."""
    order = sorted((l, s) for s, l in enumerate(lens) if l)
    out, code, prev = {}, 0, order[0][0] if order else 0
    for l, s in order:
        code <<= l - prev
        out[s] = format(code, f"0{l}b")
        code += 1
        prev = l
    return out


def _words(bits: str) -> bytes:
    bits += "0" * (-len(bits) % 32)
    return b"".join(struct.pack("<I", int(bits[k:k + 32], 2)) for k in range(0, len(bits), 32))


def compress(data: bytes, lens=None) -> bytes:
    """The stream of `data`; `lens` overrides the code lengths (to build
    streams the encoder would never write, for decoder tests)."""
    n = len(data)
    freq = [0] * 256
    for b in data:
        freq[b] += 1
    if lens is None:
        lens = lengths(freq)
    cb = codes(lens)
    N = -(-n // CHUNK)
    table, recs = b"", b""
    for i in range(N):
        chunk = data[i * CHUNK:(i + 1) * CHUNK]
        offs, bits = [], ""
        for j, b in enumerate(chunk):
            if j % SUB == 0:
                offs.append(len(bits))
            bits += cb[b]
        off = b"".join(struct.pack("<H", o) for o in offs)
        off += bytes(-len(off) % 4)
        table += struct.pack("<I", len(bits))
        recs += off + _words(bits)
    total = PRE + len(table) + len(recs)
    hdr = b"GLH1" + struct.pack("<HBBIIQQQ", 1, LIMIT, 0, CHUNK, SUB, n, N, total) + bytes(24)
    nib = bytes(lens[2 * k] | lens[2 * k + 1] << 4 for k in range(128))
    return hdr + nib + table + recs


def decompress(stream: bytes) -> bytes:
    """Decodes a valid stream (no validation beyond what decoding needs)."""
    n, N = struct.unpack_from("<QQ", stream, 16)
    lens = [stream[64 + s // 2] >> (4 * (s & 1)) & 15 for s in range(256)]
    inv = {c: s for s, c in codes(lens).items()}
    bits_tab = struct.unpack_from(f"<{N}I", stream, PRE)
    pos = PRE + 4 * N
    out = bytearray()
    for i in range(N):
        c = min(CHUNK, n - i * CHUNK)
        nsub = -(-c // SUB)
        pos += (2 * nsub + 3) // 4 * 4
        nwords = -(-bits_tab[i] // 32)
        words = struct.unpack_from(f"<{nwords}I", stream, pos)
        pos += 4 * nwords
        bits = "".join(format(w, "032b") for w in words)[:bits_tab[i]]
        cur = ""
        for bit in bits:
            cur += bit
            if cur in inv:
                out.append(inv[cur])
                cur = ""
    return bytes(out)


def cost(freq, lens) -> int:
    return sum(f * l for f, l in zip(freq, lens))


def optimal_cost(freq) -> int:
    """The least total code bits of any prefix code (no length limit): the
    sum of the weights of all joins in a Huffman tree, which does not depend
    on how ties are broken."""
    h = [f for f in freq if f]
    if len(h) == 1:
        return h[0]
    heapq.heapify(h)
    total = 0
    while len(h) > 1:
        a, b = heapq.heappop(h), heapq.heappop(h)
        total += a + b
        heapq.heappush(h, a + b)
    return total
