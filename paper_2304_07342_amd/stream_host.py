"""Host-resident inputs streamed through the GPU in data blocks (gpuLZ
section 3.3.1: inputs larger than device memory are split into blocks, 30%
of device memory by default, each compressed by its own kernel launches).

Blocks are cut at chunk boundaries, and chunks are independent, so block k's
table entries and records are exactly the ones the whole input would get:
they are copied straight to their final places in one output stream, whose
header is written last. The result is byte-identical to compressing the
whole input at once.

Pipeline (two device buffer sets, three streams): the host-to-device copy of
block k + 1 overlaps the compression of block k and the device-to-host copies
of block k - 1; pinned host staging keeps the copies asynchronous.
Decompression streams the same way: each block of chunks becomes a small
standalone stream (its own header, its slice of the table and its records)
that is decoded on the device and copied back.
"""
from __future__ import annotations

import struct

import numpy as np

from . import gpulz

HEADER = 64


def default_block_bytes(fraction: float = 0.30) -> int:
    import torch
    return int(torch.cuda.get_device_properties(0).total_memory * fraction)


def block_plan(nbytes: int, S: int, C: int, block_bytes: int):
    """[(byte offset, bytes, first chunk, chunks)] with every block but the
    last a whole number of chunks; the last one also carries the n mod S
    tail bytes."""
    chunk_bytes = C * S
    per = max(1, block_bytes // chunk_bytes)
    m = nbytes // S
    N = -(-m // C)
    out = []
    for c0 in range(0, N, per):
        c1 = min(N, c0 + per)
        off = c0 * chunk_bytes
        end = nbytes if c1 == N else c1 * chunk_bytes
        out.append((off, end - off, c0, c1 - c0))
    if not out:
        out.append((0, nbytes, 0, 0))
    return out


def header(n: int, S: int, C: int, W: int, MIN: int, policy: int, N: int, total: int,
           tail: bytes) -> bytes:
    h = b"GLZ1" + struct.pack("<HBBIHBBQQQB", 1, S, policy, C, W, MIN, 255, n, N, total,
                              len(tail))
    return h + bytes(7) + tail + bytes(8 - len(tail)) + bytes(8)


def compress_host(x: np.ndarray, S: int, C: int, W: int, MIN: int, policy: int = 0,
                  block_bytes: int | None = None) -> np.ndarray:
    """Compress a host array (any dtype; its bytes) into one stream (a host
    uint8 array)."""
    import torch
    src = np.ascontiguousarray(x).view(np.uint8).reshape(-1)
    n = src.size
    block_bytes = block_bytes or default_block_bytes()
    blocks = block_plan(n, S, C, block_bytes)
    N = -(-(n // S) // C)
    cap = gpulz.gpulz_compress_bound(n, S, C, MIN)
    out = np.empty(cap, dtype=np.uint8)
    bmax = max(b for _, b, _, _ in blocks)
    dev = [torch.empty(max(bmax, 1), dtype=torch.uint8, device="cuda") for _ in range(2)]
    pin = [torch.empty(max(bmax, 1), dtype=torch.uint8).pin_memory() for _ in range(2)]
    comps = [gpulz.Compressor(max(bmax, 1), S, C, W, MIN, policy=policy) for _ in range(2)]
    copy_in, work, copy_out = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    loaded = [torch.cuda.Event() for _ in range(2)]
    done = [torch.cuda.Event() for _ in range(2)]
    freed = [torch.cuda.Event() for _ in range(2)]
    pend = []
    rec_off = HEADER + 8 * N

    def stage(k):
        off, nb, _, _ = blocks[k]
        j = k % 2
        freed[j].synchronize()  # the pinned buffer and device buffer are free again
        pin[j][:nb].numpy()[:] = src[off:off + nb]
        with torch.cuda.stream(copy_in):
            dev[j][:nb].copy_(pin[j][:nb], non_blocking=True)
            loaded[j].record(copy_in)

    def drain(k):
        nonlocal rec_off
        j = k % 2
        _, nb, c0, nc = blocks[k]
        done[j].synchronize()
        size, status = comps[j].result()
        if status != gpulz.GPULZ_OK:
            raise gpulz.GpulzError(status, "block compress")
        with torch.cuda.stream(copy_out):
            body = comps[j].out[HEADER:size].cpu()
            freed[j].record(copy_out)
        b = body.numpy()
        out[HEADER + 8 * c0:HEADER + 8 * (c0 + nc)] = b[:8 * nc]
        rec = size - HEADER - 8 * nc
        out[rec_off:rec_off + rec] = b[8 * nc:]
        rec_off += rec

    for j in range(2):
        freed[j].record(torch.cuda.current_stream())
    if blocks:
        stage(0)
    for k in range(len(blocks)):
        j = k % 2
        _, nb, _, _ = blocks[k]
        with torch.cuda.stream(work):
            work.wait_event(loaded[j])
            comps[j].compress_async(dev[j][:nb], nb, stream=work)
            done[j].record(work)
        if k + 1 < len(blocks):
            if pend:
                drain(pend.pop(0))
            stage(k + 1)
        pend.append(k)
    while pend:
        drain(pend.pop(0))
    tail = src[n - n % S:].tobytes()
    out[:HEADER] = np.frombuffer(header(n, S, C, W, MIN, policy, N, rec_off, tail), dtype=np.uint8)
    return out[:rec_off]


def decompress_host(stream: np.ndarray, block_bytes: int | None = None) -> np.ndarray:
    """Decompress a host stream block by block; returns the host bytes."""
    import torch
    s = np.ascontiguousarray(stream).view(np.uint8).reshape(-1)
    n, S, total = gpulz.gpulz_peek_header(s[:HEADER].tobytes())
    if total != s.size:
        raise gpulz.GpulzError(gpulz.GPULZ_ERR_CORRUPT, "stream size")
    policy = int(s[7])
    C, W = struct.unpack_from("<IH", s, 8)
    MIN = int(s[14])
    N = int(struct.unpack_from("<Q", s, 24)[0])
    r = int(s[40])
    table = s[HEADER:HEADER + 8 * N].view(np.uint32).reshape(N, 2).astype(np.int64)
    rec_start = HEADER + 8 * N + np.concatenate([[0], np.cumsum(table.sum(axis=1))])
    block_bytes = block_bytes or default_block_bytes()
    out = np.empty(n, dtype=np.uint8)
    for off, nb, c0, nc in block_plan(n, S, C, block_bytes):
        tail = s[48:48 + r].tobytes() if c0 + nc == N else b""
        nb_block = nb if c0 + nc == N else nc * C * S
        recs = s[rec_start[c0]:rec_start[c0 + nc]]
        tot = HEADER + 8 * nc + recs.size
        sub = np.concatenate([
            np.frombuffer(header(nb_block, S, C, W, MIN, policy, nc, tot, tail), dtype=np.uint8),
            s[HEADER + 8 * c0:HEADER + 8 * (c0 + nc)], recs])
        d = gpulz.decompress(torch.from_numpy(sub).cuda(), nb_block)
        out[off:off + nb_block] = d.cpu().numpy()
    return out
