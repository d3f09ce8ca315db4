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
of block k - 1. Pageable input is staged into pinned buffers by a pool of
host threads (a pinned torch input is copied from directly); the output
stream is allocated pinned, so the device-to-host copies land in their final
places with no second host copy.
Decompression streams the same way: each block of chunks becomes a small
standalone stream (its own header, its slice of the table and its records)
that is decoded on the device and copied into the pinned output.

The stream format stays in the library: headers are written and read by
gpulz_write_header / gpulz_read_header, table and record positions come from
gpulz_table_offset, and the record offsets of a stream from its table by the
device scan gpulz_record_offsets.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import gpulz

_COPY_PIECE = 8 << 20


def default_block_bytes(fraction: float = 0.30) -> int:
    import torch
    return int(torch.cuda.get_device_properties(0).total_memory * fraction)


def default_threads() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


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


def _host_bytes(x):
    """(uint8 numpy view, pinned torch uint8 view or None) of a host array or
    CPU tensor."""
    import torch
    if isinstance(x, torch.Tensor):
        if x.device.type != "cpu":
            raise ValueError("host streaming takes a host array or CPU tensor")
        t = x.contiguous().view(-1).view(torch.uint8)
        return t.numpy(), (t if t.is_pinned() else None)
    return np.ascontiguousarray(x).view(np.uint8).reshape(-1), None


class _Copier:
    """Host memcpy split over a thread pool (numpy releases the GIL while it
    copies)."""

    def __init__(self, threads: int):
        self.pool = ThreadPoolExecutor(threads) if threads > 1 else None

    def __call__(self, dst: np.ndarray, src: np.ndarray) -> None:
        n = src.size
        if self.pool is None or n <= _COPY_PIECE:
            dst[:n] = src
            return
        futs = [self.pool.submit(np.copyto, dst[a:min(n, a + _COPY_PIECE)],
                                 src[a:min(n, a + _COPY_PIECE)])
                for a in range(0, n, _COPY_PIECE)]
        for f in futs:
            f.result()

    def close(self):
        if self.pool is not None:
            self.pool.shutdown()


def compress_host(x, S: int, C: int, W: int, MIN: int, policy: int = 0,
                  block_bytes: int | None = None, threads: int | None = None) -> np.ndarray:
    """Compress a host array or CPU tensor (its bytes) into one stream,
    returned as a uint8 numpy array over pinned host memory."""
    import torch
    src, src_pinned = _host_bytes(x)
    n = src.size
    block_bytes = block_bytes or default_block_bytes()
    blocks = block_plan(n, S, C, block_bytes)
    N = -(-(n // S) // C)
    cap = gpulz.gpulz_compress_bound(n, S, C, MIN)
    if cap == 0:
        raise gpulz.GpulzError(gpulz.GPULZ_ERR_INVALID_ARG, "gpulz_compress_bound")
    out_t = torch.empty(cap, dtype=torch.uint8, pin_memory=True)
    bmax = max(1, max(b for _, b, _, _ in blocks))
    dev = [torch.empty(bmax, dtype=torch.uint8, device="cuda") for _ in range(2)]
    pin = None if src_pinned is not None else \
        [torch.empty(bmax, dtype=torch.uint8, pin_memory=True) for _ in range(2)]
    comps = [gpulz.Compressor(bmax, S, C, W, MIN, policy=policy) for _ in range(2)]
    copy_in, work, copy_out = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    loaded = [torch.cuda.Event() for _ in range(2)]   # host-to-device copy of the block done
    done = [torch.cuda.Event() for _ in range(2)]     # its compression done
    copied = [torch.cuda.Event() for _ in range(2)]   # its stream copied back
    used = [False, False]
    copier = _Copier(threads or default_threads())
    at = gpulz.gpulz_table_offset
    rec_off = at(N)  # the first record of the assembled stream

    def stage(k):
        off, nb, _, _ = blocks[k]
        j = k % 2
        if used[j]:
            loaded[j].synchronize()            # the pinned staging buffer is free again
            copy_in.wait_event(done[j])        # the device buffer is free again
        if pin is None:
            host = src_pinned[off:off + nb]
        else:
            copier(pin[j].numpy(), src[off:off + nb])
            host = pin[j][:nb]
        with torch.cuda.stream(copy_in):
            dev[j][:nb].copy_(host, non_blocking=True)
            loaded[j].record(copy_in)

    def compress(k):
        _, nb, _, _ = blocks[k]
        j = k % 2
        work.wait_event(loaded[j])
        if used[j]:
            work.wait_event(copied[j])         # the previous stream in this buffer is copied out
        comps[j].compress_async(dev[j][:nb], nb, stream=work)
        done[j].record(work)
        used[j] = True

    def drain(k):
        nonlocal rec_off
        j = k % 2
        _, _, c0, nc = blocks[k]
        done[j].synchronize()
        size, status = comps[j].result()
        if status != gpulz.GPULZ_OK:
            raise gpulz.GpulzError(status, "block compress")
        # the block's stream: header, its nc table entries, its records
        rec = size - at(nc)
        body = comps[j].out
        with torch.cuda.stream(copy_out):
            out_t[at(c0):at(c0 + nc)].copy_(body[at(0):at(nc)], non_blocking=True)
            out_t[rec_off:rec_off + rec].copy_(body[at(nc):size], non_blocking=True)
            copied[j].record(copy_out)
        rec_off += rec

    try:
        stage(0)
        for k in range(len(blocks)):
            compress(k)
            if k + 1 < len(blocks):
                stage(k + 1)
            drain(k)
        copy_out.synchronize()
    finally:
        copier.close()
        torch.cuda.synchronize()
    tail = src[n - n % S:].tobytes()
    out = out_t.numpy()
    hdr = gpulz.gpulz_write_header(n, S, C, W, MIN, policy, rec_off, tail)
    out[:at(0)] = np.frombuffer(hdr, dtype=np.uint8)
    return out[:rec_off]


def decompress_host(stream, block_bytes: int | None = None,
                    threads: int | None = None) -> np.ndarray:
    """Decompress a host stream block by block; returns the bytes as a uint8
    numpy array over pinned host memory."""
    import torch
    s, _ = _host_bytes(stream)
    at = gpulz.gpulz_table_offset
    info = gpulz.gpulz_read_header(s[:at(0)].tobytes())
    if info.stream_bytes != s.size:
        raise gpulz.GpulzError(gpulz.GPULZ_ERR_CORRUPT, "stream size")
    n, S, C, W, MIN = (info.nbytes, info.symbol_bytes, info.chunk_symbols, info.window,
                       info.min_match)
    N, policy = info.chunks, info.match_policy
    tail = bytes(info.tail[:info.tail_bytes])
    # record offsets from the table, scanned on the device
    table = torch.from_numpy(s[at(0):at(N)].copy()).cuda()
    offs = torch.empty(N + 1, dtype=torch.int64, device="cuda")
    gpulz._check(gpulz.gpulz_record_offsets(table.data_ptr(), N, offs.data_ptr(),
                                            gpulz._stream_handle(torch.cuda.current_stream())),
                 "gpulz_record_offsets")
    rec_start = at(N) + offs.cpu().numpy()
    del table, offs
    if int(rec_start[-1]) != s.size:
        raise gpulz.GpulzError(gpulz.GPULZ_ERR_CORRUPT, "record sizes")
    block_bytes = block_bytes or default_block_bytes()
    blocks = block_plan(n, S, C, block_bytes)
    subs = []
    for off, nb, c0, nc in blocks:
        last = c0 + nc == N
        nb_block = nb if last else nc * C * S
        tot = at(nc) + int(rec_start[c0 + nc] - rec_start[c0])
        hdr = gpulz.gpulz_write_header(nb_block, S, C, W, MIN, policy, tot, tail if last else b"")
        subs.append((off, nb_block, c0, nc, tot, hdr))
    smax = max(1, max(t for *_, t, _ in subs))
    bmax = max(1, max(b for _, b, *_ in subs))
    out_t = torch.empty(max(n, 1), dtype=torch.uint8, pin_memory=True)
    pin = [torch.empty(smax, dtype=torch.uint8, pin_memory=True) for _ in range(2)]
    dev_in = [torch.empty(smax, dtype=torch.uint8, device="cuda") for _ in range(2)]
    dev_out = [torch.empty(bmax, dtype=torch.uint8, device="cuda") for _ in range(2)]
    ws_bytes = gpulz.gpulz_decompress_workspace_size(smax)
    ws = [torch.empty(ws_bytes, dtype=torch.uint8, device="cuda") for _ in range(2)]
    meta = torch.zeros(len(subs), 2, dtype=torch.int64, device="cuda")
    copy_in, work, copy_out = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    loaded = [torch.cuda.Event() for _ in range(2)]
    decoded = [torch.cuda.Event() for _ in range(2)]
    copied = [torch.cuda.Event() for _ in range(2)]
    used = [False, False]
    copier = _Copier(threads or default_threads())
    try:
        for k, (off, nb, c0, nc, tot, hdr) in enumerate(subs):
            j = k % 2
            if used[j]:
                loaded[j].synchronize()
                copy_in.wait_event(decoded[j])
            p = pin[j].numpy()
            p[:at(0)] = np.frombuffer(hdr, dtype=np.uint8)
            p[at(0):at(nc)] = s[at(c0):at(c0 + nc)]
            copier(p[at(nc):tot], s[rec_start[c0]:rec_start[c0 + nc]])
            with torch.cuda.stream(copy_in):
                dev_in[j][:tot].copy_(pin[j][:tot], non_blocking=True)
                loaded[j].record(copy_in)
            work.wait_event(loaded[j])
            if used[j]:
                work.wait_event(copied[j])
            st = gpulz.gpulz_decompress(dev_in[j].data_ptr(), tot, dev_out[j].data_ptr(), nb,
                                        meta[k].data_ptr(), meta[k].data_ptr() + 8,
                                        ws[j].data_ptr(), ws_bytes, gpulz._stream_handle(work))
            gpulz._check(st, "gpulz_decompress")
            decoded[j].record(work)
            with torch.cuda.stream(copy_out):
                copy_out.wait_event(decoded[j])
                out_t[off:off + nb].copy_(dev_out[j][:nb], non_blocking=True)
                copied[j].record(copy_out)
            used[j] = True
        copy_out.synchronize()
    finally:
        copier.close()
        torch.cuda.synchronize()
    m = meta.cpu().numpy()
    for k, (_, nb, *_rest) in enumerate(subs):
        status = int(m[k, 1]) & 0xFFFFFFFF
        if status != gpulz.GPULZ_OK:
            raise gpulz.GpulzError(status, f"block {k} decompress")
        if int(m[k, 0]) != nb:
            raise gpulz.GpulzError(gpulz.GPULZ_ERR_CORRUPT, f"block {k} size")
    return out_t.numpy()[:n]
