"""Python binding for libgpulz.so (the HIP kernels behind a C ABI).

Argument marshalling only: every step of compression and decompression runs
in the library's HIP kernels. The raw functions carry the C names and take
integer device pointers; `compress` / `decompress` wrap them for torch
tensors on the current HIP stream. There is no CPU fallback: if the library
is missing, loading it raises.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgpulz.so")

GPULZ_OK = 0
GPULZ_ERR_INVALID_ARG = 1
GPULZ_ERR_OUT_OF_SPACE = 2
GPULZ_ERR_CORRUPT = 3
GPULZ_ERR_WORKSPACE = 4
GPULZ_ERR_HIP = 5
GPULZ_ERR_UNSUPPORTED = 6

# Every symbol the C header declares.
EXPORTS = (
    "gpulz_abi_version", "gpulz_status_string", "gpulz_compress_bound",
    "gpulz_compress_workspace_size", "gpulz_compress", "gpulz_compress_policy", "gpulz_peek_header",
    "gpulz_decompress_workspace_size", "gpulz_decompress", "gpulz_decompress_noalloc",
    "gpulz_default_params",
    "gpulz_set_default_params", "gpulz_compress_batch_workspace_size", "gpulz_compress_batch",
    "gpulz_decompress_batch_workspace_size", "gpulz_decompress_batch", "gpulz_profile_enable",
    "gpulz_profile_read", "gpulz_huff_compress_bound", "gpulz_huff_compress_workspace_size",
    "gpulz_huff_compress", "gpulz_huff_decompress_workspace_size", "gpulz_huff_decompress",
    "gpulz_table_offset", "gpulz_write_header", "gpulz_read_header", "gpulz_record_offsets",
)
KERNEL_NAMES = ("encode", "prep", "unused", "decode_prepare", "decode", "compress_batch",
                "decompress_batch", "huff_compress", "huff_decompress")


class Params(ctypes.Structure):
    """gpulz_params: per-width parameters (zero fields = library default)."""
    _fields_ = [("chunk_symbols", ctypes.c_uint32), ("window", ctypes.c_uint32),
                ("min_match", ctypes.c_uint32), ("waves_per_chunk", ctypes.c_uint32)]


ParamsArray4 = Params * 4


def params_array(by_width=None):
    """by_width: None, or {S: (chunk, window, min_match[, waves])} for any of
    S in 1, 2, 4, 8 (others default)."""
    arr = ParamsArray4()
    for S, p in (by_width or {}).items():
        w = {1: 0, 2: 1, 4: 2, 8: 3}[S]
        p = tuple(p) + (0,) * (4 - len(p))
        arr[w] = Params(*p)
    return arr


class StreamInfo(ctypes.Structure):
    """gpulz_stream_info: the fields of a stream header."""
    _fields_ = [("nbytes", ctypes.c_uint64), ("chunks", ctypes.c_uint64),
                ("stream_bytes", ctypes.c_uint64), ("symbol_bytes", ctypes.c_uint32),
                ("chunk_symbols", ctypes.c_uint32), ("window", ctypes.c_uint32),
                ("min_match", ctypes.c_uint32), ("match_policy", ctypes.c_uint32),
                ("tail_bytes", ctypes.c_uint32), ("tail", ctypes.c_uint8 * 8)]


class GpulzError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2304_07342_amd/build.py")
        # torch carries its own HIP runtime, which it loads by file name; the
        # library asks for the runtime by soname. Loading torch first makes
        # the library bind to that same runtime: loaded the other way round,
        # the process would hold two HIP runtimes and the library's would
        # find no device.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        u32, u64, i32, sz, vp = (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_size_t,
                                 ctypes.c_void_p)
        L.gpulz_abi_version.restype = u32
        L.gpulz_abi_version.argtypes = []
        L.gpulz_status_string.restype = ctypes.c_char_p
        L.gpulz_status_string.argtypes = [i32]
        L.gpulz_compress_bound.restype = u64
        L.gpulz_compress_bound.argtypes = [u64, u32, u32, u32]
        L.gpulz_compress_workspace_size.restype = ctypes.c_int
        L.gpulz_compress_workspace_size.argtypes = [u64, u32, u32, ctypes.POINTER(sz)]
        L.gpulz_compress.restype = ctypes.c_int
        L.gpulz_compress.argtypes = [vp, u64, u32, u32, u32, u32, vp, u64, vp, vp, vp, sz, vp]
        L.gpulz_compress_policy.restype = ctypes.c_int
        L.gpulz_compress_policy.argtypes = [vp, u64, u32, u32, u32, u32, u32, vp, u64, vp, vp, vp,
                                            sz, vp]
        L.gpulz_peek_header.restype = ctypes.c_int
        L.gpulz_peek_header.argtypes = [ctypes.c_char_p, sz, ctypes.POINTER(u64),
                                        ctypes.POINTER(u32), ctypes.POINTER(u64)]
        L.gpulz_decompress_workspace_size.restype = ctypes.c_int
        L.gpulz_decompress_workspace_size.argtypes = [u64, u64, ctypes.POINTER(sz)]
        L.gpulz_decompress.restype = ctypes.c_int
        L.gpulz_decompress.argtypes = [vp, u64, vp, u64, vp, vp, vp, sz, vp]
        L.gpulz_decompress_noalloc.restype = ctypes.c_int
        L.gpulz_decompress_noalloc.argtypes = [vp, u64, vp, u64, vp, vp, vp]
        L.gpulz_default_params.restype = ctypes.c_int
        L.gpulz_default_params.argtypes = [u32, ctypes.POINTER(Params)]
        L.gpulz_set_default_params.restype = ctypes.c_int
        L.gpulz_set_default_params.argtypes = [u32, ctypes.POINTER(Params)]
        L.gpulz_compress_batch_workspace_size.restype = ctypes.c_int
        L.gpulz_compress_batch_workspace_size.argtypes = [u64, u64, ctypes.POINTER(Params),
                                                         ctypes.POINTER(sz)]
        L.gpulz_compress_batch.restype = ctypes.c_int
        L.gpulz_compress_batch.argtypes = [u64, vp, vp, vp, ctypes.POINTER(Params), vp, vp, vp, vp,
                                           u64, vp, sz, vp]
        L.gpulz_decompress_batch_workspace_size.restype = ctypes.c_int
        L.gpulz_decompress_batch_workspace_size.argtypes = [u64, u64, ctypes.POINTER(sz)]
        L.gpulz_decompress_batch.restype = ctypes.c_int
        L.gpulz_decompress_batch.argtypes = [u64, vp, vp, vp, vp, vp, vp, u64, vp, sz, vp]
        L.gpulz_profile_enable.restype = ctypes.c_int
        L.gpulz_profile_enable.argtypes = [ctypes.c_int]
        L.gpulz_profile_read.restype = ctypes.c_int
        L.gpulz_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u64),
                                         ctypes.c_int]
        L.gpulz_huff_compress_bound.restype = u64
        L.gpulz_huff_compress_bound.argtypes = [u64]
        L.gpulz_huff_compress_workspace_size.restype = ctypes.c_int
        L.gpulz_huff_compress_workspace_size.argtypes = [u64, ctypes.POINTER(sz)]
        L.gpulz_huff_compress.restype = ctypes.c_int
        L.gpulz_huff_compress.argtypes = [vp, u64, vp, vp, u64, vp, vp, vp, sz, vp]
        L.gpulz_huff_decompress_workspace_size.restype = ctypes.c_int
        L.gpulz_huff_decompress_workspace_size.argtypes = [u64, ctypes.POINTER(sz)]
        L.gpulz_huff_decompress.restype = ctypes.c_int
        L.gpulz_huff_decompress.argtypes = [vp, u64, vp, u64, vp, vp, vp, sz, vp]
        L.gpulz_table_offset.restype = u64
        L.gpulz_table_offset.argtypes = [u64]
        L.gpulz_write_header.restype = ctypes.c_int
        L.gpulz_write_header.argtypes = [vp, u64, u32, u32, u32, u32, u32, u64, ctypes.c_char_p]
        L.gpulz_read_header.restype = ctypes.c_int
        L.gpulz_read_header.argtypes = [ctypes.c_char_p, sz, ctypes.POINTER(StreamInfo)]
        L.gpulz_record_offsets.restype = ctypes.c_int
        L.gpulz_record_offsets.argtypes = [vp, u64, vp, vp]
        _lib = L
    return _lib


# ---- raw C ABI (same names as include/gpulz.h) ------------------------------

def gpulz_abi_version() -> int:
    return lib().gpulz_abi_version()


def status_string(status: int) -> str:
    return lib().gpulz_status_string(status).decode()


gpulz_status_string = status_string


def gpulz_compress_bound(nbytes: int, symbol_bytes: int, chunk_symbols: int, min_match: int) -> int:
    return lib().gpulz_compress_bound(nbytes, symbol_bytes, chunk_symbols, min_match)


def gpulz_compress_workspace_size(nbytes: int, symbol_bytes: int, chunk_symbols: int) -> int:
    ws = ctypes.c_size_t(0)
    st = lib().gpulz_compress_workspace_size(nbytes, symbol_bytes, chunk_symbols, ctypes.byref(ws))
    if st != GPULZ_OK:
        raise GpulzError(st, "gpulz_compress_workspace_size")
    return ws.value


def gpulz_compress(d_in: int, nbytes: int, symbol_bytes: int, chunk_symbols: int, window: int,
                   min_match: int, d_out: int, out_capacity: int, d_out_bytes: int, d_status: int,
                   d_workspace: int, ws_bytes: int, stream: int = 0) -> int:
    return lib().gpulz_compress(d_in, nbytes, symbol_bytes, chunk_symbols, window, min_match, d_out,
                                out_capacity, d_out_bytes, d_status, d_workspace, ws_bytes, stream)


def gpulz_compress_policy(d_in: int, nbytes: int, symbol_bytes: int, chunk_symbols: int,
                          window: int, min_match: int, match_policy: int, d_out: int,
                          out_capacity: int, d_out_bytes: int, d_status: int, d_workspace: int,
                          ws_bytes: int, stream: int = 0) -> int:
    return lib().gpulz_compress_policy(d_in, nbytes, symbol_bytes, chunk_symbols, window,
                                       min_match, match_policy, d_out, out_capacity, d_out_bytes,
                                       d_status, d_workspace, ws_bytes, stream)


def gpulz_peek_header(header: bytes):
    n, s, total = ctypes.c_uint64(0), ctypes.c_uint32(0), ctypes.c_uint64(0)
    st = lib().gpulz_peek_header(bytes(header), len(header), ctypes.byref(n), ctypes.byref(s),
                                 ctypes.byref(total))
    if st != GPULZ_OK:
        raise GpulzError(st, "gpulz_peek_header")
    return n.value, s.value, total.value


def gpulz_table_offset(chunk: int) -> int:
    return lib().gpulz_table_offset(chunk)


def gpulz_write_header(nbytes: int, symbol_bytes: int, chunk_symbols: int, window: int,
                       min_match: int, match_policy: int, stream_bytes: int,
                       tail: bytes = b"") -> bytes:
    """The 64-byte header of a stream with these fields (host memory)."""
    buf = ctypes.create_string_buffer(64)
    st = lib().gpulz_write_header(buf, nbytes, symbol_bytes, chunk_symbols, window, min_match,
                                  match_policy, stream_bytes, bytes(tail) if tail else None)
    if st != GPULZ_OK:
        raise GpulzError(st, "gpulz_write_header")
    return buf.raw


def gpulz_read_header(header: bytes) -> StreamInfo:
    info = StreamInfo()
    st = lib().gpulz_read_header(bytes(header), len(header), ctypes.byref(info))
    if st != GPULZ_OK:
        raise GpulzError(st, "gpulz_read_header")
    return info


def gpulz_record_offsets(d_table: int, chunks: int, d_offsets: int, stream: int = 0) -> int:
    return lib().gpulz_record_offsets(d_table, chunks, d_offsets, stream)


def gpulz_decompress_workspace_size(comp_bytes: int, nbytes: int = 0) -> int:
    ws = ctypes.c_size_t(0)
    st = lib().gpulz_decompress_workspace_size(comp_bytes, nbytes, ctypes.byref(ws))
    if st != GPULZ_OK:
        raise GpulzError(st, "gpulz_decompress_workspace_size")
    return ws.value


def gpulz_decompress(d_in: int, in_bytes: int, d_out: int, out_capacity: int, d_out_bytes: int,
                     d_status: int, d_workspace: int, ws_bytes: int, stream: int = 0) -> int:
    return lib().gpulz_decompress(d_in, in_bytes, d_out, out_capacity, d_out_bytes, d_status,
                                  d_workspace, ws_bytes, stream)


def gpulz_decompress_noalloc(d_in: int, in_bytes: int, d_out: int, out_capacity: int,
                             d_out_bytes: int, d_status: int, stream: int = 0) -> int:
    return lib().gpulz_decompress_noalloc(d_in, in_bytes, d_out, out_capacity, d_out_bytes,
                                          d_status, stream)


def gpulz_huff_compress_bound(nbytes: int) -> int:
    return int(lib().gpulz_huff_compress_bound(nbytes))


def gpulz_huff_compress_workspace_size(max_bytes: int) -> int:
    ws = ctypes.c_size_t(0)
    st = lib().gpulz_huff_compress_workspace_size(max_bytes, ctypes.byref(ws))
    if st != GPULZ_OK:
        raise GpulzError(st, "gpulz_huff_compress_workspace_size")
    return ws.value


def gpulz_huff_compress(d_in: int, nbytes: int, d_nbytes, d_out: int, out_capacity: int,
                        d_out_bytes: int, d_status: int, d_workspace: int, ws_bytes: int,
                        stream: int = 0) -> int:
    return lib().gpulz_huff_compress(d_in, nbytes, d_nbytes, d_out, out_capacity, d_out_bytes,
                                     d_status, d_workspace, ws_bytes, stream)


def gpulz_huff_decompress_workspace_size(stream_bytes: int) -> int:
    ws = ctypes.c_size_t(0)
    st = lib().gpulz_huff_decompress_workspace_size(stream_bytes, ctypes.byref(ws))
    if st != GPULZ_OK:
        raise GpulzError(st, "gpulz_huff_decompress_workspace_size")
    return ws.value


def gpulz_huff_decompress(d_in: int, in_bytes: int, d_out: int, out_capacity: int,
                          d_out_bytes: int, d_status: int, d_workspace: int, ws_bytes: int,
                          stream: int = 0) -> int:
    return lib().gpulz_huff_decompress(d_in, in_bytes, d_out, out_capacity, d_out_bytes, d_status,
                                       d_workspace, ws_bytes, stream)


def gpulz_default_params(symbol_bytes: int):
    p = Params()
    _check(lib().gpulz_default_params(symbol_bytes, ctypes.byref(p)), "gpulz_default_params")
    return (p.chunk_symbols, p.window, p.min_match, p.waves_per_chunk)


def gpulz_set_default_params(symbol_bytes: int, chunk_symbols: int, window: int, min_match: int,
                             waves_per_chunk: int = 4) -> None:
    p = Params(chunk_symbols, window, min_match, waves_per_chunk)
    _check(lib().gpulz_set_default_params(symbol_bytes, ctypes.byref(p)), "gpulz_set_default_params")


def gpulz_compress_batch_workspace_size(nbufs: int, max_total_in_bytes: int, params=None) -> int:
    ws = ctypes.c_size_t(0)
    arr = params if isinstance(params, ParamsArray4) else params_array(params)
    _check(lib().gpulz_compress_batch_workspace_size(nbufs, max_total_in_bytes, arr, ctypes.byref(ws)),
           "gpulz_compress_batch_workspace_size")
    return ws.value


def gpulz_compress_batch(nbufs, d_in_ptrs, d_in_bytes, d_symbol_bytes, params, d_out_ptrs, d_out_caps,
                         d_out_bytes, d_status, max_total_in_bytes, d_workspace, ws_bytes,
                         stream: int = 0) -> int:
    arr = params if isinstance(params, ParamsArray4) else params_array(params)
    return lib().gpulz_compress_batch(nbufs, d_in_ptrs, d_in_bytes, d_symbol_bytes, arr, d_out_ptrs,
                                      d_out_caps, d_out_bytes, d_status, max_total_in_bytes,
                                      d_workspace, ws_bytes, stream)


def gpulz_decompress_batch_workspace_size(nbufs: int, max_total_in_bytes: int) -> int:
    ws = ctypes.c_size_t(0)
    _check(lib().gpulz_decompress_batch_workspace_size(nbufs, max_total_in_bytes, ctypes.byref(ws)),
           "gpulz_decompress_batch_workspace_size")
    return ws.value


def gpulz_decompress_batch(nbufs, d_in_ptrs, d_in_bytes, d_out_ptrs, d_out_caps, d_out_bytes,
                           d_status, max_total_in_bytes, d_workspace, ws_bytes,
                           stream: int = 0) -> int:
    return lib().gpulz_decompress_batch(nbufs, d_in_ptrs, d_in_bytes, d_out_ptrs, d_out_caps,
                                        d_out_bytes, d_status, max_total_in_bytes, d_workspace,
                                        ws_bytes, stream)


def gpulz_profile_enable(enable: bool) -> None:
    _check(lib().gpulz_profile_enable(1 if enable else 0), "gpulz_profile_enable")


def gpulz_profile_read():
    """{kernel name: (total ms, launches)} for the calls made while enabled."""
    n = len(KERNEL_NAMES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_uint64 * n)()
    _check(lib().gpulz_profile_read(ms, cnt, n), "gpulz_profile_read")
    return {k: (ms[i], int(cnt[i])) for i, k in enumerate(KERNEL_NAMES)}


# ---- torch convenience wrappers --------------------------------------------

def _torch():
    import torch
    return torch


def _stream_handle(stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _check(st: int, what: str):
    if st != GPULZ_OK:
        raise GpulzError(st, what)


class Compressor:
    """Reusable device buffers for compressing inputs of up to `max_bytes`.

    `compress_async` only enqueues kernels on the stream; `result` reads
    back the size and status (synchronising the stream)."""

    def __init__(self, max_bytes: int, symbol_bytes: int, chunk_symbols: int, window: int,
                 min_match: int, device="cuda", policy: int = 0):
        torch = _torch()
        self.S, self.C, self.W, self.MIN = symbol_bytes, chunk_symbols, window, min_match
        self.policy = policy
        self.capacity = gpulz_compress_bound(max_bytes, symbol_bytes, chunk_symbols, min_match)
        if self.capacity == 0:
            raise GpulzError(GPULZ_ERR_INVALID_ARG, "gpulz_compress_bound")
        self.ws_bytes = gpulz_compress_workspace_size(max_bytes, symbol_bytes, chunk_symbols)
        self.out = torch.empty(self.capacity, dtype=torch.uint8, device=device)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.meta = torch.zeros(2, dtype=torch.int64, device=device)  # [out_bytes, status]

    def compress_async(self, x, nbytes: int | None = None, stream=None) -> None:
        nbytes = x.numel() * x.element_size() if nbytes is None else nbytes
        st = gpulz_compress_policy(x.data_ptr(), nbytes, self.S, self.C, self.W, self.MIN,
                                   self.policy, self.out.data_ptr(), self.capacity,
                                   self.meta.data_ptr(), self.meta.data_ptr() + 8,
                                   self.ws.data_ptr(), self.ws_bytes, _stream_handle(stream))
        _check(st, "gpulz_compress_policy")

    def result(self):
        """(stream bytes, device status)."""
        meta = self.meta.cpu()
        return int(meta[0]), int(meta[1]) & 0xFFFFFFFF


def compress(x, symbol_bytes: int, chunk_symbols: int, window: int, min_match: int, stream=None,
             policy: int = 0):
    """Compress a device tensor's bytes; returns a uint8 device tensor.
    policy 0 = exact longest match, 1 = the paper's single window pass."""
    nbytes = x.numel() * x.element_size()
    c = Compressor(max(nbytes, 1), symbol_bytes, chunk_symbols, window, min_match, device=x.device,
                   policy=policy)
    c.compress_async(x, nbytes, stream)
    size, status = c.result()
    _check(status, "gpulz_compress (device status)")
    return c.out[:size]


def decompress(s, out_capacity: int | None = None, stream=None, return_status: bool = False):
    """Decompress a uint8 device tensor holding one stream."""
    torch = _torch()
    in_bytes = s.numel()
    if out_capacity is None:
        hdr = bytes(s[:64].cpu().numpy()) if in_bytes >= 64 else b""
        try:
            out_capacity = gpulz_peek_header(hdr)[0]
        except GpulzError:
            out_capacity = 0
    ws_bytes = gpulz_decompress_workspace_size(in_bytes)
    out = torch.empty(max(out_capacity, 1), dtype=torch.uint8, device=s.device)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=s.device)
    meta = torch.zeros(2, dtype=torch.int64, device=s.device)
    st = gpulz_decompress(s.data_ptr(), in_bytes, out.data_ptr(), out_capacity, meta.data_ptr(),
                          meta.data_ptr() + 8, ws.data_ptr(), ws_bytes, _stream_handle(stream))
    _check(st, "gpulz_decompress")
    m = meta.cpu()
    n, status = int(m[0]), int(m[1]) & 0xFFFFFFFF
    if return_status:
        return status, out[:n] if status == GPULZ_OK else None
    _check(status, "gpulz_decompress (device status)")
    return out[:n]


# ---- entropy stage (Huffman) -----------------------------------------------------

class HuffCompressor:
    """Reusable device buffers for Huffman-coding inputs of up to
    `max_bytes`. `compress_async` only enqueues kernels; `result` reads back
    the size and status (synchronising)."""

    def __init__(self, max_bytes: int, device="cuda"):
        torch = _torch()
        self.max_bytes = max_bytes
        self.capacity = gpulz_huff_compress_bound(max_bytes)
        if self.capacity == 0:
            raise GpulzError(GPULZ_ERR_INVALID_ARG, "gpulz_huff_compress_bound")
        self.ws_bytes = gpulz_huff_compress_workspace_size(max_bytes)
        self.out = torch.empty(self.capacity, dtype=torch.uint8, device=device)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.meta = torch.zeros(2, dtype=torch.int64, device=device)  # [out_bytes, status]

    def compress_async(self, x, nbytes: int | None = None, d_nbytes: int | None = None,
                       stream=None) -> None:
        """`x` is a device tensor (or an integer device pointer with `nbytes`);
        `d_nbytes` is an optional device pointer to the actual size (u64),
        read by the kernels, with `nbytes` its maximum."""
        ptr = x if isinstance(x, int) else x.data_ptr()
        if nbytes is None:
            nbytes = x.numel() * x.element_size()
        st = gpulz_huff_compress(ptr, nbytes, d_nbytes, self.out.data_ptr(), self.capacity,
                                 self.meta.data_ptr(), self.meta.data_ptr() + 8, self.ws.data_ptr(),
                                 self.ws_bytes, _stream_handle(stream))
        _check(st, "gpulz_huff_compress")

    def result(self):
        meta = self.meta.cpu()
        return int(meta[0]), int(meta[1]) & 0xFFFFFFFF


def huff_compress(x, stream=None):
    """Huffman-code a device tensor's bytes; returns a uint8 device tensor."""
    nbytes = x.numel() * x.element_size()
    c = HuffCompressor(max(nbytes, 1), device=x.device)
    c.compress_async(x, nbytes, stream=stream)
    size, status = c.result()
    _check(status, "gpulz_huff_compress (device status)")
    return c.out[:size]


def huff_stream_size(s) -> int:
    """n, the decoded size, from a Huffman stream's header (device tensor)."""
    if s.numel() < 64:
        return 0
    h = bytes(s[:64].cpu().numpy())
    return int.from_bytes(h[16:24], "little") if h[:4] == b"GLH1" else 0


def huff_decompress(s, out_capacity: int | None = None, stream=None, return_status: bool = False):
    """Decode a Huffman stream held in a uint8 device tensor."""
    torch = _torch()
    in_bytes = s.numel()
    if out_capacity is None:
        out_capacity = huff_stream_size(s)
    ws_bytes = gpulz_huff_decompress_workspace_size(in_bytes)
    out = torch.empty(max(out_capacity, 1), dtype=torch.uint8, device=s.device)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=s.device)
    meta = torch.zeros(2, dtype=torch.int64, device=s.device)
    st = gpulz_huff_decompress(s.data_ptr(), in_bytes, out.data_ptr(), out_capacity,
                               meta.data_ptr(), meta.data_ptr() + 8, ws.data_ptr(), ws_bytes,
                               _stream_handle(stream))
    _check(st, "gpulz_huff_decompress")
    m = meta.cpu()
    n, status = int(m[0]), int(m[1]) & 0xFFFFFFFF
    if return_status:
        return status, out[:n] if status == GPULZ_OK else None
    _check(status, "gpulz_huff_decompress (device status)")
    return out[:n]


def compress_entropy(x, symbol_bytes: int, chunk_symbols: int, window: int, min_match: int,
                     stream=None, policy: int = 0):
    """LZSS, then Huffman coding of the LZSS stream, enqueued back to back on
    one stream (the Huffman stage reads the LZSS size on the device).
    Returns (Huffman stream, LZSS stream bytes) as (device tensor, int)."""
    nbytes = x.numel() * x.element_size()
    lz = Compressor(max(nbytes, 1), symbol_bytes, chunk_symbols, window, min_match,
                    device=x.device, policy=policy)
    hc = HuffCompressor(lz.capacity, device=x.device)
    lz.compress_async(x, nbytes, stream)
    hc.compress_async(lz.out.data_ptr(), lz.capacity, d_nbytes=lz.meta.data_ptr(), stream=stream)
    lz_size, lz_status = lz.result()
    _check(lz_status, "gpulz_compress (device status)")
    size, status = hc.result()
    _check(status, "gpulz_huff_compress (device status)")
    return hc.out[:size], lz_size


def decompress_entropy(s, stream=None):
    """Inverse of compress_entropy: Huffman decoding, then LZSS decoding."""
    return decompress(huff_decompress(s, stream=stream), stream=stream)


# ---- batches ------------------------------------------------------------------

def _ptr_array(tensors, device):
    torch = _torch()
    return torch.tensor([t.data_ptr() for t in tensors], dtype=torch.int64, device=device)


class BatchCompressor:
    """One gpulz_compress_batch call over fixed device buffers.

    inputs: uint8 device tensors (16-byte aligned, as torch allocates);
    widths: symbol width per buffer; params: {S: (chunk, window, min_match[,
    waves])} or None. Output buffers are sized by gpulz_compress_bound. The
    call can be replayed eagerly (`run`) or captured once in a HIP graph
    (`capture`) and replayed (`replay`); either way the inputs' current
    contents are compressed."""

    def __init__(self, inputs, widths, params=None, device="cuda"):
        torch = _torch()
        self.inputs = list(inputs)
        self.n = len(self.inputs)
        self.params = params_array(params)
        self.sizes = [t.numel() for t in self.inputs]
        self.widths = list(widths)
        total = sum(self.sizes)
        self.max_total = max(total, 1)
        caps = []
        for nb, S in zip(self.sizes, self.widths):
            C, W, MIN, _ = self.resolved(S)
            caps.append(gpulz_compress_bound(nb, S, C, MIN) if S in (1, 2, 4, 8) else 64)
        self.outputs = [torch.empty(max(c, 1), dtype=torch.uint8, device=device) for c in caps]
        self.caps = caps
        self.d_in_ptrs = _ptr_array(self.inputs, device)
        self.d_in_bytes = torch.tensor(self.sizes, dtype=torch.int64, device=device)
        self.d_widths = torch.tensor(self.widths, dtype=torch.uint8, device=device)
        self.d_out_ptrs = _ptr_array(self.outputs, device)
        self.d_out_caps = torch.tensor(caps, dtype=torch.int64, device=device)
        self.d_out_bytes = torch.zeros(self.n, dtype=torch.int64, device=device)
        self.d_status = torch.zeros(self.n, dtype=torch.int32, device=device)
        self.ws_bytes = gpulz_compress_batch_workspace_size(self.n, self.max_total, self.params)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.graph = None

    def resolved(self, S):
        if S not in (1, 2, 4, 8):
            return (1, 1, 1, 4)
        p = self.params[{1: 0, 2: 1, 4: 2, 8: 3}[S]]
        d = gpulz_default_params(S)
        return tuple(v if v else dv for v, dv in
                     zip((p.chunk_symbols, p.window, p.min_match, p.waves_per_chunk), d))

    def run(self, stream=None) -> None:
        st = gpulz_compress_batch(self.n, self.d_in_ptrs.data_ptr(), self.d_in_bytes.data_ptr(),
                                  self.d_widths.data_ptr(), self.params, self.d_out_ptrs.data_ptr(),
                                  self.d_out_caps.data_ptr(), self.d_out_bytes.data_ptr(),
                                  self.d_status.data_ptr(), self.max_total, self.ws.data_ptr(),
                                  self.ws_bytes, _stream_handle(stream))
        _check(st, "gpulz_compress_batch")

    def capture(self) -> None:
        torch = _torch()
        self.run()  # warm up outside the capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g

    def replay(self) -> None:
        self.graph.replay()

    def results(self):
        """[(status, stream bytes as a uint8 device tensor or None)]"""
        sizes = self.d_out_bytes.cpu().tolist()
        stats = self.d_status.cpu().tolist()
        return [(st, self.outputs[i][:sizes[i]] if st == GPULZ_OK else None)
                for i, st in enumerate(stats)]


class BatchDecompressor:
    """One gpulz_decompress_batch call over fixed device streams."""

    def __init__(self, streams, out_caps, device="cuda"):
        torch = _torch()
        self.streams = list(streams)
        self.n = len(self.streams)
        self.sizes = [t.numel() for t in self.streams]
        self.max_total = max(sum(self.sizes), 1)
        self.outputs = [torch.empty(max(c, 1), dtype=torch.uint8, device=device) for c in out_caps]
        self.d_in_ptrs = _ptr_array(self.streams, device)
        self.d_in_bytes = torch.tensor(self.sizes, dtype=torch.int64, device=device)
        self.d_out_ptrs = _ptr_array(self.outputs, device)
        self.d_out_caps = torch.tensor(list(out_caps), dtype=torch.int64, device=device)
        self.d_out_bytes = torch.zeros(self.n, dtype=torch.int64, device=device)
        self.d_status = torch.zeros(self.n, dtype=torch.int32, device=device)
        self.ws_bytes = gpulz_decompress_batch_workspace_size(self.n, self.max_total)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def run(self, stream=None) -> None:
        st = gpulz_decompress_batch(self.n, self.d_in_ptrs.data_ptr(), self.d_in_bytes.data_ptr(),
                                    self.d_out_ptrs.data_ptr(), self.d_out_caps.data_ptr(),
                                    self.d_out_bytes.data_ptr(), self.d_status.data_ptr(),
                                    self.max_total, self.ws.data_ptr(), self.ws_bytes,
                                    _stream_handle(stream))
        _check(st, "gpulz_decompress_batch")

    def results(self):
        sizes = self.d_out_bytes.cpu().tolist()
        stats = self.d_status.cpu().tolist()
        return [(st, self.outputs[i][:sizes[i]] if st == GPULZ_OK else None)
                for i, st in enumerate(stats)]
