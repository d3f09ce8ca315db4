"""CPU oracle for chunked multi-byte LZSS (gpuLZ, Zhang et al., ICS'23) and
the Huffman stage that follows it.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. The product library
(``paper_2304_07342_amd``) never imports, loads or calls it, and the two
share no code.

The oracle is plain C99 (``gpulz_oracle.c`` for LZSS, ``huff_oracle.c`` for
the Huffman stage; the two files are independent) built with gcc into
``libgpulz_oracle.so`` and loaded here with ctypes. See the C headers for
what each computes and which passage of the paper each step follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gpulz_oracle.c")
_HUFF_SRC = os.path.join(_HERE, "huff_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libgpulz_oracle.so")

OK = 0
ERR_INVALID_ARG = 1
ERR_OUT_OF_SPACE = 2
ERR_CORRUPT = 3
ERR_NOMEM = 7


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no vectorisation pragmas)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-shared", "-fPIC",
             "-pthread", _SRC, _HUFF_SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.oracle_compress_bound.restype = ctypes.c_uint64
        lib.oracle_compress_bound.argtypes = [ctypes.c_uint64, ctypes.c_uint32,
                                              ctypes.c_uint32, ctypes.c_uint32]
        lib.oracle_compress.restype = ctypes.c_int
        lib.oracle_compress.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_uint32, ctypes.c_uint32, u8p, ctypes.c_uint64,
                                        u64p]
        lib.oracle_compress_mt.restype = ctypes.c_int
        lib.oracle_compress_mt.argtypes = lib.oracle_compress.argtypes + [ctypes.c_int]
        lib.oracle_compress_policy_mt.restype = ctypes.c_int
        lib.oracle_compress_policy_mt.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint32,
                                                  ctypes.c_uint32, ctypes.c_uint32,
                                                  ctypes.c_uint32, ctypes.c_uint32, u8p,
                                                  ctypes.c_uint64, u64p, ctypes.c_int]
        lib.oracle_parse_chunk_policy.restype = ctypes.c_int64
        lib.oracle_parse_chunk_policy.argtypes = [u8p, ctypes.c_uint32, ctypes.c_uint32,
                                                  ctypes.c_uint32, ctypes.c_uint32,
                                                  ctypes.c_uint32, u32p, u32p]
        lib.oracle_decompress.restype = ctypes.c_int
        lib.oracle_decompress.argtypes = [u8p, ctypes.c_uint64, u8p, ctypes.c_uint64, u64p]
        lib.oracle_parse_chunk.restype = ctypes.c_int64
        lib.oracle_parse_chunk.argtypes = [u8p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                           ctypes.c_uint32, u32p, u32p]
        lib.oracle_huff_lengths.restype = ctypes.c_int
        lib.oracle_huff_lengths.argtypes = [u64p, ctypes.c_uint32, u8p]
        lib.oracle_huff_codes.restype = None
        lib.oracle_huff_codes.argtypes = [u8p, u32p]
        lib.oracle_huff_bound.restype = ctypes.c_uint64
        lib.oracle_huff_bound.argtypes = [ctypes.c_uint64]
        lib.oracle_huff_compress.restype = ctypes.c_int
        lib.oracle_huff_compress.argtypes = [u8p, ctypes.c_uint64, u8p, ctypes.c_uint64, u64p]
        lib.oracle_huff_decompress.restype = ctypes.c_int
        lib.oracle_huff_decompress.argtypes = [u8p, ctypes.c_uint64, u8p, ctypes.c_uint64, u64p]
        _lib = lib
    return _lib


def _u8(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _as_bytes(data) -> np.ndarray:
    if isinstance(data, np.ndarray):
        return np.ascontiguousarray(data).view(np.uint8).reshape(-1)
    return np.frombuffer(bytes(data), dtype=np.uint8)


def compress_bound(nbytes: int, symbol_bytes: int, chunk_symbols: int, min_match: int) -> int:
    return int(_load().oracle_compress_bound(nbytes, symbol_bytes, chunk_symbols, min_match))


def compress_status(data, symbol_bytes: int, chunk_symbols: int, window: int, min_match: int,
                    capacity: int | None = None, threads: int = 1, policy: int = 0):
    """Return (status, stream_bytes_or_None, required_size). policy 0 = exact
    longest match, 1 = the paper's single-pass window scan."""
    lib = _load()
    x = _as_bytes(data)
    n = x.size
    bound = lib.oracle_compress_bound(n, symbol_bytes, chunk_symbols, min_match)
    cap = bound if capacity is None else capacity
    out = np.zeros(max(cap, 1), dtype=np.uint8)
    out_len = ctypes.c_uint64(0)
    xin = x if n else np.zeros(1, dtype=np.uint8)
    if policy != 0:
        st = lib.oracle_compress_policy_mt(_u8(xin), n, symbol_bytes, chunk_symbols, window,
                                           min_match, policy, _u8(out), cap,
                                           ctypes.byref(out_len), max(1, threads))
    elif threads > 1:
        st = lib.oracle_compress_mt(_u8(xin), n, symbol_bytes, chunk_symbols, window, min_match,
                                    _u8(out), cap, ctypes.byref(out_len), threads)
    else:
        st = lib.oracle_compress(_u8(xin), n, symbol_bytes, chunk_symbols, window, min_match,
                                 _u8(out), cap, ctypes.byref(out_len))
    if st == OK:
        return st, out[: out_len.value].tobytes(), out_len.value
    return st, None, out_len.value


def compress(data, symbol_bytes: int, chunk_symbols: int, window: int, min_match: int,
             threads: int = 1, policy: int = 0) -> bytes:
    st, stream, _ = compress_status(data, symbol_bytes, chunk_symbols, window, min_match,
                                    threads=threads, policy=policy)
    if st != OK:
        raise ValueError(f"oracle_compress failed with status {st}")
    return stream


def decompress_status(stream, capacity: int | None = None):
    """Return (status, original_bytes_or_None, n)."""
    lib = _load()
    s = _as_bytes(stream)
    if capacity is None:
        capacity = int.from_bytes(bytes(s[16:24]), "little") if s.size >= 64 else 0
        capacity = min(capacity, 1 << 34)
    out = np.zeros(max(capacity, 1), dtype=np.uint8)
    out_len = ctypes.c_uint64(0)
    sin = s if s.size else np.zeros(1, dtype=np.uint8)
    st = lib.oracle_decompress(_u8(sin), s.size, _u8(out), capacity, ctypes.byref(out_len))
    if st == OK:
        return st, out[: out_len.value].tobytes(), out_len.value
    return st, None, out_len.value


def decompress(stream) -> bytes:
    st, data, _ = decompress_status(stream)
    if st != OK:
        raise ValueError(f"oracle_decompress failed with status {st}")
    return data


def parse_chunk(chunk, symbol_bytes: int, window: int, min_match: int, policy: int = 0):
    """Tokens of one chunk as a list of (length, offset); length 0 = literal."""
    lib = _load()
    x = _as_bytes(chunk)
    c = x.size // symbol_bytes
    lengths = np.zeros(max(c, 1), dtype=np.uint32)
    offsets = np.zeros(max(c, 1), dtype=np.uint32)
    xin = x if x.size else np.zeros(1, dtype=np.uint8)
    t = lib.oracle_parse_chunk_policy(_u8(xin), c, symbol_bytes, window, min_match, policy,
                                      lengths.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                      offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    if t < 0:
        raise ValueError("invalid parameters")
    return [(int(lengths[i]), int(offsets[i])) for i in range(t)]


# ---- Huffman stage ------------------------------------------------------------

def huff_lengths(freq, max_len: int = 15):
    """Code lengths (list of 256) for byte frequencies; None if max_len
    cannot hold the present symbols."""
    f = np.zeros(256, dtype=np.uint64)
    f[:len(freq)] = np.asarray(freq, dtype=np.uint64)
    out = np.zeros(256, dtype=np.uint8)
    st = _load().oracle_huff_lengths(f.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), max_len,
                                     _u8(out))
    return None if st else [int(v) for v in out]


def huff_codes(lengths):
    ln = np.zeros(256, dtype=np.uint8)
    ln[:len(lengths)] = lengths
    out = np.zeros(256, dtype=np.uint32)
    _load().oracle_huff_codes(_u8(ln), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    return [int(v) for v in out]


def huff_bound(nbytes: int) -> int:
    return int(_load().oracle_huff_bound(nbytes))


def huff_compress(data) -> bytes:
    lib = _load()
    x = _as_bytes(data)
    cap = lib.oracle_huff_bound(x.size)
    out = np.zeros(cap, dtype=np.uint8)
    out_len = ctypes.c_uint64(0)
    xin = x if x.size else np.zeros(1, dtype=np.uint8)
    st = lib.oracle_huff_compress(_u8(xin), x.size, _u8(out), cap, ctypes.byref(out_len))
    if st != OK:
        raise ValueError(f"oracle_huff_compress failed with status {st}")
    return out[: out_len.value].tobytes()


def huff_decompress_status(stream, capacity: int | None = None):
    """Return (status, original_bytes_or_None, n)."""
    lib = _load()
    s = _as_bytes(stream)
    if capacity is None:
        capacity = int.from_bytes(bytes(s[16:24]), "little") if s.size >= 64 else 0
        capacity = min(capacity, 1 << 34)
    out = np.zeros(max(capacity, 1), dtype=np.uint8)
    out_len = ctypes.c_uint64(0)
    sin = s if s.size else np.zeros(1, dtype=np.uint8)
    st = lib.oracle_huff_decompress(_u8(sin), s.size, _u8(out), capacity, ctypes.byref(out_len))
    if st == OK:
        return st, out[: out_len.value].tobytes(), out_len.value
    return st, None, out_len.value


def huff_decompress(stream) -> bytes:
    st, data, _ = huff_decompress_status(stream)
    if st != OK:
        raise ValueError(f"oracle_huff_decompress failed with status {st}")
    return data
