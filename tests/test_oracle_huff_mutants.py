"""Shows the Huffman-stage pins are not vacuous: plausible mistakes are
planted in a temporary copy of the oracle's huff_oracle.c, each copy is
compiled with gcc, and a compact selection of the pins must reject it."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import huffref
import oracle
from huff_golden import all_vectors

SRC = os.path.join(os.path.dirname(oracle.__file__), "huff_oracle.c")

MUTANTS = {
    "ties_to_internal_nodes": ("if (best < 0 || weight[x] < weight[best])",
                               "if (best < 0 || weight[x] <= weight[best])"),
    "limit_halves_down": ("w[s] = (w[s] + 1) / 2;", "w[s] = w[s] > 1 ? w[s] / 2 : 1;"),
    "canonical_first_code_not_shifted": ("c = (c + count[l - 1]) << 1;", "c = c + count[l - 1];"),
    "canonical_descending_symbols": ("for (int s = 0; s < 256; ++s) code[s] = len[s] ? next[len[s]]++ : 0;",
                                     "for (int s = 255; s >= 0; --s) code[s] = len[s] ? next[len[s]]++ : 0;"),
    "bits_lsb_first": ("get_u32(wp) | (1u << (31 - bit % 32));", "get_u32(wp) | (1u << (bit % 32));"),
    "code_lsb_first": ("for (int b = len[s] - 1; b >= 0; --b, ++bit) {\n        if ((code[s] >> b) & 1u) {",
                       "for (int b = 0; b < len[s]; ++b, ++bit) {\n        if ((code[s] >> b) & 1u) {"),
    "subblock_offset_after_symbol": ("if (j % HO_SUB == 0) put_u16(rec + 2 * (j / HO_SUB), (uint32_t)bit);",
                                     "if (j % HO_SUB == 1) put_u16(rec + 2 * (j / HO_SUB), (uint32_t)bit);"),
    "offsets_not_padded": ("return (2ull * nsub + 3) / 4 * 4;", "return 2ull * nsub;"),
    "nibbles_swapped": ("buf[HO_HDR + s / 2] |= (uint8_t)(len[s] << (4 * (s & 1)));",
                        "buf[HO_HDR + s / 2] |= (uint8_t)(len[s] << (4 - 4 * (s & 1)));"),
    "single_symbol_length_0": ("      if (w[s]) len[s] = 1;", "      if (w[s]) len[s] = 2;"),
    "decoder_accepts_incomplete_code": ("!(present == 1 ? count[1] == 1 : kraft == (1ull << 15))",
                                        "!(present == 1 ? count[1] == 1 : kraft <= (1ull << 15))"),
    "decoder_ignores_padding": ("      if (code_bit(words, b)) return HO_CORRUPT;", "      (void)0;"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    msrc = tmp_path / f"{name}.c"
    msrc.write_text(src.replace(old, new))
    lib = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-std=c99", "-O1", "-shared", "-fPIC",
                           "-I", os.path.dirname(SRC), str(msrc), "-o", str(lib)])
    L = ctypes.CDLL(str(lib))
    u8p, u64p = ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_uint64)
    L.oracle_huff_bound.restype = ctypes.c_uint64
    L.oracle_huff_bound.argtypes = [ctypes.c_uint64]
    for f in (L.oracle_huff_compress, L.oracle_huff_decompress):
        f.restype = ctypes.c_int
        f.argtypes = [u8p, ctypes.c_uint64, u8p, ctypes.c_uint64, u64p]
    return L


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _compress(L, data):
    x = np.frombuffer(data, np.uint8) if data else np.zeros(1, np.uint8)
    cap = L.oracle_huff_bound(len(data))
    out = np.zeros(cap, np.uint8)
    n = ctypes.c_uint64()
    st = L.oracle_huff_compress(_u8(x), len(data), _u8(out), cap, ctypes.byref(n))
    return out[:n.value].tobytes() if st == 0 else None


def _decompress_status(L, s):
    x = np.frombuffer(s, np.uint8)
    n0 = int.from_bytes(s[16:24], "little")
    out = np.zeros(max(n0, 1), np.uint8)
    n = ctypes.c_uint64()
    return L.oracle_huff_decompress(_u8(x), len(s), _u8(out), n0, ctypes.byref(n))


def _pins_pass(L):
    for v in all_vectors():
        if _compress(L, v["input"]) != v["stream"]:
            return False
        if _decompress_status(L, v["stream"]) != 0:
            return False
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    rng = np.random.default_rng(5)
    data = bytes(np.minimum(rng.geometric(0.2, 9000), 255).astype(np.uint8))
    if _compress(L, data) != huffref.compress(data):
        return False
    # symbol s repeated fib(s + 1) times for 18 symbols: the tree is 17 deep,
    # so the length limit applies
    fib_data = b"".join(bytes([s]) * f for s, f in enumerate(fib[:18]))
    if _compress(L, fib_data) != huffref.compress(fib_data):
        return False
    # an incomplete code (a, b, c of length 2) whose data still decodes
    lens = [0] * 256
    for ch in b"abc":
        lens[ch] = 2
    if _decompress_status(L, huffref.compress(b"abcabc", lens)) != 3:
        return False
    # corrupt streams: an incomplete code, and a set padding bit
    s = bytearray(oracle.huff_compress(b"abracadabra" * 50))
    s[64 + ord("a") // 2] ^= 0x10
    if _decompress_status(L, bytes(s)) != 3:
        return False
    s = bytearray(oracle.huff_compress(b"abracadabra" * 50))
    s[-4] ^= 1
    if _decompress_status(L, bytes(s)) != 3:
        return False
    return True


def test_unmutated_copy_passes(tmp_path):
    assert _pins_pass(_build(tmp_path, "same", "#define HO_OK 0", "#define HO_OK 0"))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    assert not _pins_pass(_build(tmp_path, name, old, new))
