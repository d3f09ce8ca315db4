"""Shows the oracle's pins are not vacuous: plausible mistakes are planted in
a temporary copy of the oracle's C source, each copy is compiled with gcc,
and the hand vectors plus a slice of the brute-force sweep must reject it."""
import ctypes
import itertools
import os
import subprocess

import pytest

import oracle
import refimpl
from golden import all_vectors

SRC = os.path.join(os.path.dirname(oracle.__file__), "gpulz_oracle.c")

MUTANTS = {
    "tie_to_smallest_offset": ("if (L > bestL) {", "if (L >= bestL) {"),
    "no_length_le_offset": ("uint32_t cap = d < lim ? d : lim;", "uint32_t cap = lim;"),
    "no_255_cap": ("if (lim > MAX_MATCH) lim = MAX_MATCH;", ""),
    "window_off_by_one": ("uint32_t dmax = p < W ? p : W;", "uint32_t dmax = p < W ? p : W - 1;"),
    "min_match_strict": ("if (L >= MIN) {", "if (L > MIN) {"),
    "flag_msb_first": ("rec[t >> 3] |= (uint8_t)(1u << (t & 7));",
                       "rec[t >> 3] |= (uint8_t)(0x80u >> (t & 7));"),
    "offset_minus_one": ("(uint8_t)(offsets[t] & 0xFFu);", "(uint8_t)((offsets[t] - 1) & 0xFFu);"),
    "pointer_fields_swapped": ("rec[F + P] = (uint8_t)lengths[t];", "rec[F + P] = (uint8_t)offsets[t];"),
    "table_fields_swapped": ("put_u32(out + HDR_BYTES + 8 * i, F[i]);",
                             "put_u32(out + HDR_BYTES + 8 * i, P[i]);"),
    "tail_dropped": ("h[48 + k] = tail[k];", "h[48 + k] = 0;"),
    "decode_offset_256": ("O = pay[used + 1] ? pay[used + 1] : 256u;", "O = pay[used + 1];"),
    "decode_no_length_le_offset_check": ("|| L > O ||", "||"),
    # match policy 1 (the paper's single window pass)
    "scan_retries_failed_slot": ("      len = 0;\n      off = 0;\n      b = p;",
                                 "      w -= len;\n      len = 0;\n      off = 0;\n      b = p;"),
    "scan_drops_open_run": ("  if (len > bestL) {\n    bestL = len;\n    bestd = off;\n  }\n  *L_out",
                            "  *L_out"),
    "scan_ties_to_newest": ("      if (len > bestL) {", "      if (len >= bestL) {"),
    "scan_no_255_cap": ("if (len < MAX_MATCH && sym_eq(chunk, b, w, S)) {",
                        "if (sym_eq(chunk, b, w, S)) {"),
}


def _build_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    msrc = tmp_path / f"{name}.c"
    msrc.write_text(src.replace(old, new))
    lib = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-std=c99", "-O1", "-shared", "-fPIC", "-pthread",
                           "-I", os.path.dirname(SRC), str(msrc), "-o", str(lib)])
    return str(lib)


def _pins_pass():
    """A compact selection of the pins: hand vectors (compress + decode), the
    binary brute-force sweep, and a corrupt-stream check."""
    for v in all_vectors():
        n = len(v["input"])
        N = -(-(n // v["S"]) // v["C"])
        exp = refimpl.header(n, v["S"], v["C"], v["W"], v["MIN"], N, v["total"], v["tail"],
                             v["policy"]) + v["body"]
        if oracle.compress(v["input"], v["S"], v["C"], v["W"], v["MIN"], policy=v["policy"]) != exp:
            return False
        st, got, _ = oracle.decompress_status(exp)
        if st != oracle.OK or got != v["input"]:
            return False
    for n in range(9):
        for t in itertools.product(b"AB", repeat=n):
            s = bytes(t)
            for C, W, MIN in [(16, 256, 2), (4, 2, 1), (16, 3, 2)]:
                if oracle.compress(s, 1, C, W, MIN) != refimpl.compress(s, 1, C, W, MIN):
                    return False
    # a pointer longer than its offset must be rejected
    bad = refimpl.header(4, 1, 8, 4, 2, 1, 64 + 8 + 4, b"") + bytes.fromhex("0100000003000000") \
        + bytes.fromhex("02 41 03 01")
    st, _, _ = oracle.decompress_status(bad)
    if st != oracle.ERR_CORRUPT:
        return False
    return True


def test_unmutated_oracle_passes_pins():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, monkeypatch):
    path = _build_mutant(tmp_path, name, *MUTANTS[name])
    real = oracle._load()
    mlib = ctypes.CDLL(path)
    for fn in ("oracle_compress_bound", "oracle_compress", "oracle_compress_mt",
               "oracle_compress_policy_mt", "oracle_decompress", "oracle_parse_chunk",
               "oracle_parse_chunk_policy"):
        getattr(mlib, fn).restype = getattr(real, fn).restype
        getattr(mlib, fn).argtypes = getattr(real, fn).argtypes
    monkeypatch.setattr(oracle, "_lib", mlib)
    assert not _pins_pass(), f"planted mistake {name} was not caught"
