"""Pins the Huffman-stage oracle to what the definitions fix: hand-worked
streams (tests/golden/huff_*.txt), the textbook frequency example, optimal
cost (an independent heap construction, and exhaustive search over complete
codes for small alphabets), the canonical-code properties, the length limit
on a hand-worked case, an independent Python encoder and decoder, round
trips, and rejection of corrupted streams."""
import itertools
import struct

import numpy as np
import pytest

import huffref
import oracle
from huff_golden import all_vectors

VECTORS = all_vectors()


@pytest.mark.parametrize("v", VECTORS, ids=[v["name"] for v in VECTORS])
def test_oracle_stream_matches_hand_vector(v):
    assert oracle.huff_compress(v["input"]).hex() == v["stream"].hex()


@pytest.mark.parametrize("v", VECTORS, ids=[v["name"] for v in VECTORS])
def test_oracle_lengths_match_hand_vector(v):
    freq = np.bincount(np.frombuffer(v["input"], np.uint8), minlength=256)
    lens = oracle.huff_lengths(freq)
    assert {s: l for s, l in enumerate(lens) if l} == v["lengths"]


@pytest.mark.parametrize("v", VECTORS, ids=[v["name"] for v in VECTORS])
def test_oracle_decodes_hand_vector(v):
    assert oracle.huff_decompress(v["stream"]) == v["input"]


@pytest.mark.parametrize("v", VECTORS, ids=[v["name"] for v in VECTORS])
def test_python_reference_matches_hand_vector(v):
    assert huffref.compress(v["input"]).hex() == v["stream"].hex()
    assert huffref.decompress(v["stream"]) == v["input"]


def test_textbook_frequencies():
    # the classic six-symbol example (frequencies 45 13 12 16 9 5, no ties):
    # lengths 1 3 3 3 4 4 and 224 bits per 100 symbols
    f = [45, 13, 12, 16, 9, 5]
    lens = oracle.huff_lengths(f)
    assert lens[:6] == [1, 3, 3, 3, 4, 4] and not any(lens[6:])
    assert huffref.cost(f, lens) == 224


def test_length_limit_hand_case():
    # weights 1 1 2 4 8 give depths 4 4 3 2 1; with a limit of 3 they become
    # ceil(w/2) = 1 1 1 2 4: joins s0+s1 -> X(2), s2(1)+s3(2, a leaf before X)
    # -> Y(3), X+Y -> Z(5), s4(4)+Z -> root: depths 3 3 3 3 1
    assert oracle.huff_lengths([1, 1, 2, 4, 8])[:5] == [4, 4, 3, 2, 1]
    assert oracle.huff_lengths([1, 1, 2, 4, 8], 3)[:5] == [3, 3, 3, 3, 1]
    assert oracle.huff_lengths([1] * 9, 3) is None


def _kraft(lens):
    return sum(2.0 ** -l for l in lens if l)


def _hist(kind, rng, k=256):
    if kind == "uniform":
        return rng.integers(1, 1000, k)
    if kind == "geometric":
        return np.maximum(1, (1e6 * 0.7 ** np.arange(k))).astype(np.int64)[rng.permutation(k)]
    if kind == "sparse":
        f = np.zeros(k, np.int64)
        idx = rng.choice(k, 7, replace=False)
        f[idx] = rng.integers(1, 50, 7)
        return f
    return np.maximum(0, rng.integers(-50, 5000, k)) ** 2  # some zeros, wide range


@pytest.mark.parametrize("kind", ["uniform", "geometric", "sparse", "wide"])
@pytest.mark.parametrize("seed", range(6))
def test_cost_is_optimal(kind, seed):
    rng = np.random.default_rng(seed)
    f = [int(x) for x in _hist(kind, rng)]
    lens = oracle.huff_lengths(f)
    if max(huffref.lengths(f, limit=99)) <= 15:
        assert huffref.cost(f, lens) == huffref.optimal_cost(f)
    else:
        assert max(lens) <= 15 and huffref.cost(f, lens) > huffref.optimal_cost(f)
    assert abs(_kraft(lens) - 1.0) < 1e-12
    assert all((l > 0) == (x > 0) for l, x in zip(lens, f))


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6])
def test_cost_equals_exhaustive_search(k):
    rng = np.random.default_rng(k)
    for _ in range(8):
        f = [int(x) for x in rng.integers(1, 30, k)]
        best = min(sum(a * b for a, b in zip(f, ls))
                   for ls in itertools.product(range(1, k), repeat=k)
                   if sum(2.0 ** -l for l in ls) == 1.0)
        assert huffref.cost(f, oracle.huff_lengths(f)) == best


def test_canonical_code_properties():
    rng = np.random.default_rng(3)
    for _ in range(20):
        f = [int(x) for x in _hist("wide", rng)]
        lens = oracle.huff_lengths(f)
        code = oracle.huff_codes(lens)
        words = {s: format(code[s], f"0{lens[s]}b") for s in range(256) if lens[s]}
        # prefix-free
        ws = sorted(words.values())
        assert all(not b.startswith(a) for a, b in zip(ws, ws[1:]))
        # codes of one length are consecutive in symbol order, and every code
        # of a shorter length sorts before every code of a longer one
        by_len = {}
        for s in sorted(words):
            by_len.setdefault(lens[s], []).append(code[s])
        for vals in by_len.values():
            assert vals == list(range(vals[0], vals[0] + len(vals)))
        seq = [words[s] for s in sorted(words, key=lambda s: (lens[s], s))]
        assert seq == sorted(seq)
        assert words == huffref.codes(lens)


def test_limit_holds_on_fibonacci_weights():
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    unlimited = huffref.lengths(fib, limit=99)
    assert max(unlimited) > 15
    lens = oracle.huff_lengths(fib)
    assert max(lens) == 15 and abs(_kraft(lens) - 1.0) < 1e-12
    assert huffref.cost(fib, lens) >= huffref.optimal_cost(fib)
    assert lens == huffref.lengths(fib)


def _inputs():
    rng = np.random.default_rng(11)
    yield "empty", b""
    yield "one", b"\x07"
    yield "single_symbol", b"q" * (3 * 4096 + 5)
    yield "two_symbols", bytes(rng.choice([3, 250], 5000, p=[0.9, 0.1]).astype(np.uint8))
    yield "all_bytes", bytes(rng.integers(0, 256, 9000).astype(np.uint8))
    zipf = np.minimum(rng.zipf(1.3, 4096 * 3 + 200), 256) - 1
    yield "zipf_3chunks_ragged", bytes(zipf.astype(np.uint8))
    for n in (127, 128, 129, 4095, 4096, 4097):
        yield f"geom_{n}", bytes(np.minimum(rng.geometric(0.2, n), 255).astype(np.uint8))


INPUTS = list(_inputs())


@pytest.mark.parametrize("name,data", INPUTS, ids=[n for n, _ in INPUTS])
def test_oracle_matches_python_reference(name, data):
    s = oracle.huff_compress(data)
    assert s == huffref.compress(data)
    assert huffref.decompress(s) == data
    assert oracle.huff_decompress(s) == data
    assert len(s) <= oracle.huff_bound(len(data))


def _corrupt_cases(s):
    N = struct.unpack_from("<Q", s, 24)[0]
    rec0 = 192 + 4 * N
    yield "magic", 0, 0x01
    yield "version", 4, 0x02
    yield "limit", 6, 0x01
    yield "chunk", 9, 0x01
    yield "reserved", 50, 0x01
    yield "length_nibble", 64 + ord("a") // 2, 0x10   # a's length 1 -> 0: incomplete code
    yield "table_bits", 192, 0x01
    yield "first_offset", rec0, 0x01
    yield "padding_bit", len(s) - 4, 0x01           # last word's lowest bit is padding


@pytest.mark.parametrize("case", ["magic", "version", "limit", "chunk", "reserved",
                                  "length_nibble", "table_bits", "first_offset", "padding_bit"])
def test_corrupt_streams_are_rejected(case):
    data = b"abracadabra" * 50
    s = oracle.huff_compress(data)
    assert oracle.huff_decompress_status(s)[0] == oracle.OK
    (name, at, mask), = [c for c in _corrupt_cases(s) if c[0] == case]
    bad = bytearray(s)
    bad[at] ^= mask
    assert oracle.huff_decompress_status(bytes(bad))[0] == oracle.ERR_CORRUPT


def test_incomplete_code_is_rejected_even_if_the_data_decodes():
    lens = [0] * 256
    for ch in b"abc":
        lens[ch] = 2  # Kraft sum 3/4
    s = huffref.compress(b"abcabc", lens)
    assert huffref.decompress(s) == b"abcabc"
    assert oracle.huff_decompress_status(s)[0] == oracle.ERR_CORRUPT


def test_length_limit_applies_on_data():
    # symbol s repeated fib(s + 1) times for 18 symbols: a 17-deep tree
    fib = [1, 1]
    while len(fib) < 18:
        fib.append(fib[-1] + fib[-2])
    data = b"".join(bytes([s]) * f for s, f in enumerate(fib))
    assert max(huffref.lengths(fib, limit=99)) == 17
    s = oracle.huff_compress(data)
    lens = [s[64 + k // 2] >> 4 * (k & 1) & 15 for k in range(256)]
    assert lens == oracle.huff_lengths(fib) and 0 < max(lens) <= 15
    assert s == huffref.compress(data)
    assert oracle.huff_decompress(s) == data


def test_truncated_and_small_capacity():
    s = oracle.huff_compress(b"hello world" * 100)
    assert oracle.huff_decompress_status(s[:-1])[0] == oracle.ERR_CORRUPT
    st, _, need = oracle.huff_decompress_status(s, capacity=10)
    assert st == oracle.ERR_OUT_OF_SPACE and need == 1100
