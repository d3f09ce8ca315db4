"""Pins the oracle's longest-match search and greedy parse: exhaustive
agreement with the slice-enumerating brute-force reference (refimpl.py) on
every string over small alphabets."""
import itertools
import random

import pytest

import oracle
import refimpl


def _all_strings(alphabet, max_len):
    for n in range(max_len + 1):
        for t in itertools.product(alphabet, repeat=n):
            yield b"".join(t)


BINARY_PARAMS = [(16, 256, 2), (16, 3, 2), (4, 4, 2), (3, 2, 1), (5, 8, 3), (1, 1, 1),
                 (2, 1, 1), (16, 1, 2), (7, 5, 1)]


@pytest.mark.parametrize("C,W,MIN", BINARY_PARAMS)
def test_exhaustive_binary_bytes(C, W, MIN):
    for s in _all_strings([b"A", b"B"], 12):
        assert oracle.compress(s, 1, C, W, MIN) == refimpl.compress(s, 1, C, W, MIN), s


@pytest.mark.parametrize("C,W,MIN", [(16, 256, 2), (4, 2, 1), (16, 3, 3), (6, 4, 2)])
def test_exhaustive_ternary_bytes(C, W, MIN):
    for s in _all_strings([b"A", b"B", b"C"], 8):
        assert oracle.compress(s, 1, C, W, MIN) == refimpl.compress(s, 1, C, W, MIN), s


@pytest.mark.parametrize("C,W,MIN", [(16, 256, 2), (3, 2, 1), (8, 3, 2)])
def test_exhaustive_u16_symbols(C, W, MIN):
    # 16-bit symbols whose bytes overlap, so a byte-level match is not a
    # symbol-level match; optional odd tail byte.
    alphabet = [b"\x01\x00", b"\x00\x01", b"\x01\x01"]
    for s in _all_strings(alphabet, 6):
        for tail in (b"", b"\x01"):
            x = s + tail
            assert oracle.compress(x, 2, C, W, MIN) == refimpl.compress(x, 2, C, W, MIN), x


@pytest.mark.parametrize("S", [4, 8])
def test_random_wide_symbols(S):
    rng = random.Random(1234 + S)
    vals = [bytes(rng.randrange(256) for _ in range(S)) for _ in range(3)]
    for _ in range(400):
        m = rng.randrange(0, 24)
        x = b"".join(rng.choice(vals) for _ in range(m)) + bytes(rng.randrange(S))
        C = rng.choice([1, 2, 3, 5, 8, 32])
        W = rng.choice([1, 2, 3, 7, 256])
        MIN = rng.choice([1, 2, 3])
        assert oracle.compress(x, S, C, W, MIN) == refimpl.compress(x, S, C, W, MIN)


def test_random_longer_runs_bytes():
    # long enough for matches near the 255 cap and offsets near 256
    rng = random.Random(99)
    for _ in range(6):
        base = bytes(rng.randrange(4) for _ in range(rng.randrange(1, 40)))
        x = (base * (700 // len(base) + 1))[:rng.randrange(300, 700)]
        x = bytearray(x)
        for _ in range(rng.randrange(0, 5)):
            x[rng.randrange(len(x))] = rng.randrange(4)
        x = bytes(x)
        W = rng.choice([200, 255, 256])
        assert oracle.compress(x, 1, 1024, W, 2) == refimpl.compress(x, 1, 1024, W, 2)
