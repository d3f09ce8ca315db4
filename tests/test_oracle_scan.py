"""Pins the oracle's match policy 1 (the paper's single window pass, section
3.3.2): exhaustive agreement with the independent Python walk on tiny
inputs, and invariants that hold for any parse the walk can produce: every
pointer is a real match within the window with length <= offset and <= 255,
never longer than the exact longest match at that position, and every
stream decodes back to its input. The hand vectors E-P1..E-P4 are in
tests/golden/."""
import itertools
import random

import pytest

import oracle
import refimpl


@pytest.mark.parametrize("C,W,MIN", [(64, 8, 1), (64, 8, 2), (5, 3, 2), (64, 256, 3)])
def test_exhaustive_binary_bytes(C, W, MIN):
    for n in range(11):
        for t in itertools.product(b"AB", repeat=n):
            s = bytes(t)
            assert oracle.compress(s, 1, C, W, MIN, policy=1) == refimpl.compress(s, 1, C, W, MIN, 1), s


@pytest.mark.parametrize("C,W,MIN", [(64, 4, 2), (6, 8, 1)])
def test_exhaustive_ternary_bytes(C, W, MIN):
    for n in range(8):
        for t in itertools.product(b"ABC", repeat=n):
            s = bytes(t)
            assert oracle.compress(s, 1, C, W, MIN, policy=1) == refimpl.compress(s, 1, C, W, MIN, 1), s


@pytest.mark.parametrize("S", [2, 4, 8])
def test_random_wide_symbols(S):
    rng = random.Random(S)
    for _ in range(60):
        alpha = [bytes(rng.randrange(256) for _ in range(S)) for _ in range(rng.choice([2, 3, 5]))]
        x = b"".join(rng.choice(alpha) for _ in range(rng.randrange(0, 120)))
        C, W, MIN = rng.choice([7, 16, 64]), rng.choice([1, 3, 16, 256]), rng.choice([1, 2, 3])
        assert oracle.compress(x, S, C, W, MIN, policy=1) == refimpl.compress(x, S, C, W, MIN, 1)


def _pointers(chunk_syms, toks):
    p = 0
    for L, d in toks:
        if L:
            yield p, L, d
            p += L
        else:
            p += 1


@pytest.mark.parametrize("seed", range(4))
def test_pointers_are_valid_and_never_beat_the_exact_match(seed):
    rng = random.Random(seed)
    for _ in range(40):
        S = rng.choice([1, 2])
        alpha = [bytes(rng.randrange(256) for _ in range(S)) for _ in range(rng.choice([2, 3, 4]))]
        syms = [rng.choice(alpha) for _ in range(rng.randrange(1, 300))]
        W, MIN = rng.choice([4, 32, 200, 256]), rng.choice([1, 2, 3])
        toks = oracle.parse_chunk(b"".join(syms), S, W, MIN, policy=1)
        for p, L, d in _pointers(syms, toks):
            assert MIN <= L <= d <= min(W, p) and L <= 255
            assert syms[p:p + L] == syms[p - d:p - d + L]
            assert L <= refimpl.brute_best(syms, p, W)[0]


@pytest.mark.parametrize("seed", range(3))
def test_streams_round_trip_and_record_the_policy(seed):
    rng = random.Random(100 + seed)
    for _ in range(20):
        S = rng.choice([1, 2, 4, 8])
        x = bytes(rng.choice(b"ABC") for _ in range(rng.randrange(0, 3000)))
        C, W, MIN = rng.choice([16, 256, 1000]), rng.choice([8, 128, 256]), rng.choice([1, 2, 4])
        s = oracle.compress(x, S, C, W, MIN, policy=1)
        assert s[7] == 1
        assert oracle.decompress(s) == x
        assert refimpl.decompress(s) == x
