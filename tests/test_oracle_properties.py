"""Pins the oracle with closed forms, a per-token greedy-longest certificate,
round trips through an independent decoder, format invariants and decoder
fuzzing."""
import random
import struct

import numpy as np
import pytest

import oracle
import refimpl


def constant_ladder(c, W, MIN):
    """Closed form for a chunk of c equal symbols: at coding position p the
    offsets 1..min(W, p) all match, a match may not exceed its offset, 255, or
    the chunk end, so L = min(W, p, 255, c - p) with the largest offset
    d = min(W, p) (ties to the largest offset); p = 0 has an empty window."""
    toks = []
    p = 0
    while p < c:
        L = min(W, p, 255, c - p)
        if p > 0 and L >= MIN:
            toks.append((L, min(W, p)))
            p += L
        else:
            toks.append((0, 0))
            p += 1
    return toks


@pytest.mark.parametrize("S", [1, 2, 4, 8])
@pytest.mark.parametrize("W", [1, 2, 5, 64, 128, 255, 256])
@pytest.mark.parametrize("MIN", [1, 2, 3, 7])
def test_constant_input_closed_form(S, W, MIN):
    c = 1000
    x = bytes(range(11, 11 + S)) * c
    assert oracle.parse_chunk(x, S, W, MIN) == constant_ladder(c, W, MIN)


@pytest.mark.parametrize("S", [1, 2, 4, 8])
def test_all_distinct_closed_form(S):
    # strictly increasing symbols never repeat: every token is a literal, so
    # F_i = ceil(c_i/8) zero bytes and the payload is the chunk verbatim
    m, C = 3000, 512
    vals = np.arange(1000, 1000 + m, dtype=np.uint64) * 7919
    x = b"".join(int(v).to_bytes(8, "little")[:S] for v in vals)
    if S == 1:
        x = bytes(range(256))[:200] * 1  # 200 distinct bytes
        m = 200
    s = oracle.compress(x, S, C, 256, 2)
    N = -(-m // C)
    pos = 64 + 8 * N
    for i in range(N):
        F, P = struct.unpack_from("<II", s, 64 + 8 * i)
        c = min(C, m - i * C)
        assert F == (c + 7) // 8 and P == S * c
        assert s[pos:pos + F] == bytes(F)
        assert s[pos + F:pos + F + P] == x[i * C * S:(i * C + c) * S]
        pos += F + P
    assert pos == len(s)


def _greedy_certificate(chunk_syms, toks, W, MIN):
    """Check that every token is what a greedy longest-match parse must emit.
    For each coding position the match length at every offset is computed
    with numpy from the element-wise equality of the shifted symbol arrays."""
    a = np.array(chunk_syms)
    c = len(a)
    p = 0
    for L, d in toks:
        best = (0, 0)
        for dd in range(1, min(W, p) + 1):
            cap = min(dd, 255, c - p)
            eq = a[p:p + cap] == a[p - dd:p - dd + cap]
            run = cap if eq.all() else int(np.argmin(eq))
            if (run, dd) > best:
                best = (run, dd)
        if best[0] >= MIN:
            assert (L, d) == best, (p, (L, d), best)
            p += L
        else:
            assert L == 0, (p, (L, d), best)
            p += 1
    assert p == c


def _syms_as_ints(data, S):
    m = len(data) // S
    return np.frombuffer(data[:m * S], dtype={1: np.uint8, 2: np.uint16, 4: np.uint32,
                                              8: np.uint64}[S])


def _random_input(rng, S, m):
    kind = rng.randrange(4)
    if kind == 0:
        v = [rng.randrange(3) for _ in range(m)]
    elif kind == 1:
        v = [rng.randrange(1 << (8 * S)) for _ in range(m)]
    elif kind == 2:
        v = [int(rng.gauss(0, 2)) & ((1 << (8 * S)) - 1) for _ in range(m)]
    else:  # copies of earlier runs
        v = [rng.randrange(16) for _ in range(m)]
        for _ in range(m // 8):
            L = rng.randrange(2, 40)
            o = rng.randrange(1, 300)
            dst = rng.randrange(0, max(1, m - L))
            for k in range(L):
                if 0 <= dst - o + k < m and dst + k < m:
                    v[dst + k] = v[dst - o + k]
    return b"".join(int(t).to_bytes(S, "little") for t in v) + bytes(rng.randrange(S))


@pytest.mark.parametrize("seed", range(6))
def test_greedy_certificate_and_round_trip(seed):
    rng = random.Random(seed)
    for _ in range(4):
        S = rng.choice([1, 2, 4, 8])
        m = rng.randrange(0, 1500)
        x = _random_input(rng, S, m)
        C = rng.choice([1, 7, 64, 300, 512, 2048])
        W = rng.choice([1, 3, 32, 128, 255, 256])
        MIN = rng.choice([1, 2, 3, 4])
        s = oracle.compress(x, S, C, W, MIN)
        params, chunks = refimpl.tokens(s)  # validates every format rule
        assert params["n"] == len(x)
        syms = _syms_as_ints(x, S)
        for i, toks in enumerate(chunks):
            _greedy_certificate(list(syms[i * C:(i + 1) * C]), toks, W, MIN)
        assert oracle.decompress(s) == x
        assert refimpl.decompress(s) == x
        assert len(s) <= oracle.compress_bound(len(x), S, C, MIN)


@pytest.mark.parametrize("n,S", [(0, 1), (0, 8), (1, 2), (3, 4), (7, 8), (8, 8), (9, 8)])
def test_empty_and_sub_symbol_inputs(n, S):
    x = bytes(range(1, n + 1))
    s = oracle.compress(x, S, 16, 8, 2)
    m = n // S
    N = -(-m // 16)
    assert len(s) == 64 + 8 * N + sum(F + P for F, P in
                                      (struct.unpack_from("<II", s, 64 + 8 * i) for i in range(N)))
    assert s[48:48 + n % S] == x[m * S:]
    assert oracle.decompress(s) == x
    assert refimpl.decompress(s) == x


def test_bound_is_reached_by_worst_cases():
    # The bound never fails on random inputs ...
    for S, MIN in [(1, 1), (1, 2), (2, 1), (4, 2), (8, 3)]:
        x = bytes(random.Random(S).randrange(256) for _ in range(S * 5000))
        assert len(oracle.compress(x, S, 333, 256, MIN)) <= oracle.compress_bound(len(x), S, 333, MIN)
    # ... and is met with equality by its all-literal case: symbols that are
    # all distinct (strictly increasing u32) have no match, so every chunk of
    # c symbols costs ceil(c/8) + 4c bytes.
    x = np.arange(1, 2 * 333 + 57, dtype=np.uint32).tobytes() + b"\x07\x08"
    assert len(oracle.compress(x, 4, 333, 256, 2)) == oracle.compress_bound(len(x), 4, 333, 2)
    # The S = 1, MIN = 1 case prices every token as a 2-byte pointer of length
    # 1. With W = 1 only d = 1 exists and L <= d = 1, so on constant bytes
    # every token after a chunk's first (a literal, the window being empty)
    # is exactly such a pointer: the stream is the bound less one byte per
    # chunk (ragged last chunk included).
    for n, C in [(3000, 1000), (2999, 1000), (1, 7), (64, 8)]:
        x = b"\x5a" * n
        s = oracle.compress(x, 1, C, 1, 1)
        N = -(-n // C)
        assert len(s) == oracle.compress_bound(n, 1, C, 1) - N
        toks = [(L, d) for L, d in oracle.parse_chunk(x[:min(C, n)], 1, 1, 1)]
        assert toks == [(0, 0)] + [(1, 1)] * (min(C, n) - 1)
        assert oracle.decompress(s) == x


def test_out_of_space_reports_required_size():
    x = bytes(range(200)) * 3
    full = oracle.compress(x, 1, 64, 32, 2)
    st, stream, need = oracle.compress_status(x, 1, 64, 32, 2, capacity=len(full) - 1)
    assert st == oracle.ERR_OUT_OF_SPACE and stream is None and need == len(full)
    st, data, need = oracle.decompress_status(full, capacity=len(x) - 1)
    assert st == oracle.ERR_OUT_OF_SPACE and need == len(x)


@pytest.mark.parametrize("S,C,W,MIN", [(3, 8, 8, 2), (2, 0, 8, 2), (2, 8, 0, 2), (2, 8, 257, 2),
                                       (2, 8, 8, 0), (2, 8, 8, 256), (16, 8, 8, 2)])
def test_invalid_parameters(S, C, W, MIN):
    st, _, _ = oracle.compress_status(b"abcd" * 10, S, C, W, MIN)
    assert st == oracle.ERR_INVALID_ARG


def _mutations(s, rng, k):
    for _ in range(k):
        b = bytearray(s)
        op = rng.randrange(4)
        if op == 0:
            i = rng.randrange(len(b))
            b[i] ^= 1 << rng.randrange(8)
        elif op == 1:
            b = b[:rng.randrange(len(b))]
        elif op == 2:
            i = rng.randrange(len(b))
            b[i] = rng.randrange(256)
        else:
            b += bytes([rng.randrange(256)])
        yield bytes(b)


@pytest.mark.parametrize("seed", range(3))
def test_decoder_fuzz_agrees_with_reference(seed):
    rng = random.Random(seed + 100)
    for _ in range(6):
        S = rng.choice([1, 2, 4, 8])
        x = _random_input(rng, S, rng.randrange(0, 300))
        s = oracle.compress(x, S, rng.choice([5, 40, 128]), rng.choice([4, 64, 256]), 2)
        for mut in _mutations(s, rng, 150):
            try:
                ref = refimpl.decompress(mut)
            except refimpl.Corrupt:
                ref = None
            st, got, _ = oracle.decompress_status(mut, capacity=len(x) + 64)
            if ref is None:
                assert st == oracle.ERR_CORRUPT
            elif len(ref) > len(x) + 64:
                assert st == oracle.ERR_OUT_OF_SPACE
            else:
                assert st == oracle.OK and got == ref
