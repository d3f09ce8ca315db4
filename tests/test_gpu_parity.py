"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer work: streams must match byte for byte, decoded data exactly.
"""
import random
import struct

import numpy as np
import pytest

import oracle
from golden import all_vectors
from gpu_helpers import gpu_compress, gpu_decompress
from paper_2304_07342_amd import gpulz, synth

pytestmark = pytest.mark.gpu

VECTORS = all_vectors()


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("v", VECTORS, ids=[v["name"] for v in VECTORS])
def test_hand_vectors(v):
    _say("hand vector", v["name"])
    st, s, _, canary = gpu_compress(v["input"], v["S"], v["C"], v["W"], v["MIN"])
    assert st == gpulz.GPULZ_OK and canary
    assert s == oracle.compress(v["input"], v["S"], v["C"], v["W"], v["MIN"])
    st, d, n, canary = gpu_decompress(s, len(v["input"]))
    assert st == gpulz.GPULZ_OK and canary and d == v["input"]


def _random_case(seed):
    rng = random.Random(seed)
    S = rng.choice([1, 2, 4, 8])
    C = rng.choice([1, 7, 64, 100, 512, 2048, 4096])
    W = rng.choice([1, 2, 63, 64, 65, 128, 200, 255, 256])
    MIN = rng.choice([1, 2, 2, 3, 8])
    n = rng.choice([0, 1, 5, 17, 1000, 30000, 100000, 150001])
    x = synth.mixed(n, S, seed)
    return x, S, C, W, MIN


@pytest.mark.parametrize("seed", range(40))
def test_random_parity_and_round_trip(seed):
    x, S, C, W, MIN = _random_case(seed)
    _say("random case", seed, "n", x.size, "S", S, "C", C, "W", W, "MIN", MIN)
    st, s, _, canary = gpu_compress(x, S, C, W, MIN)
    assert st == gpulz.GPULZ_OK and canary
    ref = oracle.compress(x, S, C, W, MIN)
    assert len(s) == len(ref)
    assert s == ref
    st, d, n, canary = gpu_decompress(s, x.size)
    assert st == gpulz.GPULZ_OK and canary and d == x.tobytes()


@pytest.mark.parametrize("S", [1, 2, 4, 8])
@pytest.mark.parametrize("W", [1, 64, 129, 256])
def test_runs_and_caps(S, W):
    # long constant and periodic runs: 255 cap, length <= offset, offset 256
    x = synth.runs(40000 // S, S, seed=S * 1000 + W)
    _say("runs", S, W)
    for C in (1000, 4096 // S * 4):
        st, s, _, _ = gpu_compress(x, S, C, W, 2)
        assert st == gpulz.GPULZ_OK
        assert s == oracle.compress(x, S, C, W, 2)
        st, d, _, _ = gpu_decompress(s, x.size)
        assert st == gpulz.GPULZ_OK and d == x.tobytes()


@pytest.mark.parametrize("S", [1, 2, 4, 8])
def test_largest_chunk(S):
    C = 48 * 1024 // S
    x = synth.mixed(3 * C * S + 7, S, seed=S)
    _say("largest chunk", S, C)
    st, s, _, _ = gpu_compress(x, S, C, 256, 2)
    assert st == gpulz.GPULZ_OK and s == oracle.compress(x, S, C, 256, 2)
    st, d, _, _ = gpu_decompress(s, x.size)
    assert st == gpulz.GPULZ_OK and d == x.tobytes()


def test_codes_1mib_full():
    cfg = synth.WORKLOADS[synth.CODES_1MIB]
    x = cfg["make"]()
    _say("codes 1 MiB")
    st, s, _, _ = gpu_compress(x, cfg["S"], cfg["C"], cfg["W"], cfg["MIN"])
    assert st == gpulz.GPULZ_OK
    assert s == oracle.compress(x, cfg["S"], cfg["C"], cfg["W"], cfg["MIN"])
    st, d, _, _ = gpu_decompress(s, x.nbytes)
    assert st == gpulz.GPULZ_OK and d == x.tobytes()


def test_field_256mib_full_stream():
    """256 MiB float32 field at full size with the benchmark's parameters and
    launch: the whole stream (all 16,384 chunks) equals the oracle's, computed
    over 16 threads, and the GPU round trip is exact."""
    import torch
    cfg = synth.WORKLOADS[synth.FIELD_256MIB]
    S, C, W, MIN = cfg["S"], cfg["C"], cfg["W"], cfg["MIN"]
    x = cfg["make"]().view(np.uint8).reshape(-1)
    _say("field 256 MiB")
    c = gpulz.Compressor(x.size, S, C, W, MIN)
    d_in = torch.from_numpy(x).cuda()
    c.compress_async(d_in)
    size, status = c.result()
    assert status == gpulz.GPULZ_OK
    s = c.out[:size].cpu().numpy().tobytes()
    _say("field 256 MiB: oracle over 16 threads")
    ref = oracle.compress(x, S, C, W, MIN, threads=16)
    assert len(s) == len(ref)
    if s != ref:
        a = np.frombuffer(s, dtype=np.uint8)
        b = np.frombuffer(ref, dtype=np.uint8)
        first = int(np.flatnonzero(a != b)[0])
        raise AssertionError(f"stream differs from the oracle first at byte {first}")
    d = gpulz.decompress(c.out[:size])
    assert torch.equal(d, d_in)


@pytest.mark.parametrize("n,S", [(0, 1), (0, 8), (1, 2), (3, 4), (7, 8), (9, 8), (4097, 4)])
def test_tiny_and_ragged(n, S):
    x = synth.mixed(n, S, seed=n + S)
    _say("tiny", n, S)
    st, s, _, _ = gpu_compress(x, S, 1024, 64, 2)
    assert st == gpulz.GPULZ_OK and s == oracle.compress(x, S, 1024, 64, 2)
    st, d, _, _ = gpu_decompress(s, max(n, 0))
    assert st == gpulz.GPULZ_OK and d == x.tobytes()


# OUT_OF_SPACE: the required size is reported and no byte at or past the
# capacity is written, for capacities from the header alone up to one byte
# short, on both encoders (split parse with few chunks, per-chunk otherwise),
# and for an input of no chunk at all.
@pytest.mark.parametrize("n,C", [(50000, 512), (600000, 256)])
def test_compress_out_of_space_writes_nothing_past_capacity(n, C):
    x = synth.mixed(n, 2, seed=5)
    ref = oracle.compress(x, 2, C, 128, 2)
    N = -(-(n // 2) // C)
    for cap in (0, 63, 64, 64 + 8 * N - 1, 64 + 8 * N + 100, len(ref) // 2, len(ref) - 1):
        _say("out of space", n, C, cap)
        st, s, need, canary = gpu_compress(x, 2, C, 128, 2, capacity=cap)
        assert st == gpulz.GPULZ_ERR_OUT_OF_SPACE and need == len(ref) and canary, cap
    st, s, need, canary = gpu_compress(x, 2, C, 128, 2, capacity=len(ref))
    assert st == gpulz.GPULZ_OK and s == ref and canary
    st, s, need, canary = gpu_compress(x[:1], 2, C, 128, 2, capacity=63)
    assert st == gpulz.GPULZ_ERR_OUT_OF_SPACE and need == 64 and canary


def test_decompress_out_of_space():
    x = synth.mixed(20000, 4, seed=6)
    s = oracle.compress(x, 4, 512, 128, 2)
    st, d, n, canary = gpu_decompress(s, x.size - 1)
    assert st == gpulz.GPULZ_ERR_OUT_OF_SPACE and n == x.size and canary


def test_deterministic_repeats():
    x = synth.mixed(300000, 4, seed=11)
    _say("determinism")
    outs = {gpu_compress(x, 4, 2048, 256, 2)[1] for _ in range(3)}
    assert len(outs) == 1


def _mutations(s, rng, k):
    for _ in range(k):
        b = bytearray(s)
        op = rng.randrange(3)
        if op == 0:
            i = rng.randrange(len(b))
            b[i] ^= 1 << rng.randrange(8)
        elif op == 1:
            b = b[:rng.randrange(len(b))]
        else:
            i = rng.randrange(64, len(b))
            b[i] = rng.randrange(256)
        yield bytes(b)


@pytest.mark.parametrize("seed", range(3))
def test_decoder_rejects_what_the_oracle_rejects(seed):
    rng = random.Random(seed)
    S = [1, 2, 4][seed]
    x = synth.mixed(3000, S, seed=seed + 50)
    s = oracle.compress(x, S, 256, 64, 2)
    _say("decoder fuzz", seed)
    for mut in _mutations(s, rng, 60):
        cap = x.size + 64
        ost, odata, _ = oracle.decompress_status(mut, capacity=cap)
        gst, gdata, _, canary = gpu_decompress(mut, cap)
        assert canary
        # the oracle's status codes use the library's numbering: the two must
        # give the same verdict (OK, CORRUPT or OUT_OF_SPACE)
        assert gst == ost
        if ost == oracle.OK:
            assert gdata == odata


# Chunks beyond the workgroup decoder's limits (more than 4096 symbols, or
# more than 16 KiB) are decoded one wavefront per chunk; fuzz that path too.
@pytest.mark.parametrize("S,C", [(1, 6000), (4, 4500)])
def test_wave_decoder_rejects_what_the_oracle_rejects(S, C):
    rng = random.Random(S * 7 + C)
    x = synth.mixed(3 * C * S // 2, S, seed=S + 90)
    s = oracle.compress(x, S, C, 200, 2)
    _say("wave decoder fuzz", S, C)
    st, d, _, canary = gpu_decompress(s, x.size)
    assert st == gpulz.GPULZ_OK and canary and d == x.tobytes()
    for mut in _mutations(s, rng, 40):
        cap = x.size + 64
        ost, odata, _ = oracle.decompress_status(mut, capacity=cap)
        gst, gdata, _, canary = gpu_decompress(mut, cap)
        assert canary
        # the oracle's status codes use the library's numbering: the two must
        # give the same verdict (OK, CORRUPT or OUT_OF_SPACE)
        assert gst == ost
        if ost == oracle.OK:
            assert gdata == odata


# 70000 symbols at C = 64 are 1094 chunks, more than the split-parse launch
# takes (1024 for S <= 2, 512 for S >= 4), so the per-chunk encoder runs with
# each waves-per-chunk setting; every result is compared with the oracle.
@pytest.mark.parametrize("S", [1, 2, 4, 8])
def test_waves_per_chunk_does_not_change_bytes(S):
    n_sym, C = 70000, 64
    x = synth.mixed(n_sym * S, S, seed=S + 40)
    assert -(-n_sym // C) > 1024
    saved = gpulz.gpulz_default_params(S)
    try:
        for W, MIN in ((200, 2), (64, 1)):
            ref = oracle.compress(x, S, C, W, MIN)
            for w in (1, 2, 4):
                _say("waves", S, W, MIN, w)
                gpulz.gpulz_set_default_params(S, saved[0], saved[1], saved[2], w)
                st, s, _, canary = gpu_compress(x, S, C, W, MIN)
                assert st == gpulz.GPULZ_OK and canary and s == ref, (S, W, MIN, w)
    finally:
        gpulz.gpulz_set_default_params(S, *saved)


def _repetitive(n_sym, S, seed):
    """Long periodic runs (matches that cross many 1/16-chunk segments), broken
    by random symbols."""
    rng = np.random.default_rng(seed)
    period = rng.integers(1, 40, size=1)[0]
    base = rng.integers(0, 256, size=(period, S), dtype=np.uint8)
    x = np.tile(base, (n_sym // period + 1, 1))[:n_sym].copy()
    noise = rng.random(n_sym) < 0.01
    x[noise] = rng.integers(0, 256, size=(int(noise.sum()), S), dtype=np.uint8)
    return x.reshape(-1)


# Launches with few chunks split each chunk's parse across 16 waves: segments
# of a chunk with C < 16 are partly empty, long pointers cross several
# segments, and chunk counts on either side of the launch rule take the two
# encoders; all must give the oracle's stream.
@pytest.mark.parametrize("S,C,n_sym,kind", [
    (1, 1, 500, "mixed"), (2, 3, 700, "rep"), (4, 15, 1200, "rep"), (8, 16, 800, "mixed"),
    (1, 17, 5000, "rep"), (2, 100, 20000, "rep"), (2, 4096, 30000, "rep"), (1, 4096, 60000, "mixed"),
    (2, 64, 1024 * 64, "mixed"), (2, 64, 1025 * 64, "mixed"), (4, 64, 512 * 64, "rep"),
    (4, 64, 513 * 64, "rep"), (8, 4096, 3 * 4096 + 5, "rep")])
def test_split_parse_matches_oracle(S, C, n_sym, kind):
    x = _repetitive(n_sym, S, C + n_sym) if kind == "rep" else synth.mixed(n_sym * S, S, C)
    for W, MIN in ((256, 2), (37, 1), (64, 3)):
        _say("split parse", S, C, n_sym, kind, W, MIN)
        st, s, _, canary = gpu_compress(x, S, C, W, MIN)
        assert st == gpulz.GPULZ_OK and canary
        assert s == oracle.compress(x, S, C, W, MIN)
        st, d, n, canary = gpu_decompress(s, x.size)
        assert st == gpulz.GPULZ_OK and canary and d == x.tobytes()


# Chunks without a pointer take a shortcut in the workgroup decoder (the
# payload is the chunk). Random symbols with a long minimum match give such
# chunks at every record alignment; the record sizes, flags and payloads
# are then mutated and every verdict compared with the oracle's.
@pytest.mark.parametrize("S,C,W,MIN", [(1, 250, 16, 6), (2, 300, 64, 2), (4, 256, 64, 2),
                                       (8, 100, 32, 2)])
def test_literal_only_chunks(S, C, W, MIN):
    rng = random.Random(S * 131 + C)
    n = 7 * C + C // 3
    x = synth.uniform_bytes(n * S, seed=S + 300)
    s = oracle.compress(x, S, C, W, MIN)
    N = (n + C - 1) // C
    lit_only = 64 + 8 * N + sum((min(C, n - i * C) + 7) // 8 + min(C, n - i * C) * S for i in range(N))
    assert len(s) == lit_only  # no pointer anywhere
    _say("literal-only chunks", S, C)
    st, d, _, canary = gpu_decompress(s, x.size)
    assert st == gpulz.GPULZ_OK and canary and d == x.tobytes()
    muts = list(_mutations(s, rng, 30))
    for k in range(N):  # each table entry's F or P off by one
        for field, delta in ((0, 1), (0, -1), (4, 1), (4, -1)):
            b = bytearray(s)
            off = 64 + 8 * k + field
            v = struct.unpack_from("<I", b, off)[0]
            struct.pack_into("<I", b, off, (v + delta) & 0xFFFFFFFF)
            muts.append(bytes(b))
        # size moves that keep the table's sum: flag bytes <-> payload bytes in
        # one entry, and payload bytes between neighbouring entries
        moves = [((64 + 8 * k, 1), (68 + 8 * k, -1)), ((64 + 8 * k, -1), (68 + 8 * k, 1))]
        if k + 1 < N:
            moves += [((68 + 8 * k, 1), (68 + 8 * k + 8, -1)), ((68 + 8 * k, -1), (68 + 8 * k + 8, 1))]
        for (o1, d1), (o2, d2) in moves:
            b = bytearray(s)
            for off, delta in ((o1, d1), (o2, d2)):
                v = struct.unpack_from("<I", b, off)[0]
                struct.pack_into("<I", b, off, (v + delta) & 0xFFFFFFFF)
            muts.append(bytes(b))
    for mut in muts:
        cap = x.size + 64
        ost, odata, _ = oracle.decompress_status(mut, capacity=cap)
        gst, gdata, _, canary = gpu_decompress(mut, cap)
        assert canary
        # the oracle's status codes use the library's numbering: the two must
        # give the same verdict (OK, CORRUPT or OUT_OF_SPACE)
        assert gst == ost
        if ost == oracle.OK:
            assert gdata == odata


# The exact search for 1- and 2-byte symbols (equality steps over offset
# masks, lengths from the last step) on the inputs that stress it: two- and
# three-symbol alphabets, constant and periodic runs, windows on both sides of
# each 64-offset column, lengths near the 255 cap and chunk ends, both the
# split-parse launch (few chunks) and the one-wave launch (many chunks).
def test_narrow_symbol_search_against_oracle():
    rng = random.Random(2024)
    cases = []
    for k in range(120):
        S = rng.choice([1, 2])
        C = rng.choice([1, 7, 64, 100, 257, 1000, 2048, 4096])
        W = rng.choice([1, 2, 3, 4, 5, 31, 63, 64, 65, 127, 128, 129, 200, 255, 256])
        MIN = rng.choice([1, 2, 3, 4, 7])
        cases.append((S, C, W, MIN, rng.randint(1, 6000), k))
    for k in range(4):  # more than 1024 chunks: the one-wave launch
        cases.append((1 + k % 2, 64, rng.choice([63, 64, 65, 256]), 2, 70000, 500 + k))
    for S, C, W, MIN, m, seed in cases:
        kind = seed % 4
        if kind == 0:
            x = synth.small_alphabet(m, S, seed=seed, alphabet=2)
        elif kind == 1:
            x = synth.small_alphabet(m, S, seed=seed, alphabet=3)
        elif kind == 2:
            x = synth.runs(m, S, seed=seed)
        else:
            x = synth.mixed(m * S, S, seed=seed)
        _say("narrow search", S, C, W, MIN, x.size, seed)
        ref = oracle.compress(x, S, C, W, MIN)
        st, s, _, canary = gpu_compress(x, S, C, W, MIN)
        assert st == gpulz.GPULZ_OK and canary and s == ref, (S, C, W, MIN, seed)
        dst, d, _, canary = gpu_decompress(s, x.size)
        assert dst == gpulz.GPULZ_OK and canary and d == np.ascontiguousarray(x).tobytes()
