"""GPU parity of the dense-chunk parse (1- and 2-byte symbols, MIN <= 2,
one wave per chunk). A chunk whose first bitmap block is mostly hits is
parsed position by position, every position compared once with its whole
window, instead of candidate by candidate. The inputs mix dense segments
(Zipf bytes or Laplace codes, two- and three-symbol alphabets) with
constant and periodic runs, so that tokens whose length the cap L <= d
decides (they are recomputed by the per-column search), the 255 cap, the
window edge at the chunk start, partial dword groups and chunk tails all
occur. Streams must equal the oracle's byte for byte and decode to the
input; the bench-shaped inputs are compared whole with the 16-thread
oracle."""
import numpy as np
import pytest

import oracle
from gpu_helpers import gpu_compress, gpu_decompress
from paper_2304_07342_amd import gpulz, synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def dense_mix(m: int, S: int, seed: int) -> np.ndarray:
    """m S-byte symbols: segments of 50..600 symbols cycling through a dense
    source (Zipf bytes / Laplace codes), a two-symbol alphabet, runs
    (constant and periodic, periods 1..257) and a three-symbol alphabet."""
    rng = np.random.default_rng(seed)
    parts, k, left = [], 0, m
    while left > 0:
        L = min(left, int(rng.integers(50, 600)))
        kind = k % 4
        if kind == 0:
            if S == 1:
                seg = synth.zipf_text(L, seed=seed * 97 + k)
            else:
                seg = synth.laplace_codes(L, seed=seed * 97 + k).view(np.uint8)
        elif kind == 1:
            seg = synth.small_alphabet(L, S, seed * 97 + k, alphabet=2)
        elif kind == 2:
            seg = synth.runs(L, S, seed * 97 + k)
        else:
            seg = synth.small_alphabet(L, S, seed * 97 + k, alphabet=3)
        parts.append(np.asarray(seg, dtype=np.uint8).reshape(-1)[: L * S])
        left -= L
        k += 1
    return np.concatenate(parts)


CASES = [(S, W, MIN, C)
         for S in (1, 2)
         for W in (1, 2, 3, 5, 64, 127, 128, 129, 200, 256)
         for MIN in (1, 2)
         for C in ((1025, 2048, 4096) if S == 1 else (513, 2048, 4096))]


@pytest.mark.parametrize("S,W,MIN,C", CASES)
def test_dense_parse_matches_oracle(S, W, MIN, C):
    saved = gpulz.gpulz_default_params(S)
    gpulz.gpulz_set_default_params(S, saved[0], saved[1], saved[2], 1)
    try:
        m = 3 * C + 37
        x = np.concatenate([dense_mix(m, S, seed=S * 1000 + W * 10 + MIN),
                            np.arange(S - 1, dtype=np.uint8)])  # n mod S = S - 1
        _say("dense", S, W, MIN, C, x.size)
        st, s, _, canary = gpu_compress(x, S, C, W, MIN)
        assert st == gpulz.GPULZ_OK and canary
        assert s == oracle.compress(x, S, C, W, MIN)
        st, d, _, canary = gpu_decompress(s, x.size)
        assert st == gpulz.GPULZ_OK and canary and d == x.tobytes()
    finally:
        gpulz.gpulz_set_default_params(S, *saved)


@pytest.mark.parametrize("kind,S,C,W", [("zipf-u8", 1, 2048, 256), ("zipf-u8", 1, 4096, 128),
                                        ("laplace-u16", 2, 2048, 128),
                                        ("laplace-u16", 2, 4096, 256)])
def test_dense_bench_shapes_whole_stream(kind, S, C, W):
    import torch
    size = 32 << 20
    host = synth.POOL_KINDS[kind][1](size, 11)[:size]
    saved = gpulz.gpulz_default_params(S)
    gpulz.gpulz_set_default_params(S, saved[0], saved[1], saved[2], 1)
    try:
        _say("dense bench shape", kind, C, W)
        x = torch.from_numpy(host).to("cuda")
        s = gpulz.compress(x, S, C, W, 2)
        got = s.cpu().numpy().tobytes()
    finally:
        gpulz.gpulz_set_default_params(S, *saved)
    _say("oracle over 16 threads")
    assert got == oracle.compress(host, S, C, W, 2, threads=16)
    assert torch.equal(gpulz.decompress(s), x)
