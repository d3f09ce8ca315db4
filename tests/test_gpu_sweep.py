"""GPU parity on the symbol-width sweep: 1 GiB per width (Zipf bytes, uint16
Laplace codes, sorted uint32 indices, the float64 field), each compressed at
the (C, W, waves per chunk) the autotuner picks on its first 64 MiB.

Chunks are independent (section 3.3.1), so a sampled chunk's table entry and
record are checked against the oracle run on that chunk alone; the two
literal-dominated inputs (sorted indices and the float64 field) are checked
against the oracle's whole stream. Every input round-trips exactly.
"""
import struct

import numpy as np
import pytest

import oracle
from paper_2304_07342_amd import autotune, gpulz, synth

pytestmark = pytest.mark.gpu

SIZE = 1 << 30
KINDS = {1: "zipf-u8", 2: "laplace-u16", 4: "sorted-u32", 8: "field-f64"}
FULL_ORACLE = {4, 8}
SAMPLED_CHUNKS = 64


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("S", [1, 2, 4, 8])
def test_sweep_width_at_autotuned_parameters(S):
    import torch
    kind = KINDS[S]
    _say("sweep", kind, "generating 1 GiB")
    host = synth.POOL_KINDS[kind][1](SIZE, 200 + S)[:SIZE]
    x = torch.from_numpy(host).to("cuda")
    saved = gpulz.gpulz_default_params(S)
    try:
        tuned = autotune.tune_width(x[: 64 << 20], S, reps=1)
        C, W, MIN, waves = (tuned["chunk_symbols"], tuned["window"], tuned["min_match"],
                            tuned["waves_per_chunk"])
        _say("sweep", kind, "autotuned C", C, "W", W, "waves", waves)
        autotune.apply({S: tuned})  # the single-buffer call runs with these waves
        comp = gpulz.Compressor(SIZE, S, C, W, MIN)
        comp.compress_async(x)
        size, status = comp.result()
    finally:
        gpulz.gpulz_set_default_params(S, *saved)
    assert status == gpulz.GPULZ_OK
    s = comp.out[:size].cpu().numpy().tobytes()
    n, SS, total = gpulz.gpulz_peek_header(s[:64])
    assert (n, SS, total) == (SIZE, S, len(s))
    N = -(-(SIZE // S) // C)
    table = np.frombuffer(s, dtype=np.uint32, count=2 * N, offset=64).reshape(N, 2)
    offs = 64 + 8 * N + np.concatenate([[0], np.cumsum(table.sum(axis=1).astype(np.int64))])
    assert offs[-1] == len(s)
    if S in FULL_ORACLE:
        _say("sweep", kind, "whole stream against the oracle over 16 threads")
        ref = oracle.compress(host, S, C, W, MIN, threads=16)
        assert s == ref
    else:
        rng = np.random.default_rng(S)
        sample = sorted(set(rng.choice(N, size=SAMPLED_CHUNKS - 2, replace=False).tolist())
                        | {0, N - 1})
        _say("sweep", kind, len(sample), "sampled chunks against the oracle")
        for i in sample:
            chunk = host[i * C * S:(i + 1) * C * S]
            ref = oracle.compress(chunk, S, C, W, MIN)
            F, P = struct.unpack_from("<II", ref, 64)
            assert (F, P) == tuple(table[i]), i
            assert s[offs[i]:offs[i + 1]] == ref[72:72 + F + P], i
    _say("sweep", kind, "round trip")
    d = gpulz.decompress(comp.out[:size])
    assert torch.equal(d, x)
    del x, comp, d
    torch.cuda.empty_cache()
