"""The candidate list of sparse 4- and 8-byte chunks (each of a chunk's
waves lists the candidates of its quarter of the hit bitmap, up to 32, and
runs their searches before the parse): per quarter 0 candidates, 31-32 (at
the limit), 33 and 34 (over it: the chunk then searches in the parse), 79,
and repeats at quarter starts whose candidate pair straddles two quarters;
all byte-equal to the oracle and round-tripped. (The counts follow from the
planted repeats: each makes its even position and the one before it
candidates.)"""
import numpy as np
import pytest

import oracle
from gpu_helpers import gpu_compress, gpu_decompress
from paper_2304_07342_amd import gpulz

pytestmark = pytest.mark.gpu


def _planted(S, C, nchunks, hits_per_quarter, seed):
    """Random symbols (no chance repeat within a window for S >= 4) with
    `h` planted repeats in quarter q of every chunk: symbol p copied from
    p - 5 at even p, which makes p and p - 1 candidates (two per repeat)."""
    rng = np.random.default_rng(seed)
    dt = np.uint32 if S == 4 else np.uint64
    x = rng.integers(0, np.iinfo(dt).max, size=C * nchunks, dtype=dt)
    q = C // 4
    for ch in range(nchunks):
        for quarter, h in enumerate(hits_per_quarter):
            lo = ch * C + quarter * q
            # spread the repeats over the quarter, at even positions, the first
            # at the quarter's start (a pair straddling the previous quarter)
            for k in range(h):
                p = lo + (k * (q // max(1, h))) // 2 * 2
                if p - 5 >= ch * C:
                    x[p] = x[p - 5]
    return x


@pytest.mark.parametrize("S,C", [(4, 4096), (8, 2048)])
@pytest.mark.parametrize("hits", [(0, 0, 0, 0), (16, 16, 16, 16), (18, 0, 16, 3), (0, 17, 0, 0),
                                  (0, 40, 0, 0), (1, 2, 3, 4)])
def test_candidate_list_limits(S, C, hits):
    # more chunks than the split-parse launch takes, so the per-chunk
    # encoder (four waves per chunk) runs
    nchunks = 520
    x = _planted(S, C, nchunks, hits, seed=S * 1000 + sum(hits))
    print("candidate list", S, C, hits, flush=True)
    for W in (256, 7):
        st, s, _, canary = gpu_compress(x, S, C, W, 2)
        assert st == gpulz.GPULZ_OK and canary
        assert s == oracle.compress(x, S, C, W, 2, threads=16)
        st, d, _, canary = gpu_decompress(s, x.nbytes)
        assert st == gpulz.GPULZ_OK and canary and d == x.tobytes()
