"""Block planning for host-resident streaming (CPU only): blocks tile the
input, start on chunk boundaries, and only the last holds the tail."""
import pytest

from paper_2304_07342_amd import stream_host


@pytest.mark.parametrize("n,S,C,bb", [(0, 1, 16, 64), (3, 4, 2, 8), (10, 4, 2, 8),
                                      (1000003, 4, 100, 40000), (65536, 2, 4096, 8192),
                                      (12345, 8, 7, 1)])
def test_blocks_tile_the_input_on_chunk_boundaries(n, S, C, bb):
    blocks = stream_host.block_plan(n, S, C, bb)
    assert sum(b for _, b, _, _ in blocks) == n
    pos, chunk = 0, 0
    for i, (off, nb, c0, nc) in enumerate(blocks):
        assert off == pos and c0 == chunk
        if i + 1 < len(blocks):
            assert nb == nc * C * S and nc >= 1
        pos += nb
        chunk += nc
    assert chunk == -(-(n // S) // C)


@pytest.mark.parametrize("n,S,C,W,MIN,policy", [
    (0, 4, 16, 8, 2, 0), (3, 4, 16, 8, 2, 0), (10, 4, 2, 8, 2, 1), (100003, 8, 100, 32, 1, 0),
    (65537, 2, 1024, 128, 2, 0), (5000, 1, 256, 256, 3, 1)])
def test_library_header_is_the_oracles(n, S, C, W, MIN, policy):
    """gpulz_write_header against the header of the oracle's stream of the
    same input (the oracle writes its own), and gpulz_read_header back."""
    import numpy as np
    import oracle
    from paper_2304_07342_amd import gpulz
    x = np.random.default_rng(n).integers(0, 4, size=n, dtype=np.uint8)
    s = oracle.compress(x.tobytes(), S, C, W, MIN, policy=policy)
    tail = x[n - n % S:].tobytes()
    assert gpulz.gpulz_write_header(n, S, C, W, MIN, policy, len(s), tail) == s[:64]
    info = gpulz.gpulz_read_header(s[:64])
    assert (info.nbytes, info.symbol_bytes, info.chunk_symbols, info.window, info.min_match,
            info.match_policy, info.stream_bytes) == (n, S, C, W, MIN, policy, len(s))
    assert info.chunks == -(-(n // S) // C) and bytes(info.tail[:info.tail_bytes]) == tail
    assert gpulz.gpulz_table_offset(info.chunks) == 64 + 8 * info.chunks


def test_read_header_rejects_what_the_decoder_rejects():
    import oracle
    from paper_2304_07342_amd import gpulz
    h = bytearray(oracle.compress(bytes(range(200)) * 5, 2, 64, 32, 2)[:64])
    assert gpulz.gpulz_read_header(bytes(h)).chunks == 8
    for at, v in [(0, ord("X")), (4, 2), (6, 3), (7, 2), (15, 7), (24, 9), (40, 1), (44, 1),
                  (60, 1)]:
        bad = bytearray(h)
        bad[at] = v
        with pytest.raises(gpulz.GpulzError):
            gpulz.gpulz_read_header(bytes(bad))
    with pytest.raises(gpulz.GpulzError):
        gpulz.gpulz_write_header(10, 3, 16, 8, 2, 0, 100)   # S = 3
    with pytest.raises(gpulz.GpulzError):
        gpulz.gpulz_write_header(10, 4, 16, 8, 2, 0, 70)    # smaller than header + table
