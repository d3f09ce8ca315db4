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


def test_header_layout():
    h = stream_host.header(10, 4, 2, 8, 2, 1, 1, 99, b"\x01\x02")
    assert len(h) == 64 and h[:4] == b"GLZ1" and h[6] == 4 and h[7] == 1 and h[40] == 2
    assert h[48:50] == b"\x01\x02" and h[50:] == bytes(14)


def test_record_sizes_must_cover_the_stream():
    import numpy as np
    import oracle
    from paper_2304_07342_amd import gpulz
    x = np.arange(4096, dtype=np.uint32)
    s = bytearray(oracle.compress(x.tobytes(), 4, 256, 64, 2))
    s[64] ^= 1    # first chunk's flag-byte count no longer matches the records
    with pytest.raises(gpulz.GpulzError):
        stream_host.decompress_host(np.frombuffer(bytes(s), np.uint8), block_bytes=4096)
