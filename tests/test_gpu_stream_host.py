"""Host-resident inputs streamed through the GPU in blocks: the assembled
stream is byte-identical to the oracle's stream of the whole input (both
match policies), and block-streamed decompression gives the input back."""
import numpy as np
import pytest

import oracle
from paper_2304_07342_amd import stream_host, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("S,C,W,MIN,policy,block", [
    (4, 256, 64, 2, 0, 64 << 10), (2, 1024, 128, 2, 0, 100 << 10),
    (1, 2048, 256, 3, 0, 1 << 20), (8, 100, 32, 1, 0, 8 << 10), (4, 512, 200, 2, 1, 48 << 10)])
def test_blocks_give_the_whole_input_stream(S, C, W, MIN, policy, block):
    x = synth.mixed(1_000_003, S, seed=S * 10 + policy)
    print("host stream", S, C, W, MIN, policy, block, flush=True)
    s = stream_host.compress_host(x, S, C, W, MIN, policy=policy, block_bytes=block)
    assert s.tobytes() == oracle.compress(x, S, C, W, MIN, policy=policy)
    d = stream_host.decompress_host(s, block_bytes=block // 2 + 1)
    assert d.tobytes() == x.tobytes()


@pytest.mark.parametrize("n", [0, 3, 17])
def test_tiny_inputs(n):
    x = synth.uniform_bytes(n, seed=n)
    s = stream_host.compress_host(x, 4, 16, 8, 2, block_bytes=64)
    assert s.tobytes() == oracle.compress(x, 4, 16, 8, 2)
    assert stream_host.decompress_host(s, block_bytes=64).tobytes() == x.tobytes()


def test_pinned_tensor_input_is_copied_from_directly():
    import torch
    x = synth.mixed(600_001, 4, seed=5)
    t = torch.from_numpy(x.view(np.uint8).copy()).pin_memory()
    s = stream_host.compress_host(t, 4, 512, 128, 2, block_bytes=40 << 10, threads=4)
    assert s.tobytes() == oracle.compress(x, 4, 512, 128, 2)
    d = stream_host.decompress_host(torch.from_numpy(s.copy()), block_bytes=70 << 10, threads=3)
    assert d.tobytes() == x.tobytes()


def test_corrupt_record_in_one_block_is_reported():
    from paper_2304_07342_amd import gpulz
    x = synth.mixed(200_000, 4, seed=9)
    s = bytearray(oracle.compress(x, 4, 256, 64, 2))
    N = -(-(x.nbytes // 4) // 256)
    table = np.frombuffer(bytes(s[64:64 + 8 * N]), np.uint32).reshape(N, 2).astype(np.int64)
    k = 150   # a chunk of a later block (32 chunks per block below)
    rec = 64 + 8 * N + int(table[:k].sum())
    s[rec] ^= 0xFF   # its first flag byte: the token kinds no longer fit the payload size
    with pytest.raises(gpulz.GpulzError):
        stream_host.decompress_host(np.frombuffer(bytes(s), np.uint8), block_bytes=32 << 10)


@pytest.mark.parametrize("n,S,C", [(0, 4, 16), (3000, 1, 7), (1_000_003, 4, 256), (4_000_000, 2, 64)])
def test_record_offsets_scan_the_table(n, S, C):
    """gpulz_record_offsets against the running sum of the oracle stream's
    table entries."""
    import torch
    from paper_2304_07342_amd import gpulz
    x = synth.mixed(n, S, seed=n)
    s = np.frombuffer(oracle.compress(x, S, C, 64, 2), np.uint8)
    N = -(-(n // S) // C)
    print("record offsets", n, S, C, N, flush=True)
    sizes = s[64:64 + 8 * N].view(np.uint32).reshape(N, 2).astype(np.uint64).sum(axis=1)
    want = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    table = torch.from_numpy(s[64:64 + 8 * N].copy()).cuda()
    got = torch.full((N + 1,), -1, dtype=torch.int64, device="cuda")
    st = gpulz.gpulz_record_offsets(table.data_ptr(), N, got.data_ptr(),
                                    torch.cuda.current_stream().cuda_stream)
    assert st == gpulz.GPULZ_OK
    assert np.array_equal(got.cpu().numpy().astype(np.uint64), want)
    assert 64 + 8 * N + int(want[-1]) == s.size


def test_record_sizes_must_cover_the_stream():
    """The device scan of a corrupted table no longer ends at the stream's
    end: decompress_host refuses before decoding any block."""
    from paper_2304_07342_amd import gpulz
    x = np.arange(4096, dtype=np.uint32)
    s = bytearray(oracle.compress(x.tobytes(), 4, 256, 64, 2))
    s[64] ^= 1    # first chunk's flag-byte count no longer matches the records
    with pytest.raises(gpulz.GpulzError):
        stream_host.decompress_host(np.frombuffer(bytes(s), np.uint8), block_bytes=4096)
