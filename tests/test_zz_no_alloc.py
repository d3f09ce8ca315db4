"""gpulz_decompress_noalloc (the decompression for callers that cannot
allocate) against gpulz_decompress on the same streams, through the C ABI:
two calls in a row on the same GPU, the second with a smaller stream, each
checked byte for byte (integer work: identical outputs, sizes and
statuses), plus a corrupted stream (same verdict) and the size limit."""
import numpy as np
import pytest

import oracle
from gpu_helpers import to_device
from paper_2304_07342_amd import gpulz, synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _run(fn_noalloc, stream_bytes: bytes, capacity: int):
    import torch
    s = to_device(np.frombuffer(stream_bytes, dtype=np.uint8))
    n = len(stream_bytes)
    out = torch.full((capacity + 64,), 0xA5, dtype=torch.uint8, device="cuda")
    meta = torch.zeros(2, dtype=torch.int64, device="cuda")
    cs = torch.cuda.current_stream().cuda_stream
    if fn_noalloc:
        st = gpulz.gpulz_decompress_noalloc(s.data_ptr(), n, out.data_ptr(), capacity,
                                            meta.data_ptr(), meta.data_ptr() + 8, cs)
    else:
        ws_bytes = gpulz.gpulz_decompress_workspace_size(n)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        st = gpulz.gpulz_decompress(s.data_ptr(), n, out.data_ptr(), capacity, meta.data_ptr(),
                                    meta.data_ptr() + 8, ws.data_ptr(), ws_bytes, cs)
    assert st == gpulz.GPULZ_OK, gpulz.status_string(st)
    torch.cuda.synchronize()
    m = meta.cpu().numpy()
    return int(m[0]), int(m[1]) & 0xFFFFFFFF, out.cpu().numpy().tobytes()


def test_noalloc_matches_decompress_two_calls():
    big = synth.laplace_codes(3 << 20, seed=5).view(np.uint8)       # 6 MiB, 1536 chunks
    small = synth.zipf_text(300_001, seed=6)                          # ragged, fewer chunks
    cases = [(big, 2, 2048, 128), (small, 1, 4096, 255)]
    for x, S, C, W in cases:
        s = oracle.compress(x, S, C, W, 2)
        _say("noalloc", x.size, len(s))
        got = _run(True, s, x.size)
        ref = _run(False, s, x.size)
        assert got == ref
        assert got[0] == x.size and got[1] == gpulz.GPULZ_OK
        assert got[2][:x.size] == x.tobytes()


def test_noalloc_corrupt_and_capacity_verdicts():
    x = synth.laplace_codes(1 << 16, seed=7).view(np.uint8)
    s = bytearray(oracle.compress(x, 2, 2048, 128, 2))
    # a table entry that no longer sums to the stream size
    s[64] ^= 1
    got = _run(True, bytes(s), x.size)
    ref = _run(False, bytes(s), x.size)
    assert got[:2] == ref[:2] and got[1] == gpulz.GPULZ_ERR_CORRUPT
    s[64] ^= 1
    got = _run(True, bytes(s), x.size - 1)
    ref = _run(False, bytes(s), x.size - 1)
    assert got[:2] == ref[:2] and got[1] == gpulz.GPULZ_ERR_OUT_OF_SPACE


def test_noalloc_rejects_streams_over_the_limit():
    # checked on the host before anything is launched
    st = gpulz.gpulz_decompress_noalloc(0x1000, (1 << 30) + 1, 0x1000, 1, 0x1000, 0x1008, 0)
    assert st == gpulz.GPULZ_ERR_WORKSPACE
