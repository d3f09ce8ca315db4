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
