"""Single-buffer calls captured in a HIP graph: the LZSS encoder (both the
split-parse path for few chunks and the per-chunk path) and the LZSS ->
Huffman chain, whose Huffman stage reads the LZSS size on the device. Each
graph is replayed several times with new input contents and eager work in
between; every replay must give the oracle's stream."""
import numpy as np
import pytest

import oracle
from paper_2304_07342_amd import gpulz, synth

pytestmark = pytest.mark.gpu


def _fill(t, x):
    import torch
    t.copy_(torch.from_numpy(np.ascontiguousarray(x).view(np.uint8).reshape(-1).copy()).cuda())


@pytest.mark.parametrize("n_sym", [1 << 19, 1 << 22])  # 256 chunks (split parse), 2048 chunks
def test_compress_graph_replays(n_sym):
    import torch
    S, C, W, MIN = 2, 2048, 128, 2
    x = torch.empty(2 * n_sym, dtype=torch.uint8, device="cuda")
    _fill(x, synth.laplace_codes(n_sym, seed=1))
    comp = gpulz.Compressor(x.numel(), S, C, W, MIN)
    comp.compress_async(x)  # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        comp.compress_async(x)
    for rep in range(3):
        src = synth.laplace_codes(n_sym, seed=50 + rep)
        _fill(x, src)
        torch.cuda.synchronize()
        _ = torch.arange(1000, device="cuda").sum().item()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        size, st = comp.result()
        assert st == gpulz.GPULZ_OK
        assert comp.out[:size].cpu().numpy().tobytes() == oracle.compress(src, S, C, W, MIN,
                                                                           threads=8), rep


def test_lz_huffman_chain_graph_replays():
    import torch
    S, C, W, MIN = 2, 2048, 128, 2
    n_sym = 1 << 20
    x = torch.empty(2 * n_sym, dtype=torch.uint8, device="cuda")
    _fill(x, synth.laplace_codes(n_sym, seed=2))
    lz = gpulz.Compressor(x.numel(), S, C, W, MIN)
    hc = gpulz.HuffCompressor(lz.capacity)

    def chain():
        lz.compress_async(x)
        hc.compress_async(lz.out.data_ptr(), lz.capacity, d_nbytes=lz.meta.data_ptr())

    chain()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        chain()
    for rep in range(3):
        src = synth.laplace_codes(n_sym, seed=80 + rep)
        _fill(x, src)
        torch.cuda.synchronize()
        _ = torch.arange(1000, device="cuda").sum().item()
        g.replay()
        torch.cuda.synchronize()
        size, st = hc.result()
        assert st == gpulz.GPULZ_OK
        ref = oracle.huff_compress(oracle.compress(src, S, C, W, MIN, threads=8))
        assert hc.out[:size].cpu().numpy().tobytes() == ref, rep
