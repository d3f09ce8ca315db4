"""GPU parity of the batch entry points: every buffer's stream equals the
oracle's (and the single-buffer path's), errors stay with their buffer, a
captured HIP graph replays correctly with new contents."""
import random

import numpy as np
import pytest

import oracle
from gpu_helpers import gpu_compress, to_device
from paper_2304_07342_amd import gpulz, synth

pytestmark = pytest.mark.gpu

PARAMS = {1: (4096, 128, 2), 2: (2048, 128, 2), 4: (1024, 256, 2), 8: (512, 64, 3)}


def _say(*a):
    print(*a, flush=True)


def _make_batch(seed, nbufs, max_bytes):
    rng = random.Random(seed)
    bufs, widths = [], []
    for b in range(nbufs):
        S = rng.choice([1, 2, 4, 8])
        n = rng.choice([0, 1, 7, rng.randrange(8, max_bytes)])
        bufs.append(synth.mixed(n, S, seed * 1000 + b))
        widths.append(S)
    return bufs, widths


def _expected(x, S, params):
    C, W, MIN = params[S][:3]
    return oracle.compress(x, S, C, W, MIN)


@pytest.mark.parametrize("seed", range(3))
def test_batch_matches_oracle_and_round_trips(seed):
    import torch
    bufs, widths = _make_batch(seed, 40, 60000)
    _say("batch", seed, sum(b.size for b in bufs))
    ins = [to_device(b)[: b.size] for b in bufs]
    bc = gpulz.BatchCompressor(ins, widths, PARAMS)
    bc.run()
    res = bc.results()
    for x, S, (st, s) in zip(bufs, widths, res):
        assert st == gpulz.GPULZ_OK
        assert s.cpu().numpy().tobytes() == _expected(x, S, PARAMS)
    # batch decompress of the batch's own streams
    bd = gpulz.BatchDecompressor([s for _, s in res], [b.size for b in bufs])
    bd.run()
    for x, (st, d) in zip(bufs, bd.results()):
        assert st == gpulz.GPULZ_OK and d.cpu().numpy().tobytes() == x.tobytes()
    torch.cuda.synchronize()


def test_batch_equals_single_buffer_path():
    bufs, widths = _make_batch(7, 12, 90000)
    ins = [to_device(b)[: b.size] for b in bufs]
    bc = gpulz.BatchCompressor(ins, widths, PARAMS)
    bc.run()
    for x, S, (st, s) in zip(bufs, widths, bc.results()):
        C, W, MIN = PARAMS[S]
        st1, s1, _, _ = gpu_compress(x, S, C, W, MIN)
        assert st == st1 == gpulz.GPULZ_OK and s.cpu().numpy().tobytes() == s1


def test_batch_default_params():
    bufs, widths = _make_batch(11, 8, 40000)
    ins = [to_device(b)[: b.size] for b in bufs]
    bc = gpulz.BatchCompressor(ins, widths, None)
    bc.run()
    for x, S, (st, s) in zip(bufs, widths, bc.results()):
        C, W, MIN, _ = gpulz.gpulz_default_params(S)
        assert st == gpulz.GPULZ_OK and s.cpu().numpy().tobytes() == oracle.compress(x, S, C, W, MIN)


def test_batch_errors_stay_with_their_buffer():
    import torch
    bufs, widths = _make_batch(3, 10, 30000)
    widths[2] = 3                         # invalid symbol width
    ins = [to_device(b)[: b.size] for b in bufs]
    bc = gpulz.BatchCompressor(ins, widths, PARAMS)
    small = 4 if bufs[5].size < 64 else 5
    bc.d_out_caps[small] = 10                    # too small for any stream
    bc.outputs[small].fill_(0xA5)
    bc.run()
    res = bc.results()
    assert res[2][0] == gpulz.GPULZ_ERR_INVALID_ARG
    assert res[small][0] == gpulz.GPULZ_ERR_OUT_OF_SPACE
    assert bool((bc.outputs[small] == 0xA5).all())
    for i, (x, S, (st, s)) in enumerate(zip(bufs, widths, res)):
        if i in (2, small):
            continue
        assert st == gpulz.GPULZ_OK and s.cpu().numpy().tobytes() == _expected(x, S, PARAMS)
    torch.cuda.synchronize()


def test_batch_graph_replays_with_new_contents():
    import torch
    bufs, widths = _make_batch(21, 16, 50000)
    ins = [to_device(b)[: b.size] for b in bufs]
    bc = gpulz.BatchCompressor(ins, widths, PARAMS)
    bc.capture()
    for rep in range(3):
        new = [synth.mixed(b.size, S, 777 + rep * 100 + i) for i, (b, S) in enumerate(zip(bufs, widths))]
        for t, x in zip(ins, new):
            if x.size:
                t.copy_(torch.from_numpy(x.copy()).cuda())
        torch.cuda.synchronize()
        _ = torch.arange(1000, device="cuda").sum().item()  # eager work between replays
        bc.replay()
        torch.cuda.synchronize()
        for x, S, (st, s) in zip(new, widths, bc.results()):
            assert st == gpulz.GPULZ_OK
            assert s.cpu().numpy().tobytes() == _expected(x, S, PARAMS), rep


def test_batch_decompress_isolates_corrupt_stream():
    import torch
    bufs, widths = _make_batch(31, 8, 20000)
    streams = [_expected(x, S, PARAMS) for x, S in zip(bufs, widths)]
    bad = bytearray(streams[3])
    bad[16] ^= 0x40                                   # header field n
    streams[3] = bytes(bad)
    dev = [to_device(np.frombuffer(s, dtype=np.uint8))[: len(s)] for s in streams]
    bd = gpulz.BatchDecompressor(dev, [b.size + 64 for b in bufs])
    bd.run()
    res = bd.results()
    for i, (x, (st, d)) in enumerate(zip(bufs, res)):
        if i == 3:
            assert st == gpulz.GPULZ_ERR_CORRUPT
        else:
            assert st == gpulz.GPULZ_OK and d.cpu().numpy().tobytes() == x.tobytes()
    torch.cuda.synchronize()


def test_batch_large_buffers_span_many_chunks():
    # a few buffers of several MB next to tiny ones (load balance at chunk grain)
    rng = random.Random(5)
    bufs, widths = [], []
    for b in range(12):
        S = [1, 2, 4, 8][b % 4]
        n = rng.choice([3 << 20, 100, 5000, 1 << 20])
        bufs.append(synth.mixed(n, S, 900 + b))
        widths.append(S)
    ins = [to_device(b)[: b.size] for b in bufs]
    bc = gpulz.BatchCompressor(ins, widths, PARAMS)
    bc.run()
    for x, S, (st, s) in zip(bufs, widths, bc.results()):
        assert st == gpulz.GPULZ_OK and s.cpu().numpy().tobytes() == _expected(x, S, PARAMS)


# Every waves-per-chunk setting (1, 2 or 4 wavefronts per chunk encoder) for
# every width, passed explicitly: the bytes are the oracle's.
@pytest.mark.parametrize("waves", [1, 2, 4])
def test_batch_explicit_waves_match_oracle(waves):
    bufs, widths = _make_batch(40 + waves, 24, 70000)
    params = {S: tuple(PARAMS[S]) + (waves,) for S in PARAMS}
    _say("batch waves", waves)
    ins = [to_device(b)[: b.size] for b in bufs]
    bc = gpulz.BatchCompressor(ins, widths, params)
    bc.run()
    for x, S, (st, s) in zip(bufs, widths, bc.results()):
        assert st == gpulz.GPULZ_OK
        assert s.cpu().numpy().tobytes() == _expected(x, S, PARAMS), (S, x.size, waves)
