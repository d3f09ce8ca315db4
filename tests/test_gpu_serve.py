"""Serving on the GPU: every result produced in the mix of a continuous-
batching run equals the same request run alone (byte for byte), and every
compress result equals the oracle's stream for its bytes and parameters; the
plain backend (one gpulz_compress / gpulz_decompress per request, same
admission) gives the same results for the same trace."""
import numpy as np
import pytest

import oracle
from gpu_helpers import to_device
from paper_2304_07342_amd import gpulz, serve, synth

pytestmark = pytest.mark.gpu


def _setup(rng):
    rng = np.random.default_rng(9)
    pools = {k: to_device(g(4 << 20, 300 + i))[: 4 << 20]
             for i, (k, (S, g)) in enumerate(synth.POOL_KINDS.items())}
    # decompress sources: a few prepared streams
    streams, origs = [], []
    for j in range(6):
        S = [1, 2, 4, 8][j % 4]
        x = synth.mixed(int(rng.integers(1000, 300000)), S, 500 + j)
        C, W, MIN, _ = gpulz.gpulz_default_params(S)
        s = oracle.compress(x, S, C, W, MIN)
        streams.append((to_device(np.frombuffer(s, dtype=np.uint8))[: len(s)], x.size))
        origs.append(x)
    trace = serve.make_trace(rate=4000.0, duration=0.05, seed=11, lo=1 << 10, hi=2 << 20)
    return pools, streams, origs, trace


def _run(backend_cls, pools, streams, trace):
    import torch
    reqs = serve.build_requests(trace, pools, streams)
    print(backend_cls.__name__, "requests", len(reqs), flush=True)
    backend = backend_cls(nstreams=3, keep_results=True)
    sched = serve.serve(reqs, backend, budget_bytes=64 << 20, slots=3, max_batch=8)
    torch.cuda.synchronize()
    assert not sched.rejected and len(reqs) > 20
    assert all(r.done is not None and r.done >= r.arrival for r in reqs)
    return reqs


def test_results_identical_alone_and_in_the_mix():
    rng = np.random.default_rng(9)
    pools, streams, origs, trace = _setup(rng)
    reqs = _run(serve.DeviceBackend, pools, streams, trace)
    for r in reqs:
        assert r.status == gpulz.GPULZ_OK, r
        got = r.result.cpu().numpy().tobytes()
        if r.op == serve.COMPRESS:
            C, W, MIN, _ = gpulz.gpulz_default_params(r.symbol_bytes)
            alone = gpulz.compress(r.src, r.symbol_bytes, C, W, MIN)
            # and the oracle on the same bytes with the width's parameters
            src = r.src.cpu().numpy()
            assert got == oracle.compress(src, r.symbol_bytes, C, W, MIN, threads=8), r.rid
        else:
            alone = gpulz.decompress(r.src)
        assert got == alone.cpu().numpy().tobytes(), r.rid
        if r.op == serve.DECOMPRESS:
            k = [s.data_ptr() for s, _ in streams].index(r.src.data_ptr())
            assert got == origs[k].tobytes()


def test_plain_backend_gives_the_same_results():
    rng = np.random.default_rng(9)
    pools, streams, origs, trace = _setup(rng)
    batched = _run(serve.DeviceBackend, pools, streams, trace)
    plain = _run(serve.PlainBackend, pools, streams, trace)
    assert len(batched) == len(plain)
    for a, b in zip(batched, plain):
        assert a.status == b.status == gpulz.GPULZ_OK, (a, b)
        assert a.result.cpu().numpy().tobytes() == b.result.cpu().numpy().tobytes(), a.rid
