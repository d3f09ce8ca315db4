"""The adaptive rule of section 3.2.3 on real data: uint16 codes compress
well with 2-byte symbols and keep them (window 2 x 128); strictly increasing
uint32 indices do not (ratio below 1.5 with 4-byte symbols) and fall back to
single bytes. The streams it writes are the oracle's for the chosen
parameters and decode back."""
import numpy as np
import pytest

import oracle
from gpu_helpers import to_device
from paper_2304_07342_amd import adaptive, gpulz, synth

pytestmark = pytest.mark.gpu


def _fields(arrays):
    return [to_device(a.view(np.uint8).reshape(-1)) for a in arrays]


def test_codes_keep_two_byte_symbols():
    arrays = [synth.laplace_codes(20000, seed=s) for s in range(3)]
    plan, streams = adaptive.compress(_fields(arrays), 2, level=3)
    assert plan.symbol_bytes == 2 and plan.window == 256 and plan.multi_byte_ratio >= 1.5
    for a, s in zip(arrays, streams):
        x = a.view(np.uint8).reshape(-1)
        assert s.cpu().numpy().tobytes() == oracle.compress(x, 2, plan.chunk_symbols, 256, 2)
        assert gpulz.decompress(s).cpu().numpy().tobytes() == x.tobytes()


def test_sorted_indices_fall_back_to_bytes():
    arrays = [synth.sorted_indices(20000, seed=s) for s in range(3)]
    plan, streams = adaptive.compress(_fields(arrays), 4, level=2)
    assert plan.symbol_bytes == 1 and plan.window == 64 and plan.multi_byte_ratio < 1.5
    for a, s in zip(arrays, streams):
        x = a.view(np.uint8).reshape(-1)
        assert s.cpu().numpy().tobytes() == oracle.compress(x, 1, plan.chunk_symbols, 64, 2)
        assert gpulz.decompress(s).cpu().numpy().tobytes() == x.tobytes()
