"""The adaptive width / window rule of section 3.2.3, on the CPU: the
decision depends only on the element width, the level and the measured
multi-byte ratio."""
import pytest

from paper_2304_07342_amd import adaptive

CHUNKS = {1: 4096, 2: 2048, 4: 4096, 8: 2048}


def _decide(S, level, ratio):
    return adaptive.decide(S, level, ratio, chunk_for=CHUNKS.get)


@pytest.mark.parametrize("level,W", [(1, 32), (2, 64), (3, 128), (4, 255)])
def test_levels_set_the_base_window(level, W):
    p = _decide(1, level, None)
    assert (p.symbol_bytes, p.window, p.chunk_symbols) == (1, W, 4096)


@pytest.mark.parametrize("S", [2, 4, 8])
def test_multi_byte_kept_with_an_enlarged_window(S):
    for level, base in adaptive.LEVEL_WINDOWS.items():
        p = _decide(S, level, 1.5)
        assert p.symbol_bytes == S and p.window == min(256, S * base)
        assert p.chunk_symbols == CHUNKS[S]


@pytest.mark.parametrize("S", [2, 4, 8])
def test_low_ratio_switches_to_single_bytes(S):
    p = _decide(S, 3, 1.4999)
    assert (p.symbol_bytes, p.window, p.chunk_symbols) == (1, 128, 4096)


def test_rejects_bad_levels():
    with pytest.raises(ValueError):
        _decide(4, 5, 2.0)
