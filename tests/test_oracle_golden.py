"""Pins the oracle to hand-worked vectors (tests/golden/*.txt)."""
import pytest

import oracle
import refimpl
from golden import all_vectors

VECTORS = all_vectors()


def expected_stream(v):
    n = len(v["input"])
    S, C = v["S"], v["C"]
    N = -(-(n // S) // C)
    hdr = refimpl.header(n, S, C, v["W"], v["MIN"], N, v["total"], v["tail"], v["policy"])
    return hdr + v["body"]


@pytest.mark.parametrize("v", VECTORS, ids=[v["name"] for v in VECTORS])
def test_fixture_is_self_consistent(v):
    assert len(expected_stream(v)) == v["total"]
    assert len(v["input"]) % v["S"] == len(v["tail"])


@pytest.mark.parametrize("v", VECTORS, ids=[v["name"] for v in VECTORS])
def test_oracle_stream_matches_hand_vector(v):
    got = oracle.compress(v["input"], v["S"], v["C"], v["W"], v["MIN"], policy=v["policy"])
    assert got.hex() == expected_stream(v).hex()


@pytest.mark.parametrize("v", VECTORS, ids=[v["name"] for v in VECTORS])
def test_oracle_tokens_match_hand_vector(v):
    S, C = v["S"], v["C"]
    data = v["input"]
    m = len(data) // S
    for i, toks in enumerate(v["tokens"]):
        chunk = data[i * C * S:min(m, (i + 1) * C) * S]
        got = oracle.parse_chunk(chunk, S, v["W"], v["MIN"], policy=v["policy"])
        assert got == toks


@pytest.mark.parametrize("v", VECTORS, ids=[v["name"] for v in VECTORS])
def test_oracle_decodes_hand_vector(v):
    assert oracle.decompress(expected_stream(v)) == v["input"]


@pytest.mark.parametrize("v", VECTORS, ids=[v["name"] for v in VECTORS])
def test_bruteforce_reference_matches_hand_vector(v):
    if len(v["input"]) > 700:
        pytest.skip("brute force too slow")
    got = refimpl.compress(v["input"], v["S"], v["C"], v["W"], v["MIN"], v["policy"])
    assert got.hex() == expected_stream(v).hex()
