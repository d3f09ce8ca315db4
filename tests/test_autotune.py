"""Autotuner host logic (selection rule, candidate space, cache round trip)."""
import json

from paper_2304_07342_amd import autotune, gpulz


def test_candidates_fit_the_chunk_limit():
    for S in (1, 2, 4, 8):
        c = autotune.candidates(S)
        assert c and all(C * S <= autotune.MAX_CHUNK_BYTES for C, _, _ in c)
    assert all(C <= 6144 for C, _, _ in autotune.candidates(8))


def test_choose_fastest_within_ratio_tolerance():
    res = [(1024, 32, 1, 1.0, 1.50), (1024, 256, 1, 5.0, 2.00), (2048, 128, 4, 2.0, 1.97),
           (4096, 64, 4, 1.5, 1.90)]
    assert autotune.choose(res, 0.02)[:3] == (2048, 128, 4)   # 1.97 >= 0.98 * 2.0, fastest such
    assert autotune.choose(res, 0.30)[:3] == (1024, 32, 1)
    assert autotune.choose(res, 0.0)[:3] == (1024, 256, 1)


def test_cache_round_trip_installs_defaults(tmp_path):
    saved = {S: gpulz.gpulz_default_params(S) for S in (1, 2, 4, 8)}
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"device": "x", "ratio_tol": 0.02, "widths": {
        "2": {"chunk_symbols": 1024, "window": 64, "min_match": 2, "waves_per_chunk": 1}}}))
    try:
        got = autotune.load(str(path))
        assert got[2]["window"] == 64
        assert gpulz.gpulz_default_params(2) == (1024, 64, 2, 1)
        assert autotune.load(str(tmp_path / "missing.json")) is None
    finally:
        for S, p in saved.items():
            gpulz.gpulz_set_default_params(S, *p)
