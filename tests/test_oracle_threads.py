"""Pins the oracle's threaded drivers (oracle_compress_mt,
oracle_compress_policy_mt) against single-threaded results.

Chunks are independent (section 3.3.1), so splitting them over threads must
not change a byte. Policy 0 is compared with the plain single-threaded
oracle_compress; policy 1 (which only has the threaded driver) with a stream
assembled here, chunk by chunk, from oracle_parse_chunk_policy's tokens and
the independent Python serialiser in refimpl. Thread counts cover fewer
chunks than threads, exactly as many, counts that do not divide the chunks,
no chunk at all, and ragged tails (a short last chunk and n not a multiple
of S).
"""
import struct

import numpy as np
import pytest

import oracle
import refimpl

THREADS = (2, 3, 7, 16)


def _input(seed, n):
    rng = np.random.default_rng(seed)
    # small alphabet with copied runs: many pointers, so the records differ
    # in size from chunk to chunk and a misplaced record shows
    x = rng.integers(0, 6, n, dtype=np.uint8)
    for _ in range(n // 40):
        L = int(rng.integers(2, 30))
        o = int(rng.integers(1, 64))
        d = int(rng.integers(o, max(o + 1, n - L)))
        if d + L <= n:
            for k in range(L):
                x[d + k] = x[d - o + k]
    return x.tobytes()


def _assembled_policy1(x, S, C, W, MIN):
    m = len(x) // S
    table, recs = b"", b""
    N = 0
    for cs in range(0, m, C):
        ch = x[cs * S:min(cs + C, m) * S]
        toks = oracle.parse_chunk(ch, S, W, MIN, policy=1)
        syms = [ch[j * S:(j + 1) * S] for j in range(len(ch) // S)]
        rec, F, P = refimpl.record(syms, toks, S)
        table += struct.pack("<II", F, P)
        recs += rec
        N += 1
    total = 64 + len(table) + len(recs)
    return refimpl.header(len(x), S, C, W, MIN, N, total, x[m * S:], policy=1) + table + recs


# (S, C, n): N = 0 (n < S and n = 0), N = 1, N = 2 < k, N = 7, N = 16, N = 23
# (not divisible by 2, 3, 7 or 16) and N = 100, each with a ragged tail
CASES = [(4, 64, 0), (4, 64, 3), (2, 50, 61), (1, 40, 75), (2, 31, 2 * 31 * 6 + 9),
         (1, 37, 37 * 15 + 11), (8, 16, 8 * 16 * 22 + 8 * 5 + 7), (1, 50, 50 * 99 + 1)]


@pytest.mark.parametrize("S,C,n", CASES)
@pytest.mark.parametrize("k", THREADS)
def test_threaded_policy0_equals_single_thread(S, C, n, k):
    x = _input(S * 1000 + n, n)
    ref = oracle.compress(x, S, C, 32, 2)
    assert oracle.compress(x, S, C, 32, 2, threads=k) == ref
    # MIN = 1 (two-byte pointers for S = 1) and a full window
    ref1 = oracle.compress(x, S, C, 256, 1)
    assert oracle.compress(x, S, C, 256, 1, threads=k) == ref1


@pytest.mark.parametrize("S,C,n", CASES)
@pytest.mark.parametrize("k", THREADS)
def test_threaded_policy1_equals_per_chunk_assembly(S, C, n, k):
    x = _input(S * 2000 + n, n)
    ref = _assembled_policy1(x, S, C, 32, 2)
    assert oracle.compress(x, S, C, 32, 2, threads=1, policy=1) == ref
    assert oracle.compress(x, S, C, 32, 2, threads=k, policy=1) == ref


def test_threaded_policy1_matches_python_reference():
    # the whole policy-1 stream, threaded, against the slice-walking reference
    for S, C, n in [(1, 9, 100), (2, 7, 2 * 50 + 1), (4, 5, 4 * 23 + 3)]:
        x = _input(n, n)
        want = refimpl.compress(x, S, C, 8, 2, policy=1)
        for k in THREADS:
            assert oracle.compress(x, S, C, 8, 2, threads=k, policy=1) == want


@pytest.mark.parametrize("k", THREADS)
def test_threaded_out_of_space_and_required_size(k):
    x = _input(5, 3000)
    full = oracle.compress(x, 1, 64, 32, 2)
    for policy in (0, 1):
        want = oracle.compress(x, 1, 64, 32, 2, policy=policy)
        st, s, need = oracle.compress_status(x, 1, 64, 32, 2, capacity=len(want) - 1, threads=k,
                                             policy=policy)
        assert st == oracle.ERR_OUT_OF_SPACE and s is None and need == len(want)
        st, s, need = oracle.compress_status(x, 1, 64, 32, 2, capacity=len(want), threads=k,
                                             policy=policy)
        assert st == oracle.OK and s == want
    assert oracle.decompress(full) == x


# ---- the pins above are not vacuous: mistakes planted in the threaded split
# of a temporary copy of the oracle (compiled with gcc) must fail them, while
# the single-threaded oracle (threads = 1) stays correct in each copy

SPLIT_MUTANTS = {
    # the last N mod k chunks belong to no job (F, P made zero-initialised so
    # the copy stays memory-safe)
    "split_drops_remainder": [
        ("jobs[t].last = N * (uint64_t)(t + 1) / (uint64_t)threads;",
         "jobs[t].last = (N / (uint64_t)threads) * (uint64_t)(t + 1);"),
        ("F = (uint32_t*)malloc(sizeof(uint32_t) * (N ? N : 1));",
         "F = (uint32_t*)calloc(N ? N : 1, sizeof(uint32_t));"),
        ("P = (uint32_t*)malloc(sizeof(uint32_t) * (N ? N : 1));",
         "P = (uint32_t*)calloc(N ? N : 1, sizeof(uint32_t));"),
    ],
    # each job reads its chunks from the start of the input
    "job_reads_from_input_start": [
        ("uint64_t cs = i * j->C;", "uint64_t cs = (i - j->first) * j->C;"),
    ],
    # each job writes its records from the first scratch slot
    "job_record_slot_from_zero": [
        ("j->recs + i * j->slot", "j->recs + (i - j->first) * j->slot"),
    ],
}


def _build_split_mutant(tmp_path, name):
    import os
    import subprocess
    src = open(os.path.join(os.path.dirname(oracle.__file__), "gpulz_oracle.c")).read()
    for old, new in SPLIT_MUTANTS[name]:
        assert src.count(old) == 1, (name, old)
        src = src.replace(old, new)
    msrc = tmp_path / f"{name}.c"
    msrc.write_text(src)
    lib = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-std=c99", "-O1", "-shared", "-fPIC", "-pthread",
                           "-I", os.path.dirname(oracle.__file__), str(msrc), "-o", str(lib)])
    return str(lib)


def _thread_pins_pass():
    try:
        for S, C, n in CASES:
            x = _input(S * 1000 + n, n)
            ref = oracle.compress(x, S, C, 32, 2)
            for k in THREADS:
                if oracle.compress(x, S, C, 32, 2, threads=k) != ref:
                    return False
                if oracle.compress(x, S, C, 32, 2, threads=k, policy=1) != \
                        _assembled_policy1(x, S, C, 32, 2):
                    return False
    except ValueError:
        return False
    return True


def test_unmutated_threads_pass():
    assert _thread_pins_pass()


@pytest.mark.parametrize("name", sorted(SPLIT_MUTANTS))
def test_split_mutant_is_caught(name, tmp_path, monkeypatch):
    import ctypes
    path = _build_split_mutant(tmp_path, name)
    real = oracle._load()
    mlib = ctypes.CDLL(path)
    for fn in ("oracle_compress_bound", "oracle_compress", "oracle_compress_mt",
               "oracle_compress_policy_mt", "oracle_decompress", "oracle_parse_chunk",
               "oracle_parse_chunk_policy"):
        getattr(mlib, fn).restype = getattr(real, fn).restype
        getattr(mlib, fn).argtypes = getattr(real, fn).argtypes
    monkeypatch.setattr(oracle, "_lib", mlib)
    # single-threaded results are untouched by the planted mistake ...
    x = _input(9, 500)
    assert mlib is oracle._load()
    assert oracle.compress(x, 1, 37, 32, 2) == refimpl.compress(x, 1, 37, 32, 2)
    # ... and the thread pins catch it
    assert not _thread_pins_pass(), f"planted mistake {name} was not caught"
