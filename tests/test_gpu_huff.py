"""Huffman stage on the GPU against the oracle: byte-identical streams on the
hand-worked vectors and on seeded inputs (ragged chunks, one and two symbols,
all 256 bytes, the length limit), decoding of oracle streams, rejection of
corrupted streams, the LZSS -> Huffman chain at the benchmark's full size,
and the device-resident size path."""
import struct

import numpy as np
import pytest

import huffref
import oracle
from huff_golden import all_vectors
from paper_2304_07342_amd import gpulz, synth

pytestmark = pytest.mark.gpu

VECTORS = all_vectors()


def _dev(data: bytes):
    import torch
    return torch.from_numpy(np.frombuffer(data, np.uint8).copy()).to("cuda")


def _gpu_stream(data: bytes) -> bytes:
    return gpulz.huff_compress(_dev(data)).cpu().numpy().tobytes()


@pytest.mark.parametrize("v", VECTORS, ids=[v["name"] for v in VECTORS])
def test_hand_vectors(v):
    print("huff hand vector", v["name"], flush=True)
    assert _gpu_stream(v["input"]).hex() == v["stream"].hex()
    assert gpulz.huff_decompress(_dev(v["stream"])).cpu().numpy().tobytes() == v["input"]


def _inputs():
    rng = np.random.default_rng(21)
    yield "empty", b""
    yield "one", b"\x07"
    yield "single_symbol", b"q" * (3 * 4096 + 5)
    yield "two_symbols", bytes(rng.choice([3, 250], 50001, p=[0.9, 0.1]).astype(np.uint8))
    yield "all_bytes", bytes(rng.integers(0, 256, 90001).astype(np.uint8))
    zipf = np.minimum(rng.zipf(1.3, 4096 * 37 + 200), 256) - 1
    yield "zipf_ragged", bytes(zipf.astype(np.uint8))
    for n in (127, 128, 129, 4095, 4096, 4097, 8 * 4096 * 3 + 1):
        yield f"geom_{n}", bytes(np.minimum(rng.geometric(0.2, n), 255).astype(np.uint8))
    fib = [1, 1]
    while len(fib) < 18:
        fib.append(fib[-1] + fib[-2])
    yield "length_limit", b"".join(bytes([s]) * f for s, f in enumerate(fib))
    # counts 2^17 .. 2^0 and 22 singletons: code lengths 11 through 15 (the
    # two-level decoding table)
    yield "long_codes", b"".join(bytes([s]) * (1 << (17 - s)) for s in range(18)) + bytes(range(18, 40))
    x = synth.laplace_codes(1 << 19, seed=4)
    yield "lz_stream_of_codes", oracle.compress(x, 2, 2048, 128, 2)


INPUTS = list(_inputs())


@pytest.mark.parametrize("name,data", INPUTS, ids=[n for n, _ in INPUTS])
def test_streams_match_oracle(name, data):
    print("huff parity", name, len(data), flush=True)
    ref = oracle.huff_compress(data)
    assert _gpu_stream(data) == ref
    back = gpulz.huff_decompress(_dev(ref)).cpu().numpy().tobytes()
    assert back == data


def _corrupt(s: bytes, case: str) -> bytes:
    N = struct.unpack_from("<Q", s, 24)[0]
    at, mask = {"magic": (0, 1), "version": (4, 2), "limit": (6, 1), "chunk": (9, 1),
                "reserved": (50, 1), "length_nibble": (64 + ord("a") // 2, 0x10),
                "table_bits": (192, 1), "first_offset": (192 + 4 * N, 1),
                "padding_bit": (len(s) - 4, 1)}[case]
    b = bytearray(s)
    b[at] ^= mask
    return bytes(b)


@pytest.mark.parametrize("case", ["magic", "version", "limit", "chunk", "reserved",
                                  "length_nibble", "table_bits", "first_offset", "padding_bit"])
def test_corrupt_streams_rejected_like_the_oracle(case):
    s = _corrupt(oracle.huff_compress(b"abracadabra" * 50), case)
    assert oracle.huff_decompress_status(s)[0] == oracle.ERR_CORRUPT
    st, _ = gpulz.huff_decompress(_dev(s), out_capacity=550, return_status=True)
    assert st == gpulz.GPULZ_ERR_CORRUPT


def test_incomplete_code_and_bad_offsets_rejected():
    lens = [0] * 256
    for ch in b"abc":
        lens[ch] = 2
    s = huffref.compress(b"abcabc", lens)
    assert gpulz.huff_decompress(_dev(s), out_capacity=6, return_status=True)[0] == \
        gpulz.GPULZ_ERR_CORRUPT
    # a later sub-block's start bit moved by one: the sub-blocks no longer meet
    data = bytes(np.random.default_rng(2).integers(0, 40, 5000).astype(np.uint8))
    s = bytearray(oracle.huff_compress(data))
    N = struct.unpack_from("<Q", s, 24)[0]
    rec0 = 192 + 4 * N
    s[rec0 + 2 * 5] ^= 1
    assert oracle.huff_decompress_status(bytes(s))[0] == oracle.ERR_CORRUPT
    assert gpulz.huff_decompress(_dev(bytes(s)), out_capacity=5000, return_status=True)[0] == \
        gpulz.GPULZ_ERR_CORRUPT


def test_small_output_capacity():
    s = oracle.huff_compress(b"hello world" * 100)
    st, _ = gpulz.huff_decompress(_dev(s), out_capacity=10, return_status=True)
    assert st == gpulz.GPULZ_ERR_OUT_OF_SPACE


def test_device_size_larger_than_maximum_is_rejected():
    import torch
    x = _dev(b"abc" * 1000)
    hc = gpulz.HuffCompressor(3000)
    n_dev = torch.tensor([3001], dtype=torch.int64, device="cuda")
    hc.compress_async(x, 3000, d_nbytes=n_dev.data_ptr())
    size, st = hc.result()
    assert st == gpulz.GPULZ_ERR_INVALID_ARG and size == 0
    n_dev.fill_(2000)
    hc.compress_async(x, 3000, d_nbytes=n_dev.data_ptr())
    size, st = hc.result()
    assert st == gpulz.GPULZ_OK
    assert hc.out[:size].cpu().numpy().tobytes() == oracle.huff_compress(b"abc" * 666 + b"ab")


def test_chain_at_benchmark_size():
    """256 MiB of uint16 quantization codes: LZSS (S=2, C=2048, W=128,
    MIN=2) then Huffman, as the benchmark times it; the chained stream
    equals the oracle's Huffman stream of the oracle's LZSS stream."""
    x = synth.laplace_codes_pool(1 << 27, seed=7)
    print("huff chain 256 MiB", flush=True)
    lz_ref = oracle.compress(x, 2, 2048, 128, 2, threads=16)
    ref = oracle.huff_compress(lz_ref)
    import torch
    d = torch.from_numpy(x.view(np.uint8).copy()).to("cuda")
    s, lz_size = gpulz.compress_entropy(d, 2, 2048, 128, 2)
    assert lz_size == len(lz_ref)
    assert s.numel() == len(ref)
    assert s.cpu().numpy().tobytes() == ref
    back = gpulz.decompress_entropy(s)
    assert torch.equal(back, d)
