"""Reads the hand-worked Huffman vectors tests/golden/huff_*.txt.

Fields: `input_ascii` or `input_hex` (the input), `lengths` (hex symbol =
code length, for every symbol with a code), `stream_hex` (the whole expected
stream; repeated lines concatenate, spaces are ignored, `XX*K` is byte XX
repeated K times). Lines starting with # explain the derivation."""
import glob
import os

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _hex(tokens):
    out = b""
    for tok in tokens:
        if "*" in tok:
            b, k = tok.split("*")
            out += bytes.fromhex(b) * int(k)
        else:
            out += bytes.fromhex(tok)
    return out


def load(path):
    v = {"name": os.path.basename(path)[:-4], "stream": b""}
    for line in open(path):
        line = line.rstrip("\n")
        if not line or line.startswith("#"):
            continue
        key, val = line.split(":", 1)
        if key == "input_ascii":
            v["input"] = val.strip().encode()
        elif key == "input_hex":
            v["input"] = _hex(val.split())
        elif key == "lengths":
            v["lengths"] = {int(a, 16): int(b) for a, b in (t.split("=") for t in val.split())}
        elif key == "stream_hex":
            v["stream"] += _hex(val.split())
    return v


def all_vectors():
    return [load(p) for p in sorted(glob.glob(os.path.join(HERE, "huff_*.txt")))]
