"""Loader for the hand-worked vectors under tests/golden/."""
from __future__ import annotations

import glob
import os

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _hexlist(items):
    out = b""
    for it in items:
        if "*" in it:
            h, k = it.split("*")
            out += bytes.fromhex(h) * int(k)
        else:
            out += bytes.fromhex(it)
    return out


def _tokens(items):
    chunks = [[]]
    for it in items:
        if it == "|":
            chunks.append([])
            continue
        rep = 1
        if "*" in it:
            it, k = it.split("*")
            rep = int(k)
        tok = (0, 0) if it == "lit" else tuple(int(v) for v in it.split(","))
        chunks[-1].extend([tok] * rep)
    return chunks


def load(path):
    v = {"name": os.path.basename(path), "tail": b"", "policy": 0}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, _, rest = line.partition(" ")
        items = rest.split()
        if key in ("S", "C", "W", "MIN", "total", "policy"):
            v[key] = int(items[0])
        elif key in ("input", "body", "tail"):
            v[key] = _hexlist(items)
        elif key == "tokens":
            v[key] = _tokens(items)
    return v


def all_vectors():
    return [load(p) for p in sorted(glob.glob(os.path.join(GOLDEN_DIR, "e*.txt")))]
