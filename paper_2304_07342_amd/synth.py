"""Seeded synthetic inputs shaped like the paper's workloads.

The paper measures on cuSZ quantisation codes (uint16), TPC-H int32 and
string columns, and the RTM float32 seismic field (section 4.1, datasets);
none of those datasets is available, so these generators stand in for them.
This module only draws data: it holds none of the compression method's
arithmetic, and both the GPU path and the CPU oracle consume its output.

Every generator takes an explicit seed and uses numpy's PCG64.
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def laplace_codes(m: int, seed: int = 0, copy_fraction: float = 0.30) -> np.ndarray:
    """uint16 quantisation-code stand-in: 512 + rint(Laplace(0, 2)) clipped to
    [0, 1023]; then random earlier runs are copied forward (length U{2..32},
    source offset U{1..128}, copied element by element so a short offset
    repeats a period) until at least `copy_fraction` of the positions have
    been overwritten."""
    rng = _rng(seed)
    v = np.clip(512 + np.rint(rng.laplace(0.0, 2.0, size=m)), 0, 1023).astype(np.uint16)
    if m < 40:
        return v
    written = np.zeros(m, dtype=bool)
    count = 0
    target = int(np.ceil(copy_fraction * m))
    batch = 4096
    while count < target:
        Ls = rng.integers(2, 33, size=batch)
        os_ = rng.integers(1, 129, size=batch)
        us = rng.random(size=batch)
        for L, o, u in zip(Ls.tolist(), os_.tolist(), us.tolist()):
            hi = m - L
            if hi < o:
                continue
            dst = o + int(u * (hi - o + 1))
            if o >= L:
                v[dst:dst + L] = v[dst - o:dst - o + L]
            else:
                for k in range(L):
                    v[dst + k] = v[dst - o + k]
            seg = written[dst:dst + L]
            count += L - int(np.count_nonzero(seg))
            seg[:] = True
            if count >= target:
                break
    return v


def sinusoid_field(shape=(512, 512, 256), seed: int = 1, dtype=np.float32,
                   n_waves: int = 8, noise: float = 1e-3, quantum: float = 1e-4) -> np.ndarray:
    """Smooth 3-D field (RTM seismic stand-in): a sum of `n_waves` plane waves
    a*sin(2*pi*f*(u . r) + phi) with a ~ U(0.1, 1), f ~ U(1, 16) cycles over
    the domain, u a random unit vector and r the coordinates scaled to
    [0, 1); plus N(0, noise) noise, rounded to multiples of `quantum` in
    float64 and cast to `dtype`, C order."""
    rng = _rng(seed)
    a = rng.uniform(0.1, 1.0, size=n_waves)
    f = rng.uniform(1.0, 16.0, size=n_waves)
    u = rng.normal(size=(n_waves, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    phi = rng.uniform(0.0, 2 * np.pi, size=n_waves)
    nx, ny, nz = shape
    out = np.empty(shape, dtype=dtype)
    ys = (np.arange(ny) / ny)[:, None]
    zs = (np.arange(nz) / nz)[None, :]
    noise_rng = _rng(seed + 1_000_003)
    for i in range(nx):
        x = i / nx
        acc = np.zeros((ny, nz), dtype=np.float64)
        for k in range(n_waves):
            arg = 2 * np.pi * f[k] * (u[k, 0] * x + u[k, 1] * ys + u[k, 2] * zs) + phi[k]
            acc += a[k] * np.sin(arg)
        acc += noise_rng.normal(0.0, noise, size=(ny, nz))
        out[i] = (np.rint(acc / quantum) * quantum).astype(dtype)
    return out


def zipf_text(n: int, seed: int = 2, s: float = 1.2, ranks: int = 64) -> np.ndarray:
    """uint8 text-like bytes (TPC-H string stand-in): rank r in 1..`ranks`
    drawn with probability proportional to r**-s (inverse CDF of uniform
    draws, 16 Mi at a time), byte = 0x20 + r - 1."""
    rng = _rng(seed)
    p = np.arange(1, ranks + 1, dtype=np.float64) ** -s
    cdf = np.cumsum(p / p.sum())
    cdf[-1] = 1.0
    out = np.empty(n, dtype=np.uint8)
    step = 1 << 24
    for i in range(0, n, step):
        u = rng.random(min(step, n - i))
        out[i:i + u.size] = 0x20 + np.searchsorted(cdf, u, side="right")
    return out


def sorted_indices(m: int, seed: int = 2, p: float = 0.3) -> np.ndarray:
    """uint32 strictly increasing indices (TPC-H int32 stand-in): the
    cumulative sum of Geometric(p) gaps (each gap >= 1), 16 Mi at a time."""
    rng = _rng(seed)
    out = np.empty(m, dtype=np.uint32)
    carry = np.uint64(0)
    step = 1 << 24
    for i in range(0, m, step):
        c = np.cumsum(rng.geometric(p, size=min(step, m - i)), dtype=np.uint64) + carry
        out[i:i + c.size] = c.astype(np.uint32)
        carry = c[-1]
    return out


def laplace_codes_pool(m: int, seed: int, copy_fraction: float = 0.30,
                       batch: int = 1 << 15) -> np.ndarray:
    """Large-scale variant of `laplace_codes` for benchmark pools: the same
    Laplace codes and the same copy distributions (length U{2..32}, source
    offset U{1..128}, periodic when the offset is shorter than the length),
    but copies are applied `batch` at a time, each batch reading the codes as
    they were before it (so copies within a batch do not see each other)."""
    rng = _rng(seed)
    v = np.clip(512 + np.rint(rng.laplace(0.0, 2.0, size=m)), 0, 1023).astype(np.uint16)
    if m < 200:
        return v
    target = int(np.ceil(copy_fraction * m))
    written = 0
    while written < target:
        L = rng.integers(2, 33, size=batch)
        o = rng.integers(1, 129, size=batch)
        dst = o + (rng.random(batch) * (m - 32 - o)).astype(np.int64)
        k = np.arange(32)[None, :]
        valid = k < L[:, None]
        src = dst[:, None] - o[:, None] + (k % o[:, None])
        d = (dst[:, None] + k)[valid]
        v[d] = v[src[valid]]
        written += int(L.sum())
    return v


def uniform_bytes(n: int, seed: int) -> np.ndarray:
    return _rng(seed).integers(0, 256, size=n, dtype=np.uint8)


def small_alphabet(m: int, S: int, seed: int, alphabet: int = 4) -> np.ndarray:
    """S-byte symbols drawn from `alphabet` random distinct values: dense in
    matches of every length and offset."""
    rng = _rng(seed)
    vals = rng.integers(0, 256, size=(alphabet, S), dtype=np.uint8)
    return vals[rng.integers(0, alphabet, size=m)].reshape(-1)


def runs(m: int, S: int, seed: int) -> np.ndarray:
    """Long constant and periodic runs (stresses the 255 length cap, the
    length <= offset cap and offsets up to 256)."""
    rng = _rng(seed)
    out = np.empty((m, S), dtype=np.uint8)
    j = 0
    while j < m:
        L = int(rng.integers(1, 700))
        period = int(rng.choice([1, 2, 3, 64, 200, 256, 257]))
        pat = rng.integers(0, 256, size=(period, S), dtype=np.uint8)
        seg = pat[np.arange(min(L, m - j)) % period]
        out[j:j + len(seg)] = seg
        j += len(seg)
    return out.reshape(-1)


def mixed(nbytes: int, S: int, seed: int) -> np.ndarray:
    """Concatenation of the small-case generators above (for parity tests)."""
    rng = _rng(seed)
    parts = []
    left = nbytes
    k = 0
    while left > 0:
        take = min(left, int(rng.integers(1, max(2, nbytes // 3 + 1))))
        m = max(1, take // S)
        kind = k % 4
        if kind == 0:
            part = small_alphabet(m, S, seed * 131 + k)
        elif kind == 1:
            part = runs(m, S, seed * 131 + k)
        elif kind == 2:
            part = uniform_bytes(m * S, seed * 131 + k)
        else:
            part = laplace_codes(max(1, (m * S) // 2), seed * 131 + k).view(np.uint8)
        parts.append(part[:left])
        left -= len(parts[-1])
        k += 1
    return np.concatenate(parts)[:nbytes] if parts else np.zeros(0, dtype=np.uint8)


# ---- the two single-buffer benchmark workloads ------------------------------

def codes_1mib() -> np.ndarray:
    """1 MiB of uint16 Laplace codes with 30% copied runs, seed 0."""
    return laplace_codes(1 << 19, seed=0)


def field_256mib() -> np.ndarray:
    """256 MiB float32 field 512 x 512 x 256, seed 1."""
    return sinusoid_field((512, 512, 256), seed=1, dtype=np.float32)


def field64(shape=(256, 512, 256), seed: int = 8) -> np.ndarray:
    """float64 version of the smooth field (same recipe)."""
    return sinusoid_field(shape, seed=seed, dtype=np.float64)


# Pools for the batched and serving workloads: one per content kind, device
# buffers are slices of these (kind -> (symbol width, generator)).
POOL_KINDS = {
    "zipf-u8": (1, lambda nbytes, seed: zipf_text(nbytes, seed=seed)),
    "laplace-u16": (2, lambda nbytes, seed: laplace_codes_pool(nbytes // 2, seed=seed).view(np.uint8)),
    "sorted-u32": (4, lambda nbytes, seed: sorted_indices(nbytes // 4, seed=seed).view(np.uint8)),
    "field-f32": (4, lambda nbytes, seed: sinusoid_field((nbytes // (4 * 512 * 256), 512, 256),
                                                         seed=seed).view(np.uint8).reshape(-1)),
    "field-f64": (8, lambda nbytes, seed: sinusoid_field((nbytes // (8 * 512 * 256), 512, 256),
                                                         seed=seed, dtype=np.float64)
                  .view(np.uint8).reshape(-1)),
}
# content kinds drawn for each symbol width (uniformly)
WIDTH_KINDS = {1: ["zipf-u8"], 2: ["laplace-u16"], 4: ["sorted-u32", "field-f32"], 8: ["field-f64"]}


def batch_spec(nbufs: int, seed: int, lo: int = 4 << 10, hi: int = 64 << 20,
               pool_bytes: int = 256 << 20):
    """Buffers for the batched workload: size log-uniform in [lo, hi] rounded
    down to the symbol width, width uniform over {1, 2, 4, 8}, content kind by
    width, and a random 16-byte aligned slice of that kind's pool. Returns a
    list of (kind, width, offset, nbytes)."""
    rng = _rng(seed)
    out = []
    for _ in range(nbufs):
        S = int(rng.choice([1, 2, 4, 8]))
        kind = WIDTH_KINDS[S][int(rng.integers(0, len(WIDTH_KINDS[S])))]
        n = int(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        n = max(S, min(n, pool_bytes) // S * S)
        off = int(rng.integers(0, pool_bytes - n + 1)) // 16 * 16
        out.append((kind, S, off, n))
    return out


# The two single-buffer workloads by name: 1 MiB of uint16 codes (small
# enough for the oracle in seconds) and the 256 MiB float32 field.
WORKLOADS = {
    "laplace-u16-1MiB": dict(name="laplace-u16-1MiB", S=2, C=2048, W=128, MIN=2, make=codes_1mib),
    "field-f32-256MiB": dict(name="field-f32-256MiB", S=4, C=4096, W=256, MIN=2, make=field_256mib),
}
CODES_1MIB, FIELD_256MIB = "laplace-u16-1MiB", "field-f32-256MiB"
