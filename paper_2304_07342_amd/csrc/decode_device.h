// Device code of the decoder, shared by the single-buffer and batch kernels.
//
// The paper states that decompression exists and is easy to parallelise
// (section 4.4) without describing it; this decoder follows from the stream
// layout:
//   header   one thread checks every header field;
//   table    the table's F_i + P_i are prefix-summed once per group of 64
//            chunks (one u64 per group; the sum must end exactly at the
//            stream's end); a chunk's record offset is its group's offset
//            plus a 64-lane prefix sum over the group's table entries;
//   chunk    one wavefront per chunk walks the tokens 64 at a time: lane l
//            takes token t + l, its flag bit gives its kind, mbcnt over the
//            literal / pointer ballots gives its payload offset, a wave scan
//            of the token lengths gives its output position. Literals are
//            written into an LDS ring of recent symbols; pointers are then
//            resolved in token order, each copied by all 64 lanes (a pointer
//            never overlaps itself because its length never exceeds its
//            offset). Finished symbols stream out to HBM. The ring keeps the
//            last 256 symbols (the largest offset), so LDS use does not
//            depend on the chunk size.
// Every rule the encoder guarantees is checked; a broken one makes the
// stream GPULZ_ERR_CORRUPT.
#pragma once

#include "gpulz_internal.h"
#include "wave.h"

namespace gpulz {
namespace dec {

constexpr uint32_t kGroup = 64;  // chunks per record-offset group

__device__ inline uint64_t rd_u64(const uint8_t* p) {
  uint64_t v = 0;
  for (int k = 7; k >= 0; --k) v = (v << 8) | p[k];
  return v;
}
__device__ inline uint32_t rd_u32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

// Checks the header of a stream of in_bytes bytes; fills p (p.status = kOk or
// kCorrupt). One thread.
__device__ inline void parse_header(const uint8_t* h, uint64_t in_bytes, DecodeParams& p) {
  p = DecodeParams{};
  bool ok = in_bytes >= kHeaderBytes;
  if (ok) {
    ok = h[0] == 'G' && h[1] == 'L' && h[2] == 'Z' && h[3] == '1' && h[4] == 1 && h[5] == 0 &&
         h[7] == 0 && h[15] == kMaxMatch;
    p.S = h[6];
    p.C = rd_u32(h + 8);
    p.W = (uint32_t)h[12] | ((uint32_t)h[13] << 8);
    p.MIN = h[14];
    p.n = rd_u64(h + 16);
    p.N = rd_u64(h + 24);
    const uint64_t total = rd_u64(h + 32);
    p.r = h[40];
    ok = ok && (p.S == 1 || p.S == 2 || p.S == 4 || p.S == 8) && p.C >= 1 && p.C <= (1u << 24) &&
         p.W >= 1 && p.W <= kMaxWindow && p.MIN >= 1;
    if (ok) {
      p.m = p.n / p.S;
      ok = p.r == p.n % p.S && p.N == (p.m + p.C - 1) / p.C && total == in_bytes &&
           p.N <= decode_max_chunks(in_bytes);
      for (uint32_t k = 41; k < 48; ++k) ok = ok && h[k] == 0;
      for (uint32_t k = 48 + p.r; k < 64; ++k) ok = ok && h[k] == 0;
    }
  }
  p.status = ok ? kOk : kCorrupt;
}

// Workgroup-wide: group_off[g] = absolute offset of the first record of chunk
// group g (g = 0 .. ceil(N / 64)); returns the end of the last record. Any
// blockDim that is a multiple of 64. `scratch` holds blockDim/64 + 1 u64.
__device__ inline uint64_t scan_table_groups(const uint8_t* in, uint64_t N, uint64_t* group_off,
                                             uint64_t* scratch) {
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
  const uint32_t nw = blockDim.x >> 6;
  const uint64_t ngroups = (N + kGroup - 1) / kGroup;
  const uint8_t* table = in + kHeaderBytes;
  uint64_t carry = kHeaderBytes + 8 * N;
  // each wave sums one group of 64 entries; then the block scans nw groups
  for (uint64_t g0 = 0; g0 < ngroups; g0 += nw) {
    const uint64_t g = g0 + wid;
    uint64_t sum = 0;
    if (g < ngroups) {
      const uint64_t i = g * kGroup + lane;
      uint64_t v = 0;
      if (i < N) {
        const uint32_t* e = reinterpret_cast<const uint32_t*>(table + 8 * i);
        v = (uint64_t)e[0] + e[1];
      }
      sum = wave_incl_scan_u64(v);  // lane 63 holds the group's sum
    }
    if (lane == 63) scratch[wid] = sum;
    __syncthreads();
    if (wid == 0) {
      const uint64_t w = lane < nw ? scratch[lane] : 0;
      const uint64_t wi = wave_incl_scan_u64(w);
      if (lane < nw && g0 + lane < ngroups) group_off[g0 + lane] = carry + wi - w;
      if (lane == nw - 1) scratch[nw] = wi;
    }
    __syncthreads();
    carry += scratch[nw];
    __syncthreads();
  }
  if (tid == 0) group_off[ngroups] = carry;
  return carry;
}

// Wave-wide: absolute record offset of chunk i.
__device__ inline uint64_t record_offset(const uint8_t* in, const uint64_t* group_off, uint64_t i) {
  const uint32_t lane = lane_id();
  const uint64_t g = i / kGroup;
  const uint32_t k = (uint32_t)(i % kGroup);
  uint64_t v = 0;
  if (lane < k) {
    const uint32_t* e = reinterpret_cast<const uint32_t*>(in + kHeaderBytes + 8 * (g * kGroup + lane));
    v = (uint64_t)e[0] + e[1];
  }
  const uint64_t s = wave_incl_scan_u64(v);
  return group_off[g] + __shfl(s, 63, 64);
}

// Decode one chunk (wave-wide); returns false if the chunk breaks a rule.
template <int S>
__device__ bool decode_chunk(const uint8_t* flags, uint32_t F, uint32_t P, uint32_t c, uint32_t W,
                             uint32_t MIN, typename SymType<S>::T* out, uint8_t* ring_raw) {
  using T = typename SymType<S>::T;
  constexpr uint32_t R = kDecodeRingBytes / S;    // ring capacity in symbols
  constexpr uint32_t SPAN = R - 2 * kMaxWindow;   // new symbols per step
  T* ring = reinterpret_cast<T*>(ring_raw);
  const uint8_t* pay = flags + F;
  const uint32_t lane = lane_id();
  uint32_t q = 0, u = 0;
  uint64_t t = 0;
  while (q < c) {
    const uint64_t tok = t + lane;
    const bool has = tok < 8ull * F;
    const bool ptr = has && ((flags[tok >> 3] >> (tok & 7)) & 1u);
    const uint64_t pm = ballot(ptr);
    const uint64_t lm = ballot(has && !ptr);
    const uint32_t off = u + S * mbcnt(lm) + 2u * mbcnt(pm);
    bool ok = has && off + (ptr ? 2u : (uint32_t)S) <= P;
    uint32_t L = 1, O = 1;
    if (ptr && ok) {
      L = pay[off];
      O = pay[off + 1] ? pay[off + 1] : 256u;
    }
    const uint32_t len = has ? L : 0;
    const uint32_t pos = q + wave_incl_scan(len) - len;
    const uint32_t lim = min(c, q + SPAN);
    const bool take = has && pos < lim;
    const uint64_t tm = ballot(take);
    if (tm == 0) return false;  // flags exhausted before the chunk is complete
    if (ptr) ok = ok && L >= MIN && O <= W && O <= pos && L <= O && pos + L <= c;
    if (ballot(take && !ok)) return false;
    if (take && !ptr) {
      uint64_t v = 0;
#pragma unroll
      for (int b = 0; b < S; ++b) v |= (uint64_t)pay[off + b] << (8 * b);
      ring[pos & (R - 1)] = (T)v;
    }
    wave_sync();
    uint64_t mt = pm & tm;
    while (mt) {
      const uint32_t j = (uint32_t)__ffsll((unsigned long long)mt) - 1;
      mt &= mt - 1;
      const uint32_t pj = readlane(pos, j), Lj = readlane(L, j), Oj = readlane(O, j);
      for (uint32_t k = lane; k < Lj; k += 64) ring[(pj + k) & (R - 1)] = ring[(pj - Oj + k) & (R - 1)];
      wave_sync();
    }
    const uint32_t last = 63u - (uint32_t)__clzll(tm);
    const uint32_t nq = readlane(pos + len, last);
    for (uint32_t k = q + lane; k < nq; k += 64) out[k] = ring[k & (R - 1)];
    wave_sync();
    t += popc64(tm);
    u += S * popc64(lm & tm) + 2u * popc64(pm & tm);
    q = nq;
  }
  if ((t + 7) / 8 != F || u != P) return false;
  if (t < 8ull * F && (flags[F - 1] >> (uint32_t)(t - 8ull * (F - 1))) != 0) return false;
  return true;
}

// Decode chunk i of a validated stream (wave-wide); false if it is corrupt.
__device__ inline bool decode_stream_chunk(const uint8_t* in, const DecodeParams& p,
                                           const uint64_t* group_off, uint64_t i, uint8_t* out,
                                           uint8_t* ring) {
  const uint8_t* e = in + kHeaderBytes + 8 * i;
  const uint32_t F = *reinterpret_cast<const uint32_t*>(e);
  const uint32_t P = *reinterpret_cast<const uint32_t*>(e + 4);
  const uint8_t* rec = in + record_offset(in, group_off, i);
  const uint64_t cs = i * p.C;
  const uint32_t c = (uint32_t)min<uint64_t>(p.C, p.m - cs);
  uint8_t* dst = out + cs * p.S;
  switch (p.S) {
    case 1: return decode_chunk<1>(rec, F, P, c, p.W, p.MIN, reinterpret_cast<uint8_t*>(dst), ring);
    case 2: return decode_chunk<2>(rec, F, P, c, p.W, p.MIN, reinterpret_cast<uint16_t*>(dst), ring);
    case 4: return decode_chunk<4>(rec, F, P, c, p.W, p.MIN, reinterpret_cast<uint32_t*>(dst), ring);
    default: return decode_chunk<8>(rec, F, P, c, p.W, p.MIN, reinterpret_cast<uint64_t*>(dst), ring);
  }
}

}  // namespace dec
}  // namespace gpulz
