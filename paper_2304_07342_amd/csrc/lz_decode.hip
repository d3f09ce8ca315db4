// Decoder. The paper states that decompression exists and is easy to
// parallelise (section 4.4) without describing it; this one follows from
// the stream layout:
//   prepare  one workgroup validates the header and prefix-sums the table
//            into absolute record offsets (checking that the records exactly
//            fill the stream);
//   decode   one wavefront per chunk walks the tokens 64 at a time: lane l
//            takes token t + l, its flag bit gives its kind, mbcnt over the
//            literal / pointer ballots gives its payload offset, a wave scan
//            of the token lengths gives its output position. Literals are
//            written into an LDS ring of recent symbols; pointers are then
//            resolved in token order, each copied by all 64 lanes (a pointer
//            never overlaps itself because its length never exceeds its
//            offset). Finished symbols stream out to HBM. The ring keeps the
//            last 256 symbols (the largest offset), so LDS use does not depend
//            on the chunk size.
// Every rule the encoder guarantees is checked; a broken one sets
// GPULZ_ERR_CORRUPT and stops that chunk.
#include "gpulz_internal.h"
#include "wave.h"

namespace gpulz {
namespace {

constexpr uint32_t kPrepThreads = 1024;
constexpr uint32_t kPrepItems = 8;
constexpr uint32_t kDecodeBlocks = 256 * 16;

__device__ uint64_t rd_u64(const uint8_t* p) {
  uint64_t v = 0;
  for (int k = 7; k >= 0; --k) v = (v << 8) | p[k];
  return v;
}
__device__ uint32_t rd_u32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

__global__ __launch_bounds__(kPrepThreads) void decode_prepare_kernel(DecodePrepArgs a) {
  __shared__ DecodeParams P;
  __shared__ uint64_t wave_pre[kPrepThreads / 64];
  __shared__ uint64_t tile_total;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
  if (tid == 0) {
    DecodeParams p = {};
    bool ok = a.in_bytes >= kHeaderBytes;
    if (ok) {
      const uint8_t* h = a.in;
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
        ok = p.r == p.n % p.S && p.N == (p.m + p.C - 1) / p.C && total == a.in_bytes &&
             p.N <= a.max_chunks;
        for (uint32_t k = 41; k < 48; ++k) ok = ok && h[k] == 0;
        for (uint32_t k = 48 + p.r; k < 64; ++k) ok = ok && h[k] == 0;
      }
    }
    p.status = ok ? kOk : kCorrupt;
    P = p;
  }
  __syncthreads();
  if (P.status != kOk) {
    if (tid == 0) {
      *a.params = P;
      *a.out_bytes = 0;
      *a.status = kCorrupt;
    }
    return;
  }
  const uint64_t N = P.N;
  const uint64_t first = kHeaderBytes + 8 * N;
  const uint64_t tile = (uint64_t)kPrepThreads * kPrepItems;
  uint64_t carry = 0;
  for (uint64_t base = 0; base < N; base += tile) {
    uint64_t v[kPrepItems];
    uint64_t local = 0;
#pragma unroll
    for (uint32_t j = 0; j < kPrepItems; ++j) {
      const uint64_t i = base + (uint64_t)tid * kPrepItems + j;
      v[j] = 0;
      if (i < N) {
        const uint32_t* e = reinterpret_cast<const uint32_t*>(a.in + kHeaderBytes + 8 * i);
        v[j] = (uint64_t)e[0] + e[1];
      }
      local += v[j];
    }
    const uint64_t incl = wave_incl_scan_u64(local);
    if (lane == 63) wave_pre[wid] = incl;
    __syncthreads();
    if (wid == 0) {
      const uint64_t w = lane < kPrepThreads / 64 ? wave_pre[lane] : 0;
      const uint64_t wi = wave_incl_scan_u64(w);
      if (lane < kPrepThreads / 64) wave_pre[lane] = wi - w;
      if (lane == kPrepThreads / 64 - 1) tile_total = wi;
    }
    __syncthreads();
    uint64_t run = first + carry + wave_pre[wid] + incl - local;
#pragma unroll
    for (uint32_t j = 0; j < kPrepItems; ++j) {
      const uint64_t i = base + (uint64_t)tid * kPrepItems + j;
      if (i < N) a.offsets[i] = run;
      run += v[j];
    }
    carry += tile_total;
    __syncthreads();
  }
  if (tid == 0) {
    DecodeParams p = P;
    if (first + carry != a.in_bytes) {
      p.status = kCorrupt;
      *a.out_bytes = 0;
    } else {
      p.status = a.capacity < p.n ? kOutOfSpace : kOk;
      *a.out_bytes = p.n;
    }
    a.offsets[N] = first + carry;
    *a.params = p;
    *a.status = p.status;
  }
}

// Decode one chunk; returns false if the chunk breaks a rule.
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

__global__ __launch_bounds__(64) void decode_kernel(DecodeArgs a) {
  __shared__ __align__(16) uint8_t ring[kDecodeRingBytes];
  const DecodeParams p = *a.params;
  if (p.status != kOk) return;
  if (blockIdx.x == 0 && threadIdx.x < p.r) a.out[p.m * p.S + threadIdx.x] = a.in[48 + threadIdx.x];
  for (uint64_t i = blockIdx.x; i < p.N; i += gridDim.x) {
    const uint8_t* e = a.in + kHeaderBytes + 8 * i;
    const uint32_t F = *reinterpret_cast<const uint32_t*>(e);
    const uint32_t P = *reinterpret_cast<const uint32_t*>(e + 4);
    const uint8_t* rec = a.in + a.offsets[i];
    const uint64_t cs = i * p.C;
    const uint32_t c = (uint32_t)min<uint64_t>(p.C, p.m - cs);
    uint8_t* dst = a.out + cs * p.S;
    bool ok;
    switch (p.S) {
      case 1: ok = decode_chunk<1>(rec, F, P, c, p.W, p.MIN, reinterpret_cast<uint8_t*>(dst), ring); break;
      case 2: ok = decode_chunk<2>(rec, F, P, c, p.W, p.MIN, reinterpret_cast<uint16_t*>(dst), ring); break;
      case 4: ok = decode_chunk<4>(rec, F, P, c, p.W, p.MIN, reinterpret_cast<uint32_t*>(dst), ring); break;
      default: ok = decode_chunk<8>(rec, F, P, c, p.W, p.MIN, reinterpret_cast<uint64_t*>(dst), ring); break;
    }
    if (!ok && lane_id() == 0) atomicExch(a.status, kCorrupt);
  }
}

}  // namespace

hipError_t launch_decode_prepare(const DecodePrepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(decode_prepare_kernel, dim3(1), dim3(kPrepThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_decode_chunks(const DecodeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(decode_kernel, dim3(kDecodeBlocks), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace gpulz
