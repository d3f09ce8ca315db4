// Device helpers for writing streams: the header and record compaction.
#pragma once

#include "gpulz_internal.h"
#include "wave.h"

namespace gpulz {
namespace stream {

// Byte b (0..63) of the stream header; `tail` holds the n mod S bytes after
// the last whole symbol. The one definition of the header layout, used by
// the kernels and by the host entry point gpulz_write_header.
__host__ __device__ inline uint8_t header_byte(uint32_t b, uint64_t n, uint32_t S, uint32_t C,
                                               uint32_t W, uint32_t MIN, uint32_t policy,
                                               uint64_t N, uint64_t total, const uint8_t* tail) {
  const uint32_t r = (uint32_t)(n % S);
  switch (b) {
    case 0: return 'G';
    case 1: return 'L';
    case 2: return 'Z';
    case 3: return '1';
    case 4: return 1;  // version
    case 6: return (uint8_t)S;
    case 7: return (uint8_t)policy;  // match policy
    case 14: return (uint8_t)MIN;
    case 15: return (uint8_t)kMaxMatch;
    case 40: return (uint8_t)r;
    default: break;
  }
  if (b >= 8 && b < 12) return (uint8_t)(C >> (8 * (b - 8)));
  if (b >= 12 && b < 14) return (uint8_t)(W >> (8 * (b - 12)));
  if (b >= 16 && b < 24) return (uint8_t)(n >> (8 * (b - 16)));
  if (b >= 24 && b < 32) return (uint8_t)(N >> (8 * (b - 24)));
  if (b >= 32 && b < 40) return (uint8_t)(total >> (8 * (b - 32)));
  if (b >= 48 && b < 48 + r) return tail[b - 48];
  return 0;
}

// Copies len bytes from a 16-byte aligned source to any destination: bytes
// up to the first 16-byte aligned destination word, whole aligned 16-byte
// words in between (each funnel-shifted from two source words), then the
// last bytes. Edge bytes are written one by one so that neighbouring records
// that share a destination word never overwrite each other. The source may
// be read up to 16 bytes past its end (scratch slots keep that slack).
__device__ inline void copy_bytes(uint8_t* dst, const uint8_t* src, uint32_t len, uint32_t tid,
                                  uint32_t nthreads) {
  // bytes up to dst's first 16-byte boundary
  uint32_t head = (uint32_t)((16u - ((uintptr_t)dst & 15u)) & 15u);
  if (head > len) head = len;
  for (uint32_t b = tid; b < head; b += nthreads) dst[b] = src[b];
  // whole 16-byte words of dst; each one's source starts `head` bytes into
  // a 16-byte source word (the same for all), so it is funnel-shifted out of
  // two aligned source words
  const uint32_t nw = (len - head) / 16;
  uint4* d4 = reinterpret_cast<uint4*>(dst + head);
  const uint4* s4 = reinterpret_cast<const uint4*>(src);
  const uint32_t r = head & 3u;
  switch (head >> 2) {
#define GPULZ_COPY_CASE(Q)                                                                   \
  case Q:                                                                                    \
    for (uint32_t k = tid; k < nw; k += nthreads) {                                          \
      const uint4 a = s4[k];                                                                 \
      const uint4 b = (Q == 0 && r == 0) ? a : s4[k + 1];                                    \
      const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};                        \
      uint4 o;                                                                               \
      o.x = __builtin_amdgcn_alignbyte(w[Q + 1], w[Q], r);                                   \
      o.y = __builtin_amdgcn_alignbyte(w[Q + 2], w[Q + 1], r);                               \
      o.z = __builtin_amdgcn_alignbyte(w[Q + 3], w[Q + 2], r);                               \
      o.w = __builtin_amdgcn_alignbyte(w[Q + 4], w[Q + 3], r);                               \
      d4[k] = o;                                                                             \
    }                                                                                        \
    break;
    GPULZ_COPY_CASE(0)
    GPULZ_COPY_CASE(1)
    GPULZ_COPY_CASE(2)
    GPULZ_COPY_CASE(3)
#undef GPULZ_COPY_CASE
  }
  // the rest
  for (uint32_t b = head + 16 * nw + tid; b < len; b += nthreads) dst[b] = src[b];
}

// Writes len zero bytes at any destination: bytes up to the first 16-byte
// boundary, aligned 16-byte words, then the last bytes (the edges never touch
// a neighbour's bytes).
__device__ inline void fill_zero(uint8_t* dst, uint64_t len, uint32_t tid, uint32_t nthreads) {
  uint64_t head = (16u - ((uintptr_t)dst & 15u)) & 15u;
  if (head > len) head = len;
  for (uint64_t b = tid; b < head; b += nthreads) dst[b] = 0;
  const uint64_t nw = (len - head) / 16;
  uint4* d4 = reinterpret_cast<uint4*>(dst + head);
  for (uint64_t k = tid; k < nw; k += nthreads) d4[k] = make_uint4(0u, 0u, 0u, 0u);
  for (uint64_t b = head + 16 * nw + tid; b < len; b += nthreads) dst[b] = 0;
}

// Workgroup-wide exclusive scan of F_i + P_i over N chunks (sizes holds
// {F, P} pairs) into offs; returns the total. blockDim is a multiple of 64;
// `scratch` holds blockDim/64 + 1 u64.
template <uint32_t ITEMS>
__device__ inline uint64_t scan_record_sizes(const uint32_t* sizes, uint64_t N, uint64_t* offs,
                                             uint64_t* scratch) {
  static_assert(ITEMS % 2 == 0, "items come in pairs (16-byte loads)");
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
  const uint32_t nw = blockDim.x >> 6;
  const uint64_t tile = (uint64_t)blockDim.x * ITEMS;
  // a tile's record bytes fit in 32 bits (records are at most ~104 KB), so
  // the scans inside a tile are 32-bit register (DPP) scans
  // 16-byte loads and stores when both arrays are 16-byte aligned (a
  // thread's first item index is a multiple of ITEMS, which is even)
  const bool vec = (((uintptr_t)sizes | (uintptr_t)offs) & 15u) == 0;
  uint64_t carry = 0;
  for (uint64_t base = 0; base < N; base += tile) {
    const uint64_t i0 = base + (uint64_t)tid * ITEMS;  // this thread's first item
    uint32_t v[ITEMS];
    uint32_t local = 0;
    if (vec && i0 + ITEMS <= N) {
      const uint4* s4 = reinterpret_cast<const uint4*>(sizes + 2 * i0);
#pragma unroll
      for (uint32_t j = 0; j < ITEMS / 2; ++j) {
        const uint4 q = s4[j];
        v[2 * j] = q.x + q.y;
        v[2 * j + 1] = q.z + q.w;
      }
    } else {
#pragma unroll
      for (uint32_t j = 0; j < ITEMS; ++j) {
        const uint64_t i = i0 + j;
        v[j] = i < N ? sizes[2 * i] + sizes[2 * i + 1] : 0u;
      }
    }
#pragma unroll
    for (uint32_t j = 0; j < ITEMS; ++j) local += v[j];
    const uint32_t incl = wave_incl_scan(local);
    if (lane == 63) scratch[wid] = incl;
    __syncthreads();
    uint64_t before = 0, total = 0;
    for (uint32_t w = 0; w < nw; ++w) {
      const uint64_t x = scratch[w];
      before += w < wid ? x : 0ull;
      total += x;
    }
    uint64_t run = carry + before + incl - local;
    if (vec && i0 + ITEMS <= N) {
      uint4* o4 = reinterpret_cast<uint4*>(offs + i0);
#pragma unroll
      for (uint32_t j = 0; j < ITEMS / 2; ++j) {
        const uint64_t a = run, b = run + v[2 * j];
        run = b + v[2 * j + 1];
        o4[j] = make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32));
      }
    } else {
#pragma unroll
      for (uint32_t j = 0; j < ITEMS; ++j) {
        const uint64_t i = i0 + j;
        if (i < N) offs[i] = run;
        run += v[j];
      }
    }
    carry += total;
    __syncthreads();
  }
  return carry;
}

}  // namespace stream
}  // namespace gpulz
