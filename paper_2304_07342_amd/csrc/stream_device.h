// Device helpers for writing streams: the header and record compaction.
#pragma once

#include "gpulz_internal.h"
#include "wave.h"

namespace gpulz {
namespace stream {

// Byte b (0..63) of the stream header.
__device__ inline uint8_t header_byte(uint32_t b, uint64_t n, uint32_t S, uint32_t C, uint32_t W,
                                      uint32_t MIN, uint64_t N, uint64_t total,
                                      const uint8_t* in) {
  const uint32_t r = (uint32_t)(n % S);
  switch (b) {
    case 0: return 'G';
    case 1: return 'L';
    case 2: return 'Z';
    case 3: return '1';
    case 4: return 1;  // version
    case 6: return (uint8_t)S;
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
  if (b >= 48 && b < 48 + r) return in[n - r + (b - 48)];
  return 0;
}

// Copies len bytes from a 4-byte aligned source to any destination: bytes up
// to the first aligned destination word, whole aligned words in between
// (each funnel-shifted from two source words), then the last bytes. Edge
// bytes are written one by one so that neighbouring records that share a
// destination word never overwrite each other. The source may be read up to
// 4 bytes past its end.
__device__ inline void copy_bytes(uint8_t* dst, const uint8_t* src, uint32_t len, uint32_t tid,
                                  uint32_t nthreads) {
  uint32_t head = (uint32_t)((4u - ((uintptr_t)dst & 3u)) & 3u);
  if (head > len) head = len;
  if (tid < head) dst[tid] = src[tid];
  const uint32_t body = (len - head) / 4;
  uint32_t* dw = reinterpret_cast<uint32_t*>(dst + head);
  const uint32_t* sw = reinterpret_cast<const uint32_t*>(src);
  const uint32_t sh = head & 3u;
  for (uint32_t k = tid; k < body; k += nthreads) {
    const uint32_t o = (head + 4 * k) >> 2;
    const uint32_t lo = sw[o];
    dw[k] = sh ? __builtin_amdgcn_alignbyte(sw[o + 1], lo, sh) : lo;
  }
  const uint32_t done = head + 4 * body;
  if (tid < len - done) dst[done + tid] = src[done + tid];
}

// Workgroup-wide exclusive scan of F_i + P_i over N chunks (sizes holds
// {F, P} pairs) into offs; returns the total. blockDim is a multiple of 64;
// `scratch` holds blockDim/64 + 1 u64.
template <uint32_t ITEMS>
__device__ inline uint64_t scan_record_sizes(const uint32_t* sizes, uint64_t N, uint64_t* offs,
                                             uint64_t* scratch) {
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
  const uint32_t nw = blockDim.x >> 6;
  const uint64_t tile = (uint64_t)blockDim.x * ITEMS;
  uint64_t carry = 0;
  for (uint64_t base = 0; base < N; base += tile) {
    uint64_t v[ITEMS];
    uint64_t local = 0;
#pragma unroll
    for (uint32_t j = 0; j < ITEMS; ++j) {
      const uint64_t i = base + (uint64_t)tid * ITEMS + j;
      v[j] = i < N ? (uint64_t)sizes[2 * i] + sizes[2 * i + 1] : 0;
      local += v[j];
    }
    const uint64_t incl = wave_incl_scan_u64(local);
    if (lane == 63) scratch[wid] = incl;
    __syncthreads();
    if (wid == 0) {
      const uint64_t w = lane < nw ? scratch[lane] : 0;
      const uint64_t wi = wave_incl_scan_u64(w);
      if (lane < nw) scratch[lane] = wi - w;
      if (lane == nw - 1) scratch[nw] = wi;
    }
    __syncthreads();
    uint64_t run = carry + scratch[wid] + incl - local;
#pragma unroll
    for (uint32_t j = 0; j < ITEMS; ++j) {
      const uint64_t i = base + (uint64_t)tid * ITEMS + j;
      if (i < N) offs[i] = run;
      run += v[j];
    }
    carry += scratch[nw];
    __syncthreads();
  }
  return carry;
}

}  // namespace stream
}  // namespace gpulz
