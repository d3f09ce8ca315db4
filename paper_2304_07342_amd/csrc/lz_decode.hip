// Single-buffer decoder kernels (the steps are in decode_device.h):
//   decode_prepare_kernel  one workgroup checks the header, prefix-sums the
//                          table into per-group record offsets, checks the
//                          sums and the output capacity;
//   decode_kernel          one workgroup of 256 threads per chunk, grid-stride
//                          over chunks.
#include "decode_device.h"

namespace gpulz {
namespace {

constexpr uint32_t kPrepThreads = 1024;
constexpr uint32_t kDecodeBlocks = 256 * 4;  // 4 workgroups of ~33 KiB LDS per CU

__global__ __launch_bounds__(kPrepThreads) void decode_prepare_kernel(DecodePrepArgs a) {
  __shared__ DecodeParams P;
  __shared__ uint64_t scratch[kPrepThreads / 64 + 1];
  if (threadIdx.x == 0) dec::parse_header(a.in, a.in_bytes, P);
  __syncthreads();
  if (P.status != kOk) {
    if (threadIdx.x == 0) {
      *a.params = P;
      *a.out_bytes = 0;
      *a.status = kCorrupt;
    }
    return;
  }
  const uint64_t end = dec::scan_table_groups(a.in, P.N, a.group_off, scratch);
  if (threadIdx.x == 0) {
    DecodeParams p = P;
    if (end != a.in_bytes) {
      p.status = kCorrupt;
      *a.out_bytes = 0;
    } else {
      p.status = a.capacity < p.n ? kOutOfSpace : kOk;
      *a.out_bytes = p.n;
    }
    *a.params = p;
    *a.status = p.status;
  }
}

__global__ __launch_bounds__(dec::kDecThreads, 4) void decode_kernel(DecodeArgs a) {
  __shared__ __align__(16) dec::BlockLds sm;
  const DecodeParams p = *a.params;
  if (p.status != kOk) return;
  if (blockIdx.x == 0 && threadIdx.x < p.r) a.out[p.m * p.S + threadIdx.x] = a.in[48 + threadIdx.x];
  for (uint64_t i = blockIdx.x; i < p.N; i += gridDim.x) {
    const bool ok = dec::decode_stream_chunk_block(a.in, a.in_bytes, p, a.group_off, i, a.out, sm);
    if (!ok && threadIdx.x == 0) atomicExch(a.status, kCorrupt);
  }
}

// One workgroup: tiles of 4 entries per thread, a wave scan and a scan of
// the wave totals per tile, the running total carried across tiles.
__global__ __launch_bounds__(kPrepThreads) void record_offsets_kernel(const uint32_t* table,
                                                                      uint64_t chunks,
                                                                      uint64_t* offsets) {
  constexpr uint32_t kPer = 4;
  __shared__ uint64_t wsum[kPrepThreads / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
  const uint32_t nw = blockDim.x >> 6;
  const uint64_t tile = (uint64_t)blockDim.x * kPer;
  uint64_t carry = 0;
  for (uint64_t base = 0; base < chunks; base += tile) {
    const uint64_t i0 = base + (uint64_t)tid * kPer;
    uint64_t sz[kPer];
    uint64_t v = 0;
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
      sz[k] = i0 + k < chunks ? (uint64_t)table[2 * (i0 + k)] + table[2 * (i0 + k) + 1] : 0ull;
      v += sz[k];
    }
    const uint64_t incl = wave_incl_scan_u64(v);
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    uint64_t before = 0, total = 0;
    for (uint32_t w = 0; w < nw; ++w) {
      const uint64_t x = wsum[w];
      before += w < wid ? x : 0ull;
      total += x;
    }
    uint64_t o = carry + before + incl - v;
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
      if (i0 + k < chunks) offsets[i0 + k] = o;
      o += sz[k];
    }
    carry += total;
    __syncthreads();
  }
  if (tid == 0) offsets[chunks] = carry;
}

}  // namespace

hipError_t launch_record_offsets(const uint32_t* table, uint64_t chunks, uint64_t* offsets,
                                 hipStream_t s) {
  hipLaunchKernelGGL(record_offsets_kernel, dim3(1), dim3(kPrepThreads), 0, s, table, chunks,
                     offsets);
  return hipGetLastError();
}

hipError_t launch_decode_prepare(const DecodePrepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(decode_prepare_kernel, dim3(1), dim3(kPrepThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_decode_chunks(const DecodeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(decode_kernel, dim3(kDecodeBlocks), dim3(dec::kDecThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace gpulz
