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

}  // namespace

hipError_t launch_decode_prepare(const DecodePrepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(decode_prepare_kernel, dim3(1), dim3(kPrepThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_decode_chunks(const DecodeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(decode_kernel, dim3(kDecodeBlocks), dim3(dec::kDecThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace gpulz
