// Global prefix sum over chunk record sizes, stream header, and compaction
// of the per-chunk records into one stream (gpuLZ sections 3.2.2 and 3.3.3:
// the second pass of the two-pass prefix sum; section 3.3.4: deflating).
//
// The paper scans flag sizes and payload sizes separately and writes two
// output regions; here each chunk's record is flags followed by payload, so
// a single scan of F_i + P_i gives every record's position.
#include "stream_device.h"

namespace gpulz {
namespace {

constexpr uint32_t kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void scan_kernel(ScanArgs a) {
  __shared__ uint64_t scratch[kScanThreads / 64 + 1];
  const uint64_t sum = stream::scan_record_sizes<16>(a.sizes, a.N, a.offsets, scratch);
  const uint64_t total = kHeaderBytes + 8 * a.N + sum;
  const uint32_t tid = threadIdx.x;
  if (tid == 0) {
    a.offsets[a.N] = sum;
    *a.out_bytes = total;
    *a.status = total <= a.capacity ? kOk : kOutOfSpace;
  }
  if (total <= a.capacity && tid < kHeaderBytes)
    a.out[tid] = stream::header_byte(tid, a.nbytes, a.S, a.C, a.W, a.MIN, a.policy, a.N, total, a.in);
}

__global__ __launch_bounds__(256) void scatter_kernel(ScatterArgs a) {
  const uint64_t i = blockIdx.x;
  const uint64_t total = kHeaderBytes + 8 * a.N + a.offsets[a.N];
  if (total > a.capacity) return;
  const uint32_t F = a.sizes[2 * i], P = a.sizes[2 * i + 1];
  const uint32_t tid = threadIdx.x;
  if (tid < 8) {
    const uint32_t v = tid < 4 ? F : P;
    a.out[kHeaderBytes + 8 * i + tid] = (uint8_t)(v >> (8 * (tid & 3u)));
  }
  uint8_t* rec = a.out + kHeaderBytes + 8 * a.N + a.offsets[i];
  const uint8_t* slot = a.slots + i * a.slot_bytes;
  stream::copy_bytes(rec, slot, F, tid, blockDim.x);
  stream::copy_bytes(rec + F, slot + a.flag_area, P, tid, blockDim.x);
}

}  // namespace

hipError_t launch_scan(const ScanArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(kScanThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_scatter(const ScatterArgs& a, hipStream_t s) {
  if (a.N == 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_kernel, dim3((uint32_t)a.N), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace gpulz
