// Global prefix sum over chunk record sizes, stream header, and compaction
// of the per-chunk records into one stream (gpuLZ sections 3.2.2 and 3.3.3:
// the second pass of the two-pass prefix sum; section 3.3.4: deflating).
//
// The paper scans flag sizes and payload sizes separately and writes two
// output regions; here each chunk's record is flags followed by payload, so
// a single scan of F_i + P_i gives every record's position.
#include "gpulz_internal.h"
#include "wave.h"

namespace gpulz {
namespace {

constexpr uint32_t kScanThreads = 1024;
constexpr uint32_t kScanItems = 16;

__device__ uint8_t header_byte(uint32_t b, const ScanArgs& a, uint64_t total) {
  const uint32_t r = (uint32_t)(a.nbytes % a.S);
  const uint64_t N = a.N;
  switch (b) {
    case 0: return 'G';
    case 1: return 'L';
    case 2: return 'Z';
    case 3: return '1';
    case 4: return 1;  // version
    case 6: return (uint8_t)a.S;
    case 14: return (uint8_t)a.MIN;
    case 15: return (uint8_t)kMaxMatch;
    case 40: return (uint8_t)r;
    default: break;
  }
  if (b >= 8 && b < 12) return (uint8_t)(a.C >> (8 * (b - 8)));
  if (b >= 12 && b < 14) return (uint8_t)(a.W >> (8 * (b - 12)));
  if (b >= 16 && b < 24) return (uint8_t)(a.nbytes >> (8 * (b - 16)));
  if (b >= 24 && b < 32) return (uint8_t)(N >> (8 * (b - 24)));
  if (b >= 32 && b < 40) return (uint8_t)(total >> (8 * (b - 32)));
  if (b >= 48 && b < 48 + r) return a.in[a.nbytes - r + (b - 48)];
  return 0;
}

__global__ __launch_bounds__(kScanThreads) void scan_kernel(ScanArgs a) {
  __shared__ uint64_t wave_pre[kScanThreads / 64];
  __shared__ uint64_t tile_total;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
  const uint64_t tile = (uint64_t)kScanThreads * kScanItems;
  uint64_t carry = 0;
  for (uint64_t base = 0; base < a.N; base += tile) {
    uint64_t v[kScanItems];
    uint64_t local = 0;
#pragma unroll
    for (uint32_t j = 0; j < kScanItems; ++j) {
      const uint64_t i = base + (uint64_t)tid * kScanItems + j;
      v[j] = i < a.N ? (uint64_t)a.sizes[2 * i] + a.sizes[2 * i + 1] : 0;
      local += v[j];
    }
    const uint64_t incl = wave_incl_scan_u64(local);
    if (lane == 63) wave_pre[wid] = incl;
    __syncthreads();
    if (wid == 0) {
      const uint64_t w = lane < kScanThreads / 64 ? wave_pre[lane] : 0;
      const uint64_t wi = wave_incl_scan_u64(w);
      if (lane < kScanThreads / 64) wave_pre[lane] = wi - w;
      if (lane == kScanThreads / 64 - 1) tile_total = wi;
    }
    __syncthreads();
    uint64_t run = carry + wave_pre[wid] + incl - local;
#pragma unroll
    for (uint32_t j = 0; j < kScanItems; ++j) {
      const uint64_t i = base + (uint64_t)tid * kScanItems + j;
      if (i < a.N) a.offsets[i] = run;
      run += v[j];
    }
    carry += tile_total;
    __syncthreads();
  }
  const uint64_t total = kHeaderBytes + 8 * a.N + carry;
  if (tid == 0) {
    a.offsets[a.N] = carry;
    *a.out_bytes = total;
    *a.status = total <= a.capacity ? kOk : kOutOfSpace;
  }
  if (total <= a.capacity && tid < kHeaderBytes) a.out[tid] = header_byte(tid, a, total);
}

// Copies len bytes from a 4-byte aligned source to any destination: bytes up
// to the first aligned destination word, whole aligned words in between
// (each funnel-shifted from two source words), then the last bytes. Edge
// bytes are written one by one so that neighbouring records that share a
// destination word never overwrite each other. The source may be read up to
// 4 bytes past its end.
__device__ void copy_bytes(uint8_t* dst, const uint8_t* src, uint32_t len, uint32_t tid,
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
  copy_bytes(rec, slot, F, tid, blockDim.x);
  copy_bytes(rec + F, slot + a.flag_area, P, tid, blockDim.x);
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
