// Single-buffer chunk encoder kernels: one workgroup of 1, 2 or 4 wavefronts
// per chunk (see encode_device.h for the steps), for match policy 0 (exact
// longest match) and 1 (the paper's single window pass).
#include "encode_device.h"

namespace gpulz {
namespace {

// Launches of at most this many chunks take the split-parse encoder (measured
// crossovers on 256 CUs: about 1.5-2.5 K chunks for 1- and 2-byte symbols,
// 512 for 4-byte ones).
constexpr uint64_t kSpecMaxChunksNarrow = 1024;  // S <= 2
constexpr uint64_t kSpecMaxChunksWide = 512;     // S >= 4

template <int S, int WC>
__global__ __launch_bounds__(64 * enc::kEncodeWaves) void encode_kernel(EncodeArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  const uint64_t chunk = blockIdx.x;
  const uint64_t cs = chunk * a.C;
  enc::ChunkJob job;
  job.src = a.in + cs * S;
  job.src_avail = a.nbytes - cs * S;
  job.c = (uint32_t)min<uint64_t>(a.C, a.m - cs);
  job.C = a.C;
  job.W = a.W;
  job.MIN = a.MIN;
  job.slot = a.slots + chunk * a.slot_bytes;
  job.flag_area = a.flag_area;
  job.sizes = a.sizes + 2 * chunk;
  enc::encode_chunk<S, WC>(job, lds);
}

// The same encoder with the parse split across kSpecWaves waves, for
// launches with few chunks (then the serial parse of one chunk per CU is the
// whole run time).
template <int S, int WC>
__global__ __launch_bounds__(64 * enc::kSpecWaves) void encode_spec_kernel(EncodeArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  const uint64_t chunk = blockIdx.x;
  const uint64_t cs = chunk * a.C;
  enc::ChunkJob job;
  job.src = a.in + cs * S;
  job.src_avail = a.nbytes - cs * S;
  job.c = (uint32_t)min<uint64_t>(a.C, a.m - cs);
  job.C = a.C;
  job.W = a.W;
  job.MIN = a.MIN;
  job.slot = a.slots + chunk * a.slot_bytes;
  job.flag_area = a.flag_area;
  job.sizes = a.sizes + 2 * chunk;
  enc::encode_chunk_spec<S, WC>(job, lds);
}

template <int S, int WC>
hipError_t launch_sw(const EncodeArgs& a, uint64_t N, uint32_t waves, hipStream_t s) {
  const size_t spec_lds = enc::spec_lds_bytes<S, WC>(a.C);
  const uint64_t spec_max = S <= 2 ? kSpecMaxChunksNarrow : kSpecMaxChunksWide;
  if (N <= spec_max && a.C <= enc::kSpecMaxSyms && spec_lds <= kMaxGroupLdsBytes) {
    hipLaunchKernelGGL((encode_spec_kernel<S, WC>), dim3((uint32_t)N), dim3(64 * enc::kSpecWaves),
                       spec_lds, s, a);
    return hipGetLastError();
  }
  const size_t lds = enc::lds_bytes<S, WC>(a.C);
  hipLaunchKernelGGL((encode_kernel<S, WC>), dim3((uint32_t)N), dim3(64 * waves), lds, s, a);
  return hipGetLastError();
}
template <int S>
hipError_t launch_s(const EncodeArgs& a, uint64_t N, uint32_t waves, hipStream_t s) {
  switch ((a.W + 63) / 64) {
    case 1: return launch_sw<S, 1>(a, N, waves, s);
    case 2: return launch_sw<S, 2>(a, N, waves, s);
    case 3: return launch_sw<S, 3>(a, N, waves, s);
    default: return launch_sw<S, 4>(a, N, waves, s);
  }
}

// Policy-1 chunk encoder kernel: one workgroup per chunk.
template <int S>
__global__ __launch_bounds__(64 * enc::kEncodeWaves) void encode_scan_kernel(EncodeArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  const uint64_t chunk = blockIdx.x;
  const uint64_t cs = chunk * a.C;
  enc::ChunkJob job;
  job.src = a.in + cs * S;
  job.src_avail = a.nbytes - cs * S;
  job.c = (uint32_t)min<uint64_t>(a.C, a.m - cs);
  job.C = a.C;
  job.W = a.W;
  job.MIN = a.MIN;
  job.slot = a.slots + chunk * a.slot_bytes;
  job.flag_area = a.flag_area;
  job.sizes = a.sizes + 2 * chunk;
  enc::encode_chunk_scan<S>(job, lds);
}

template <int S>
hipError_t launch_scan_s(const EncodeArgs& a, uint64_t N, uint32_t waves, hipStream_t s) {
  const size_t lds = enc::scan_lds_bytes(a.C, S);
  hipLaunchKernelGGL((encode_scan_kernel<S>), dim3((uint32_t)N), dim3(64 * waves), lds, s, a);
  return hipGetLastError();
}

}  // namespace

size_t encode_scan_lds_bytes(uint32_t C, uint32_t S) { return enc::scan_lds_bytes(C, S); }

hipError_t launch_encode_scan(const EncodeArgs& a, uint32_t S, uint64_t N, uint32_t waves,
                              hipStream_t s) {
  if (N == 0) return hipSuccess;
  switch (S) {
    case 1: return launch_scan_s<1>(a, N, waves, s);
    case 2: return launch_scan_s<2>(a, N, waves, s);
    case 4: return launch_scan_s<4>(a, N, waves, s);
    default: return launch_scan_s<8>(a, N, waves, s);
  }
}

size_t encode_lds_bytes(uint32_t C, uint32_t S, uint32_t W) {
  return enc::encode_lds(C, S, (W + 63) / 64);
}

hipError_t launch_encode(const EncodeArgs& a, uint32_t S, uint64_t N, uint32_t waves, hipStream_t s) {
  if (N == 0) return hipSuccess;
  switch (S) {
    case 1: return launch_s<1>(a, N, waves, s);
    case 2: return launch_s<2>(a, N, waves, s);
    case 4: return launch_s<4>(a, N, waves, s);
    default: return launch_s<8>(a, N, waves, s);
  }
}

}  // namespace gpulz
