// Single-buffer compression in one pass over the records: a preparation
// kernel, then the chunk encoders (one workgroup per chunk; see
// encode_device.h for the steps), which take chunk ids from an atomic ticket,
// find their record offsets by decoupled look-back and write the table entry
// and record straight into the stream. Match policy 0 (exact longest match)
// and 1 (the paper's single window pass).
#include "encode_device.h"

namespace gpulz {
namespace {

// Launches of at most this many chunks take the split-parse encoder (measured
// crossovers on 256 CUs: about 1.5-2.5 K chunks for 1- and 2-byte symbols,
// 512 for 4-byte ones).
constexpr uint64_t kSpecMaxChunksNarrow = 1024;  // S <= 2
constexpr uint64_t kSpecMaxChunksWide = 512;     // S >= 4

__global__ __launch_bounds__(256) void prep_kernel(FusedArgs a) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = t; k < a.N; k += stride) a.desc[k] = 0;
  if (t < kMaxTickets) a.tickets[t] = 0;
  if (a.N == 0 && blockIdx.x == 0) {
    // no chunk: the stream is the header alone
    const uint64_t total = kHeaderBytes;
    const bool fits = total <= a.capacity;
    if (threadIdx.x == 0) {
      *a.out_bytes = total;
      *a.status = fits ? kOk : kOutOfSpace;
    }
    if (fits && threadIdx.x < kHeaderBytes)
      a.out[threadIdx.x] = stream::header_byte(threadIdx.x, a.nbytes, a.S, a.C, a.W, a.MIN,
                                               a.policy, 0, total, a.in + a.nbytes / a.S * a.S);
  }
}

// The chunk this workgroup encodes: the next ticket of this launch (so chunk
// ids follow the order in which workgroups start, which the look-back needs),
// with its stream context.
__device__ __forceinline__ enc::ChunkJob take_chunk(const FusedArgs& a, uint32_t S,
                                                    uint64_t* shared_item) {
  if (threadIdx.x == 0)
    *shared_item = a.chunk0 + atomicAdd((unsigned long long*)&a.tickets[a.launch], 1ull);
  __syncthreads();
  const uint64_t i = *shared_item;
  const uint64_t cs = i * a.C;
  enc::ChunkJob job;
  job.src = a.in + cs * S;
  job.src_avail = a.nbytes - cs * S;
  job.c = (uint32_t)min<uint64_t>(a.C, a.m - cs);
  job.C = a.C;
  job.W = a.W;
  job.MIN = a.MIN;
  job.slot = a.slots + i * a.slot_bytes;
  job.flag_area = a.flag_area;
  job.sizes = nullptr;
  job.i = i;
  job.N = a.N;
  job.desc = a.desc;
  job.out = a.out;
  job.capacity = a.capacity;
  job.in = a.in;
  job.nbytes = a.nbytes;
  job.S = S;
  job.policy = a.policy;
  job.out_bytes = a.out_bytes;
  job.status = a.status;
  return job;
}

template <int S, int WC>
__global__ __launch_bounds__(64 * enc::kEncodeWaves) void encode_kernel(FusedArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ uint64_t item;
  const enc::ChunkJob job = take_chunk(a, S, &item);
  enc::encode_chunk<S, WC, true>(job, lds);
}

// The same encoder with the parse split across kSpecWaves waves, for
// launches with few chunks (then the serial parse of one chunk per CU is the
// whole run time).
template <int S, int WC>
__global__ __launch_bounds__(64 * enc::kSpecWaves) void encode_spec_kernel(FusedArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ uint64_t item;
  const enc::ChunkJob job = take_chunk(a, S, &item);
  enc::encode_chunk_spec<S, WC>(job, lds);
}

// Policy-1 chunk encoder kernel: one workgroup per chunk.
template <int S>
__global__ __launch_bounds__(64 * enc::kEncodeWaves) void encode_scan_kernel(FusedArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ uint64_t item;
  const enc::ChunkJob job = take_chunk(a, S, &item);
  enc::encode_chunk_scan<S>(job, lds);
}

template <int S, int WC>
hipError_t launch_sw(const FusedArgs& a, uint32_t waves, hipStream_t s) {
  const size_t spec_lds = enc::spec_lds_bytes<S, WC>(a.C);
  const uint64_t spec_max = S <= 2 ? kSpecMaxChunksNarrow : kSpecMaxChunksWide;
  if (a.N <= spec_max && a.C <= enc::kSpecMaxSyms && spec_lds <= kMaxGroupLdsBytes) {
    hipLaunchKernelGGL((encode_spec_kernel<S, WC>), dim3((uint32_t)a.nchunks),
                       dim3(64 * enc::kSpecWaves), spec_lds, s, a);
    return hipGetLastError();
  }
  const size_t lds = enc::lds_bytes<S, WC>(a.C, waves);
  hipLaunchKernelGGL((encode_kernel<S, WC>), dim3((uint32_t)a.nchunks), dim3(64 * waves), lds, s, a);
  return hipGetLastError();
}

template <int S>
hipError_t launch_s(const FusedArgs& a, uint32_t waves, hipStream_t s) {
  if (a.policy == 1) {
    const size_t lds = enc::scan_lds_bytes(a.C, S);
    hipLaunchKernelGGL((encode_scan_kernel<S>), dim3((uint32_t)a.nchunks), dim3(64 * waves), lds,
                       s, a);
    return hipGetLastError();
  }
  switch ((a.W + 63) / 64) {
    case 1: return launch_sw<S, 1>(a, waves, s);
    case 2: return launch_sw<S, 2>(a, waves, s);
    case 3: return launch_sw<S, 3>(a, waves, s);
    default: return launch_sw<S, 4>(a, waves, s);
  }
}

}  // namespace

size_t encode_scan_lds_bytes(uint32_t C, uint32_t S) { return enc::scan_lds_bytes(C, S); }

size_t encode_lds_bytes(uint32_t C, uint32_t S, uint32_t W, uint32_t waves) {
  return enc::encode_lds(C, S, (W + 63) / 64, waves);
}

hipError_t launch_fused_prep(const FusedArgs& a, hipStream_t s) {
  const uint64_t want = (a.N + 2047) / 2048 + 1;
  const uint64_t blocks = want < 1024 ? want : 1024;
  hipLaunchKernelGGL(prep_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fused_encode(const FusedArgs& a, uint32_t waves, hipStream_t s) {
  if (a.nchunks == 0) return hipSuccess;
  switch (a.S) {
    case 1: return launch_s<1>(a, waves, s);
    case 2: return launch_s<2>(a, waves, s);
    case 4: return launch_s<4>(a, waves, s);
    default: return launch_s<8>(a, waves, s);
  }
}

}  // namespace gpulz
