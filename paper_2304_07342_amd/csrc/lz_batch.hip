// Batches: many buffers of different sizes and symbol widths in one pass.
//
// Compression, all on the stream with no host round trip (so the whole call
// can be captured in a HIP graph):
//   plan     one workgroup validates every buffer, counts its chunks and
//            prefix-sums chunk counts and scratch sizes over the buffers;
//   encode   one persistent launch per symbol width: each workgroup takes
//            (buffer, chunk) work items of that width from the width's atomic
//            ticket, so thousands of uneven buffers balance at chunk grain,
//            and every width runs with its own waves per chunk and LDS size
//            (dense widths parse fastest with many 1-wave workgroups);
//   scan     one workgroup per buffer prefix-sums its chunks' record sizes
//            and writes its header, size and status;
//   scatter  grid-stride over all chunks: table entry and record into the
//            buffer's stream.
// Every buffer's stream is byte-identical to gpulz_compress on that buffer.
//
// Decompression: per-buffer header checks, a prefix sum over buffers of
// chunk counts and record-offset groups, one workgroup per buffer for its
// table, then a persistent decoder over all chunks.
#include "decode_device.h"
#include "encode_device.h"
#include "stream_device.h"

namespace gpulz {
namespace {

constexpr uint32_t kPlanThreads = 1024;

__device__ inline uint32_t width_index(uint32_t S) {
  return S == 1 ? 0u : S == 2 ? 1u : S == 4 ? 2u : 3u;
}

// Largest b with base(b) <= g (base non-decreasing, base(0) = 0).
template <typename F>
__device__ inline uint64_t find_buffer(uint64_t nbufs, uint64_t g, F base) {
  uint64_t lo = 0, hi = nbufs - 1;
  while (lo < hi) {
    const uint64_t mid = (lo + hi + 1) / 2;
    if (base(mid) <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Block-wide exclusive scan of one u64 per thread; returns this thread's
// exclusive prefix and writes the block total to *total.
__device__ inline uint64_t block_excl_scan(uint64_t v, uint64_t* scratch, uint64_t* total) {
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
  const uint32_t nw = blockDim.x >> 6;
  const uint64_t incl = wave_incl_scan_u64(v);
  if (lane == 63) scratch[wid] = incl;
  __syncthreads();
  if (wid == 0) {
    const uint64_t w = lane < nw ? scratch[lane] : 0;
    const uint64_t wi = wave_incl_scan_u64(w);
    if (lane < nw) scratch[lane] = wi - w;
    if (lane == nw - 1) scratch[nw] = wi;
  }
  __syncthreads();
  const uint64_t r = scratch[wid] + incl - v;
  *total = scratch[nw];
  __syncthreads();
  return r;
}

// ---- compression --------------------------------------------------------------

__global__ __launch_bounds__(kPlanThreads) void batch_enc_plan_kernel(BatchEncArgs a) {
  __shared__ uint64_t scratch[kPlanThreads / 64 + 1];
  uint64_t chunk_carry = 0, slot_carry = 0, byte_carry = 0;
  uint64_t width_carry[4] = {0, 0, 0, 0};
  for (uint64_t b0 = 0; b0 < a.nbufs; b0 += blockDim.x) {
    const uint64_t b = b0 + threadIdx.x;
    BatchEncBuf e = {};
    e.status = kOk;
    uint64_t nb = 0;
    uint32_t wi = 4;
    if (b < a.nbufs) {
      const uint32_t S = a.symbol_bytes[b];
      nb = a.in_bytes[b];
      const uintptr_t ip = (uintptr_t)a.in_ptrs[b], op = (uintptr_t)a.out_ptrs[b];
      const bool ok = (S == 1 || S == 2 || S == 4 || S == 8) && (ip & 15) == 0 && (op & 15) == 0 &&
                      (nb == 0 || ip != 0) && (a.out_caps[b] == 0 || op != 0);
      e.n = nb;
      if (ok) {
        const uint32_t w = width_index(S);
        wi = w;
        e.S = S;
        e.C = a.wp.C[w];
        e.W = a.wp.W[w];
        e.MIN = a.wp.MIN[w];
        e.slot_bytes = (uint32_t)a.wp.slot_bytes[w];
        e.flag_area = (uint32_t)a.wp.flag_area[w];
        e.N = (nb / S + e.C - 1) / e.C;
      } else {
        e.status = kInvalidArg;
      }
    }
    uint64_t t_chunks, t_slots, t_bytes;
    const uint64_t xc = block_excl_scan(e.N, scratch, &t_chunks);
    const uint64_t xs = block_excl_scan(e.N * e.slot_bytes, scratch, &t_slots);
    block_excl_scan(nb, scratch, &t_bytes);
#pragma unroll
    for (uint32_t w = 0; w < 4; ++w) {
      uint64_t t_w;
      const uint64_t xw = block_excl_scan(wi == w ? e.N : 0, scratch, &t_w);
      e.width_base[w] = width_carry[w] + xw;
      width_carry[w] += t_w;
    }
    if (b < a.nbufs) {
      e.chunk_base = chunk_carry + xc;
      e.slot_base = slot_carry + xs;
      a.bufs[b] = e;
    }
    chunk_carry += t_chunks;
    slot_carry += t_slots;
    byte_carry += t_bytes;
  }
  const bool fits = chunk_carry <= a.max_chunks && slot_carry <= a.slot_cap &&
                    byte_carry <= a.max_total_in_bytes;
  __syncthreads();
  if (!fits) {
    // the workspace was sized for fewer bytes: no buffer is processed
    for (uint64_t b = threadIdx.x; b < a.nbufs; b += blockDim.x) {
      a.bufs[b].N = 0;
      a.bufs[b].status = kWorkspace;
    }
  }
  if (threadIdx.x < 4) {
    a.ctrl->ticket[threadIdx.x] = 0;
    a.ctrl->T[threadIdx.x] = fits ? width_carry[threadIdx.x] : 0;
  }
  if (threadIdx.x == 0) {
    a.ctrl->T_all = fits ? chunk_carry : 0;
    a.ctrl->slot_total = fits ? slot_carry : 0;
  }
}

template <int S, int WC>
__device__ __forceinline__ void encode_item(const BatchEncArgs& a, uint64_t b, const BatchEncBuf& e,
                                            uint64_t i, uint8_t* lds) {
  const uint64_t cs = i * e.C;
  enc::ChunkJob job;
  job.src = static_cast<const uint8_t*>(a.in_ptrs[b]) + cs * S;
  job.src_avail = e.n - cs * S;
  job.c = (uint32_t)min<uint64_t>(e.C, e.n / S - cs);
  job.C = e.C;
  job.W = e.W;
  job.MIN = e.MIN;
  job.slot = a.slots + e.slot_base + i * e.slot_bytes;
  job.flag_area = e.flag_area;
  job.sizes = a.sizes + 2 * (e.chunk_base + i);
  enc::encode_chunk<S, WC>(job, lds);
}

// Persistent encoder for the chunks of symbol width S (width index WI); the
// window spans WC columns of 64 offsets (one window per width in a batch).
// At least 6 waves per SIMD: the 1-byte encoder then fits in 80 VGPRs (82
// otherwise, 5 waves) without spilling; the other widths need fewer.
template <int S, uint32_t WI, int WC>
__global__ __launch_bounds__(64 * enc::kEncodeWaves) __attribute__((amdgpu_waves_per_eu(6)))
void batch_encode_kernel(BatchEncArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ uint64_t item;
  const uint64_t T = a.ctrl->T[WI];
  if (T == 0) return;
  for (;;) {
    if (threadIdx.x == 0) item = atomicAdd((unsigned long long*)&a.ctrl->ticket[WI], 1ull);
    __syncthreads();
    const uint64_t g = item;
    __syncthreads();
    if (g >= T) break;
    const uint64_t b = find_buffer(a.nbufs, g, [&](uint64_t k) { return a.bufs[k].width_base[WI]; });
    const BatchEncBuf& e = a.bufs[b];
    encode_item<S, WC>(a, b, e, g - e.width_base[WI], lds);
    __syncthreads();
  }
}

__global__ __launch_bounds__(1024) void batch_enc_scan_kernel(BatchEncArgs a) {
  __shared__ uint64_t scratch[1024 / 64 + 1];
  const uint64_t b = blockIdx.x;
  BatchEncBuf& e = a.bufs[b];
  if (e.status != kOk) {
    if (threadIdx.x == 0) {
      a.out_bytes[b] = 0;
      a.status[b] = e.status;
    }
    return;
  }
  const uint64_t sum = stream::scan_record_sizes<4>(a.sizes + 2 * e.chunk_base, e.N,
                                                    a.offs + e.chunk_base, scratch);
  const uint64_t total = kHeaderBytes + 8 * e.N + sum;
  const bool fits = total <= a.out_caps[b];
  if (threadIdx.x < kHeaderBytes && fits) {
    static_cast<uint8_t*>(a.out_ptrs[b])[threadIdx.x] = stream::header_byte(
        threadIdx.x, e.n, e.S, e.C, e.W, e.MIN, 0, e.N, total,
        static_cast<const uint8_t*>(a.in_ptrs[b]) + e.n / e.S * e.S);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a.out_bytes[b] = total;
    a.status[b] = fits ? kOk : kOutOfSpace;
    e.status = fits ? kOk : kOutOfSpace;
  }
}

__global__ __launch_bounds__(256) void batch_scatter_kernel(BatchEncArgs a) {
  const uint64_t T = a.ctrl->T_all;
  for (uint64_t g = blockIdx.x; g < T; g += gridDim.x) {
    const uint64_t b = find_buffer(a.nbufs, g, [&](uint64_t k) { return a.bufs[k].chunk_base; });
    const BatchEncBuf& e = a.bufs[b];
    if (e.status != kOk) continue;
    const uint64_t i = g - e.chunk_base;
    const uint32_t F = a.sizes[2 * g], P = a.sizes[2 * g + 1];
    uint8_t* out = static_cast<uint8_t*>(a.out_ptrs[b]);
    const uint32_t tid = threadIdx.x;
    if (tid < 8) {
      const uint32_t v = tid < 4 ? F : P;
      out[kHeaderBytes + 8 * i + tid] = (uint8_t)(v >> (8 * (tid & 3u)));
    }
    uint8_t* rec = out + kHeaderBytes + 8 * e.N + a.offs[g];
    const uint8_t* slot = a.slots + e.slot_base + i * e.slot_bytes;
    stream::copy_bytes(rec, slot, F, tid, blockDim.x);
    stream::copy_bytes(rec + F, slot + e.flag_area, P, tid, blockDim.x);
  }
}

// ---- decompression ------------------------------------------------------------

__global__ __launch_bounds__(256) void batch_dec_header_kernel(BatchDecArgs a) {
  const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.nbufs) return;
  BatchDecBuf e = {};
  const uintptr_t ip = (uintptr_t)a.in_ptrs[b], op = (uintptr_t)a.out_ptrs[b];
  const uint64_t nb = a.in_bytes[b];
  if ((ip & 15) != 0 || (op & 15) != 0 || (nb != 0 && ip == 0)) {
    e.p.status = kInvalidArg;
  } else {
    dec::parse_header(static_cast<const uint8_t*>(a.in_ptrs[b]), nb, e.p);
  }
  if (e.p.status == kOk) e.groups = (e.p.N + dec::kGroup - 1) / dec::kGroup + 1;
  a.bufs[b] = e;
}

__global__ __launch_bounds__(kPlanThreads) void batch_dec_plan_kernel(BatchDecArgs a) {
  __shared__ uint64_t scratch[kPlanThreads / 64 + 1];
  uint64_t chunk_carry = 0, group_carry = 0, byte_carry = 0;
  for (uint64_t b0 = 0; b0 < a.nbufs; b0 += blockDim.x) {
    const uint64_t b = b0 + threadIdx.x;
    uint64_t n_chunks = 0, n_groups = 0, nb = 0;
    if (b < a.nbufs) {
      nb = a.in_bytes[b];
      if (a.bufs[b].p.status == kOk) {
        n_chunks = a.bufs[b].p.N;
        n_groups = a.bufs[b].groups;
      }
    }
    uint64_t t_c, t_g, t_b;
    const uint64_t xc = block_excl_scan(n_chunks, scratch, &t_c);
    const uint64_t xg = block_excl_scan(n_groups, scratch, &t_g);
    block_excl_scan(nb, scratch, &t_b);
    if (b < a.nbufs) {
      a.bufs[b].chunk_base = chunk_carry + xc;
      a.bufs[b].group_base = group_carry + xg;
    }
    chunk_carry += t_c;
    group_carry += t_g;
    byte_carry += t_b;
  }
  const bool fits = group_carry <= a.group_cap && byte_carry <= a.max_total_in_bytes;
  __syncthreads();
  if (!fits) {
    for (uint64_t b = threadIdx.x; b < a.nbufs; b += blockDim.x) {
      a.bufs[b].p.status = kWorkspace;
      a.bufs[b].p.N = 0;
    }
  }
  if (threadIdx.x == 0) a.ctrl->T_all = fits ? chunk_carry : 0;
}

__global__ __launch_bounds__(256) void batch_dec_table_kernel(BatchDecArgs a) {
  __shared__ uint64_t scratch[256 / 64 + 1];
  const uint64_t b = blockIdx.x;
  BatchDecBuf& e = a.bufs[b];
  int32_t st = e.p.status;
  if (st == kOk) {
    const uint8_t* in = static_cast<const uint8_t*>(a.in_ptrs[b]);
    const uint64_t end = dec::scan_table_groups(in, e.p.N, a.group_off + e.group_base, scratch);
    if (end != a.in_bytes[b]) st = kCorrupt;
    else if (a.out_caps[b] < e.p.n) st = kOutOfSpace;
    else if (e.p.n != 0 && a.out_ptrs[b] == nullptr) st = kInvalidArg;
    if (st == kOk && threadIdx.x < e.p.r)
      static_cast<uint8_t*>(a.out_ptrs[b])[e.p.m * e.p.S + threadIdx.x] = in[48 + threadIdx.x];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const bool sized = st == kOk || st == kOutOfSpace;
    a.out_bytes[b] = sized ? e.p.n : 0;
    a.status[b] = st;
    e.p.status = st;
  }
}

__global__ __launch_bounds__(dec::kDecThreads, 4) void batch_decode_kernel(BatchDecArgs a) {
  __shared__ __align__(16) dec::BlockLds sm;
  const uint64_t T = a.ctrl->T_all;
  for (uint64_t g = blockIdx.x; g < T; g += gridDim.x) {
    const uint64_t b = find_buffer(a.nbufs, g, [&](uint64_t k) { return a.bufs[k].chunk_base; });
    const BatchDecBuf& e = a.bufs[b];
    if (e.p.status != kOk) continue;
    const bool ok = dec::decode_stream_chunk_block(
        static_cast<const uint8_t*>(a.in_ptrs[b]), a.in_bytes[b], e.p, a.group_off + e.group_base,
        g - e.chunk_base, static_cast<uint8_t*>(a.out_ptrs[b]), sm);
    if (!ok && threadIdx.x == 0) atomicExch(&a.status[b], kCorrupt);
  }
}

int device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

}  // namespace

template <int S, uint32_t WI, int WC>
hipError_t launch_width_wc(const BatchEncArgs& a, hipStream_t s) {
  const uint32_t threads = 64 * a.wp.waves[WI];
  const size_t lds = encode_lds_bytes(a.wp.C[WI], S, a.wp.W[WI], a.wp.waves[WI]);
  int per_cu = 0;
  hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, batch_encode_kernel<S, WI, WC>, threads, lds);
  if (err != hipSuccess) return err;
  if (per_cu < 1) per_cu = 1;
  hipLaunchKernelGGL((batch_encode_kernel<S, WI, WC>), dim3(device_cus() * per_cu), dim3(threads),
                     lds, s, a);
  return hipGetLastError();
}

template <int S, uint32_t WI>
hipError_t launch_width(const BatchEncArgs& a, hipStream_t s) {
  switch ((a.wp.W[WI] + 63) / 64) {
    case 1: return launch_width_wc<S, WI, 1>(a, s);
    case 2: return launch_width_wc<S, WI, 2>(a, s);
    case 3: return launch_width_wc<S, WI, 3>(a, s);
    default: return launch_width_wc<S, WI, 4>(a, s);
  }
}

hipError_t launch_compress_batch(const BatchEncArgs& a, hipStream_t s) {
  if (a.nbufs == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_enc_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  if ((err = launch_width<1, 0>(a, s)) != hipSuccess) return err;
  if ((err = launch_width<2, 1>(a, s)) != hipSuccess) return err;
  if ((err = launch_width<4, 2>(a, s)) != hipSuccess) return err;
  if ((err = launch_width<8, 3>(a, s)) != hipSuccess) return err;
  hipLaunchKernelGGL(batch_enc_scan_kernel, dim3((uint32_t)a.nbufs), dim3(1024), 0, s, a);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  hipLaunchKernelGGL(batch_scatter_kernel, dim3(device_cus() * 16), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_decompress_batch(const BatchDecArgs& a, hipStream_t s) {
  if (a.nbufs == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_dec_header_kernel, dim3((uint32_t)((a.nbufs + 255) / 256)), dim3(256),
                     0, s, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(batch_dec_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, a);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  hipLaunchKernelGGL(batch_dec_table_kernel, dim3((uint32_t)a.nbufs), dim3(256), 0, s, a);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  hipLaunchKernelGGL(batch_decode_kernel, dim3(device_cus() * 4), dim3(dec::kDecThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace gpulz
