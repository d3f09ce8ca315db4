// Internal declarations shared by the HIP kernel files and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpulz {

constexpr uint32_t kHeaderBytes = 64;
constexpr uint32_t kMaxMatch = 255;
constexpr uint32_t kMaxWindow = 256;
// Largest chunk (C * S bytes) the encoder stages in LDS; with the window pad
// and the hit bitmap this stays under 64 KiB of LDS per workgroup.
constexpr uint32_t kMaxChunkBytes = 48 * 1024;
// Per-wave LDS ring the decoder rebuilds symbols in (independent of C).
constexpr uint32_t kDecodeRingBytes = 16 * 1024;
constexpr uint64_t kMaxGroupLdsBytes = 64 * 1024;  // LDS one workgroup may allocate

// Device status values (same numbering as gpulz_status).
enum : int32_t {
  kOk = 0, kInvalidArg = 1, kOutOfSpace = 2, kCorrupt = 3, kWorkspace = 4,
  kInternal = 5  // a bounded device-side wait gave up (reported as GPULZ_ERR_HIP)
};

__host__ __device__ constexpr uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

// ---- compress ---------------------------------------------------------------

// Per-chunk scratch record laid out as [flag area | payload area | slack].
struct SlotLayout {
  uint64_t flag_area;   // bytes reserved for flags (multiple of 16)
  uint64_t slot_bytes;  // full slot (multiple of 16)
};

__host__ __device__ inline SlotLayout slot_layout(uint32_t C, uint32_t S, uint32_t min_match) {
  const uint64_t k = (S == 1 && min_match == 1) ? 2 : S;
  SlotLayout l;
  l.flag_area = align_up(align_up(C, 64) / 8, 16);
  l.slot_bytes = align_up(l.flag_area + (uint64_t)C * k + 16, 16);
  return l;
}

// ---- single-pass compress: records written once at their final offset ----
//
// Chunk ids come from an atomic ticket in the order workgroups start, and
// every chunk publishes its record size in a look-back descriptor
// (u64: state in bits 62-63, value in bits 0-61). State 1: the value is this
// chunk's record bytes; state 2: the record bytes of chunks 0..i (inclusive
// prefix). A chunk sums its predecessors' values back to the nearest
// inclusive prefix, so its record offset needs no separate scan pass.
constexpr uint64_t kDescAgg = 1ull << 62;
constexpr uint64_t kDescPrefix = 2ull << 62;
constexpr uint64_t kDescValue = (1ull << 62) - 1;  // also the "failed" prefix value
// Blocks per launch of the chunk encoders (launches of more chunks are
// split; every work-item count then stays far below 2^32).
constexpr uint64_t kMaxChunksPerLaunch = 1ull << 22;

// Workspace = ctrl (256 B: one ticket per launch) | desc[N] (u64) | slots[N].
// A slot only receives a chunk's 64-token groups from its first pointer on;
// all-literal groups before it are copied from the staged chunk.
constexpr uint32_t kMaxTickets = 32;
struct FusedWorkspace {
  uint64_t desc_off, slots_off, total;
};

__host__ __device__ inline FusedWorkspace fused_workspace(uint64_t N, uint32_t C, uint32_t S,
                                                          uint32_t min_match) {
  FusedWorkspace w;
  w.desc_off = 256;
  w.slots_off = w.desc_off + align_up(8 * N, 256);
  w.total = w.slots_off + N * slot_layout(C, S, min_match).slot_bytes + 256;
  return w;
}

struct FusedArgs {
  const uint8_t* in;
  uint64_t nbytes, m, N;
  uint32_t S, C, W, MIN, policy;
  uint8_t* out;
  uint64_t capacity;
  uint64_t* out_bytes;
  int32_t* status;
  uint64_t* tickets;   // kMaxTickets counters, one per launch
  uint64_t* desc;      // N look-back descriptors
  uint8_t* slots;
  uint64_t slot_bytes, flag_area;
  uint64_t chunk0;     // first chunk of this launch
  uint64_t nchunks;    // chunks of this launch
  uint32_t launch;     // index of this launch (its ticket)
};

// Zeroes the descriptors and tickets; for N = 0 also writes the header, size
// and status (one small kernel).
hipError_t launch_fused_prep(const FusedArgs& a, hipStream_t s);
// Encodes chunks [a.chunk0, a.chunk0 + a.nchunks) (at most
// kMaxChunksPerLaunch) with ticket a.launch, for match policy a.policy.
hipError_t launch_fused_encode(const FusedArgs& a, uint32_t waves, hipStream_t s);


size_t encode_lds_bytes(uint32_t C, uint32_t S, uint32_t W, uint32_t waves);
size_t encode_scan_lds_bytes(uint32_t C, uint32_t S);

// ---- decompress -------------------------------------------------------------

struct DecodeParams {
  int32_t status;
  uint32_t S, C, W, MIN, r;
  uint64_t n, m, N;
};

// Upper bound on the chunks of a valid stream: every chunk costs at least 8
// table bytes, 1 flag byte and 1 payload byte.
__host__ __device__ constexpr uint64_t decode_max_chunks(uint64_t stream_bytes) {
  return stream_bytes > kHeaderBytes ? (stream_bytes - kHeaderBytes) / 10 : 0;
}

// Record offsets are kept for every 64th chunk (a chunk's own offset is its
// group's plus a wave prefix sum over the group's table entries).
__host__ __device__ constexpr uint64_t decode_group_slots(uint64_t stream_bytes) {
  return (decode_max_chunks(stream_bytes) + 63) / 64 + 1;
}

// Workspace = DecodeParams (256 B) | group offsets[decode_group_slots] (u64).
struct DecodePrepArgs {
  const uint8_t* in;
  uint64_t in_bytes;
  uint64_t capacity;
  DecodeParams* params;
  uint64_t* group_off;
  uint64_t* out_bytes;
  int32_t* status;
};

struct DecodeArgs {
  const uint8_t* in;
  uint64_t in_bytes;
  const DecodeParams* params;
  const uint64_t* group_off;
  uint8_t* out;
  int32_t* status;
};

hipError_t launch_decode_prepare(const DecodePrepArgs& a, hipStream_t s);
// offsets[i] = sum of table[2k] + table[2k+1] over k < i, for i = 0 .. chunks
hipError_t launch_record_offsets(const uint32_t* table, uint64_t chunks, uint64_t* offsets,
                                 hipStream_t s);
hipError_t launch_decode_chunks(const DecodeArgs& a, hipStream_t s);

// ---- batches ----------------------------------------------------------------

// Per-width parameters as the kernels see them (index = log2 S).
// Per symbol width (index 0..3 for S = 1, 2, 4, 8).
struct WidthParams {
  uint32_t C[4], W[4], MIN[4], waves[4];
  uint64_t slot_bytes[4], flag_area[4];
};

struct BatchCtrl {
  uint64_t ticket[4];   // next work item of each width's persistent encoder
  uint64_t T[4];        // work items (chunks) of each width
  uint64_t T_all;       // work items in the batch
  uint64_t slot_total;  // scratch slot bytes used
};

struct BatchEncBuf {
  uint64_t chunk_base;     // first work item of this buffer
  uint64_t width_base[4];  // chunks of each width in the buffers before this one
  uint64_t slot_base;   // its first scratch slot (bytes into the slot region)
  uint64_t n;           // input bytes
  uint64_t N;           // chunks
  uint32_t S, C, W, MIN;
  uint32_t slot_bytes, flag_area;
  int32_t status;
  uint32_t pad;
};

struct BatchEncLayout {
  uint64_t ctrl_off, bufs_off, sizes_off, offs_off, slots_off, total;
  uint64_t max_chunks, slot_cap;
};

struct BatchEncArgs {
  uint64_t nbufs;
  const void* const* in_ptrs;
  const uint64_t* in_bytes;
  const uint8_t* symbol_bytes;
  void* const* out_ptrs;
  const uint64_t* out_caps;
  uint64_t* out_bytes;
  int32_t* status;
  uint64_t max_total_in_bytes;
  WidthParams wp;
  BatchCtrl* ctrl;
  BatchEncBuf* bufs;
  uint32_t* sizes;      // 2 per work item
  uint64_t* offs;       // per work item, offset of its record within its stream's records
  uint8_t* slots;
  uint64_t max_chunks, slot_cap;
};

struct BatchDecBuf {
  DecodeParams p;
  uint64_t chunk_base;  // first work item of this buffer
  uint64_t group_base;  // first record-offset group slot
  uint64_t groups;      // group slots used (ceil(N / 64) + 1), 0 if the header is bad
};

struct BatchDecArgs {
  uint64_t nbufs;
  const void* const* in_ptrs;
  const uint64_t* in_bytes;
  void* const* out_ptrs;
  const uint64_t* out_caps;
  uint64_t* out_bytes;
  int32_t* status;
  uint64_t max_total_in_bytes;
  BatchCtrl* ctrl;
  BatchDecBuf* bufs;
  uint64_t* group_off;
  uint64_t group_cap;
};

hipError_t launch_compress_batch(const BatchEncArgs& a, hipStream_t s);
hipError_t launch_decompress_batch(const BatchDecArgs& a, hipStream_t s);

}  // namespace gpulz
