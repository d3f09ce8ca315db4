// C ABI: argument checks, workspace layout, kernel launches.
#include "gpulz.h"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "gpulz_internal.h"
#include "huff_internal.h"
#include "stream_device.h"

using namespace gpulz;

namespace {

// ---- optional per-kernel event timing ---------------------------------------
constexpr int kProfKernels = 9;
struct EventPair {
  int kernel;
  hipEvent_t start, stop;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<EventPair> g_prof_events;

// Records `start` before a launch when profiling; returns the pair index or -1.
int prof_begin(int kernel, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_on) return -1;
  EventPair e{kernel, nullptr, nullptr};
  if (hipEventCreate(&e.start) != hipSuccess || hipEventCreate(&e.stop) != hipSuccess) return -1;
  hipEventRecord(e.start, s);
  g_prof_events.push_back(e);
  return (int)g_prof_events.size() - 1;
}

void prof_end(int idx, hipStream_t s) {
  if (idx < 0) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipEventRecord(g_prof_events[idx].stop, s);
}

// Launch checks read hipGetLastError, which also holds the error of any
// earlier failed HIP call on this thread (the caller's, or a framework's);
// entry points clear it right before their first launch so that their
// return value reports their own launches only.
void clear_stale_hip_error() { (void)hipGetLastError(); }

// A failed launch or runtime call: GPULZ_ERR_HIP (with the HIP error named on
// stderr if GPULZ_DEBUG is set in the environment).
gpulz_status hip_failed(hipError_t e, const char* what) {
  if (getenv("GPULZ_DEBUG")) fprintf(stderr, "gpulz: %s: %s\n", what, hipGetErrorName(e));
  return GPULZ_ERR_HIP;
}

bool valid_params(uint32_t S, uint32_t C, uint32_t W, uint32_t MIN) {
  if (!(S == 1 || S == 2 || S == 4 || S == 8)) return false;
  if (C < 1 || C > (1u << 24)) return false;
  if (W < 1 || W > kMaxWindow) return false;
  if (MIN < 1 || MIN > kMaxMatch) return false;
  return true;
}

bool aligned(const void* p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

uint64_t num_chunks(uint64_t nbytes, uint32_t S, uint32_t C) {
  const uint64_t m = nbytes / S;
  return (m + C - 1) / C;
}

// ---- per-width defaults and batch layouts ------------------------------------

std::mutex g_defaults_mu;
// Small chunks of dense (match-rich) data parse fastest with one wave per
// workgroup (more chunks resident per CU); large literal-heavy chunks with
// four (the hit bitmap is split across them).
gpulz_params g_defaults[4] = {
    {4096, 128, 2, 1},  // S = 1
    {2048, 128, 2, 1},  // S = 2
    {4096, 256, 2, 4},  // S = 4
    {2048, 256, 2, 4},  // S = 8
};

int width_index(uint32_t S) { return S == 1 ? 0 : S == 2 ? 1 : S == 4 ? 2 : S == 8 ? 3 : -1; }

bool valid_waves(uint32_t w) { return w == 1 || w == 2 || w == 4; }

// Fills zero fields from the defaults and checks the result.
bool resolve_params(const gpulz_params* in, WidthParams& wp) {
  std::lock_guard<std::mutex> lk(g_defaults_mu);
  for (int w = 0; w < 4; ++w) {
    const uint32_t S = 1u << w;
    gpulz_params p = in ? in[w] : gpulz_params{0, 0, 0, 0};
    if (p.chunk_symbols == 0) p.chunk_symbols = g_defaults[w].chunk_symbols;
    if (p.window == 0) p.window = g_defaults[w].window;
    if (p.min_match == 0) p.min_match = g_defaults[w].min_match;
    if (p.waves_per_chunk == 0) p.waves_per_chunk = g_defaults[w].waves_per_chunk;
    if (!valid_params(S, p.chunk_symbols, p.window, p.min_match) || !valid_waves(p.waves_per_chunk))
      return false;
    if ((uint64_t)p.chunk_symbols * S > kMaxChunkBytes) return false;
    wp.C[w] = p.chunk_symbols;
    wp.W[w] = p.window;
    wp.MIN[w] = p.min_match;
    wp.waves[w] = p.waves_per_chunk;
    const SlotLayout sl = slot_layout(p.chunk_symbols, S, p.min_match);
    wp.slot_bytes[w] = sl.slot_bytes;
    wp.flag_area[w] = sl.flag_area;
  }
  return true;
}

BatchEncLayout batch_enc_layout(uint64_t nbufs, uint64_t max_total, const WidthParams& wp) {
  uint64_t min_sc = ~0ull, max_slot = 0;
  double max_ratio = 0;
  for (int w = 0; w < 4; ++w) {
    const uint64_t sc = (uint64_t)wp.C[w] << w;
    min_sc = sc < min_sc ? sc : min_sc;
    max_slot = wp.slot_bytes[w] > max_slot ? wp.slot_bytes[w] : max_slot;
    const double r = (double)wp.slot_bytes[w] / (double)sc;
    max_ratio = r > max_ratio ? r : max_ratio;
  }
  BatchEncLayout l;
  l.max_chunks = max_total / min_sc + nbufs;
  l.slot_cap = (uint64_t)((double)max_total * max_ratio) + nbufs * max_slot + 4096;
  static_assert(sizeof(BatchCtrl) <= 256, "control block");
  l.ctrl_off = 0;
  l.bufs_off = 256;
  l.sizes_off = l.bufs_off + align_up(nbufs * sizeof(BatchEncBuf), 256);
  l.offs_off = l.sizes_off + align_up(8 * l.max_chunks, 256);
  l.slots_off = l.offs_off + align_up(8 * l.max_chunks, 256);
  l.total = l.slots_off + align_up(l.slot_cap, 256) + 256;
  return l;
}

struct BatchDecLayout {
  uint64_t bufs_off, groups_off, total, group_cap;
};

BatchDecLayout batch_dec_layout(uint64_t nbufs, uint64_t max_total) {
  BatchDecLayout l;
  l.group_cap = max_total / 640 + 2 * nbufs + 16;
  l.bufs_off = 256;
  l.groups_off = l.bufs_off + align_up(nbufs * sizeof(BatchDecBuf), 256);
  l.total = l.groups_off + align_up(8 * l.group_cap, 256);
  return l;
}

}  // namespace

extern "C" {

uint32_t gpulz_abi_version(void) { return 102; }

const char* gpulz_status_string(gpulz_status status) {
  switch (status) {
    case GPULZ_OK: return "ok";
    case GPULZ_ERR_INVALID_ARG: return "invalid argument";
    case GPULZ_ERR_OUT_OF_SPACE: return "output capacity too small";
    case GPULZ_ERR_CORRUPT: return "corrupt stream";
    case GPULZ_ERR_WORKSPACE: return "workspace too small";
    case GPULZ_ERR_HIP: return "HIP runtime error";
    case GPULZ_ERR_UNSUPPORTED: return "unsupported on this device";
    default: return "unknown status";
  }
}

uint64_t gpulz_compress_bound(uint64_t nbytes, uint32_t S, uint32_t C, uint32_t MIN) {
  if (!valid_params(S, C, 1, MIN)) return 0;
  const uint64_t m = nbytes / S;
  const uint64_t k = (S == 1 && MIN == 1) ? 2 : S;
  const uint64_t full = m / C, last = m % C;
  uint64_t total = kHeaderBytes + 8 * num_chunks(nbytes, S, C);
  total += full * ((C + 7) / 8 + (uint64_t)C * k);
  if (last) total += (last + 7) / 8 + last * k;
  return total;
}

gpulz_status gpulz_compress_workspace_size(uint64_t nbytes, uint32_t S, uint32_t C,
                                           size_t* ws_bytes) {
  if (!ws_bytes || !valid_params(S, C, 1, 1)) return GPULZ_ERR_INVALID_ARG;
  // the slot size depends on min_match only for S == 1; size for the worst
  *ws_bytes = (size_t)fused_workspace(num_chunks(nbytes, S, C), C, S, 1).total;
  return GPULZ_OK;
}

gpulz_status gpulz_compress_policy(const void* d_in, uint64_t nbytes, uint32_t S, uint32_t C,
                                   uint32_t W, uint32_t MIN, uint32_t policy, void* d_out,
                                   uint64_t out_capacity, uint64_t* d_out_bytes, int32_t* d_status,
                                   void* d_ws, size_t ws_bytes, hipStream_t stream) {
  if (!valid_params(S, C, W, MIN) || policy > 1) return GPULZ_ERR_INVALID_ARG;
  if ((nbytes && !d_in) || !d_out_bytes || !d_status || (out_capacity && !d_out))
    return GPULZ_ERR_INVALID_ARG;
  if (!aligned(d_in, 16) || !aligned(d_out, 16) || !aligned(d_ws, 256)) return GPULZ_ERR_INVALID_ARG;
  if ((uint64_t)C * S > kMaxChunkBytes) return GPULZ_ERR_UNSUPPORTED;
  if (policy == 1 && encode_scan_lds_bytes(C, S) > kMaxGroupLdsBytes) return GPULZ_ERR_UNSUPPORTED;
  const uint64_t N = num_chunks(nbytes, S, C);
  if (N > (uint64_t)kMaxTickets * kMaxChunksPerLaunch) return GPULZ_ERR_UNSUPPORTED;
  const FusedWorkspace w = fused_workspace(N, C, S, 1);
  if (!d_ws || ws_bytes < w.total) return GPULZ_ERR_WORKSPACE;
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  const SlotLayout sl = slot_layout(C, S, 1);

  FusedArgs a;
  a.in = static_cast<const uint8_t*>(d_in);
  a.nbytes = nbytes;
  a.m = nbytes / S;
  a.N = N;
  a.S = S;
  a.C = C;
  a.W = W;
  a.MIN = MIN;
  a.policy = policy;
  a.out = static_cast<uint8_t*>(d_out);
  a.capacity = out_capacity;
  a.out_bytes = d_out_bytes;
  a.status = d_status;
  a.tickets = reinterpret_cast<uint64_t*>(ws);
  a.desc = reinterpret_cast<uint64_t*>(ws + w.desc_off);
  a.slots = ws + w.slots_off;
  a.slot_bytes = sl.slot_bytes;
  a.flag_area = sl.flag_area;
  a.chunk0 = 0;
  a.nchunks = 0;
  a.launch = 0;
  uint32_t waves;
  {
    std::lock_guard<std::mutex> lk(g_defaults_mu);
    waves = g_defaults[width_index(S)].waves_per_chunk;
  }
  int pi = prof_begin(1, stream);
  clear_stale_hip_error();
  hipError_t err = launch_fused_prep(a, stream);
  if (err != hipSuccess) return hip_failed(err, "compress prepare launch");
  prof_end(pi, stream);
  pi = prof_begin(0, stream);
  for (uint64_t c0 = 0; c0 < N; c0 += kMaxChunksPerLaunch) {
    a.chunk0 = c0;
    a.nchunks = N - c0 < kMaxChunksPerLaunch ? N - c0 : kMaxChunksPerLaunch;
    if ((err = launch_fused_encode(a, waves, stream)) != hipSuccess)
      return hip_failed(err, "compress encode launch");
    ++a.launch;
  }
  prof_end(pi, stream);
  return GPULZ_OK;
}

gpulz_status gpulz_compress(const void* d_in, uint64_t nbytes, uint32_t S, uint32_t C, uint32_t W,
                            uint32_t MIN, void* d_out, uint64_t out_capacity, uint64_t* d_out_bytes,
                            int32_t* d_status, void* d_ws, size_t ws_bytes, hipStream_t stream) {
  return gpulz_compress_policy(d_in, nbytes, S, C, W, MIN, 0, d_out, out_capacity, d_out_bytes,
                               d_status, d_ws, ws_bytes, stream);
}

gpulz_status gpulz_peek_header(const void* h_header, size_t header_bytes, uint64_t* nbytes,
                               uint32_t* symbol_bytes, uint64_t* stream_bytes) {
  if (!h_header || header_bytes < kHeaderBytes) return GPULZ_ERR_INVALID_ARG;
  const uint8_t* h = static_cast<const uint8_t*>(h_header);
  if (memcmp(h, "GLZ1", 4) != 0 || h[4] != 1 || h[5] != 0) return GPULZ_ERR_CORRUPT;
  uint64_t n = 0, total = 0;
  uint32_t C = 0;
  for (int k = 7; k >= 0; --k) n = (n << 8) | h[16 + k];
  for (int k = 7; k >= 0; --k) total = (total << 8) | h[32 + k];
  for (int k = 3; k >= 0; --k) C = (C << 8) | h[8 + k];
  const uint32_t W = (uint32_t)h[12] | ((uint32_t)h[13] << 8);
  if (!valid_params(h[6], C, W, h[14]) || h[7] > 1 || h[15] != kMaxMatch) return GPULZ_ERR_CORRUPT;
  if (nbytes) *nbytes = n;
  if (symbol_bytes) *symbol_bytes = h[6];
  if (stream_bytes) *stream_bytes = total;
  return GPULZ_OK;
}

uint64_t gpulz_table_offset(uint64_t chunk) { return kHeaderBytes + 8 * chunk; }

gpulz_status gpulz_write_header(void* h_header, uint64_t nbytes, uint32_t S, uint32_t C, uint32_t W,
                                uint32_t MIN, uint32_t policy, uint64_t stream_bytes,
                                const void* h_tail) {
  if (!h_header || !valid_params(S, C, W, MIN) || policy > 1) return GPULZ_ERR_INVALID_ARG;
  const uint64_t N = num_chunks(nbytes, S, C);
  const uint32_t r = (uint32_t)(nbytes % S);
  if (stream_bytes < kHeaderBytes + 8 * N || (r && !h_tail)) return GPULZ_ERR_INVALID_ARG;
  uint8_t* h = static_cast<uint8_t*>(h_header);
  const uint8_t* tail = static_cast<const uint8_t*>(h_tail);
  for (uint32_t b = 0; b < kHeaderBytes; ++b)
    h[b] = stream::header_byte(b, nbytes, S, C, W, MIN, policy, N, stream_bytes, tail);
  return GPULZ_OK;
}

gpulz_status gpulz_read_header(const void* h_header, size_t header_bytes, gpulz_stream_info* info) {
  if (!h_header || !info || header_bytes < kHeaderBytes) return GPULZ_ERR_INVALID_ARG;
  const uint8_t* h = static_cast<const uint8_t*>(h_header);
  auto u64 = [&](int at) {
    uint64_t v = 0;
    for (int k = 7; k >= 0; --k) v = (v << 8) | h[at + k];
    return v;
  };
  gpulz_stream_info f{};
  f.symbol_bytes = h[6];
  f.match_policy = h[7];
  f.chunk_symbols = (uint32_t)h[8] | ((uint32_t)h[9] << 8) | ((uint32_t)h[10] << 16) |
                    ((uint32_t)h[11] << 24);
  f.window = (uint32_t)h[12] | ((uint32_t)h[13] << 8);
  f.min_match = h[14];
  f.nbytes = u64(16);
  f.chunks = u64(24);
  f.stream_bytes = u64(32);
  f.tail_bytes = h[40];
  bool ok = memcmp(h, "GLZ1", 4) == 0 && h[4] == 1 && h[5] == 0 && f.match_policy <= 1 &&
            h[15] == kMaxMatch &&
            valid_params(f.symbol_bytes, f.chunk_symbols, f.window, f.min_match);
  if (ok) {
    ok = f.tail_bytes == f.nbytes % f.symbol_bytes &&
         f.chunks == num_chunks(f.nbytes, f.symbol_bytes, f.chunk_symbols) &&
         f.chunks <= decode_max_chunks(f.stream_bytes) &&
         f.stream_bytes >= kHeaderBytes + 8 * f.chunks;
    for (int k = 41; k < 48; ++k) ok = ok && h[k] == 0;
    for (uint32_t k = 48 + f.tail_bytes; k < kHeaderBytes; ++k) ok = ok && h[k] == 0;
  }
  if (!ok) return GPULZ_ERR_CORRUPT;
  for (uint32_t k = 0; k < f.tail_bytes; ++k) f.tail[k] = h[48 + k];
  *info = f;
  return GPULZ_OK;
}

gpulz_status gpulz_record_offsets(const void* d_table, uint64_t chunks, uint64_t* d_offsets,
                                  hipStream_t stream) {
  if (!d_offsets || !aligned(d_offsets, 8) || (chunks && (!d_table || !aligned(d_table, 4))))
    return GPULZ_ERR_INVALID_ARG;
  clear_stale_hip_error();
  const hipError_t err = launch_record_offsets(static_cast<const uint32_t*>(d_table), chunks,
                                               d_offsets, stream);
  return err != hipSuccess ? hip_failed(err, "record offsets launch") : GPULZ_OK;
}

gpulz_status gpulz_decompress_workspace_size(uint64_t comp_bytes, uint64_t nbytes,
                                             size_t* ws_bytes) {
  if (!ws_bytes) return GPULZ_ERR_INVALID_ARG;
  // one record-offset slot per 64 chunks of the most a stream of comp_bytes
  // can hold (the decoder accepts no header claiming more); the size does
  // not depend on nbytes
  (void)nbytes;
  *ws_bytes = (size_t)(256 + 8 * decode_group_slots(comp_bytes));
  return GPULZ_OK;
}

gpulz_status gpulz_decompress(const void* d_in, uint64_t in_bytes, void* d_out, uint64_t out_capacity,
                              uint64_t* d_out_bytes, int32_t* d_status, void* d_ws, size_t ws_bytes,
                              hipStream_t stream) {
  if ((in_bytes && !d_in) || !d_out_bytes || !d_status || (out_capacity && !d_out))
    return GPULZ_ERR_INVALID_ARG;
  if (!aligned(d_in, 16) || !aligned(d_out, 16) || !aligned(d_ws, 256)) return GPULZ_ERR_INVALID_ARG;
  size_t need = 0;
  gpulz_decompress_workspace_size(in_bytes, 0, &need);
  if (!d_ws || ws_bytes < need) return GPULZ_ERR_WORKSPACE;
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  DecodePrepArgs pa;
  pa.in = static_cast<const uint8_t*>(d_in);
  pa.in_bytes = in_bytes;
  pa.capacity = out_capacity;
  pa.params = reinterpret_cast<DecodeParams*>(ws);
  pa.group_off = reinterpret_cast<uint64_t*>(ws + 256);
  pa.out_bytes = d_out_bytes;
  pa.status = d_status;
  DecodeArgs da;
  da.in = pa.in;
  da.in_bytes = in_bytes;
  da.params = pa.params;
  da.group_off = pa.group_off;
  da.out = static_cast<uint8_t*>(d_out);
  da.status = d_status;
  int pi = prof_begin(3, stream);
  clear_stale_hip_error();
  hipError_t err = launch_decode_prepare(pa, stream);
  if (err != hipSuccess) return hip_failed(err, "decompress prepare launch");
  prof_end(pi, stream);
  pi = prof_begin(4, stream);
  if ((err = launch_decode_chunks(da, stream)) != hipSuccess)
    return hip_failed(err, "decompress launch");
  prof_end(pi, stream);
  return GPULZ_OK;
}

// ---- decompression without allocation ---------------------------------------
//
// gpulz_decompress_noalloc takes its workspace from a file-scope device
// array instead of a caller's buffer. Each GPU the library runs on holds its
// own copy until the process ends. Host code never passes the array's name
// to a kernel (in host code it is a stand-in, not a device address): its
// device address is looked up once per device, with that device current,
// and kept. The decoder writes every byte of its workspace it later reads
// (the stream parameters, then every record-offset group), so nothing has to
// be cleared between calls.
constexpr uint64_t kNoAllocMaxStreamBytes = 1ull << 30;
constexpr size_t kNoAllocScratchBytes =
    (size_t)align_up(256 + 8 * decode_group_slots(kNoAllocMaxStreamBytes), 256);
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// This device's scratch address (looked up on the device's first call).
gpulz_status current_scratch(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GPULZ_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GPULZ_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GPULZ_OK;
}

}  // namespace

gpulz_status gpulz_decompress_noalloc(const void* d_in, uint64_t in_bytes, void* d_out,
                                      uint64_t out_capacity, uint64_t* d_out_bytes,
                                      int32_t* d_status, hipStream_t stream) {
  if (in_bytes > kNoAllocMaxStreamBytes) return GPULZ_ERR_WORKSPACE;
  size_t need = 0;
  gpulz_decompress_workspace_size(in_bytes, 0, &need);
  if (need > kNoAllocScratchBytes) return GPULZ_ERR_WORKSPACE;
  void* ws = nullptr;
  const gpulz_status st = current_scratch(&ws);
  if (st != GPULZ_OK) return st;
  return gpulz_decompress(d_in, in_bytes, d_out, out_capacity, d_out_bytes, d_status, ws, need,
                          stream);
}

gpulz_status gpulz_default_params(uint32_t S, gpulz_params* params) {
  const int w = width_index(S);
  if (w < 0 || !params) return GPULZ_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_defaults_mu);
  *params = g_defaults[w];
  return GPULZ_OK;
}

gpulz_status gpulz_set_default_params(uint32_t S, const gpulz_params* params) {
  const int w = width_index(S);
  if (w < 0 || !params) return GPULZ_ERR_INVALID_ARG;
  const gpulz_params& p = *params;
  if (!valid_params(S, p.chunk_symbols, p.window, p.min_match) || !valid_waves(p.waves_per_chunk) ||
      (uint64_t)p.chunk_symbols * S > kMaxChunkBytes)
    return GPULZ_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_defaults_mu);
  g_defaults[w] = p;
  return GPULZ_OK;
}

gpulz_status gpulz_compress_batch_workspace_size(uint64_t nbufs, uint64_t max_total_in_bytes,
                                                 const gpulz_params params_by_width[4],
                                                 size_t* ws_bytes) {
  WidthParams wp;
  if (!ws_bytes || !resolve_params(params_by_width, wp)) return GPULZ_ERR_INVALID_ARG;
  *ws_bytes = (size_t)batch_enc_layout(nbufs, max_total_in_bytes, wp).total;
  return GPULZ_OK;
}

gpulz_status gpulz_compress_batch(uint64_t nbufs, const void* const* d_in_ptrs,
                                  const uint64_t* d_in_bytes, const uint8_t* d_symbol_bytes,
                                  const gpulz_params params_by_width[4], void* const* d_out_ptrs,
                                  const uint64_t* d_out_caps, uint64_t* d_out_bytes,
                                  int32_t* d_status, uint64_t max_total_in_bytes, void* d_ws,
                                  size_t ws_bytes, hipStream_t stream) {
  if (nbufs == 0) return GPULZ_OK;
  if (!d_in_ptrs || !d_in_bytes || !d_symbol_bytes || !d_out_ptrs || !d_out_caps || !d_out_bytes ||
      !d_status || nbufs > 0xFFFFFFFFull)
    return GPULZ_ERR_INVALID_ARG;
  WidthParams wp;
  if (!resolve_params(params_by_width, wp)) return GPULZ_ERR_INVALID_ARG;
  if (!aligned(d_ws, 256)) return GPULZ_ERR_INVALID_ARG;
  const BatchEncLayout l = batch_enc_layout(nbufs, max_total_in_bytes, wp);
  if (!d_ws || ws_bytes < l.total) return GPULZ_ERR_WORKSPACE;
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  BatchEncArgs a;
  a.nbufs = nbufs;
  a.in_ptrs = d_in_ptrs;
  a.in_bytes = d_in_bytes;
  a.symbol_bytes = d_symbol_bytes;
  a.out_ptrs = d_out_ptrs;
  a.out_caps = d_out_caps;
  a.out_bytes = d_out_bytes;
  a.status = d_status;
  a.max_total_in_bytes = max_total_in_bytes;
  a.wp = wp;
  a.ctrl = reinterpret_cast<BatchCtrl*>(ws + l.ctrl_off);
  a.bufs = reinterpret_cast<BatchEncBuf*>(ws + l.bufs_off);
  a.sizes = reinterpret_cast<uint32_t*>(ws + l.sizes_off);
  a.offs = reinterpret_cast<uint64_t*>(ws + l.offs_off);
  a.slots = ws + l.slots_off;
  a.max_chunks = l.max_chunks;
  a.slot_cap = l.slot_cap;
  int pi = prof_begin(5, stream);
  clear_stale_hip_error();
  const hipError_t err = launch_compress_batch(a, stream);
  if (err != hipSuccess) return hip_failed(err, "compress batch launch");
  prof_end(pi, stream);
  return GPULZ_OK;
}

gpulz_status gpulz_decompress_batch_workspace_size(uint64_t nbufs, uint64_t max_total_in_bytes,
                                                   size_t* ws_bytes) {
  if (!ws_bytes) return GPULZ_ERR_INVALID_ARG;
  *ws_bytes = (size_t)batch_dec_layout(nbufs, max_total_in_bytes).total;
  return GPULZ_OK;
}

gpulz_status gpulz_decompress_batch(uint64_t nbufs, const void* const* d_in_ptrs,
                                    const uint64_t* d_in_bytes, void* const* d_out_ptrs,
                                    const uint64_t* d_out_caps, uint64_t* d_out_bytes,
                                    int32_t* d_status, uint64_t max_total_in_bytes, void* d_ws,
                                    size_t ws_bytes, hipStream_t stream) {
  if (nbufs == 0) return GPULZ_OK;
  if (!d_in_ptrs || !d_in_bytes || !d_out_ptrs || !d_out_caps || !d_out_bytes || !d_status ||
      nbufs > 0xFFFFFFFFull)
    return GPULZ_ERR_INVALID_ARG;
  if (!aligned(d_ws, 256)) return GPULZ_ERR_INVALID_ARG;
  const BatchDecLayout l = batch_dec_layout(nbufs, max_total_in_bytes);
  if (!d_ws || ws_bytes < l.total) return GPULZ_ERR_WORKSPACE;
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  BatchDecArgs a;
  a.nbufs = nbufs;
  a.in_ptrs = d_in_ptrs;
  a.in_bytes = d_in_bytes;
  a.out_ptrs = d_out_ptrs;
  a.out_caps = d_out_caps;
  a.out_bytes = d_out_bytes;
  a.status = d_status;
  a.max_total_in_bytes = max_total_in_bytes;
  a.ctrl = reinterpret_cast<BatchCtrl*>(ws);
  a.bufs = reinterpret_cast<BatchDecBuf*>(ws + l.bufs_off);
  a.group_off = reinterpret_cast<uint64_t*>(ws + l.groups_off);
  a.group_cap = l.group_cap;
  int pi = prof_begin(6, stream);
  clear_stale_hip_error();
  const hipError_t err = launch_decompress_batch(a, stream);
  if (err != hipSuccess) return hip_failed(err, "decompress batch launch");
  prof_end(pi, stream);
  return GPULZ_OK;
}

gpulz_status gpulz_profile_enable(int enable) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& e : g_prof_events) {
    hipEventSynchronize(e.stop);
    hipEventDestroy(e.start);
    hipEventDestroy(e.stop);
  }
  g_prof_events.clear();
  g_prof_on = enable != 0;
  return GPULZ_OK;
}

// ---- entropy stage ------------------------------------------------------------

uint64_t gpulz_huff_compress_bound(uint64_t nbytes) {
  return nbytes > huff::kMaxInput ? 0 : huff::bound(nbytes);
}

gpulz_status gpulz_huff_compress_workspace_size(uint64_t max_bytes, size_t* ws_bytes) {
  if (!ws_bytes || max_bytes > huff::kMaxInput) return GPULZ_ERR_INVALID_ARG;
  *ws_bytes = (size_t)huff::enc_workspace(max_bytes).total;
  return GPULZ_OK;
}

gpulz_status gpulz_huff_compress(const void* d_in, uint64_t nbytes, const uint64_t* d_nbytes,
                                 void* d_out, uint64_t out_capacity, uint64_t* d_out_bytes,
                                 int32_t* d_status, void* d_ws, size_t ws_bytes,
                                 hipStream_t stream) {
  if ((nbytes && !d_in) || !d_out || !d_out_bytes || !d_status || nbytes > huff::kMaxInput)
    return GPULZ_ERR_INVALID_ARG;
  if (!aligned(d_in, 16) || !aligned(d_out, 16) || !aligned(d_ws, 256)) return GPULZ_ERR_INVALID_ARG;
  if (out_capacity < huff::bound(nbytes)) return GPULZ_ERR_OUT_OF_SPACE;
  const huff::EncWorkspace w = huff::enc_workspace(nbytes);
  if (!d_ws || ws_bytes < w.total) return GPULZ_ERR_WORKSPACE;
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  huff::EncArgs a;
  a.in = static_cast<const uint8_t*>(d_in);
  a.max_n = nbytes;
  a.d_n = d_nbytes;
  a.hist_blocks = huff::hist_blocks(nbytes);
  a.partial = reinterpret_cast<uint32_t*>(ws + w.partial_off);
  a.codes = reinterpret_cast<uint32_t*>(ws + w.codes_off);
  a.sizes = reinterpret_cast<uint32_t*>(ws + w.sizes_off);
  a.offs = reinterpret_cast<uint64_t*>(ws + w.offs_off);
  a.out = static_cast<uint8_t*>(d_out);
  a.out_bytes = d_out_bytes;
  a.status = d_status;
  const int pi = prof_begin(7, stream);
  clear_stale_hip_error();
  const hipError_t err = huff::launch_compress(a, stream);
  if (err != hipSuccess) return hip_failed(err, "huffman compress launch");
  prof_end(pi, stream);
  return GPULZ_OK;
}

gpulz_status gpulz_huff_decompress_workspace_size(uint64_t stream_bytes, size_t* ws_bytes) {
  if (!ws_bytes) return GPULZ_ERR_INVALID_ARG;
  *ws_bytes = (size_t)huff::dec_workspace(stream_bytes).total;
  return GPULZ_OK;
}

gpulz_status gpulz_huff_decompress(const void* d_in, uint64_t in_bytes, void* d_out,
                                   uint64_t out_capacity, uint64_t* d_out_bytes, int32_t* d_status,
                                   void* d_ws, size_t ws_bytes, hipStream_t stream) {
  if ((in_bytes && !d_in) || !d_out_bytes || !d_status || (out_capacity && !d_out))
    return GPULZ_ERR_INVALID_ARG;
  if (!aligned(d_in, 16) || !aligned(d_out, 16) || !aligned(d_ws, 256)) return GPULZ_ERR_INVALID_ARG;
  const huff::DecWorkspace w = huff::dec_workspace(in_bytes);
  if (!d_ws || ws_bytes < w.total) return GPULZ_ERR_WORKSPACE;
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  huff::DecArgs a;
  a.in = static_cast<const uint8_t*>(d_in);
  a.in_bytes = in_bytes;
  a.capacity = out_capacity;
  a.tab = reinterpret_cast<huff::DecTables*>(ws);
  a.sizes = reinterpret_cast<uint32_t*>(ws + w.sizes_off);
  a.offs = reinterpret_cast<uint64_t*>(ws + w.offs_off);
  a.out = static_cast<uint8_t*>(d_out);
  a.out_bytes = d_out_bytes;
  a.status = d_status;
  const int pi = prof_begin(8, stream);
  clear_stale_hip_error();
  const hipError_t err = huff::launch_decompress(a, stream);
  if (err != hipSuccess) return hip_failed(err, "huffman decompress launch");
  prof_end(pi, stream);
  return GPULZ_OK;
}

gpulz_status gpulz_profile_read(double* total_ms, uint64_t* launches, int nkernels) {
  if (nkernels < 0) return GPULZ_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  double ms[kProfKernels] = {0};
  uint64_t cnt[kProfKernels] = {0};
  for (auto& e : g_prof_events) {
    float t = 0.f;
    if (hipEventSynchronize(e.stop) != hipSuccess) return GPULZ_ERR_HIP;
    if (hipEventElapsedTime(&t, e.start, e.stop) != hipSuccess) return GPULZ_ERR_HIP;
    ms[e.kernel] += t;
    cnt[e.kernel] += 1;
  }
  for (int k = 0; k < nkernels && k < kProfKernels; ++k) {
    if (total_ms) total_ms[k] = ms[k];
    if (launches) launches[k] = cnt[k];
  }
  return GPULZ_OK;
}

}  // extern "C"
