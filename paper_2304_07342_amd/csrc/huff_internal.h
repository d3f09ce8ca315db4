// Entropy stage after LZSS: Huffman coding of bytes, chunked for parallel
// decoding. gpuLZ section 4.5 runs LZSS in front of a Huffman coder; the
// coder itself is not specified there, so the stream follows these rules:
//   * one code for the whole input, from its byte frequencies: Huffman's
//     algorithm with ties broken by (weight, node index), leaves indexed by
//     symbol before internal nodes in creation order; lengths limited to 15
//     by halving every weight (rounding up) and building again;
//   * canonical codes (RFC 1951 section 3.2.2);
//   * 4096-byte chunks; each chunk's record holds the start bit of each of
//     its 128-symbol sub-blocks, then its code bits MSB-first in
//     little-endian u32 words.
// The byte layout is documented with gpulz_huff_compress in gpulz.h.
#pragma once

#include "gpulz_internal.h"

namespace gpulz {
namespace huff {

constexpr uint32_t kChunk = 4096;            // symbols (bytes) per chunk
constexpr uint32_t kSub = 128;               // symbols per sub-block
constexpr uint32_t kSubs = kChunk / kSub;    // sub-blocks per full chunk
constexpr uint32_t kLimit = 15;              // longest code
constexpr uint32_t kLutBits = 11;            // decoder lookup table index bits
// Codes longer than 11 bits cover at most 256 x 8 fifteen-bit slots, i.e. 128
// eleven-bit prefixes (129 when unaligned): the second-level subtables.
constexpr uint32_t kMaxSubtables = 136;
constexpr uint32_t kPre = 192;               // header + code lengths
constexpr uint32_t kMaxWords = (kChunk * kLimit + 31) / 32;  // code words of a full chunk
constexpr uint32_t kMaxHistBlocks = 512;
constexpr uint32_t kMaxLimitRounds = 48;     // cap on rebuilds by the length limit
constexpr uint64_t kMaxInput = 1ull << 40;

__host__ __device__ inline uint64_t chunks(uint64_t n) { return (n + kChunk - 1) / kChunk; }
__host__ __device__ inline uint32_t offsets_bytes(uint32_t nsub) { return (2 * nsub + 3) / 4 * 4; }

__host__ __device__ inline uint64_t bound(uint64_t n) {
  return kPre + chunks(n) * (4 + offsets_bytes(kSubs) + 4ull * kMaxWords);
}

// Histogram workgroups for inputs of up to max_n bytes (~64 KiB each).
__host__ inline uint32_t hist_blocks(uint64_t max_n) {
  const uint64_t b = (max_n + 65535) / 65536;
  return (uint32_t)(b < 1 ? 1 : b > kMaxHistBlocks ? kMaxHistBlocks : b);
}

// Compress workspace: partial histograms | code table (256 codes + a build
// status word) | record sizes (u32
// pairs: sub-block offset bytes, code word bytes) | record offsets (N + 1).
struct EncWorkspace {
  uint64_t partial_off, codes_off, sizes_off, offs_off, total;
};

__host__ inline EncWorkspace enc_workspace(uint64_t max_n) {
  const uint64_t N = chunks(max_n);
  EncWorkspace w;
  w.partial_off = 0;
  w.codes_off = align_up(4ull * 256 * hist_blocks(max_n), 256);
  w.sizes_off = w.codes_off + 2048;
  w.offs_off = w.sizes_off + align_up(8 * N, 256);
  w.total = w.offs_off + align_up(8 * (N + 1), 256);
  return w;
}

struct EncArgs {
  const uint8_t* in;
  uint64_t max_n;       // the host's input size, or the maximum when d_n is set
  const uint64_t* d_n;  // device-resident input size (optional)
  uint32_t hist_blocks;
  uint32_t* partial;    // hist_blocks x 256
  uint32_t* codes;      // 256 x (length << 16 | code), then the build status
  uint32_t* sizes;      // 2 per chunk
  uint64_t* offs;       // N + 1
  uint8_t* out;
  uint64_t* out_bytes;
  int32_t* status;
};

// Decoder tables, built once per stream by the prepare kernel.
struct DecTables {
  int32_t status;
  uint32_t pad;
  uint64_t n, N;
  uint32_t first[16];  // first canonical code of each length
  uint32_t count[16];  // codes of each length
  uint32_t rank0[16];  // rank of the first code of each length
  uint8_t by_rank[256];
  // two-level decoding table: lut[11-bit prefix] = length << 8 | symbol for
  // codes of up to 11 bits, 0x8000 | t for a prefix of longer codes (t-th
  // 16-entry subtable of lut2, indexed by the next 4 bits), 0 for no code
  uint16_t lut[1u << kLutBits];
  uint16_t lut2[kMaxSubtables * 16];
};

// Decompress workspace: tables | record sizes (u32 pairs) | record offsets.
struct DecWorkspace {
  uint64_t sizes_off, offs_off, total, max_chunks;
};

__host__ inline DecWorkspace dec_workspace(uint64_t stream_bytes) {
  DecWorkspace w;
  w.max_chunks = stream_bytes > kPre ? (stream_bytes - kPre) / 4 : 0;
  w.sizes_off = align_up(sizeof(DecTables), 256);
  w.offs_off = w.sizes_off + align_up(8 * w.max_chunks, 256);
  w.total = w.offs_off + align_up(8 * (w.max_chunks + 1), 256);
  return w;
}

struct DecArgs {
  const uint8_t* in;
  uint64_t in_bytes;
  uint64_t capacity;
  DecTables* tab;
  uint32_t* sizes;
  uint64_t* offs;
  uint8_t* out;
  uint64_t* out_bytes;
  int32_t* status;
};

hipError_t launch_compress(const EncArgs& a, hipStream_t s);
hipError_t launch_decompress(const DecArgs& a, hipStream_t s);

}  // namespace huff
}  // namespace gpulz
