/*
 * gpulz — chunked multi-byte LZSS compression on AMD Instinct MI355X (gfx950).
 *
 * The method is gpuLZ (Zhang, Tian, Di, Yu, Swany, Tao, Cappello, ICS'23):
 *   - the input is split into independent chunks of C symbols; no match
 *     crosses a chunk boundary (section 3.3.1, data chunks);
 *   - symbols are S = 1, 2, 4 or 8 bytes and matching compares whole symbols
 *     (section 3.2.3, multi-byte matching);
 *   - inside a chunk, the greedy LZSS parse of section 2.2 (basic steps 1-6)
 *     takes the longest match in a sliding window of W symbols; a match of
 *     at least `min_match` symbols becomes a 2-byte pointer, anything else a
 *     literal (section 3.3.2, encoding step); a match never exceeds its
 *     offset (section 3.3.2) nor 255 symbols (one-byte fields, section 2.2);
 *     among equally long matches the largest offset wins;
 *   - per-token sizes are prefix-summed inside each chunk, the chunk sizes
 *     across chunks, and the chunk records are compacted into one stream
 *     (section 3.2.2, two-pass prefix sum; section 3.3.4, deflating).
 *
 * Stream layout (little-endian), identical for every producer:
 *   bytes 0..63   header:
 *       0  u8[4] magic "GLZ1"       4  u16 version = 1
 *       6  u8    S                  7  u8  match policy: 0 exact longest, 1 single pass
 *       8  u32   C (chunk symbols) 12  u16 W (window symbols, 1..256)
 *      14  u8    min_match         15  u8  max_match = 255
 *      16  u64   n (input bytes)   24  u64 N = ceil((n / S) / C) chunks
 *      32  u64   total stream bytes
 *      40  u8    r = n mod S       41..47 zero
 *      48  u8[8] the last r input bytes, zero padded   56..63 zero
 *   64 .. 64+8N  table: per chunk {u32 flag_bytes F_i, u32 payload_bytes P_i}
 *   then the records of chunks 0..N-1 back to back, each F_i flag bytes
 *   followed by P_i payload bytes. Flag bit t of a chunk (bit t & 7 of byte
 *   t >> 3) is 1 if token t is a pointer; F_i = ceil(T_i / 8), unused bits 0.
 *   A literal's payload is its S raw bytes; a pointer's is
 *   [length][offset & 0xFF] (offset 256 is stored as 0).
 *
 * Conventions for every entry point below:
 *   - Device pointers (d_*) are caller-owned device memory (for instance
 *     torch tensors). The library never allocates or frees on the
 *     compress/decompress paths; it only launches kernels on `stream`.
 *   - d_in and d_out must be 16-byte aligned; d_workspace 256-byte aligned.
 *   - Sizes are in bytes; chunk_symbols, window and min_match in symbols.
 *   - The return value reports host-detectable problems only (invalid
 *     argument, workspace too small, chunk too large for on-chip memory,
 *     a failed HIP launch). Outcomes that depend on the data are written on
 *     the stream to *d_status (a gpulz_status) and *d_out_bytes; read them
 *     after synchronising the stream.
 *   - Calls on different streams with distinct workspaces may overlap.
 */
#ifndef GPULZ_H
#define GPULZ_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GPULZ_OK = 0,
  GPULZ_ERR_INVALID_ARG = 1,
  GPULZ_ERR_OUT_OF_SPACE = 2,
  GPULZ_ERR_CORRUPT = 3,
  GPULZ_ERR_WORKSPACE = 4,
  GPULZ_ERR_HIP = 5,
  GPULZ_ERR_UNSUPPORTED = 6
} gpulz_status;

/* Version of this interface (major * 100 + minor). */
uint32_t gpulz_abi_version(void);

/* Static string naming a status code ("unknown status" for other values). */
const char* gpulz_status_string(gpulz_status status);

/* Largest stream gpulz_compress can produce for these parameters: header,
 * table, and for every chunk of c symbols ceil(c/8) flag bytes plus c*k
 * payload bytes, k = 2 if S == 1 and min_match == 1 (every token a pointer)
 * else S (every token a literal). Returns 0 if the parameters are invalid.
 * Host-only, pure. */
uint64_t gpulz_compress_bound(uint64_t nbytes, uint32_t symbol_bytes, uint32_t chunk_symbols,
                              uint32_t min_match);

/* Workspace bytes gpulz_compress needs for an input of `nbytes`. Host-only.
 * Returns GPULZ_ERR_INVALID_ARG for invalid parameters or a NULL ws_bytes. */
gpulz_status gpulz_compress_workspace_size(uint64_t nbytes, uint32_t symbol_bytes,
                                           uint32_t chunk_symbols, size_t* ws_bytes);

/* Compress d_in[0..nbytes) into d_out as one stream (layout above).
 *   symbol_bytes  S in {1, 2, 4, 8}
 *   chunk_symbols C >= 1; the chunk must fit in on-chip memory
 *                 (C * S <= 48 KiB), else GPULZ_ERR_UNSUPPORTED
 *   window        W in [1, 256]
 *   min_match     in [1, 255]
 *   out_capacity  bytes available at d_out
 *   d_out_bytes   device u64: receives the stream size (also when it does
 *                 not fit)
 *   d_status      device i32: GPULZ_OK; GPULZ_ERR_OUT_OF_SPACE if the
 *                 stream is larger than out_capacity (then no byte at or
 *                 past out_capacity is written and d_out's contents are
 *                 unspecified); GPULZ_ERR_HIP if a device-side wait of the
 *                 record-offset look-back gave up (not expected in use)
 *   d_workspace   at least gpulz_compress_workspace_size bytes
 * The call launches one small preparation kernel and then one chunk-encoder
 * launch per 2^22 chunks: every chunk finds its record offset by decoupled
 * look-back over the sizes its predecessors publish (the global prefix sum
 * of section 3.2.2) and writes its table entry and record once, at the final
 * place (section 3.3.4's compaction needs no pass of its own). Inputs of
 * more than 2^27 chunks give GPULZ_ERR_UNSUPPORTED.
 * The chunk encoder runs with the waves_per_chunk of the width's defaults
 * (gpulz_default_params); that changes speed, never the bytes.
 * Asynchronous on `stream` (0 = null stream). Same bytes as any other
 * conforming producer for the same input and parameters. Calls that overlap
 * must use distinct workspaces. */
gpulz_status gpulz_compress(const void* d_in, uint64_t nbytes, uint32_t symbol_bytes,
                            uint32_t chunk_symbols, uint32_t window, uint32_t min_match,
                            void* d_out, uint64_t out_capacity, uint64_t* d_out_bytes,
                            int32_t* d_status, void* d_workspace, size_t ws_bytes,
                            hipStream_t stream);

/* gpulz_compress with an explicit match policy, recorded in header byte 7:
 *   0  the exact longest match (gpulz_compress);
 *   1  the paper's own single pass over the window (gpuLZ section 3.3.2,
 *      matching steps 1-4): per coding position, a window pointer walks once
 *      from the oldest slot; runs of equal symbols are candidates that win
 *      only if strictly longer; after a mismatch the look-ahead restarts at
 *      the coding position and the walk continues at the next slot (the
 *      failed slot is not retried as a start); the run still open when the
 *      walk ends counts, and runs stop at 255 symbols. Lengths never exceed
 *      offsets. Not always the longest match; cost W steps per position.
 * Other arguments, results and errors as gpulz_compress; policy > 1 gives
 * GPULZ_ERR_INVALID_ARG, and policy 1 also needs the chunk plus two bytes
 * per symbol of tables in on-chip memory (GPULZ_ERR_UNSUPPORTED when
 * C * (S + 2) exceeds about 60 KiB). Both policies decode with
 * gpulz_decompress. */
gpulz_status gpulz_compress_policy(const void* d_in, uint64_t nbytes, uint32_t symbol_bytes,
                                   uint32_t chunk_symbols, uint32_t window, uint32_t min_match,
                                   uint32_t match_policy, void* d_out, uint64_t out_capacity,
                                   uint64_t* d_out_bytes, int32_t* d_status, void* d_workspace,
                                   size_t ws_bytes, hipStream_t stream);

/* Read the fields of a stream header from a host copy of its first 64 bytes.
 * Validates magic, version and field ranges; GPULZ_ERR_CORRUPT otherwise.
 * Any output pointer may be NULL. Host-only. */
gpulz_status gpulz_peek_header(const void* h_header, size_t header_bytes, uint64_t* nbytes,
                               uint32_t* symbol_bytes, uint64_t* stream_bytes);

/* ---- stream layout, for callers that assemble or split streams ---------
 * Data blocks (section 3.3.1): an input too large for device memory is
 * compressed block by block, each block a whole number of chunks. Since
 * chunks are independent, a block's table entries and records are exactly
 * those of the whole input at its chunk and record bases, so one stream is
 * assembled from the blocks' streams with the entry points below (and split
 * into per-block streams for decompression the same way). */

/* Fields of a stream header (the layout above). */
typedef struct {
  uint64_t nbytes;        /* n: decompressed bytes */
  uint64_t chunks;        /* N */
  uint64_t stream_bytes;  /* total stream bytes */
  uint32_t symbol_bytes, chunk_symbols, window, min_match, match_policy;
  uint32_t tail_bytes;    /* r = n mod S */
  uint8_t tail[8];        /* the last r input bytes */
} gpulz_stream_info;

/* Byte offset of chunk i's table entry in a stream; with i = N, the offset
 * of chunk 0's record. Host-only. */
uint64_t gpulz_table_offset(uint64_t chunk);

/* Writes the 64-byte header of a stream with these fields into h_header
 * (host memory, 64 bytes); h_tail holds the n mod S bytes after the last
 * whole symbol (may be NULL when there are none). The chunk count is
 * derived from n, S and C. GPULZ_ERR_INVALID_ARG for parameters that
 * gpulz_compress rejects, a match policy other than 0 or 1, or a stream
 * size below 64 + 8N. Host-only. */
gpulz_status gpulz_write_header(void* h_header, uint64_t nbytes, uint32_t symbol_bytes,
                                uint32_t chunk_symbols, uint32_t window, uint32_t min_match,
                                uint32_t match_policy, uint64_t stream_bytes, const void* h_tail);

/* Reads every field of a header from a host copy of its first 64 bytes and
 * checks them as the decoder does (magic, version, parameter ranges, N from
 * n, S and C, a stream size of at least 64 + 8N, zero reserved bytes);
 * GPULZ_ERR_CORRUPT otherwise. Host-only. */
gpulz_status gpulz_read_header(const void* h_header, size_t header_bytes, gpulz_stream_info* info);

/* Record offsets from a stream's table (section 3.2.2, the prefix sum over
 * chunk sizes): d_table holds `chunks` table entries (8 bytes each, 4-byte
 * aligned, device memory), and d_offsets (device, chunks + 1 u64) receives
 * offsets[i] = F_0 + P_0 + ... + F_{i-1} + P_{i-1}, the offset of chunk i's
 * record from chunk 0's, and offsets[chunks] = all record bytes. One
 * workgroup, asynchronous on `stream`; no workspace. */
gpulz_status gpulz_record_offsets(const void* d_table, uint64_t chunks, uint64_t* d_offsets,
                                  hipStream_t stream);

/* Workspace bytes gpulz_decompress needs for a stream of `comp_bytes` whose
 * decompressed size is `nbytes` (0 if not known). The size is that of the
 * most chunks a stream of comp_bytes can hold (the decoder rejects a header
 * that claims more), so it does not depend on nbytes. Host-only. */
gpulz_status gpulz_decompress_workspace_size(uint64_t comp_bytes, uint64_t nbytes,
                                             size_t* ws_bytes);

/* Decompress the stream d_in[0..in_bytes) into d_out. The decoder checks
 * every rule of the layout (header fields, table sums, flag and payload
 * extents, each pointer within 1..W, within the symbols already decoded in
 * its chunk, not longer than its offset and not past the chunk end, unused
 * flag bits zero). On the stream it writes *d_status = GPULZ_OK,
 * GPULZ_ERR_CORRUPT (a rule is broken; d_out contents are then
 * unspecified) or GPULZ_ERR_OUT_OF_SPACE (out_capacity < n; nothing is
 * written to d_out), and *d_out_bytes = n from a valid header (0 if the
 * header is invalid). Asynchronous on `stream`. */
gpulz_status gpulz_decompress(const void* d_in, uint64_t in_bytes, void* d_out,
                              uint64_t out_capacity, uint64_t* d_out_bytes, int32_t* d_status,
                              void* d_workspace, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * decompression as gpulz_decompress, with the workspace taken from a
 * library-owned device array instead of a caller's buffer. The array holds
 * 13,422,080 bytes on each GPU the library runs on, kept until the process
 * ends; it serves streams of at most 2^30 bytes (GPULZ_ERR_WORKSPACE,
 * nothing launched, for a larger in_bytes). Calls on one GPU share that
 * array: calls that overlap on one GPU (different streams, or host threads)
 * race and must be serialised by the caller. The array needs no clearing
 * between calls (each call rewrites what it reads). Arguments, outcomes and
 * asynchrony as gpulz_decompress; the first call on a device also looks up
 * the array's address there (GPULZ_ERR_HIP if that fails). */
gpulz_status gpulz_decompress_noalloc(const void* d_in, uint64_t in_bytes, void* d_out,
                                      uint64_t out_capacity, uint64_t* d_out_bytes,
                                      int32_t* d_status, hipStream_t stream);

/* ---- batches ------------------------------------------------------------
 * Many buffers, each with its own size and symbol width, compressed or
 * decompressed by one fixed sequence of launches on one stream (a plan
 * kernel, one persistent kernel that takes (buffer, chunk) work items from a
 * device-side ticket, a per-buffer scan, a compaction), with no host round
 * trip and no allocation, so the call can be captured in a HIP graph and
 * replayed with new array contents. Each buffer's output is a standalone
 * stream, byte-identical to gpulz_compress / gpulz_decompress on that buffer
 * with the same parameters.
 * All arrays below are device memory holding one entry per buffer.
 */

/* Parameters for one symbol width; zero fields take the library default for
 * that width. waves_per_chunk is the workgroup size of the chunk encoder in
 * wavefronts (1, 2 or 4); one batch launch uses the largest value given. */
typedef struct {
  uint32_t chunk_symbols;
  uint32_t window;
  uint32_t min_match;
  uint32_t waves_per_chunk;
} gpulz_params;

/* Current defaults for symbol width S (1, 2, 4 or 8). Host-only. */
gpulz_status gpulz_default_params(uint32_t symbol_bytes, gpulz_params* params);

/* Replace the defaults for width S (e.g. with an autotuner's choice). Every
 * field must be valid (no zeros). Host-only; process-wide. */
gpulz_status gpulz_set_default_params(uint32_t symbol_bytes, const gpulz_params* params);

/* Workspace for gpulz_compress_batch of up to nbufs buffers holding up to
 * max_total_in_bytes input bytes in total. params_by_width[i] applies to
 * symbol width 1 << i; NULL means all defaults. Host-only. */
gpulz_status gpulz_compress_batch_workspace_size(uint64_t nbufs, uint64_t max_total_in_bytes,
                                                 const gpulz_params params_by_width[4],
                                                 size_t* ws_bytes);

/* Compress buffer b = d_in_ptrs[b][0 .. d_in_bytes[b]) with symbol width
 * d_symbol_bytes[b] into d_out_ptrs[b] (capacity d_out_caps[b]). Per buffer,
 * on the stream: d_out_bytes[b] = its stream size, d_status[b] = GPULZ_OK,
 * GPULZ_ERR_OUT_OF_SPACE (nothing written to that output),
 * GPULZ_ERR_INVALID_ARG (bad width, or a pointer not 16-byte aligned) or
 * GPULZ_ERR_WORKSPACE (the inputs exceed max_total_in_bytes; then every
 * buffer gets it). Host-detectable errors are returned. */
gpulz_status gpulz_compress_batch(uint64_t nbufs, const void* const* d_in_ptrs,
                                  const uint64_t* d_in_bytes, const uint8_t* d_symbol_bytes,
                                  const gpulz_params params_by_width[4], void* const* d_out_ptrs,
                                  const uint64_t* d_out_caps, uint64_t* d_out_bytes,
                                  int32_t* d_status, uint64_t max_total_in_bytes, void* d_workspace,
                                  size_t ws_bytes, hipStream_t stream);

/* Workspace for gpulz_decompress_batch of up to nbufs streams holding up to
 * max_total_in_bytes stream bytes in total. Host-only. */
gpulz_status gpulz_decompress_batch_workspace_size(uint64_t nbufs, uint64_t max_total_in_bytes,
                                                   size_t* ws_bytes);

/* Decompress stream b = d_in_ptrs[b][0 .. d_in_bytes[b]) into d_out_ptrs[b]
 * (capacity d_out_caps[b]). Per buffer, on the stream: d_out_bytes[b] = its
 * original size (0 if the header is invalid), d_status[b] = GPULZ_OK,
 * GPULZ_ERR_CORRUPT, GPULZ_ERR_OUT_OF_SPACE, GPULZ_ERR_INVALID_ARG (a pointer
 * not 16-byte aligned) or GPULZ_ERR_WORKSPACE (the streams exceed
 * max_total_in_bytes). */
gpulz_status gpulz_decompress_batch(uint64_t nbufs, const void* const* d_in_ptrs,
                                    const uint64_t* d_in_bytes, void* const* d_out_ptrs,
                                    const uint64_t* d_out_caps, uint64_t* d_out_bytes,
                                    int32_t* d_status, uint64_t max_total_in_bytes,
                                    void* d_workspace, size_t ws_bytes, hipStream_t stream);

/* ---- Entropy stage: Huffman coding of bytes ---------------------------------
 *
 * gpuLZ (section 4.5) places the LZSS stage in front of a Huffman coder; these
 * calls provide that coder for any byte buffer (an LZSS stream, or raw
 * bytes). The paper does not specify the coder, so the code is defined as:
 *   - one code for the input, from its byte frequencies, by Huffman's
 *     algorithm: repeatedly join the two nodes of smallest (weight, index),
 *     where leaves are indexed 0-255 by symbol and internal nodes 256, 257,
 *     ... in the order they are made; a symbol's length is its depth. One
 *     distinct symbol gets length 1. If a length exceeds 15, every weight w
 *     becomes ceil(w / 2) and the tree is built again;
 *   - canonical codes (RFC 1951 section 3.2.2).
 * Stream layout (little-endian):
 *   0..3 "GLH1"; 4..5 version 1; 6 15 (longest code); 7 0;
 *   8..11 4096 (chunk bytes); 12..15 128 (sub-block bytes);
 *   16..23 n; 24..31 N = ceil(n / 4096); 32..39 total stream bytes;
 *   40..63 zero;
 *   64..191 code lengths, symbol 2k in bits 0-3 and 2k + 1 in bits 4-7 of
 *           byte 64 + k;
 *   192..  N u32 bits_i (code bits of chunk i);
 *   then per chunk: ceil(c_i / 128) u16 start bits of its 128-byte
 *   sub-blocks (the first is 0), zero-padded to a multiple of 4 bytes, then
 *   ceil(bits_i / 32) u32 words, bit k of the chunk = bit 31 - (k % 32) of
 *   word k / 32, unused bits zero (c_i = min(4096, n - 4096 i)). */

/* Largest stream for an input of n bytes (0 if n exceeds 2^40). Host-only. */
uint64_t gpulz_huff_compress_bound(uint64_t nbytes);

/* Workspace bytes for gpulz_huff_compress with inputs of up to max_bytes.
 * Host-only. */
gpulz_status gpulz_huff_compress_workspace_size(uint64_t max_bytes, size_t* ws_bytes);

/* Huffman-code d_in into d_out. The input size is `nbytes`, or, when
 * d_nbytes is not NULL, the device value *d_nbytes read by the kernels
 * (then `nbytes` is its maximum; a larger value gives *d_status =
 * GPULZ_ERR_INVALID_ARG and *d_out_bytes = 0). This lets the call follow
 * gpulz_compress on the same stream with d_nbytes = that call's d_out_bytes,
 * with no host round trip. out_capacity must be at least
 * gpulz_huff_compress_bound(nbytes) (else GPULZ_ERR_OUT_OF_SPACE, nothing
 * launched). d_in and d_out 16-byte aligned, d_workspace 256-byte aligned
 * (else GPULZ_ERR_INVALID_ARG); workspace as sized above (else
 * GPULZ_ERR_WORKSPACE). Writes *d_out_bytes and *d_status = GPULZ_OK.
 * Asynchronous on `stream`; the caller owns every buffer. */
gpulz_status gpulz_huff_compress(const void* d_in, uint64_t nbytes, const uint64_t* d_nbytes,
                                 void* d_out, uint64_t out_capacity, uint64_t* d_out_bytes,
                                 int32_t* d_status, void* d_workspace, size_t ws_bytes,
                                 hipStream_t stream);

/* Workspace bytes for gpulz_huff_decompress of a stream of stream_bytes.
 * Host-only. */
gpulz_status gpulz_huff_decompress_workspace_size(uint64_t stream_bytes, size_t* ws_bytes);

/* Decode a Huffman stream d_in[0..in_bytes) into d_out. Every rule of the
 * layout is checked: header fields, a code that is complete (or one symbol
 * of length 1, or no symbol for n = 0), record sizes that tile the stream,
 * each sub-block decoding exactly its symbols from its start bit to the next
 * one's, zero padding. Writes *d_status = GPULZ_OK, GPULZ_ERR_CORRUPT (d_out
 * contents unspecified) or GPULZ_ERR_OUT_OF_SPACE (out_capacity < n; nothing
 * written), and *d_out_bytes = n (0 for a bad header). Alignment and
 * workspace rules as gpulz_huff_compress. Asynchronous on `stream`. */
gpulz_status gpulz_huff_decompress(const void* d_in, uint64_t in_bytes, void* d_out,
                                   uint64_t out_capacity, uint64_t* d_out_bytes, int32_t* d_status,
                                   void* d_workspace, size_t ws_bytes, hipStream_t stream);

/* Kernel timing for benchmarks. While enabled, every gpulz_compress and
 * gpulz_decompress call records a pair of HIP events on its own stream
 * around each kernel it launches, so the times cover exactly those kernels.
 * Kernel ids: 0 chunk encode (with the look-back and the record write-out),
 * 1 compress preparation, 2 not used, 3 decode prepare (header check + table
 * scan), 4 chunk decode, 5 a whole
 * gpulz_compress_batch call, 6 a whole gpulz_decompress_batch call, 7 a
 * whole gpulz_huff_compress call, 8 a whole gpulz_huff_decompress call.
 * gpulz_profile_enable(1) clears the accumulated times, (0) stops recording.
 * gpulz_profile_read waits for the recorded events and writes, for each of
 * the first `nkernels` ids, the summed milliseconds and the launch count
 * (either pointer may be NULL). Host-side; not for concurrent use. */
gpulz_status gpulz_profile_enable(int enable);
gpulz_status gpulz_profile_read(double* total_ms, uint64_t* launches, int nkernels);

#ifdef __cplusplus
}
#endif

#endif /* GPULZ_H */
