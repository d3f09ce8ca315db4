/*
 * CPU oracle for chunked multi-byte LZSS (gpuLZ, Zhang et al., ICS'23).
 *
 * TEST INFRASTRUCTURE ONLY. This library is the slow, obviously correct
 * reference that the GPU path is checked against. Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it. The
 * product library never links, loads or calls it, and it shares no code,
 * header, table or constant with the GPU path.
 *
 * What it computes (each function cites the passage it follows):
 *   - the textbook greedy LZSS parse of the paper's section 2.2 (basic steps
 *     1-6): at each coding position take the longest window match; emit a
 *     pointer if it is at least the minimum encode length (section 3.3.2,
 *     Kernel I encoding step), else emit one literal symbol;
 *   - symbols are S = 1, 2, 4 or 8 raw bytes (section 3.2.3, multi-byte
 *     matching);
 *   - match policy 1 replaces the longest match by the paper's own
 *     single-pass window scan (section 3.3.2, matching steps 1-4);
 *   - the input is split into independent chunks of C symbols; no match
 *     crosses a chunk boundary and the window is empty at each chunk start
 *     (section 3.3.1, data chunks; section 2.2, the window starts empty);
 *   - a match never exceeds its offset (section 3.3.2, last paragraph of the
 *     matching method) nor 255 symbols (one-byte length field, section 2.2).
 *   - Ties between equal-length matches go to the largest offset.
 *
 * Stream layout (all little-endian):
 *   header (64 B) | table of N x {u32 flag_bytes, u32 payload_bytes} |
 *   per-chunk records, record = flag bytes followed by payload bytes.
 * Flag bit t of a chunk (bit t&7 of flag byte t>>3, LSB first) is 1 for a
 * pointer token and 0 for a literal. A literal's payload is its S raw bytes;
 * a pointer's payload is two bytes [length][offset & 0xFF] (offset 256 is
 * stored as 0).
 *
 * Status codes match the product's numbering so tests can compare them.
 */
#ifndef GPULZ_ORACLE_H
#define GPULZ_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORACLE_OK = 0,
  ORACLE_ERR_INVALID_ARG = 1,
  ORACLE_ERR_OUT_OF_SPACE = 2,
  ORACLE_ERR_CORRUPT = 3,
  ORACLE_ERR_NOMEM = 7
};

/* Worst-case stream size for these parameters, or 0 on invalid arguments. */
uint64_t oracle_compress_bound(uint64_t nbytes, uint32_t symbol_bytes,
                               uint32_t chunk_symbols, uint32_t min_match);

/* Compress x[0..n). On ORACLE_OK, out[0..*out_len) holds the stream. If the
 * stream does not fit in `capacity`, returns ORACLE_ERR_OUT_OF_SPACE with
 * *out_len set to the required size and writes nothing to out. */
int oracle_compress(const uint8_t* x, uint64_t n, uint32_t symbol_bytes,
                    uint32_t chunk_symbols, uint32_t window, uint32_t min_match,
                    uint8_t* out, uint64_t capacity, uint64_t* out_len);

/* Decompress and validate a stream. On ORACLE_OK, out[0..*out_len) holds the
 * original bytes. ORACLE_ERR_CORRUPT if any format rule is broken,
 * ORACLE_ERR_OUT_OF_SPACE (with *out_len = n) if capacity < n. */
int oracle_decompress(const uint8_t* in, uint64_t in_len, uint8_t* out,
                      uint64_t capacity, uint64_t* out_len);

/* Parse one chunk only (for inspecting tokens in tests). The chunk is
 * sym[0..c) of S-byte symbols. Writes up to c tokens: lengths[t] = 0 for a
 * literal, else the pointer length; offsets[t] = pointer offset (0 for a
 * literal). Returns the token count, or -1 on invalid arguments. */
int64_t oracle_parse_chunk(const uint8_t* chunk, uint32_t c, uint32_t symbol_bytes,
                           uint32_t window, uint32_t min_match,
                           uint32_t* lengths, uint32_t* offsets);

/* Compress with match policy 0 (the exact longest match, as oracle_compress)
 * or 1 (the paper's single-pass window scan of section 3.3.2, see
 * scan_match in the source). The policy is recorded in header byte 7. */
int oracle_compress_policy(const uint8_t* x, uint64_t n, uint32_t symbol_bytes,
                           uint32_t chunk_symbols, uint32_t window, uint32_t min_match,
                           uint32_t policy, uint8_t* out, uint64_t capacity, uint64_t* out_len);
int oracle_compress_policy_mt(const uint8_t* x, uint64_t n, uint32_t symbol_bytes,
                              uint32_t chunk_symbols, uint32_t window, uint32_t min_match,
                              uint32_t policy, uint8_t* out, uint64_t capacity,
                              uint64_t* out_len, int threads);

/* oracle_parse_chunk with an explicit match policy (0 or 1). */
int64_t oracle_parse_chunk_policy(const uint8_t* chunk, uint32_t c, uint32_t symbol_bytes,
                                  uint32_t window, uint32_t min_match, uint32_t policy,
                                  uint32_t* lengths, uint32_t* offsets);

/* Compress with the input split across `threads` POSIX threads by chunk
 * range (chunks are independent). Same output as oracle_compress; used only
 * to time the oracle on several host cores. */
int oracle_compress_mt(const uint8_t* x, uint64_t n, uint32_t symbol_bytes,
                       uint32_t chunk_symbols, uint32_t window, uint32_t min_match,
                       uint8_t* out, uint64_t capacity, uint64_t* out_len,
                       int threads);

#ifdef __cplusplus
}
#endif

#endif
