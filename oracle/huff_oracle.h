/* CPU oracle for the entropy stage that follows LZSS.
 *
 * TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may use it. It shares no code with the GPU
 * library.
 *
 * gpuLZ (Zhang et al., ICS'23) section 4.5 runs the LZSS stage in front of a
 * Huffman coder (the Deflate pairing of LZSS and Huffman is recalled in the
 * paper's background section). The paper does not define that coder; the
 * readings here are:
 *
 *   code lengths   Huffman's algorithm (Huffman, 1952) over the byte
 *                  frequencies of the whole input: repeatedly join the two
 *                  live nodes of smallest key (weight, index), where leaves
 *                  are indexed 0..255 by symbol and internal nodes 256, 257,
 *                  ... in creation order (so on equal weight a leaf goes
 *                  first, then the smaller symbol or the older node). A
 *                  symbol's length is its leaf's depth. One present symbol
 *                  gets length 1; an empty input gets no lengths. If a length
 *                  exceeds the limit (15), every present weight w becomes
 *                  ceil(w / 2) and the tree is built again.
 *   codes          canonical, as in RFC 1951 section 3.2.2: codes of each
 *                  length are consecutive in symbol order, and the first
 *                  code of length l is (first(l-1) + count(l-1)) << 1.
 *   stream         all integers little-endian:
 *                    0..3   "GLH1"            4..5   version 1
 *                    6      15 (length limit)  7      0
 *                    8..11  4096 (chunk symbols)
 *                    12..15 128 (sub-block symbols)
 *                    16..23 n, input bytes      24..31 N = ceil(n / 4096)
 *                    32..39 total stream bytes  40..63 zero
 *                    64..191 code lengths, two per byte: symbol 2k in bits
 *                           0-3 of byte 64 + k, symbol 2k + 1 in bits 4-7
 *                    192    N u32: bits_i, the code bits of chunk i
 *                    then one record per chunk, in order:
 *                      nsub_i = ceil(c_i / 128) u16 start bits of its
 *                      sub-blocks (the first is 0), zero-padded to a
 *                      multiple of 4 bytes; then ceil(bits_i / 32) u32 words
 *                      of code bits: bit k of the chunk is bit 31 - (k % 32)
 *                      of word k / 32; unused bits are zero.
 *                  c_i = min(4096, n - 4096 i). Each sub-block's start lets
 *                  a decoder begin there without decoding what precedes it.
 *
 * Status values: 0 ok, 1 invalid argument, 2 output too small (*out_len
 * gets the size needed), 3 corrupt stream, 7 out of memory.
 *
 * Pins (tests/test_oracle_huff.py): hand-worked streams and lengths under
 * tests/golden/huff_*.txt, the textbook frequency example, optimal cost
 * against an independent heap-based construction and against exhaustive
 * search over complete codes for small alphabets, canonical-code
 * properties, an independent Python encoder and decoder, round trips,
 * rejection of corrupted streams, and planted mistakes.
 */
#ifndef HUFF_ORACLE_H
#define HUFF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Code lengths for 256 byte frequencies with lengths at most max_len
 * (1 <= max_len <= 15). Returns 0, or 1 if the limit cannot hold all the
 * present symbols. */
int oracle_huff_lengths(const uint64_t freq[256], uint32_t max_len, uint8_t len[256]);

/* Canonical codes (value of the code, MSB = first bit) for the lengths. */
void oracle_huff_codes(const uint8_t len[256], uint32_t code[256]);

/* Largest stream for an input of n bytes. */
uint64_t oracle_huff_bound(uint64_t n);

int oracle_huff_compress(const uint8_t* in, uint64_t n, uint8_t* out, uint64_t cap,
                         uint64_t* out_len);

int oracle_huff_decompress(const uint8_t* in, uint64_t in_bytes, uint8_t* out, uint64_t cap,
                           uint64_t* out_len);

#ifdef __cplusplus
}
#endif

#endif
