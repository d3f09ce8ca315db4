/* CPU oracle for the entropy stage (Huffman coding of bytes) that follows
 * LZSS. TEST INFRASTRUCTURE ONLY. The definitions it follows and the stream
 * layout are in huff_oracle.h. Plain, slow code: the tree is built by
 * scanning all live nodes for the two smallest keys, and decoding reads one
 * bit at a time. */
#include "huff_oracle.h"

#include <stdlib.h>
#include <string.h>

#define HO_OK 0
#define HO_INVALID 1
#define HO_SPACE 2
#define HO_CORRUPT 3
#define HO_NOMEM 7

#define HO_HDR 64
#define HO_PRE 192 /* header + code lengths */
#define HO_CHUNK 4096u
#define HO_SUB 128u
#define HO_LIMIT 15u

static void put_u16(uint8_t* p, uint32_t v) {
  p[0] = (uint8_t)v;
  p[1] = (uint8_t)(v >> 8);
}
static void put_u32(uint8_t* p, uint32_t v) {
  for (int k = 0; k < 4; ++k) p[k] = (uint8_t)(v >> (8 * k));
}
static void put_u64(uint8_t* p, uint64_t v) {
  for (int k = 0; k < 8; ++k) p[k] = (uint8_t)(v >> (8 * k));
}
static uint32_t get_u16(const uint8_t* p) { return (uint32_t)p[0] | (uint32_t)p[1] << 8; }
static uint32_t get_u32(const uint8_t* p) {
  uint32_t v = 0;
  for (int k = 3; k >= 0; --k) v = v << 8 | p[k];
  return v;
}
static uint64_t get_u64(const uint8_t* p) {
  uint64_t v = 0;
  for (int k = 7; k >= 0; --k) v = v << 8 | p[k];
  return v;
}

/* The live node of smallest key (weight, index); -1 if none. */
static int take_min(const uint64_t* weight, int* alive, int nodes) {
  int best = -1;
  for (int x = 0; x < nodes; ++x) {
    if (!alive[x]) continue;
    if (best < 0 || weight[x] < weight[best]) best = x;  /* equal weight: smaller index stays */
  }
  if (best >= 0) alive[best] = 0;
  return best;
}

int oracle_huff_lengths(const uint64_t freq[256], uint32_t max_len, uint8_t len[256]) {
  uint64_t w[256];
  int present = 0;
  memset(len, 0, 256);
  for (int s = 0; s < 256; ++s) {
    w[s] = freq[s];
    present += w[s] != 0;
  }
  if (present == 0) return 0;
  if (max_len < 1 || max_len > 15) return 1;
  if (present == 1) {
    for (int s = 0; s < 256; ++s)
      if (w[s]) len[s] = 1;
    return 0;
  }
  if (max_len < 8 && present > (1 << max_len)) return 1;
  for (;;) {
    uint64_t weight[511];
    int alive[511], parent[511];
    int nodes = 256;
    for (int s = 0; s < 256; ++s) {
      weight[s] = w[s];
      alive[s] = w[s] != 0;
      parent[s] = -1;
    }
    for (int k = 0; k < present - 1; ++k) {
      const int a = take_min(weight, alive, nodes);
      const int b = take_min(weight, alive, nodes);
      weight[nodes] = weight[a] + weight[b];
      alive[nodes] = 1;
      parent[nodes] = -1;
      parent[a] = parent[b] = nodes;
      ++nodes;
    }
    uint32_t deepest = 0;
    for (int s = 0; s < 256; ++s) {
      if (!w[s]) continue;
      uint32_t d = 0;
      for (int x = s; parent[x] >= 0; x = parent[x]) ++d;
      len[s] = (uint8_t)(d > 255 ? 255 : d);
      if (d > deepest) deepest = d;
    }
    if (deepest <= max_len) return 0;
    for (int s = 0; s < 256; ++s) w[s] = (w[s] + 1) / 2;
  }
}

void oracle_huff_codes(const uint8_t len[256], uint32_t code[256]) {
  uint32_t count[16] = {0}, next[16] = {0};
  for (int s = 0; s < 256; ++s)
    if (len[s]) ++count[len[s]];
  uint32_t c = 0;
  for (int l = 1; l <= 15; ++l) {
    c = (c + count[l - 1]) << 1;
    next[l] = c;
  }
  for (int s = 0; s < 256; ++s) code[s] = len[s] ? next[len[s]]++ : 0;
}

static uint64_t chunks_of(uint64_t n) { return (n + HO_CHUNK - 1) / HO_CHUNK; }
static uint32_t subs_of(uint32_t c) { return (c + HO_SUB - 1) / HO_SUB; }
static uint64_t offsets_bytes(uint32_t nsub) { return (2ull * nsub + 3) / 4 * 4; }
static uint64_t record_bytes(uint32_t c, uint64_t bits) {
  return offsets_bytes(subs_of(c)) + 4 * ((bits + 31) / 32);
}

uint64_t oracle_huff_bound(uint64_t n) {
  const uint64_t N = chunks_of(n);
  return HO_PRE + N * (4 + record_bytes(HO_CHUNK, (uint64_t)HO_LIMIT * HO_CHUNK));
}

int oracle_huff_compress(const uint8_t* in, uint64_t n, uint8_t* out, uint64_t cap,
                         uint64_t* out_len) {
  uint64_t freq[256] = {0};
  uint8_t len[256];
  uint32_t code[256];
  *out_len = 0;
  for (uint64_t j = 0; j < n; ++j) ++freq[in[j]];
  if (oracle_huff_lengths(freq, HO_LIMIT, len) != 0) return HO_INVALID;
  oracle_huff_codes(len, code);

  const uint64_t N = chunks_of(n);
  const uint64_t bound = oracle_huff_bound(n);
  uint8_t* buf = (uint8_t*)calloc(bound, 1);
  if (!buf) return HO_NOMEM;
  uint64_t pos = HO_PRE + 4 * N;
  for (uint64_t i = 0; i < N; ++i) {
    const uint64_t first = i * HO_CHUNK;
    const uint32_t c = (uint32_t)(n - first < HO_CHUNK ? n - first : HO_CHUNK);
    const uint32_t nsub = subs_of(c);
    uint8_t* rec = buf + pos;
    uint8_t* words = rec + offsets_bytes(nsub);
    uint64_t bit = 0;
    for (uint32_t j = 0; j < c; ++j) {
      if (j % HO_SUB == 0) put_u16(rec + 2 * (j / HO_SUB), (uint32_t)bit);
      const uint8_t s = in[first + j];
      for (int b = len[s] - 1; b >= 0; --b, ++bit) {
        if ((code[s] >> b) & 1u) {
          uint8_t* wp = words + 4 * (bit / 32);
          const uint32_t wv = get_u32(wp) | (1u << (31 - bit % 32));
          put_u32(wp, wv);
        }
      }
    }
    put_u32(buf + HO_PRE + 4 * i, (uint32_t)bit);
    pos += record_bytes(c, bit);
  }
  memcpy(buf, "GLH1", 4);
  put_u16(buf + 4, 1);
  buf[6] = HO_LIMIT;
  put_u32(buf + 8, HO_CHUNK);
  put_u32(buf + 12, HO_SUB);
  put_u64(buf + 16, n);
  put_u64(buf + 24, N);
  put_u64(buf + 32, pos);
  for (int s = 0; s < 256; ++s) buf[HO_HDR + s / 2] |= (uint8_t)(len[s] << (4 * (s & 1)));
  *out_len = pos;
  if (pos > cap) {
    free(buf);
    return HO_SPACE;
  }
  memcpy(out, buf, pos);
  free(buf);
  return HO_OK;
}

/* Bit k of a chunk's code words. */
static uint32_t code_bit(const uint8_t* words, uint64_t k) {
  return (get_u32(words + 4 * (k / 32)) >> (31 - k % 32)) & 1u;
}

int oracle_huff_decompress(const uint8_t* in, uint64_t in_bytes, uint8_t* out, uint64_t cap,
                           uint64_t* out_len) {
  *out_len = 0;
  if (in_bytes < HO_PRE || memcmp(in, "GLH1", 4) != 0) return HO_CORRUPT;
  if (get_u16(in + 4) != 1 || in[6] != HO_LIMIT || in[7] != 0 || get_u32(in + 8) != HO_CHUNK ||
      get_u32(in + 12) != HO_SUB)
    return HO_CORRUPT;
  for (int b = 40; b < HO_HDR; ++b)
    if (in[b]) return HO_CORRUPT;
  const uint64_t n = get_u64(in + 16), N = get_u64(in + 24), total = get_u64(in + 32);
  if (total != in_bytes || N != chunks_of(n) || N > (in_bytes - HO_PRE) / 4) return HO_CORRUPT;

  /* the code: none for an empty input, one symbol of length 1, or complete */
  uint8_t len[256];
  uint32_t count[16] = {0}, present = 0;
  uint64_t kraft = 0;
  for (int s = 0; s < 256; ++s) {
    len[s] = (in[HO_HDR + s / 2] >> (4 * (s & 1))) & 15u;
    if (len[s]) {
      ++present;
      ++count[len[s]];
      kraft += 1ull << (15 - len[s]);
    }
  }
  if (n == 0 ? present != 0 : !(present == 1 ? count[1] == 1 : kraft == (1ull << 15)))
    return HO_CORRUPT;

  /* record positions; every record inside the stream, and nothing after */
  uint64_t pos = HO_PRE + 4 * N;
  for (uint64_t i = 0; i < N; ++i) {
    const uint32_t c = (uint32_t)(n - i * HO_CHUNK < HO_CHUNK ? n - i * HO_CHUNK : HO_CHUNK);
    const uint64_t bits = get_u32(in + HO_PRE + 4 * i);
    if (bits > (uint64_t)HO_LIMIT * c) return HO_CORRUPT;
    const uint64_t rb = record_bytes(c, bits);
    if (rb > in_bytes - pos) return HO_CORRUPT;
    pos += rb;
  }
  if (pos != in_bytes) return HO_CORRUPT;
  if (n > cap) {
    *out_len = n;
    return HO_SPACE;
  }

  /* canonical decoding tables: first code, count and first rank per length */
  uint32_t code[256], first[16] = {0}, rank0[16] = {0};
  uint8_t by_rank[256];
  oracle_huff_codes(len, code);
  {
    uint32_t r = 0;
    for (int l = 1; l <= 15; ++l) {
      rank0[l] = r;
      for (int s = 0; s < 256; ++s)
        if (len[s] == l) {
          if (r == rank0[l]) first[l] = code[s];
          by_rank[r++] = (uint8_t)s;
        }
    }
  }

  pos = HO_PRE + 4 * N;
  for (uint64_t i = 0; i < N; ++i) {
    const uint32_t c = (uint32_t)(n - i * HO_CHUNK < HO_CHUNK ? n - i * HO_CHUNK : HO_CHUNK);
    const uint32_t nsub = subs_of(c);
    const uint64_t bits = get_u32(in + HO_PRE + 4 * i);
    const uint8_t* rec = in + pos;
    const uint8_t* words = rec + offsets_bytes(nsub);
    for (uint64_t b = 2ull * nsub; b < offsets_bytes(nsub); ++b)
      if (rec[b]) return HO_CORRUPT;
    if (get_u16(rec) != 0) return HO_CORRUPT;
    for (uint32_t k = 0; k < nsub; ++k)
      if (get_u16(rec + 2 * k) > bits) return HO_CORRUPT;
    for (uint32_t k = 0; k < nsub; ++k) {
      uint64_t p = get_u16(rec + 2 * k);
      const uint64_t end = k + 1 < nsub ? get_u16(rec + 2 * (k + 1)) : bits;
      const uint32_t cnt = k + 1 < nsub ? HO_SUB : c - HO_SUB * k;
      for (uint32_t j = 0; j < cnt; ++j) {
        uint32_t v = 0, l = 0;
        for (;;) {
          if (p >= end) return HO_CORRUPT;
          v = v << 1 | code_bit(words, p++);
          if (++l > 15) return HO_CORRUPT;
          if (count[l] && v >= first[l] && v - first[l] < count[l]) break;
        }
        out[i * HO_CHUNK + HO_SUB * k + j] = by_rank[rank0[l] + (v - first[l])];
      }
      if (p != end) return HO_CORRUPT;
    }
    for (uint64_t b = bits; b < 32 * ((bits + 31) / 32); ++b)
      if (code_bit(words, b)) return HO_CORRUPT;
    pos += record_bytes(c, bits);
  }
  *out_len = n;
  return HO_OK;
}
