/*
 * CPU oracle for chunked multi-byte LZSS (gpuLZ, Zhang et al., ICS'23).
 *
 * TEST INFRASTRUCTURE ONLY: see gpulz_oracle.h. Plain C99, no intrinsics,
 * no GPU headers, no blocking or fusion beyond the definition below, so that
 * each step can be checked against the paper by eye.
 *
 * Parity status: every function here is pinned by tests that do not reuse
 * this code (hand-worked byte vectors, a brute-force slice-comparison
 * reference on exhaustive tiny inputs, closed forms on constant and
 * all-distinct inputs, a per-token longest-match certificate check, and
 * round trips).
 */
#include "gpulz_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define HDR_BYTES 64u
#define MAX_MATCH 255u
#define MAX_CHUNK (1u << 24)

/* ---- little-endian helpers (the stream is little-endian by definition) -- */
static void put_u16(uint8_t* p, uint32_t v) {
  p[0] = (uint8_t)v;
  p[1] = (uint8_t)(v >> 8);
}
static void put_u32(uint8_t* p, uint32_t v) {
  int k;
  for (k = 0; k < 4; ++k) p[k] = (uint8_t)(v >> (8 * k));
}
static void put_u64(uint8_t* p, uint64_t v) {
  int k;
  for (k = 0; k < 8; ++k) p[k] = (uint8_t)(v >> (8 * k));
}
static uint32_t get_u16(const uint8_t* p) { return (uint32_t)p[0] | ((uint32_t)p[1] << 8); }
static uint32_t get_u32(const uint8_t* p) {
  uint32_t v = 0;
  int k;
  for (k = 3; k >= 0; --k) v = (v << 8) | p[k];
  return v;
}
static uint64_t get_u64(const uint8_t* p) {
  uint64_t v = 0;
  int k;
  for (k = 7; k >= 0; --k) v = (v << 8) | p[k];
  return v;
}

static int valid_params(uint32_t S, uint32_t C, uint32_t W, uint32_t MIN) {
  if (!(S == 1 || S == 2 || S == 4 || S == 8)) return 0;
  if (C < 1 || C > MAX_CHUNK) return 0;
  if (W < 1 || W > 256) return 0;
  if (MIN < 1 || MIN > MAX_MATCH) return 0;
  return 1;
}

/* Symbols are compared as raw S-byte strings (section 3.2.3: matching works
 * on symbols of S bytes instead of single bytes). Bitwise equality. */
static int sym_eq(const uint8_t* chunk, uint32_t a, uint32_t b, uint32_t S) {
  return memcmp(chunk + (size_t)a * S, chunk + (size_t)b * S, S) == 0;
}

/* Step 2 of the basic LZSS steps (section 2.2): find the longest match that
 * starts at coding position p. The window holds the min(W, p) symbols before
 * p inside this chunk (it starts empty at the chunk start, section 2.2, and
 * never reaches into another chunk, section 3.3.1). The match length is
 * capped by the offset (section 3.3.2: a match never exceeds its offset), by
 * 255 (one-byte length field, section 2.2) and by the end of the chunk.
 * Offsets are tried from the oldest window slot to the newest, keeping a
 * candidate only if strictly longer, so ties go to the largest offset. */
static void best_match(const uint8_t* chunk, uint32_t c, uint32_t S, uint32_t W,
                       uint32_t p, uint32_t* L_out, uint32_t* d_out) {
  uint32_t lim = c - p;
  uint32_t dmax = p < W ? p : W;
  uint32_t bestL = 0, bestd = 0, d;
  if (lim > MAX_MATCH) lim = MAX_MATCH;
  for (d = dmax; d >= 1; --d) {
    uint32_t cap = d < lim ? d : lim;
    uint32_t L = 0;
    while (L < cap && sym_eq(chunk, p + L, p - d + L, S)) ++L;
    if (L > bestL) {
      bestL = L;
      bestd = d;
    }
  }
  *L_out = bestL;
  *d_out = bestd;
}

/* Match policy 1: the paper's own single-pass search (section 3.3.2,
 * matching steps 1-4). A window pointer w starts at the oldest window slot
 * and a buffer pointer b at the coding position p. While the symbols at b
 * and w are equal both advance and the current match grows (its offset is
 * p - w at its first symbol). At a mismatch the current match replaces the
 * best one if strictly longer, b returns to p, and w still advances by one,
 * so the slot where a match failed is not retried as a match start. The
 * walk ends when w reaches p (the match never exceeds its offset) or b
 * reaches the chunk end. Readings where the paper is silent: the match in
 * progress when the walk ends is compared too, and a match stops growing at
 * 255 symbols (one-byte length field, section 2.2). */
static void scan_match(const uint8_t* chunk, uint32_t c, uint32_t S, uint32_t W, uint32_t p,
                       uint32_t* L_out, uint32_t* d_out) {
  uint32_t w = p > W ? p - W : 0, b = p, len = 0, off = 0, bestL = 0, bestd = 0;
  while (w < p && b < c) {
    if (len < MAX_MATCH && sym_eq(chunk, b, w, S)) {
      if (len == 0) off = p - w;
      ++len;
      ++b;
    } else {
      if (len > bestL) {
        bestL = len;
        bestd = off;
      }
      len = 0;
      off = 0;
      b = p;
    }
    ++w;
  }
  if (len > bestL) {
    bestL = len;
    bestd = off;
  }
  *L_out = bestL;
  *d_out = bestd;
}

/* Steps 1-6 of section 2.2 on one chunk: start at the chunk's first symbol;
 * if the longest match is at least min_match long (the encoding step of
 * section 3.3.2), emit a pointer and advance by its length, else emit one
 * literal and advance by one. */
int64_t oracle_parse_chunk_policy(const uint8_t* chunk, uint32_t c, uint32_t S, uint32_t W,
                                  uint32_t MIN, uint32_t policy, uint32_t* lengths,
                                  uint32_t* offsets) {
  uint32_t p = 0;
  int64_t t = 0;
  if (!valid_params(S, c ? c : 1, W, MIN) || policy > 1) return -1;
  while (p < c) {
    uint32_t L, d;
    if (policy == 0) best_match(chunk, c, S, W, p, &L, &d);
    else scan_match(chunk, c, S, W, p, &L, &d);
    if (L >= MIN) {
      lengths[t] = L;
      offsets[t] = d;
      p += L;
    } else {
      lengths[t] = 0;
      offsets[t] = 0;
      p += 1;
    }
    ++t;
  }
  return t;
}

int64_t oracle_parse_chunk(const uint8_t* chunk, uint32_t c, uint32_t S, uint32_t W,
                           uint32_t MIN, uint32_t* lengths, uint32_t* offsets) {
  return oracle_parse_chunk_policy(chunk, c, S, W, MIN, 0, lengths, offsets);
}

/* Serialise one parsed chunk: flag bytes (one bit per token, 1 = pointer,
 * section 2.2 flag array and section 3.3.2), then the payload: a literal is
 * its S raw bytes, a pointer is [length][offset & 0xFF]. Returns the record
 * size; F and P receive the flag and payload byte counts. `rec` may be NULL
 * to only size the record. */
static uint64_t encode_record(const uint8_t* chunk, uint32_t S, int64_t T,
                              const uint32_t* lengths, const uint32_t* offsets,
                              uint8_t* rec, uint32_t* F_out, uint32_t* P_out) {
  uint32_t F = (uint32_t)((T + 7) / 8);
  uint32_t P = 0, p = 0;
  int64_t t;
  if (rec) memset(rec, 0, F);
  for (t = 0; t < T; ++t) {
    if (lengths[t] != 0) {
      if (rec) {
        rec[t >> 3] |= (uint8_t)(1u << (t & 7));
        rec[F + P] = (uint8_t)lengths[t];
        rec[F + P + 1] = (uint8_t)(offsets[t] & 0xFFu);
      }
      P += 2;
      p += lengths[t];
    } else {
      if (rec) memcpy(rec + F + P, chunk + (size_t)p * S, S);
      P += S;
      p += 1;
    }
  }
  *F_out = F;
  *P_out = P;
  return (uint64_t)F + P;
}

uint64_t oracle_compress_bound(uint64_t n, uint32_t S, uint32_t C, uint32_t MIN) {
  uint64_t m, N, k, full, last, total;
  if (!valid_params(S, C, 1, MIN)) return 0;
  m = n / S;
  N = (m + C - 1) / C;
  k = (S == 1 && MIN == 1) ? 2 : S; /* all literals, or all length-1 pointers */
  full = m / C;
  last = m % C;
  total = HDR_BYTES + 8 * N;
  total += full * ((C + 7) / 8 + (uint64_t)C * k);
  if (last) total += (last + 7) / 8 + last * k;
  return total;
}

static void write_header(uint8_t* h, uint64_t n, uint32_t S, uint32_t C, uint32_t W,
                         uint32_t MIN, uint32_t policy, uint64_t N, uint64_t total,
                         const uint8_t* tail) {
  uint32_t r = (uint32_t)(n % S), k;
  memset(h, 0, HDR_BYTES);
  h[0] = 'G';
  h[1] = 'L';
  h[2] = 'Z';
  h[3] = '1';
  put_u16(h + 4, 1);      /* version */
  h[6] = (uint8_t)S;      /* symbol bytes */
  h[7] = (uint8_t)policy; /* match policy: 0 exact longest match, 1 single-pass scan */
  put_u32(h + 8, C);      /* chunk symbols */
  put_u16(h + 12, W);     /* window (256 fits the u16 field) */
  h[14] = (uint8_t)MIN;   /* minimum match */
  h[15] = MAX_MATCH;      /* maximum match */
  put_u64(h + 16, n);     /* original bytes */
  put_u64(h + 24, N);     /* chunk count */
  put_u64(h + 32, total); /* stream bytes */
  h[40] = (uint8_t)r;     /* tail length */
  for (k = 0; k < r; ++k) h[48 + k] = tail[k];
}

typedef struct {
  const uint8_t* x;
  uint64_t m;
  uint32_t S, C, W, MIN, policy;
  uint64_t first, last; /* chunk range [first, last) */
  uint8_t* recs;        /* records at chunk slots of `slot` bytes */
  uint64_t slot;
  uint32_t* F;
  uint32_t* P;
  int failed;
} job_t;

static void* run_job(void* arg) {
  job_t* j = (job_t*)arg;
  uint32_t* lengths = (uint32_t*)malloc(sizeof(uint32_t) * j->C);
  uint32_t* offsets = (uint32_t*)malloc(sizeof(uint32_t) * j->C);
  uint64_t i;
  if (!lengths || !offsets) {
    j->failed = 1;
    free(lengths);
    free(offsets);
    return NULL;
  }
  for (i = j->first; i < j->last; ++i) {
    uint64_t cs = i * j->C;
    uint32_t c = (uint32_t)((j->m - cs) < j->C ? (j->m - cs) : j->C);
    const uint8_t* chunk = j->x + cs * j->S;
    int64_t T = oracle_parse_chunk_policy(chunk, c, j->S, j->W, j->MIN, j->policy, lengths, offsets);
    encode_record(chunk, j->S, T, lengths, offsets, j->recs + i * j->slot, &j->F[i], &j->P[i]);
  }
  free(lengths);
  free(offsets);
  return NULL;
}

static int compress_impl(const uint8_t* x, uint64_t n, uint32_t S, uint32_t C, uint32_t W,
                         uint32_t MIN, uint32_t policy, uint8_t* out, uint64_t capacity,
                         uint64_t* out_len, int threads) {
  uint64_t m, N, slot, total, i, pos;
  uint8_t* recs;
  uint32_t *F, *P;
  int status = ORACLE_OK, t;
  if (!out_len || (n && !x) || !valid_params(S, C, W, MIN) || policy > 1)
    return ORACLE_ERR_INVALID_ARG;
  m = n / S;
  N = (m + C - 1) / C;
  slot = (C + 7) / 8 + (uint64_t)C * ((S == 1 && MIN == 1) ? 2 : S);
  recs = (uint8_t*)malloc(N ? N * slot : 1);
  F = (uint32_t*)malloc(sizeof(uint32_t) * (N ? N : 1));
  P = (uint32_t*)malloc(sizeof(uint32_t) * (N ? N : 1));
  if (!recs || !F || !P) {
    free(recs);
    free(F);
    free(P);
    return ORACLE_ERR_NOMEM;
  }
  if (threads < 1) threads = 1;
  if ((uint64_t)threads > N) threads = N ? (int)N : 1;
  {
    job_t* jobs = (job_t*)calloc((size_t)threads, sizeof(job_t));
    pthread_t* tids = (pthread_t*)calloc((size_t)threads, sizeof(pthread_t));
    if (!jobs || !tids) {
      free(jobs);
      free(tids);
      free(recs);
      free(F);
      free(P);
      return ORACLE_ERR_NOMEM;
    }
    for (t = 0; t < threads; ++t) {
      jobs[t].x = x;
      jobs[t].m = m;
      jobs[t].S = S;
      jobs[t].C = C;
      jobs[t].W = W;
      jobs[t].MIN = MIN;
      jobs[t].policy = policy;
      jobs[t].first = N * (uint64_t)t / (uint64_t)threads;
      jobs[t].last = N * (uint64_t)(t + 1) / (uint64_t)threads;
      jobs[t].recs = recs;
      jobs[t].slot = slot;
      jobs[t].F = F;
      jobs[t].P = P;
    }
    if (threads == 1) {
      run_job(&jobs[0]);
    } else {
      for (t = 0; t < threads; ++t) pthread_create(&tids[t], NULL, run_job, &jobs[t]);
      for (t = 0; t < threads; ++t) pthread_join(tids[t], NULL);
    }
    for (t = 0; t < threads; ++t)
      if (jobs[t].failed) status = ORACLE_ERR_NOMEM;
    free(jobs);
    free(tids);
  }
  if (status == ORACLE_OK) {
    total = HDR_BYTES + 8 * N;
    for (i = 0; i < N; ++i) total += (uint64_t)F[i] + P[i];
    *out_len = total;
    if (total > capacity || !out) {
      status = ORACLE_ERR_OUT_OF_SPACE;
    } else {
      write_header(out, n, S, C, W, MIN, policy, N, total, x + (n - n % S));
      pos = HDR_BYTES + 8 * N;
      for (i = 0; i < N; ++i) {
        put_u32(out + HDR_BYTES + 8 * i, F[i]);
        put_u32(out + HDR_BYTES + 8 * i + 4, P[i]);
        memcpy(out + pos, recs + i * slot, (size_t)F[i] + P[i]);
        pos += (uint64_t)F[i] + P[i];
      }
    }
  }
  free(recs);
  free(F);
  free(P);
  return status;
}

int oracle_compress(const uint8_t* x, uint64_t n, uint32_t S, uint32_t C, uint32_t W,
                    uint32_t MIN, uint8_t* out, uint64_t capacity, uint64_t* out_len) {
  return compress_impl(x, n, S, C, W, MIN, 0, out, capacity, out_len, 1);
}

int oracle_compress_policy(const uint8_t* x, uint64_t n, uint32_t S, uint32_t C, uint32_t W,
                           uint32_t MIN, uint32_t policy, uint8_t* out, uint64_t capacity,
                           uint64_t* out_len) {
  return compress_impl(x, n, S, C, W, MIN, policy, out, capacity, out_len, 1);
}

int oracle_compress_mt(const uint8_t* x, uint64_t n, uint32_t S, uint32_t C, uint32_t W,
                       uint32_t MIN, uint8_t* out, uint64_t capacity, uint64_t* out_len,
                       int threads) {
  return compress_impl(x, n, S, C, W, MIN, 0, out, capacity, out_len, threads);
}

int oracle_compress_policy_mt(const uint8_t* x, uint64_t n, uint32_t S, uint32_t C, uint32_t W,
                              uint32_t MIN, uint32_t policy, uint8_t* out, uint64_t capacity,
                              uint64_t* out_len, int threads) {
  return compress_impl(x, n, S, C, W, MIN, policy, out, capacity, out_len, threads);
}

/* Inverse of the parse: replay the tokens of every chunk. The paper only
 * states that decompression exists; the validation rules below are those
 * the stream layout implies (every field within its range, every pointer
 * inside its chunk's decoded prefix, every byte of the stream accounted
 * for). */
int oracle_decompress(const uint8_t* in, uint64_t in_len, uint8_t* out, uint64_t capacity,
                      uint64_t* out_len) {
  uint32_t S, C, W, MIN, r, k;
  uint64_t n, N, total, m, i, sum, pos;
  if (!out_len || (in_len && !in)) return ORACLE_ERR_INVALID_ARG;
  if (in_len < HDR_BYTES) return ORACLE_ERR_CORRUPT;
  /* header */
  if (in[0] != 'G' || in[1] != 'L' || in[2] != 'Z' || in[3] != '1') return ORACLE_ERR_CORRUPT;
  if (get_u16(in + 4) != 1) return ORACLE_ERR_CORRUPT;
  S = in[6];
  if (in[7] > 1) return ORACLE_ERR_CORRUPT; /* match policy 0 or 1 */
  C = get_u32(in + 8);
  W = get_u16(in + 12);
  MIN = in[14];
  if (in[15] != MAX_MATCH) return ORACLE_ERR_CORRUPT;
  if (!valid_params(S, C, W, MIN)) return ORACLE_ERR_CORRUPT;
  n = get_u64(in + 16);
  N = get_u64(in + 24);
  total = get_u64(in + 32);
  r = in[40];
  m = n / S;
  if (r != n % S) return ORACLE_ERR_CORRUPT;
  if (N != (m + C - 1) / C) return ORACLE_ERR_CORRUPT;
  for (k = 41; k < 48; ++k)
    if (in[k]) return ORACLE_ERR_CORRUPT;
  for (k = 48 + r; k < 64; ++k)
    if (in[k]) return ORACLE_ERR_CORRUPT;
  if (total != in_len) return ORACLE_ERR_CORRUPT;
  if (N > (in_len - HDR_BYTES) / 8) return ORACLE_ERR_CORRUPT;
  sum = HDR_BYTES + 8 * N;
  for (i = 0; i < N; ++i) {
    sum += (uint64_t)get_u32(in + HDR_BYTES + 8 * i) + get_u32(in + HDR_BYTES + 8 * i + 4);
    if (sum > in_len) return ORACLE_ERR_CORRUPT;
  }
  if (sum != in_len) return ORACLE_ERR_CORRUPT;
  *out_len = n;
  if (capacity < n || (n && !out)) return ORACLE_ERR_OUT_OF_SPACE;
  /* chunks */
  pos = HDR_BYTES + 8 * N;
  for (i = 0; i < N; ++i) {
    uint32_t F = get_u32(in + HDR_BYTES + 8 * i);
    uint32_t P = get_u32(in + HDR_BYTES + 8 * i + 4);
    const uint8_t* flags = in + pos;
    const uint8_t* pay = in + pos + F;
    uint64_t cs = i * (uint64_t)C;
    uint32_t c = (uint32_t)((m - cs) < C ? (m - cs) : C);
    uint8_t* dst = out + cs * S;
    uint32_t q = 0, used = 0;
    uint64_t t = 0;
    while (q < c) {
      if (t >= 8 * (uint64_t)F) return ORACLE_ERR_CORRUPT;
      if ((flags[t >> 3] >> (t & 7)) & 1u) {
        uint32_t L, O;
        if (used + 2 > P) return ORACLE_ERR_CORRUPT;
        L = pay[used];
        O = pay[used + 1] ? pay[used + 1] : 256u;
        used += 2;
        if (L < MIN || L > MAX_MATCH || O > W || O > q || L > O || L > c - q)
          return ORACLE_ERR_CORRUPT;
        for (k = 0; k < L; ++k) memcpy(dst + (size_t)(q + k) * S, dst + (size_t)(q + k - O) * S, S);
        q += L;
      } else {
        if (used + S > P) return ORACLE_ERR_CORRUPT;
        memcpy(dst + (size_t)q * S, pay + used, S);
        used += S;
        q += 1;
      }
      ++t;
    }
    if ((t + 7) / 8 != F || used != P) return ORACLE_ERR_CORRUPT;
    for (; t < 8 * (uint64_t)F; ++t)
      if ((flags[t >> 3] >> (t & 7)) & 1u) return ORACLE_ERR_CORRUPT;
    pos += (uint64_t)F + P;
  }
  for (k = 0; k < r; ++k) out[m * S + k] = in[48 + k];
  return ORACLE_OK;
}
