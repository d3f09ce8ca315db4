// Device code of the decoder, shared by the single-buffer and batch kernels.
//
// The paper states that decompression exists and is easy to parallelise
// (section 4.4) without describing it; this decoder follows from the stream
// layout:
//   header   one thread checks every header field;
//   table    the table's F_i + P_i are prefix-summed once per group of 64
//            chunks (one u64 per group; the sum must end exactly at the
//            stream's end); a chunk's record offset is its group's offset
//            plus a 64-lane prefix sum over the group's table entries;
//   chunk    (chunks of at most 4096 symbols and 16 KiB, the usual case) one
//            workgroup of 256 threads per chunk: the record is staged into
//            LDS with 16-byte loads; block-wide scans over the flag bits and
//            the token lengths give every token's payload offset and output
//            position at once, every rule is checked and the literals are
//            written into an LDS copy of the chunk; wave 0 then copies the
//            pointers in token order (a run of pointers whose sources are
//            already final is copied together), and the chunk is written to
//            HBM with 16-byte stores;
//   chunk    (any other chunk) one wavefront walks the tokens 64 at a time: lane l
//            takes token t + l, its flag bit gives its kind, mbcnt over the
//            literal / pointer ballots gives its payload offset, a wave scan
//            of the token lengths gives its output position. Literals are
//            written into an LDS ring of recent symbols; pointers are then
//            resolved in token order, each copied by all 64 lanes (a pointer
//            never overlaps itself because its length never exceeds its
//            offset). Finished symbols stream out to HBM. The ring keeps the
//            last 256 symbols (the largest offset), so LDS use does not
//            depend on the chunk size.
// Every rule the encoder guarantees is checked; a broken one makes the
// stream GPULZ_ERR_CORRUPT.
#pragma once

#include "gpulz_internal.h"
#include "wave.h"

namespace gpulz {
namespace dec {

constexpr uint32_t kGroup = 64;  // chunks per record-offset group

__device__ inline uint64_t rd_u64(const uint8_t* p) {
  uint64_t v = 0;
  for (int k = 7; k >= 0; --k) v = (v << 8) | p[k];
  return v;
}
__device__ inline uint32_t rd_u32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

// Checks the header of a stream of in_bytes bytes; fills p (p.status = kOk or
// kCorrupt). One thread.
__device__ inline void parse_header(const uint8_t* h, uint64_t in_bytes, DecodeParams& p) {
  p = DecodeParams{};
  bool ok = in_bytes >= kHeaderBytes;
  if (ok) {
    ok = h[0] == 'G' && h[1] == 'L' && h[2] == 'Z' && h[3] == '1' && h[4] == 1 && h[5] == 0 &&
         h[7] <= 1 && h[15] == kMaxMatch;  // match policy 0 or 1
    p.S = h[6];
    p.C = rd_u32(h + 8);
    p.W = (uint32_t)h[12] | ((uint32_t)h[13] << 8);
    p.MIN = h[14];
    p.n = rd_u64(h + 16);
    p.N = rd_u64(h + 24);
    const uint64_t total = rd_u64(h + 32);
    p.r = h[40];
    ok = ok && (p.S == 1 || p.S == 2 || p.S == 4 || p.S == 8) && p.C >= 1 && p.C <= (1u << 24) &&
         p.W >= 1 && p.W <= kMaxWindow && p.MIN >= 1;
    if (ok) {
      p.m = p.n / p.S;
      ok = p.r == p.n % p.S && p.N == (p.m + p.C - 1) / p.C && total == in_bytes &&
           p.N <= decode_max_chunks(in_bytes);
      for (uint32_t k = 41; k < 48; ++k) ok = ok && h[k] == 0;
      for (uint32_t k = 48 + p.r; k < 64; ++k) ok = ok && h[k] == 0;
    }
  }
  p.status = ok ? kOk : kCorrupt;
}

// Workgroup-wide: group_off[g] = absolute offset of the first record of chunk
// group g (g = 0 .. ceil(N / 64)); returns the end of the last record. Any
// blockDim that is a multiple of 64. `scratch` holds blockDim/64 + 1 u64.
__device__ inline uint64_t scan_table_groups(const uint8_t* in, uint64_t N, uint64_t* group_off,
                                             uint64_t* scratch) {
  // each thread sums 16 consecutive entries (eight 16-byte loads; the table
  // starts 16-byte aligned), so 4 threads cover a group of 64; one block-wide
  // scan per tile of 16 blockDim entries gives every group's offset
  constexpr uint32_t kPer = 16;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
  const uint32_t nw = blockDim.x >> 6;
  const uint64_t ngroups = (N + kGroup - 1) / kGroup;
  const uint8_t* table = in + kHeaderBytes;
  const uint4* t4 = reinterpret_cast<const uint4*>(table);
  const uint64_t tile = (uint64_t)blockDim.x * kPer;
  uint64_t carry = kHeaderBytes + 8 * N;
  for (uint64_t base = 0; base < N; base += tile) {
    const uint64_t i0 = base + (uint64_t)tid * kPer;
    uint64_t v = 0;
    if (i0 + kPer <= N) {
#pragma unroll
      for (uint32_t q = 0; q < kPer / 2; ++q) {
        const uint4 e = t4[i0 / 2 + q];
        v += (uint64_t)e.x + e.y + (uint64_t)e.z + e.w;
      }
    } else {
      for (uint32_t k = 0; k < kPer && i0 + k < N; ++k) {
        const uint32_t* e = reinterpret_cast<const uint32_t*>(table + 8 * (i0 + k));
        v += (uint64_t)e[0] + e[1];
      }
    }
    const uint64_t incl = wave_incl_scan_u64(v);
    if (lane == 63) scratch[wid] = incl;
    __syncthreads();
    uint64_t before = 0, total = 0;
    for (uint32_t w = 0; w < nw; ++w) {
      const uint64_t x = scratch[w];
      before += w < wid ? x : 0ull;
      total += x;
    }
    // i0 is a multiple of 64 exactly on every fourth thread
    if ((tid & 3u) == 0 && i0 < N) group_off[i0 / kGroup] = carry + before + incl - v;
    carry += total;
    __syncthreads();
  }
  if (tid == 0) group_off[ngroups] = carry;
  return carry;
}

// Wave-wide: absolute record offset of chunk i.
__device__ inline uint64_t record_offset(const uint8_t* in, const uint64_t* group_off, uint64_t i) {
  const uint32_t lane = lane_id();
  const uint64_t g = i / kGroup;
  const uint32_t k = (uint32_t)(i % kGroup);
  uint64_t v = 0;
  if (lane < k) {
    const uint32_t* e = reinterpret_cast<const uint32_t*>(in + kHeaderBytes + 8 * (g * kGroup + lane));
    v = (uint64_t)e[0] + e[1];
  }
  const uint64_t s = wave_incl_scan_u64(v);
  return group_off[g] + __shfl(s, 63, 64);
}

// Decode one chunk (wave-wide); returns false if the chunk breaks a rule.
template <int S>
__device__ bool decode_chunk(const uint8_t* flags, uint32_t F, uint32_t P, uint32_t c, uint32_t W,
                             uint32_t MIN, typename SymType<S>::T* out, uint8_t* ring_raw) {
  using T = typename SymType<S>::T;
  constexpr uint32_t R = kDecodeRingBytes / S;    // ring capacity in symbols
  constexpr uint32_t SPAN = R - 2 * kMaxWindow;   // new symbols per step
  T* ring = reinterpret_cast<T*>(ring_raw);
  const uint8_t* pay = flags + F;
  const uint32_t lane = lane_id();
  uint32_t q = 0, u = 0;
  uint64_t t = 0;
  while (q < c) {
    const uint64_t tok = t + lane;
    const bool has = tok < 8ull * F;
    const bool ptr = has && ((flags[tok >> 3] >> (tok & 7)) & 1u);
    const uint64_t pm = ballot(ptr);
    const uint64_t lm = ballot(has && !ptr);
    const uint32_t off = u + S * mbcnt(lm) + 2u * mbcnt(pm);
    bool ok = has && off + (ptr ? 2u : (uint32_t)S) <= P;
    uint32_t L = 1, O = 1;
    if (ptr && ok) {
      L = pay[off];
      O = pay[off + 1] ? pay[off + 1] : 256u;
    }
    const uint32_t len = has ? L : 0;
    const uint32_t pos = q + wave_incl_scan(len) - len;
    const uint32_t lim = min(c, q + SPAN);
    const bool take = has && pos < lim;
    const uint64_t tm = ballot(take);
    if (tm == 0) return false;  // flags exhausted before the chunk is complete
    if (ptr) ok = ok && L >= MIN && O <= W && O <= pos && L <= O && pos + L <= c;
    if (ballot(take && !ok)) return false;
    if (take && !ptr) {
      uint64_t v = 0;
#pragma unroll
      for (int b = 0; b < S; ++b) v |= (uint64_t)pay[off + b] << (8 * b);
      ring[pos & (R - 1)] = (T)v;
    }
    wave_sync();
    uint64_t mt = pm & tm;
    while (mt) {
      const uint32_t j = (uint32_t)__ffsll((unsigned long long)mt) - 1;
      mt &= mt - 1;
      const uint32_t pj = readlane(pos, j), Lj = readlane(L, j), Oj = readlane(O, j);
      for (uint32_t k = lane; k < Lj; k += 64) ring[(pj + k) & (R - 1)] = ring[(pj - Oj + k) & (R - 1)];
      wave_sync();
    }
    const uint32_t last = 63u - (uint32_t)__clzll(tm);
    const uint32_t nq = readlane(pos + len, last);
    for (uint32_t k = q + lane; k < nq; k += 64) out[k] = ring[k & (R - 1)];
    wave_sync();
    t += popc64(tm);
    u += S * popc64(lm & tm) + 2u * popc64(pm & tm);
    q = nq;
  }
  if ((t + 7) / 8 != F || u != P) return false;
  if (t < 8ull * F && (flags[F - 1] >> (uint32_t)(t - 8ull * (F - 1))) != 0) return false;
  return true;
}

// ---- workgroup decoder ------------------------------------------------------

constexpr uint32_t kDecThreads = 256;
constexpr uint32_t kFastSyms = 16 * kDecThreads;          // tokens per chunk (16 per thread)
constexpr uint32_t kFastOut = kDecodeRingBytes;           // chunk bytes kept in LDS
constexpr uint32_t kFastRec = kFastSyms / 8 + kFastOut + 32;

struct BlockLds {
  uint8_t rec[kFastRec];              // staged record (16-byte aligned copy)
  uint8_t out[kFastOut];              // the chunk; the ring of the wave decoder
  uint64_t ptrbits[kFastSyms / 64];   // pointer flags of the decoded tokens
  uint32_t scratch[16];
};

// Block-wide exclusive scan (sum) of one u32 per thread; `total` gets the sum.
__device__ inline uint32_t block_excl_scan_u32(uint32_t v, uint32_t* scratch, uint32_t& total) {
  const uint32_t lane = lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint32_t incl = wave_incl_scan(v);
  if (lane == 63) scratch[wid] = incl;
  __syncthreads();
  uint32_t before = 0;
  total = 0;
  for (uint32_t w = 0; w < nw; ++w) {
    const uint32_t x = scratch[w];
    before += w < wid ? x : 0u;
    total += x;
  }
  __syncthreads();
  return before + incl - v;
}

// Block-wide maximum and sum of one u32 each per thread, and any of a flag.
__device__ inline void block_reduce(uint32_t& mx, uint32_t& sum, bool& any, uint32_t* scratch) {
  const uint32_t lane = lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint32_t wm = wave_max_u32(mx);
  const uint32_t ws = readlane(wave_incl_scan(sum), 63);
  const bool wa = ballot(any) != 0;
  if (lane == 0) {
    scratch[wid] = wm;
    scratch[4 + wid] = ws;
    scratch[8 + wid] = wa;
  }
  __syncthreads();
  mx = 0;
  sum = 0;
  any = false;
  for (uint32_t w = 0; w < nw; ++w) {
    mx = max(mx, scratch[w]);
    sum += scratch[4 + w];
    any = any || scratch[8 + w];
  }
  __syncthreads();
}

// Whether the workgroup decoder takes a chunk of c symbols with F flag and
// P payload bytes.
__device__ inline bool fits_block(uint32_t c, uint32_t S, uint32_t F, uint32_t P) {
  return c <= kFastSyms && c * S <= kFastOut && F <= kFastSyms / 8 && F + P + 16 <= kFastRec;
}

// One symbol of S bytes at any byte address in LDS (aligned dword reads and a
// funnel shift; up to 11 bytes past the symbol are read).
template <int S>
__device__ __forceinline__ typename SymType<S>::T load_sym(const uint8_t* p) {
  const uint32_t sh = (uint32_t)(uintptr_t)p & 3u;
  const uint32_t* w = reinterpret_cast<const uint32_t*>(__builtin_assume_aligned(p - sh, 4));
  const uint32_t lo = __builtin_amdgcn_alignbyte(w[1], w[0], sh);
  if constexpr (S == 8) {
    return (uint64_t)lo | ((uint64_t)__builtin_amdgcn_alignbyte(w[2], w[1], sh) << 32);
  } else {
    return (typename SymType<S>::T)lo;
  }
}

// Sum over the waves before this one of a wave-uniform value, and the total.
__device__ inline uint32_t waves_excl(uint32_t v, uint32_t* scratch, uint32_t& total) {
  const uint32_t wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane_id() == 0) scratch[wid] = v;
  __syncthreads();
  uint32_t before = 0;
  total = 0;
  for (uint32_t w = 0; w < nw; ++w) {
    const uint32_t x = scratch[w];
    before += w < wid ? x : 0u;
    total += x;
  }
  __syncthreads();
  return before;
}

// Decode one chunk with the whole workgroup (kDecThreads threads); returns
// false (uniformly) if the chunk breaks a rule. rec: its record in HBM;
// in_end: end of the stream (no byte at or past it is read); dst: its first
// output byte.
//
// Token i (of the 8 F the flags describe) is handled by wave i / (64 R) in
// round (i / 64) % R on lane i % 64, R = ceil(8 F / 256) rounds per wave, so
// neighbouring lanes touch neighbouring LDS bytes and small chunks still
// spread over all four waves. Payload offsets come from the literal / pointer
// counts (mbcnt within a round, running totals across rounds, one exchange
// across waves); output positions likewise from the token lengths.
template <int S>
__device__ bool decode_chunk_block(const uint8_t* rec, const uint8_t* in_end, uint32_t F,
                                   uint32_t P, uint32_t c, uint32_t W, uint32_t MIN, uint8_t* dst,
                                   BlockLds& sm) {
  using T = typename SymType<S>::T;
  const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  T* out = reinterpret_cast<T*>(sm.out);

  // stage the record; the copy keeps the record's alignment within 16 bytes
  const uint32_t a = (uint32_t)((uintptr_t)rec & 15u);
  const uint8_t* g0 = rec - a;
  const uint32_t nwords = (a + F + P + 15) / 16;
  for (uint32_t k = tid; k < nwords; k += kDecThreads) {
    const uint8_t* gp = g0 + 16 * k;
    if (gp + 16 <= in_end) {
      *reinterpret_cast<uint4*>(sm.rec + 16 * k) = *reinterpret_cast<const uint4*>(gp);
    } else {
      for (uint32_t b = 0; b < 16; ++b) sm.rec[16 * k + b] = gp + b < in_end ? gp[b] : 0;
    }
  }
  __syncthreads();
  const uint8_t* fl = sm.rec + a;
  const uint8_t* pay = fl + F;
  const uint32_t nt = 8 * F;
  // R rounds of 64 tokens per wave (R <= 16), so that small chunks spread over
  // all four waves too
  const uint32_t R = nt <= 256 ? 1u : (nt + 255) / 256;
  const uint32_t tpw = 64 * R;
  const uint32_t t0 = tpw * wave + lane;

  // token i's kind: pointer flag bit (only for i < 8 F)
  auto is_ptr = [&](uint32_t i) { return i < nt && ((fl[i >> 3] >> (i & 7)) & 1u); };
  // the wave's literal / pointer counts: lane l counts the wave's tokens
  // R l .. R l + R - 1 (R flag bits at any bit offset, at most 3 bytes)
  uint32_t np, nh;
  {
    const uint32_t i = tpw * wave + R * lane;  // first of this lane's R tokens
    const uint32_t b0 = i >> 3;
    uint32_t fb = 0;
    if (b0 < F) fb = fl[b0];
    if (b0 + 1 < F) fb |= (uint32_t)fl[b0 + 1] << 8;
    if (b0 + 2 < F) fb |= (uint32_t)fl[b0 + 2] << 16;
    fb >>= (i & 7u);
    const uint32_t cnt = i >= nt ? 0u : min(R, nt - i);
    const uint32_t hmask = (1u << cnt) - 1u;
    np = readlane(wave_incl_scan((uint32_t)__popc(fb & hmask)), 63);
    nh = readlane(wave_incl_scan((uint32_t)__popc(hmask)), 63);
  }
  uint32_t tot;
  const uint32_t x1 = waves_excl((nh - np) | (np << 16), sm.scratch, tot);
  if ((tot >> 16) == 0) {
    // no pointer: the record is valid exactly when its tokens are the chunk's
    // c literals (F = ceil(c / 8) flag bytes, P = c S payload bytes), and then
    // the payload is the chunk. It is copied out of LDS with one funnel shift
    // (its start's offset within a dword is the same for every word).
    if (F != (c + 7) / 8 || P != c * S) return false;
    const uint32_t nb = c * S, base = a + F, sh = base & 3u;
    const uint32_t* w = reinterpret_cast<const uint32_t*>(sm.rec + (base - sh));
    if (((uintptr_t)dst & 15u) == 0) {
      for (uint32_t k = tid; k < nb / 16; k += kDecThreads) {
        const uint32_t* q = w + 4 * k;
        const uint32_t q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
        const uint32_t q4 = sh ? q[4] : 0u;  // read only when it holds payload bytes
        *reinterpret_cast<uint4*>(dst + 16 * k) =
            make_uint4(__builtin_amdgcn_alignbyte(q1, q0, sh), __builtin_amdgcn_alignbyte(q2, q1, sh),
                       __builtin_amdgcn_alignbyte(q3, q2, sh), __builtin_amdgcn_alignbyte(q4, q3, sh));
      }
      for (uint32_t b = (nb & ~15u) + tid; b < nb; b += kDecThreads) dst[b] = sm.rec[base + b];
    } else {
      for (uint32_t b = tid; b < nb; b += kDecThreads) dst[b] = sm.rec[base + b];
    }
    return true;
  }
  const uint32_t lit0 = x1 & 0xFFFFu, ptr0 = x1 >> 16;
  // Pointer symbols are resolved in parallel (pointer jumping, below) when the
  // chunk has many pointers and its decoded bytes leave room in `out` for a
  // 16-bit source index per symbol; otherwise wave 0 copies them in order.
  const uint32_t src_at = (c * S + 15) & ~15u;
  const bool jump = (tot >> 16) >= 64 && src_at + 2 * c <= kFastOut;
  uint16_t* src = reinterpret_cast<uint16_t*>(sm.out + src_at);

  // this wave's total length: one per token, plus L - 1 per pointer whose
  // payload is in range
  uint32_t wlen = nh;
  {
    uint32_t lit = lit0, ptr = ptr0;
    for (uint32_t j = 0; j < R; ++j) {
      const uint32_t i = t0 + 64 * j;
      const bool isp = is_ptr(i);
      const uint64_t pmj = ballot(isp), lm = ballot(i < nt && !isp);
      if (pmj) {
        const uint32_t off = S * (lit + mbcnt(lm)) + 2 * (ptr + mbcnt(pmj));
        const uint32_t e = isp && off + 2 <= P ? pay[off] - 1u : 0u;
        wlen += readlane(wave_incl_scan(e), 63);
      }
      lit += popc64(lm);
      ptr += popc64(pmj);
    }
  }
  uint32_t pos_end;
  const uint32_t wpos0 = waves_excl(wlen, sm.scratch, pos_end);

  // positions, checks and literals; taken tokens (position < c) are a prefix
  bool bad = false;
  uint32_t taken = 0, uend = 0;
  {
    uint32_t lit = lit0, ptr = ptr0, run = wpos0;
    for (uint32_t j = 0; j < R; ++j) {
      const uint32_t i = t0 + 64 * j;
      const bool has = i < nt;
      const bool isp = is_ptr(i);
      const uint64_t pmj = ballot(isp), lm = ballot(has && !isp);
      const uint32_t off = S * (lit + mbcnt(lm)) + 2 * (ptr + mbcnt(pmj));
      const uint32_t sz = isp ? 2u : (uint32_t)S;
      const bool okp = off + sz <= P;
      uint32_t L = 1, O = 1, pos;
      if (pmj) {
        if (isp && okp) {
          L = pay[off];
          O = pay[off + 1] ? pay[off + 1] : 256u;
        }
        const uint32_t len = has ? L : 0u;
        const uint32_t inc = wave_incl_scan(len);
        pos = run + inc - len;
        run += readlane(inc, 63);
      } else {
        // no pointer in this round: consecutive positions
        pos = run + lane;
        run += popc64(lm);
      }
      const bool tk = has && pos < c;
      if (tk) {
        ++taken;
        uend = max(uend, off + sz);
        if (!okp) {
          bad = true;
        } else if (isp) {
          const bool ok = L >= MIN && O <= W && O <= pos && L <= O && pos + L <= c;
          bad = bad || !ok;
          if (ok && jump)
            for (uint32_t k = 0; k < L; ++k) src[pos + k] = (uint16_t)(pos + k - O);
        } else {
          out[pos] = load_sym<S>(pay + off);
          if (jump) src[pos] = (uint16_t)pos;
        }
      }
      const uint64_t tb = ballot(tk && isp);
      if (lane == 0 && !jump) sm.ptrbits[R * wave + j] = tb;
      lit += popc64(lm);
      ptr += popc64(pmj);
    }
  }
  uint32_t Tn = taken;
  block_reduce(uend, Tn, bad, sm.scratch);
  // every rule of the wave decoder: all checks above hold, the flags cover
  // the chunk, the tokens use exactly F flag bytes and P payload bytes, and
  // the unused flag bits are zero
  if (bad || pos_end < c || (Tn + 7) / 8 != F || uend != P) return false;
  if (Tn < nt && (fl[F - 1] >> (Tn - 8 * (F - 1))) != 0) return false;

  // pointers. Symbol p of a pointer with offset O takes the value of symbol
  // p - O (always earlier, since O <= its position), which is a literal or
  // again a pointer symbol. Replacing every source by its source's source
  // (pointer jumping) reaches a literal for every symbol within
  // ceil(log2 c) <= 12 rounds: a chain of any length halves each round. The
  // update is in place: a thread that reads an entry another thread just
  // replaced still gets an earlier symbol of the same chain. Then every
  // pointer symbol copies its literal.
  if (jump) {
    for (uint32_t round = 0; round < 13; ++round) {
      bool changed = false;
      for (uint32_t p = tid; p < c; p += kDecThreads) {
        const uint32_t s0 = src[p];
        const uint32_t s1 = src[s0];
        if (s1 != s0) {
          src[p] = (uint16_t)s1;
          changed = true;
        }
      }
      if (!__syncthreads_or(changed)) break;
    }
    for (uint32_t p = tid; p < c; p += kDecThreads) {
      const uint32_t s0 = src[p];
      if (s0 != p) out[p] = out[s0];
    }
    __syncthreads();
  }

  // pointers, 64 at a time in token order, by wave 0. A pointer is copied
  // once the last uncopied pointer before it ends at or before its source
  // starts (destinations are ordered, so no uncopied output overlaps its
  // source); the first uncopied pointer always qualifies.
  if (!jump && wave == 0) {
    const uint32_t nwd = (Tn + 63) / 64;
    const uint64_t wd = lane < nwd ? sm.ptrbits[lane] : 0ull;
    const uint32_t cnt = popc64(wd);
    const uint32_t wb_incl = wave_incl_scan(cnt);
    const uint32_t wb = wb_incl - cnt;  // pointers before flag word `lane`
    const uint32_t NP = readlane(wb_incl, 63);
    uint32_t extra = 0;
    for (uint32_t g = 0; g < NP; g += 64) {
      const uint32_t o = g + lane;  // this lane's pointer ordinal
      const bool valid = o < NP;
      // its flag word: the last word whose first ordinal is <= o
      uint32_t lo = 0, hi = 63;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const uint32_t mid = (lo + hi + 1) / 2;
        if ((uint32_t)__shfl((int)wb, (int)mid, 64) <= o) lo = mid;
        else hi = mid - 1;
      }
      uint64_t m = __shfl((unsigned long long)wd, (int)lo, 64);
      uint32_t r = o - (uint32_t)__shfl((int)wb, (int)lo, 64);
      uint32_t bit = 0;
#pragma unroll
      for (uint32_t width = 32; width >= 1; width >>= 1) {
        const uint32_t lowc = popc64(m & ((1ull << width) - 1));
        if (r >= lowc) {
          r -= lowc;
          m >>= width;
          bit += width;
        }
      }
      const uint32_t t = 64 * lo + bit;
      uint32_t L = 0, O = 0;
      if (valid) {
        const uint32_t off = S * (t - o) + 2 * o;
        L = pay[off];
        O = pay[off + 1] ? pay[off + 1] : 256u;
      }
      const uint32_t e = valid ? L - 1 : 0u;
      const uint32_t inc = wave_incl_scan(e);
      const uint32_t pos = t + extra + inc - e;
      extra += readlane(inc, 63);
      const uint32_t end = pos + L, src = pos - O;
      uint64_t un = ballot(valid);
      while (un) {
        const uint64_t below = un & ((1ull << lane) - 1);
        const uint32_t lk = below ? 63u - (uint32_t)__clzll(below) : 0u;
        const uint32_t endk = (uint32_t)__shfl((int)end, (int)lk, 64);
        const bool ready = ((un >> lane) & 1u) && (below == 0 || endk <= src);
        const uint64_t rm = ballot(ready);
        if (popc64(rm) == 1) {
          const uint32_t j0 = (uint32_t)__ffsll((unsigned long long)rm) - 1;
          const uint32_t P0 = readlane(pos, j0), Lj = readlane(L, j0), Oj = readlane(O, j0);
          for (uint32_t k = lane; k < Lj; k += 64) out[P0 + k] = out[P0 - Oj + k];
        } else if (ready) {
          for (uint32_t k = 0; k < L; ++k) out[pos + k] = out[src + k];
        }
        wave_sync();
        un &= ~rm;
      }
    }
  }
  __syncthreads();

  // write the chunk out
  const uint32_t nb = c * S;
  if (((uintptr_t)dst & 15u) == 0) {
    for (uint32_t k = tid; k < nb / 16; k += kDecThreads)
      *reinterpret_cast<uint4*>(dst + 16 * k) = *reinterpret_cast<const uint4*>(sm.out + 16 * k);
    for (uint32_t b = (nb & ~15u) + tid; b < nb; b += kDecThreads) dst[b] = sm.out[b];
  } else {
    for (uint32_t b = tid; b < nb; b += kDecThreads) dst[b] = sm.out[b];
  }
  return true;
}

// 16 bytes starting sh bytes (0..3) past the dword at q (global memory),
// funnel-shifted from dword reads that never reach in_end.
__device__ __forceinline__ uint4 load_group(const uint32_t* q, uint32_t sh, const uint8_t* in_end) {
  uint32_t d[5];
  __builtin_memcpy(d, __builtin_assume_aligned(q, 4), 16);
  d[4] = 0;
  if (sh) {
    // the fifth dword holds the group's last sh bytes; at the end of the
    // stream it is read byte by byte
    const uint8_t* q4 = reinterpret_cast<const uint8_t*>(q + 4);
    if (q4 + 4 <= in_end) {
      d[4] = q[4];
    } else {
      for (uint32_t b = 0; b < sh; ++b) d[4] |= (uint32_t)q4[b] << (8 * b);
    }
  }
  return make_uint4(__builtin_amdgcn_alignbyte(d[1], d[0], sh), __builtin_amdgcn_alignbyte(d[2], d[1], sh),
                    __builtin_amdgcn_alignbyte(d[3], d[2], sh), __builtin_amdgcn_alignbyte(d[4], d[3], sh));
}

// A record sized for c literals (F = ceil(c / 8) flag bytes, P = c S payload
// bytes) whose flag bytes are all zero is valid and its payload is the chunk:
// copy it straight from the stream to the output (dword-aligned 16-byte loads,
// funnel-shifted by the payload's offset within a dword). Returns false
// (uniformly), having written nothing, if any flag bit is set. Every dword
// read holds a byte of the record; none reaches in_end.
__device__ inline bool copy_literal_chunk(const uint8_t* rec, const uint8_t* in_end, uint32_t F,
                                          uint32_t nb, uint8_t* dst) {
  const uint32_t tid = threadIdx.x;
  const uint32_t r0 = (uint32_t)((uintptr_t)rec & 3u);
  const uint32_t* fw = reinterpret_cast<const uint32_t*>(rec - r0);
  bool set = false;
  for (uint32_t k = tid; 4 * k < r0 + F; k += kDecThreads) {
    uint32_t v = 0;
    const uint8_t* wk = reinterpret_cast<const uint8_t*>(fw + k);
    if (wk + 4 <= in_end) {
      v = fw[k];
    } else {
      for (uint32_t b = 0; wk + b < in_end; ++b) v |= (uint32_t)wk[b] << (8 * b);
    }
    if (4 * k < r0) v &= ~0u << (8 * r0);                // bytes before the record
    const uint32_t in_f = r0 + F - 4 * k;                 // flag bytes in this dword, from its start
    if (in_f < 4) v &= (1u << (8 * in_f)) - 1u;           // bytes after the flags
    set = set || v != 0;
  }
  if (__syncthreads_or(set)) return false;
  const uint8_t* src = rec + F;
  const uint32_t sh = (uint32_t)((uintptr_t)src & 3u);
  const uint32_t* sw = reinterpret_cast<const uint32_t*>(src - sh);
  const uint32_t ng = ((uintptr_t)dst & 15u) == 0 ? nb / 16 : 0u;  // 16-byte groups
  // four groups per thread in flight: all loads, then all stores
  for (uint32_t k0 = tid; k0 < ng; k0 += 4 * kDecThreads) {
    uint4 g[4];
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
      const uint32_t k = k0 + j * kDecThreads;
      if (k < ng) g[j] = load_group(sw + 4 * k, sh, in_end);
    }
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
      const uint32_t k = k0 + j * kDecThreads;
      if (k < ng) *reinterpret_cast<uint4*>(dst + 16 * k) = g[j];
    }
  }
  for (uint32_t b = 16 * ng + tid; b < nb; b += kDecThreads) dst[b] = src[b];
  return true;
}

// Decode chunk i of a validated stream of in_bytes bytes with the whole
// workgroup; false (uniformly) if it is corrupt. Chunks the workgroup
// decoder does not take go to the wave decoder on wave 0.
__device__ inline bool decode_stream_chunk_block(const uint8_t* in, uint64_t in_bytes,
                                                 const DecodeParams& p, const uint64_t* group_off,
                                                 uint64_t i, uint8_t* out, BlockLds& sm) {
  const uint8_t* e = in + kHeaderBytes + 8 * i;
  const uint32_t F = *reinterpret_cast<const uint32_t*>(e);
  const uint32_t P = *reinterpret_cast<const uint32_t*>(e + 4);
  const uint8_t* rec = in + record_offset(in, group_off, i);
  const uint64_t cs = i * p.C;
  const uint32_t c = (uint32_t)min<uint64_t>(p.C, p.m - cs);
  uint8_t* dst = out + cs * p.S;
  if (F == (c + 7) / 8 && P == c * p.S && copy_literal_chunk(rec, in + in_bytes, F, P, dst)) return true;
  if (fits_block(c, p.S, F, P)) {
    switch (p.S) {
      case 1: return decode_chunk_block<1>(rec, in + in_bytes, F, P, c, p.W, p.MIN, dst, sm);
      case 2: return decode_chunk_block<2>(rec, in + in_bytes, F, P, c, p.W, p.MIN, dst, sm);
      case 4: return decode_chunk_block<4>(rec, in + in_bytes, F, P, c, p.W, p.MIN, dst, sm);
      default: return decode_chunk_block<8>(rec, in + in_bytes, F, P, c, p.W, p.MIN, dst, sm);
    }
  }
  const uint32_t wave = threadIdx.x >> 6;
  if (wave == 0) {
    bool ok;
    switch (p.S) {
      case 1: ok = decode_chunk<1>(rec, F, P, c, p.W, p.MIN, reinterpret_cast<uint8_t*>(dst), sm.out); break;
      case 2: ok = decode_chunk<2>(rec, F, P, c, p.W, p.MIN, reinterpret_cast<uint16_t*>(dst), sm.out); break;
      case 4: ok = decode_chunk<4>(rec, F, P, c, p.W, p.MIN, reinterpret_cast<uint32_t*>(dst), sm.out); break;
      default: ok = decode_chunk<8>(rec, F, P, c, p.W, p.MIN, reinterpret_cast<uint64_t*>(dst), sm.out); break;
    }
    if (lane_id() == 0) sm.scratch[15] = ok;
  }
  __syncthreads();
  const bool ok = sm.scratch[15] != 0;
  __syncthreads();
  return ok;
}

}  // namespace dec
}  // namespace gpulz
