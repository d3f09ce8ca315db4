// Device code of the chunk encoder, shared by the single-buffer kernel and
// the persistent batch kernel.
#pragma once

#include <type_traits>

#include "gpulz_internal.h"
#include "dense_asm.h"
#include "stream_device.h"
#include "wave.h"

namespace gpulz {
namespace enc {

// Chunk encoder: one workgroup of wavefronts per chunk.
//
// Steps, following gpuLZ (Zhang et al., ICS'23):
//   stage   the chunk is copied HBM -> LDS with 16-byte loads; window and
//           look-ahead live in the same LDS array (section 3.3.2, unified
//           shared buffer).
//   hits    (all waves) for every position p, whether any offset
//           d <= min(W, p) has sym[p - d] == sym[p]; a position without such
//           an offset can only be a literal. Each lane owns a 16-byte vector
//           of V = 16 / S consecutive positions; one aligned 16-byte window
//           read per V offsets feeds V x V symbol compares (v_cmp, result in
//           a 64-bit lane mask), so LDS traffic is one byte per compare.
//   parse   (wave 0) greedy LZSS (section 2.2 basic steps; section 3.3.2
//           encoding step): runs of positions without a hit become literals
//           in bulk; at a hit, the exact longest match is found with the 64
//           lanes holding window offsets (up to 4 columns of 64): the 64-bit
//           mask of offsets still matching is ANDed with the comparison at
//           each next look-ahead symbol, offsets d <= L drop out (a match
//           never exceeds its offset, section 3.3.2). Rows are computed four
//           at a time so one LDS round trip serves four extension steps. The
//           length is the number of steps before the mask empties (at most
//           255, and never past the chunk end); the offset is the highest
//           surviving bit, so ties go to the largest offset. Positions
//           covered by a pointer are never searched.
//   encode  (wave 0) every 64 tokens, one token per lane: the flag bits are
//           the ballot of the pointer lanes and each lane's payload offset is
//           S * (literal lanes below it) + 2 * (pointer lanes below it), via
//           mbcnt (the local prefix sum of section 3.2.2, over token sizes).
// The record goes to a per-chunk scratch slot; the chunk's flag and payload
// sizes go to `sizes` for the global prefix sum.


constexpr int kEncodeWaves = 4;

// Match search at a hit: 4-symbol equality steps over offset masks
// (match_key, for 1- and 2-byte symbols, whose 4 symbols fit one 32- or
// 64-bit compare) or per-row offset masks (4- and 8-byte symbols; 4% faster
// than per-lane runs on the literal-heavy 4-byte field).
template <int S> constexpr bool kRunSearch = S <= 2;

// One chunk's work.
struct ChunkJob {
  const uint8_t* src;   // first input byte of the chunk
  uint64_t src_avail;   // input bytes readable from src (bounds the 16-byte loads)
  uint32_t c;           // symbols in this chunk
  uint32_t C;           // nominal chunk symbols (LDS layout)
  uint32_t W, MIN;
  uint8_t* slot;        // scratch record: [flag area | payload]
  uint64_t flag_area;
  uint32_t* sizes;      // receives {F, P} (two-pass path)
  // single-pass path: the stream this chunk belongs to
  uint64_t i, N;        // chunk index, chunks of the stream
  uint64_t* desc;       // the stream's look-back descriptors
  uint8_t* out;         // the stream
  uint64_t capacity;
  const uint8_t* in;    // the stream's input (the header's tail bytes)
  uint64_t nbytes;
  uint32_t S, policy;
  uint64_t* out_bytes;  // written by the stream's last chunk
  int32_t* status;
};


template <int S> struct Geo {
  static constexpr int V = 16 / S;                  // symbols per 16-byte vector
  // 16-byte vectors per lane in the hit phase: two for 4- and 8-byte symbols
  // (one window read then serves 2 V positions), one for narrower ones,
  // whose single vector already holds 8 or 16
  static constexpr int R = S >= 4 ? 2 : 1;
  static constexpr uint32_t kBlock = 64u * V * R;   // positions per wave block
};

// Window columns of the streaming search (1- and 2-byte symbols): 4 / S
// offsets per lane, so one column of 64 lanes covers 256 / S offsets.
__host__ __device__ constexpr uint32_t stream_cols(uint32_t S, uint32_t wc) {
  return S == 1 ? 1u : (S == 2 ? (wc <= 2 ? 1u : 2u) : 0u);
}
// Bytes before the staged chunk: window reads reach 64 WC S bytes back (the
// per-column searches) or 256 bytes per streaming column.
__host__ __device__ constexpr uint32_t pad_for(uint32_t S, uint32_t wc) {
  const uint32_t a = 64u * wc * S, b = 256u * stream_cols(S, wc);
  return (uint32_t)align_up((a > b ? a : b) + 16u, 16);
}

// LDS layout: [pad | chunk (rounded up to whole hit blocks) + slack | hit bitmap]
template <int S, int WC>
__host__ __device__ constexpr uint32_t pad_bytes() {
  return pad_for(S, WC);
}
__host__ __device__ constexpr uint64_t chunk_lds_bytes(uint32_t C, uint32_t S) {
  return align_up((uint64_t)C * S, S >= 4 ? 2048 : 1024) + 64;  // whole hit blocks
}
__host__ __device__ constexpr uint64_t hit_words(uint32_t C, uint32_t S) {
  return align_up(C, 1024 / S) / 32 + 64;
}
// Candidate list of a sparse chunk (4- and 8-byte symbols, workgroups of
// several waves): per wave up to kListPerWave candidate positions and their
// search results, then one count per wave.
constexpr uint32_t kListPerWave = 32;
__host__ __device__ constexpr uint64_t list_lds_bytes(uint32_t S, uint32_t waves) {
  return S >= 4 && waves > 1 ? 4ull * (2 * kEncodeWaves * kListPerWave + kEncodeWaves) : 0ull;
}
// LDS of one chunk encoder with wc window columns and `waves` waves.
__host__ __device__ constexpr uint64_t encode_lds(uint32_t C, uint32_t S, uint32_t wc,
                                                  uint32_t waves) {
  return pad_for(S, wc) + chunk_lds_bytes(C, S) + 4 * hit_words(C, S) + list_lds_bytes(S, waves);
}

template <int S>
__device__ __forceinline__ typename SymType<S>::T vec_elem(const uint4& v, int e) {
  using T = typename SymType<S>::T;
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  if constexpr (S == 8) {
    return (T)w[2 * e] | ((T)w[2 * e + 1] << 32);
  } else if constexpr (S == 4) {
    return (T)w[e];
  } else if constexpr (S == 2) {
    return (T)(w[e >> 1] >> (16 * (e & 1)));
  } else {
    return (T)(w[e >> 2] >> (8 * (e & 3)));
  }
}

// 4 S bytes (S = 1 or 2) of LDS starting sh bytes (0..3) past the dword at
// p, read as aligned dwords (wide LDS reads below dword alignment are slow)
// and funnel-shifted.
template <int S>
__device__ __forceinline__ typename SymType<4 * S>::T load_run(const uint32_t* p, uint32_t sh) {
  const uint32_t w0 = p[0], w1 = p[1];
  const uint32_t lo = __builtin_amdgcn_alignbyte(w1, w0, sh);
  if constexpr (S == 1) {
    return lo;
  } else {
    return (uint64_t)lo | ((uint64_t)__builtin_amdgcn_alignbyte(p[2], w1, sh) << 32);
  }
}

// Exact longest match at chunk position h (h >= 1) over offsets
// d <= min(W, h), lanes holding offsets (column col, lane l: d = 64 col + l
// + 1). Every step compares the next four symbols of each live offset with
// those at h as one equality; an offset stays live while all four agree and
// its length, now at least L0 + 4, is still below d (a match never exceeds
// its offset). The offsets live at the start of the last step hold the
// answer: any offset that left earlier is shorter, or was capped at its own
// d, which is no longer than the length every last-step offset reaches and
// smaller than their offsets. Their exact lengths come from that step's
// data: L0 plus the leading equal symbols. The wave maximum of
// (min(length, d, lim) << 9 | d) is the longest length and, among equal
// lengths, the largest offset. Returns that key (length = key >> 9,
// offset = key & 511).
template <int S, int WC>
__device__ __forceinline__ uint32_t match_key(const typename SymType<S>::T* win, uint32_t h,
                                              uint32_t lim, uint32_t W, uint32_t lane) {
  using U = typename SymType<4 * S>::T;
  const uint8_t* wb = reinterpret_cast<const uint8_t*>(win);
  // Byte offset of this lane's run in the last column at step 0. Columns are
  // 64 S bytes apart and steps 4 S bytes, so one dword alignment serves all.
  // Positions down to h - 64 WC lie in the LDS pad before the chunk; reads
  // reach at most 4 S + 3 bytes past position h + L0 (L0 < lim <= c - h),
  // inside the slack after it.
  const int yb = ((int)h - (int)lane - 1 - 64 * (WC - 1)) * S;
  const uint32_t ysh = (uint32_t)yb & 3u;
  const uint32_t* yp = reinterpret_cast<const uint32_t*>(wb + (yb - (int)ysh));
  const uint32_t xb = h * S;
  const uint32_t xsh = xb & 3u;
  const uint32_t* xp = reinterpret_cast<const uint32_t*>(wb + (xb - xsh));
  // live offsets as wave masks, one per column
  uint64_t live[WC], start[WC];
  U yv[WC];
#pragma unroll
  for (int col = 0; col < WC; ++col) {
    const uint32_t d = 64u * col + lane + 1u;
    live[col] = ballot((d <= W) & (d <= h));
  }
  U xv;
  uint32_t L0 = 0;
  while (true) {
    xv = load_run<S>(xp + S * (L0 / 4), xsh);
    const uint32_t n0 = L0 + 4;
    uint64_t any = 0;
#pragma unroll
    for (int col = 0; col < WC; ++col) {
      yv[col] = load_run<S>(yp + S * (L0 / 4) + 16 * S * (WC - 1 - col), ysh);
      start[col] = live[col];
      // offsets d <= L0 + 4 end here
      live[col] &= ballot(yv[col] == xv) & ballot(64u * col + lane + 1u > n0);
      any |= live[col];
    }
    if (any == 0 || n0 >= lim) break;
    L0 = n0;
  }
  uint32_t key = 0;
#pragma unroll
  for (int col = 0; col < WC; ++col) {
    const uint32_t d = 64u * col + lane + 1u;
    // leading equal symbols of the last step (4 when all agree)
    const uint32_t r = (uint32_t)__builtin_ctzg(xv ^ yv[col], 32 * S) / (8u * S);
    const uint32_t Lc = min(min(L0 + r, d), lim);
    key = max(key, __builtin_amdgcn_inverse_ballot_w64(start[col]) ? (Lc << 9) | d : 0u);
  }
  return wave_max_u32(key);
}

// Token descriptors: bit 0 = pointer; literal: bits 1.. = chunk position;
// pointer: bits 1..8 = length, bits 9..16 = offset & 0xFF.
template <int S>
__device__ __forceinline__ void encode_group(uint32_t cnt, uint32_t desc, uint32_t group,
                                             const typename SymType<S>::T* win, uint8_t* slot,
                                             uint64_t flag_area, uint32_t& pay) {
  using T = typename SymType<S>::T;
  const uint32_t lane = lane_id();
  const bool valid = lane < cnt;
  const bool is_ptr = valid && (desc & 1u);
  const uint64_t pm = ballot(is_ptr);
  const uint64_t lm = ballot(valid && !(desc & 1u));
  const uint32_t off = pay + S * mbcnt(lm) + 2u * mbcnt(pm);
  uint8_t* dst = slot + flag_area + off;
  if (is_ptr) {
    dst[0] = (uint8_t)(desc >> 1);
    dst[1] = (uint8_t)(desc >> 9);
  } else if (valid) {
    T v = win[desc >> 1];
#pragma unroll
    for (int b = 0; b < S; ++b) dst[b] = (uint8_t)((uint64_t)v >> (8 * b));
  }
  if (lane == 0) *reinterpret_cast<uint64_t*>(slot + 8u * group) = pm;
  pay += S * popc64(lm) + 2u * popc64(pm);
}

// Compares this lane's V R symbols x[] with the window vectors wv[0..R]
// (wv[0] sits V k positions before the lane's first vector, wv[r] the r-th
// vector after it), for the offsets d = V (k - 1) + j, j = 1 .. jmax. In the
// chunk's first W positions (kHead) only offsets d <= p count; 4- and 8-byte
// symbols need no such mask (the bytes before the chunk hold a symbol that
// none of the first W symbols equals, see fill_pad_distinct).
template <int S, bool kHead, bool kPartial, int kStep, int R>
__device__ __forceinline__ void hit_step(const typename SymType<S>::T (&x)[16 / S * R],
                                         const uint4 (&wv)[R + 1], uint32_t dk, uint32_t jmax,
                                         uint32_t base, uint64_t (&acc)[16 / S * R]) {
  using T = typename SymType<S>::T;
  constexpr int V = Geo<S>::V;
  constexpr int VR = V * R;
  T q[(R + 1) * V];
#pragma unroll
  for (int r = 0; r <= R; ++r)
#pragma unroll
    for (int e = 0; e < V; ++e) q[r * V + e] = vec_elem<S>(wv[r], e);
  static_assert(!kHead || R == 1, "4- and 8-byte symbols run no head variant");
#pragma unroll
  for (int j = 1; j <= V; ++j) {
    if (kPartial && (uint32_t)j > jmax) break;
#pragma unroll
    for (int i = 0; i < VR; i += kStep) {
      if constexpr (kHead)
        acc[i] |= ballot((x[i] == q[i + V - j]) & (base + VR * lane_id() + i >= dk + j));
      else
        acc[i] |= ballot(x[i] == q[i + V - j]);
    }
    // with 8 or 16 positions per lane, keep at most V R compare masks live
    // (more would spill SGPRs); 4 positions schedule better without it
    if constexpr (VR >= 8) __builtin_amdgcn_sched_barrier(0);
  }
}

// Hit bitmap for one block of 64 V R positions starting at `base` (each lane
// owns R consecutive 16-byte vectors): for every kStep-th position p, bit p
// is set iff some offset d <= min(W, p) has sym[p - d] == sym[p] (the other
// bits stay 0). Step k reads the one vector V k positions back; the R before
// it come from the previous steps, held in a ring of R + 1 registers whose
// slot for step k is k mod (R + 1), so the steps are unrolled R + 1 at a time
// and every ring index is a constant.
template <int S, bool kHead, int kStep>
__device__ __forceinline__ void hit_block(const uint4* w4, uint32_t base, uint32_t W,
                                          uint32_t* hits, uint32_t kb = 1, uint32_t ke = ~0u) {
  using T = typename SymType<S>::T;
  constexpr int V = Geo<S>::V;
  constexpr int R = Geo<S>::R;
  constexpr int VR = V * R;
  const uint32_t lane = lane_id();
  const int vbase = (int)(base / V + R * lane);
  uint4 ring[R + 1];
  T x[VR];
  uint4 x0v = w4[vbase];  // with R = 1: the vector after the current step's
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const uint4 v = m == 0 ? x0v : w4[vbase + m];
    ring[(R + 1 - m) % (R + 1)] = v;  // the vector m after the lane's first: slot -m
#pragma unroll
    for (int e = 0; e < V; ++e) x[m * V + e] = vec_elem<S>(v, e);
  }
  uint64_t acc[VR];
#pragma unroll
  for (int i = 0; i < VR; ++i) acc[i] = 0;
  const uint32_t pos0 = base + VR * lane;  // this lane's first position
  const uint32_t kfull = W / V;            // steps whose V offsets are all <= W
  uint32_t k = 1;
  if constexpr (R == 1) {
    // steps [kb, ke) only (the split parse shares one block's offsets among
    // several waves); x0v is the vector after step k's
    const uint32_t kend = min(ke, kfull + 1);  // full steps end
    if (kb > 1) {
      k = kb;
      x0v = w4[vbase - (int)(kb - 1)];
    }
    // two steps per round: ring slot 1 for odd k, 0 for even k
    for (; k + 1 < kend; k += 2) {
      ring[1] = w4[vbase - (int)k];
      ring[0] = w4[vbase - (int)k - 1];
      const uint4 w1[2] = {ring[1], x0v}, w2[2] = {ring[0], ring[1]};
      hit_step<S, kHead, false, kStep, R>(x, w1, V * (k - 1), V, base, acc);
      hit_step<S, kHead, false, kStep, R>(x, w2, V * k, V, base, acc);
      x0v = ring[0];
    }
    if (k < kend) {
      const uint4 q1 = w4[vbase - (int)k];
      const uint4 w1[2] = {q1, x0v};
      hit_step<S, kHead, false, kStep, R>(x, w1, V * (k - 1), V, base, acc);
      x0v = q1;
      ++k;
    }
    if (W % V && k == kfull + 1 && k < ke) {
      const uint4 w1[2] = {w4[vbase - (int)k], x0v};
      hit_step<S, kHead, true, kStep, R>(x, w1, V * (k - 1), W % V, base, acc);
    }
  } else {
    for (; k + R <= kfull; k += R + 1) {
      uint4 nv[R + 1];
#pragma unroll
      for (int u = 0; u <= R; ++u) nv[u] = w4[vbase - (int)(k + u)];
#pragma unroll
      for (int u = 0; u <= R; ++u) {
        ring[(1 + u) % (R + 1)] = nv[u];
        uint4 wv[R + 1];
#pragma unroll
        for (int r = 0; r <= R; ++r) wv[r] = ring[(1 + u - r + 2 * (R + 1)) % (R + 1)];
        hit_step<S, kHead, false, kStep, R>(x, wv, V * (k + u - 1), V, base, acc);
      }
    }
    // at most R full steps remain, then the partial one (W % V offsets)
#pragma unroll
    for (int u = 0; u <= R; ++u) {
      const uint32_t kk = k + u;
      if (kk <= kfull || (kk == kfull + 1 && W % V)) {
        ring[(1 + u) % (R + 1)] = w4[vbase - (int)kk];
        uint4 wv[R + 1];
#pragma unroll
        for (int r = 0; r <= R; ++r) wv[r] = ring[(1 + u - r + 2 * (R + 1)) % (R + 1)];
        if (kk <= kfull)
          hit_step<S, kHead, false, kStep, R>(x, wv, V * (kk - 1), V, base, acc);
        else
          hit_step<S, kHead, true, kStep, R>(x, wv, V * (kk - 1), W % V, base, acc);
      }
    }
  }
  uint32_t bits = 0;
#pragma unroll
  for (int i = 0; i < VR; i += kStep) bits |= (uint32_t)((acc[i] >> lane) & 1u) << i;
  if (bits) atomicOr(&hits[pos0 >> 5], bits << (pos0 & 31u));
}

// 4- and 8-byte symbols: fills the `pad` bytes before the staged chunk with
// one symbol value that none of the chunk's first `lim` = min(W, c) symbols
// equals, so that compares reaching before the chunk never hit and the hit
// phase needs no per-offset mask there. At most lim <= 256 values are taken,
// so counting up from a fixed pattern finds one within lim + 1 rounds. Run
// by the one wave that builds block 0 (the only block whose window reaches
// before the chunk); the stage must be visible to it.
template <int S>
__device__ __forceinline__ void fill_pad_distinct(uint8_t* stage, uint32_t pad, uint32_t lim) {
  using T = typename SymType<S>::T;
  const T* sym = reinterpret_cast<const T*>(stage);
  const uint32_t lane = lane_id();
  T own[4];
  bool in[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    in[t] = lane + 64u * t < lim;
    own[t] = in[t] ? sym[lane + 64u * t] : (T)0;
  }
  T v = (T)0x9E3779B97F4A7C15ull;
  for (;;) {
    bool eq = false;
#pragma unroll
    for (int t = 0; t < 4; ++t) eq |= in[t] && own[t] == v;
    if (!ballot(eq)) break;
    ++v;
  }
  T* before = reinterpret_cast<T*>(stage - pad);
  for (uint32_t k = lane; k < pad / S; k += 64) before[k] = v;
  wave_sync();
}

// Hit blocks b0, b0 + step, ... below nblocks of the staged chunk.
template <int S, int WC>
__device__ __forceinline__ void build_hits(uint8_t* stage, uint32_t b0, uint32_t nblocks,
                                           uint32_t step, uint32_t W, uint32_t c, bool sampled,
                                           uint32_t* hits) {
  constexpr uint32_t kBlock = Geo<S>::kBlock;
  const uint4* w4 = reinterpret_cast<const uint4*>(stage);
  for (uint32_t b = b0; b < nblocks; b += step) {
    const uint32_t base = b * kBlock;
    if constexpr (Geo<S>::R > 1) {
      if (b == 0) fill_pad_distinct<S>(stage, pad_bytes<S, WC>(), min(W, c));
      if (sampled) hit_block<S, false, 2>(w4, base, W, hits);
      else hit_block<S, false, 1>(w4, base, W, hits);
    } else if (sampled) {
      if (base >= W) hit_block<S, false, 2>(w4, base, W, hits);
      else hit_block<S, true, 2>(w4, base, W, hits);
    } else {
      if (base >= W) hit_block<S, false, 1>(w4, base, W, hits);
      else hit_block<S, true, 1>(w4, base, W, hits);
    }
  }
}

// Word w of the candidate bitmap: the hit bitmap itself, or, when only even
// positions were tested, bit p set iff bit p or bit p + 1 of the hits is.
__device__ __forceinline__ uint32_t cand_word(const uint32_t* hits, uint32_t w, uint32_t nhw,
                                              bool sampled) {
  const uint32_t h = w < nhw ? hits[w] : 0u;
  if (!sampled) return h;
  const uint32_t next = w + 1 < nhw ? hits[w + 1] : 0u;
  return h | (h >> 1) | (next << 31);
}

// Copies the chunk HBM -> LDS with 16-byte loads (all threads); it lands
// 16-byte aligned in LDS whatever its alignment in HBM.
template <int S>
__device__ __forceinline__ void stage_chunk(const ChunkJob& job, uint8_t* stage) {
  const uint32_t tid = threadIdx.x;
  const uint32_t nbytes = job.c * S;
  if (((uintptr_t)job.src & 15) == 0) {
    const uint32_t nw = (nbytes + 15) / 16;
    // words wholly inside the input, four per thread in flight
    const uint32_t full = (uint32_t)min<uint64_t>(nw, job.src_avail / 16);
    const uint32_t step = blockDim.x;
    uint32_t k = tid;
    // (four named vectors, not an array: an array here has been left in
    // scratch memory inside the persistent batch encoder)
    for (; k + 3 * step < full; k += 4 * step) {
      const uint4* src = reinterpret_cast<const uint4*>(job.src) + k;
      const uint4 v0 = src[0], v1 = src[step], v2 = src[2 * step], v3 = src[3 * step];
      uint4* dst = reinterpret_cast<uint4*>(stage) + k;
      dst[0] = v0;
      dst[step] = v1;
      dst[2 * step] = v2;
      dst[3 * step] = v3;
    }
    for (; k < nw; k += step) {
      const uint64_t g = 16ull * k;
      if (g + 16 <= job.src_avail) {
        *reinterpret_cast<uint4*>(stage + 16 * k) = *reinterpret_cast<const uint4*>(job.src + g);
      } else {
        for (uint32_t b = 0; b < 16; ++b) stage[16 * k + b] = g + b < job.src_avail ? job.src[g + b] : 0;
      }
    }
  } else {
    for (uint32_t k = tid; k < nbytes; k += blockDim.x) stage[k] = job.src[k];
  }
}

// Cursor over a candidate bitmap: 64 consecutive words cached one per lane.
struct CandCursor {
  uint32_t hw0, hcache;
  __device__ __forceinline__ void init(const uint32_t* hits, uint32_t nhw, bool sampled) {
    hw0 = 0;
    hcache = cand_word(hits, lane_id(), nhw, sampled);
  }
  // First candidate at or after p (c if none); p never decreases between
  // calls. The first look is at p's own bit in the cached words.
  __device__ __forceinline__ uint32_t next(uint32_t p, uint32_t c, const uint32_t* hits,
                                           uint32_t nhw, bool sampled) {
    const uint32_t lane = lane_id();
    const uint32_t pw = p >> 5;  // bitmap word holding position p
    if (pw - hw0 < 64u && ((readlane(hcache, pw - hw0) >> (p & 31u)) & 1u)) return p;
    uint32_t w = pw;
    for (;;) {
      if (w >= hw0 + 64) {
        hw0 = w;
        hcache = cand_word(hits, hw0 + lane, nhw, sampled);
      }
      uint32_t mine = hcache;
      const uint32_t gw = hw0 + lane;
      if (gw < pw) mine = 0;
      else if (gw == pw) mine &= ~0u << (p & 31u);
      const uint64_t nz = ballot(mine != 0);
      if (nz) {
        const uint32_t l = (uint32_t)__ffsll((unsigned long long)nz) - 1;
        return min(c, (hw0 + l) * 32u + (uint32_t)__ffs(readlane(mine, l)) - 1u);
      }
      w = hw0 + 64;
      if (w * 32u >= c) return c;
    }
  }
};

// Cursor over the candidate list of a sparse chunk: the sub-lists of the
// waves in order (each sorted, each over a later range of positions), one
// sub-list cached per lane. next() returns the first candidate at or after p
// whose search found a match (c if none) and that result; p never decreases
// between calls. Candidates without a match are skipped: the greedy parse
// takes a literal at every position up to the next match, candidate or not,
// so those positions join the literal run before it.
struct ListCursor {
  const uint32_t* pos;
  const uint32_t* key;
  const uint32_t* cnt;
  uint32_t w, nw, n, ch, ck;
  __device__ __forceinline__ void load() {
    const uint32_t lane = lane_id();
    n = cnt[w];
    ch = lane < n ? pos[w * kListPerWave + lane] : 0u;
    ck = lane < n ? key[w * kListPerWave + lane] : 0u;
  }
  __device__ __forceinline__ void init(const uint32_t* list, uint32_t waves) {
    pos = list;
    key = list + kEncodeWaves * kListPerWave;
    cnt = key + kEncodeWaves * kListPerWave;
    w = 0;
    nw = waves;
    load();
  }
  __device__ __forceinline__ uint32_t next(uint32_t p, uint32_t c, uint32_t& k) {
    for (;;) {
      const uint64_t m = ballot(lane_id() < n && ch >= p && ck != 0u);
      if (m) {
        const uint32_t j = (uint32_t)__builtin_ctzll(m);
        k = readlane(ck, j);
        return readlane(ch, j);
      }
      if (++w >= nw) return c;
      load();
    }
  }
};

// The exact longest match at candidate h (h >= 1): L << 9 | d (offset d),
// or 0 if it is shorter than MIN. All 64 lanes take part; the result is
// wave-uniform. Lanes hold offsets (d = 64 col + lane + 1); ties go to the
// largest offset.
template <int S, int WC>
__device__ __forceinline__ uint32_t search_token(const typename SymType<S>::T* win, uint32_t h,
                                                 uint32_t c, uint32_t W, uint32_t MIN,
                                                 const uint64_t (&wmask)[WC], uint32_t lane) {
  using T = typename SymType<S>::T;
  if constexpr (kRunSearch<S>) {
    const uint32_t key = match_key<S, WC>(win, h, min(kMaxMatch, c - h), W, lane);
    return (key >> 9) >= MIN ? key : 0u;
  } else {
    // exact longest match at h. Invariant: A holds the offsets d >= L whose
    // match at h is at least L long; extending to L + 1 drops d = L and keeps
    // the offsets that also match at h + L. Rows come four per LDS round trip
    // from one per-lane base address (positions up to 3 past the chunk end
    // read slack bytes and are never used).
    uint64_t A[WC];
    if (h < 64u * WC) {
#pragma unroll
      for (int col = 0; col < WC; ++col) A[col] = wmask[col] & ballot(64u * col + lane + 1u <= h);
    } else {
#pragma unroll
      for (int col = 0; col < WC; ++col) A[col] = wmask[col];
    }
    uint32_t L = 0;
    const uint32_t lim = min(kMaxMatch, c - h);
    while (L < lim) {
      const uint32_t qb = h + L;
      // this lane's window symbol for row r, column col: win[qb + r - (64 col + lane + 1)]
      const T* wbase = win + (int)qb - (int)lane - 1 - 64 * (WC - 1);
      T xr[4], wr[4][WC];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        xr[r] = win[qb + r];
#pragma unroll
        for (int col = 0; col < WC; ++col) wr[r][col] = wbase[r + 64 * (WC - 1 - col)];
      }
      if (L + 4 <= 64) {
        // offsets d <= L (only d = L can still be present) all sit in column 0
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (L >= lim) goto found;
          uint64_t B[WC];
#pragma unroll
          for (int col = 0; col < WC; ++col) B[col] = A[col] & ballot(wr[r][col] == xr[r]);
          B[0] &= ~0ull << L;
          uint64_t any = 0;
#pragma unroll
          for (int col = 0; col < WC; ++col) any |= B[col];
          if (!any) goto found;
#pragma unroll
          for (int col = 0; col < WC; ++col) A[col] = B[col];
          ++L;
        }
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (L >= lim) goto found;
          uint64_t B[WC];
          uint64_t any = 0;
#pragma unroll
          for (int col = 0; col < WC; ++col) {
            const int sh = (int)L - 64 * col;  // offsets d <= L are too short
            const uint64_t cap = sh <= 0 ? ~0ull : (sh >= 64 ? 0ull : (~0ull << sh));
            B[col] = A[col] & ballot(wr[r][col] == xr[r]) & cap;
            any |= B[col];
          }
          if (!any) goto found;
#pragma unroll
          for (int col = 0; col < WC; ++col) A[col] = B[col];
          ++L;
        }
      }
    }
  found:
    if (L < MIN) return 0u;
    uint32_t d = 0;
#pragma unroll
    for (int col = WC - 1; col >= 0; --col) {
      if (d == 0 && A[col]) d = 64u * col + 64u - (uint32_t)__clzll(A[col]);
    }
    return L << 9 | d;
  }
}

// ---- streaming exact search for 1- and 2-byte symbols ----------------------
//
// The greedy parse asks for the longest match at each token start h. For
// 1- and 2-byte symbols the window offsets are packed K = 4 / S to a lane:
// lane l of column c holds offsets d = 64 K c + K l + K - k in its k-th byte
// (S = 1) or half (S = 2), so that the dword ending just before position q
// holds sym[q - d] for all of them (kept in registers, see StreamMatch). A
// position q is compared with its whole window at once: the dword of K
// copies of sym[q] XOR each lane's dword, reduced to one "differs" bit per
// offset (a
// byte-wise carry trick for bytes, a packed 16-bit minimum with 1 for
// halves). The offsets whose match at h is at least t symbols long are a
// live bit set: start with the offsets d <= min(W, h) that match at h, and
// clear the differing ones at h + 1, h + 2, ... until none is left or the
// length limit is reached. The token's length is the number of positions
// passed and its offset the largest survivor of the last position before
// the set emptied (ties go to the largest offset).
//
// Every position is compared once: the position where a match ends is the
// next token's start (greedy parse), so its differs bits are kept and
// reused. Only a rewind (a literal after a partial match with MIN >= 3, or
// the capped fallback below) or a jump over non-candidates reloads.
//
// The live set ignores the cap L <= d (a match never overlaps its own
// source) while it runs. If the largest survivor d has d >= L the uncapped
// result is also the capped one (it reaches length L and no offset can give
// more). Otherwise (periodic runs shorter than their length, e.g. constant
// runs) the token is recomputed by the per-column search with the cap.

template <int S> struct Pack {
  static constexpr uint32_t K = 4 / S;         // offsets per lane
  static constexpr uint32_t kPerCol = 64 * K;  // offsets per column
  // one bit per offset: bit 7 of each byte / bit 0 of each half
  static constexpr uint32_t kLive = S == 1 ? 0x80808080u : 0x00010001u;
};

constexpr uint32_t kNeedCapped = 1;  // token(): recompute with the L <= d cap

// Differs bits of K window symbols y against K copies xr of sym[q].
template <int S>
__device__ __forceinline__ uint32_t differs(uint32_t y, uint32_t xr) {
  const uint32_t e = y ^ xr;
  if constexpr (S == 1) {
    // bit 7 of a byte: it is nonzero (low 7 bits via a carry into bit 7,
    // which never crosses into the next byte, or bit 7 itself)
    return ((e & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | e;
  } else {
    uint32_t z;
    // each half: min(e, 1), i.e. 1 iff the two symbols differ
    asm("v_pk_min_u16 %0, %1, %2" : "=v"(z) : "v"(e), "s"(0x00010001u));
    return z;
  }
}

// One whole-wave shift: lane l takes src of lane l - 1, lane 0 takes `fill`.
__device__ __forceinline__ uint32_t wave_shr1(uint32_t src, uint32_t fill) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)src, 0x138, 0xF, 0xF, false);
}

template <int S, int NC>
struct StreamMatch {
  using P = Pack<S>;
  // Window registers for position q, with qa = (S q) & ~3 the byte address
  // of the dword holding q's first byte: lane l of column c holds in A[c]
  // the dword at qa - 4 (64 c + l + 1) and in B[c] the one after it, so
  // alignbyte(B, A, (S q) & 3) is the dword ending just before q's first
  // byte, whose parts are sym[q - d] for the lane's offsets. When q moves
  // into the next dword, A takes B and B shifts up one lane (lane 0 of
  // column 0 takes the dword at qa + 4, lane 0 of a higher column the old
  // lane 63 of the column below): no LDS read per position.
  const uint32_t* stage;
  uint32_t wmask[NC];  // live bits of the offsets d <= W
  uint32_t q;          // next position to compare
  uint32_t sh;         // (S q) & 3
  uint32_t A[NC], B[NC];
  uint32_t xc, xn;     // the dwords at qa and qa + 4 (same in all lanes)
  uint32_t z[NC];      // differs bits of position q - 1

  // Live bits of column c for the offsets d <= lim.
  __device__ __forceinline__ static uint32_t mask_le(uint32_t c, uint32_t lim, uint32_t lane) {
    const int32_t dmax = (int32_t)(c * P::kPerCol + P::K * lane + P::K);  // offset of part 0
    const int32_t t = dmax - (int32_t)lim;  // parts k < t hold offsets above lim
    if (t <= 0) return P::kLive;
    if (t >= (int32_t)P::K) return 0u;
    return P::kLive << (8 * S * t);
  }

  __device__ __forceinline__ void init(const uint8_t* st, uint32_t W, uint32_t lane) {
    stage = reinterpret_cast<const uint32_t*>(st);
#pragma unroll
    for (int c = 0; c < NC; ++c) wmask[c] = mask_le(c, W, lane);
    q = ~0u;
  }

  // Window registers for position pos (aligned dword reads; the pad before
  // the chunk holds the 256 NC bytes the highest offsets reach back).
  __device__ __forceinline__ void seek(uint32_t pos, uint32_t lane) {
    q = pos;
    sh = (S * pos) & 3u;
    const uint32_t* w = stage + (S * pos) / 4;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      A[c] = w[-(int32_t)(64 * c + lane + 1)];
      B[c] = w[-(int32_t)(64 * c + lane)];
    }
    xc = w[0];
    xn = w[1];
  }

  // Differs bits of position q; then q + 1.
  __device__ __forceinline__ void step() {
    const uint32_t sel = sh * 0x01010101u + (S == 1 ? 0u : 0x01000100u);
    const uint32_t xr = __builtin_amdgcn_perm(xc, xc, sel);  // K copies of sym[q]
#pragma unroll
    for (int c = 0; c < NC; ++c) z[c] = differs<S>(__builtin_amdgcn_alignbyte(B[c], A[c], sh), xr);
    ++q;
    sh += S;
    if (sh == 4) {
      sh = 0;
#pragma unroll
      for (int c = NC - 1; c >= 1; --c) {
        const uint32_t carry = readlane(B[c - 1], 63);
        A[c] = B[c];
        B[c] = wave_shr1(B[c], carry);
      }
      A[0] = B[0];
      B[0] = wave_shr1(B[0], xn);
      xc = xn;
      xn = stage[(S * q) / 4 + 1];  // stays within the slack after the chunk
    }
  }

  __device__ __forceinline__ static bool any(const uint32_t (&v)[NC]) {
    uint32_t o = v[0];
#pragma unroll
    for (int c = 1; c < NC; ++c) o |= v[c];
    return ballot(o != 0) != 0;
  }

  // Largest offset with a live bit.
  __device__ __forceinline__ static uint32_t largest(const uint32_t (&v)[NC]) {
#pragma unroll
    for (int c = NC - 1; c >= 0; --c) {
      const uint64_t b = ballot(v[c] != 0);
      if (b) {
        const uint32_t l = 63u - (uint32_t)__builtin_clzll(b);
        const uint32_t k = (uint32_t)__builtin_ctz(readlane(v[c], l)) / (8 * S);
        return c * P::kPerCol + P::K * l + P::K - k;
      }
    }
    return 0;
  }

  // The token at chunk position h < c, lim = min(255, c - h): L << 9 | d
  // for a match of at least MIN symbols, 0 for a literal, kNeedCapped if
  // the cap L <= d decides it. All lanes; the result is wave-uniform.
  __device__ __forceinline__ uint32_t token(uint32_t h, uint32_t lim, uint32_t W, uint32_t MIN,
                                            uint32_t lane) {
    if (h + 1 != q) {  // z does not hold position h yet
      if (h != q) seek(h, lane);
      step();
    }
    uint32_t live[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c)
      live[c] = (h >= W ? wmask[c] : (wmask[c] & mask_le(c, h, lane))) & ~z[c];
    if (!any(live)) return 0u;
    uint32_t t = 1;  // live: the offsets whose match at h is at least t long
    while (t < lim) {
      step();
      uint32_t nl[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) nl[c] = live[c] & ~z[c];
      if (!any(nl)) break;
#pragma unroll
      for (int c = 0; c < NC; ++c) live[c] = nl[c];
      ++t;
    }
    if (t < MIN) return 0u;
    const uint32_t d = largest(live);
    if (d < t) return kNeedCapped;
    return t << 9 | d;
  }
};

template <int S> constexpr bool kStreamSearch = S <= 2;
template <int S, int WC>
using StreamMatchFor = StreamMatch<S, (stream_cols(S, WC) ? (int)stream_cols(S, WC) : 1)>;

// The exact longest match at h through the streaming search (1- and 2-byte
// symbols, with the capped per-column search as its fallback) or the
// per-column search alone.
template <int S, int WC>
__device__ __forceinline__ uint32_t find_token(StreamMatchFor<S, WC>& sm,
                                               const typename SymType<S>::T* win, uint32_t h,
                                               uint32_t c, uint32_t W, uint32_t MIN,
                                               const uint64_t (&wmask)[WC], uint32_t lane) {
  if constexpr (kStreamSearch<S>) {
    const uint32_t key = sm.token(h, min(kMaxMatch, c - h), W, MIN, lane);
    if (key != kNeedCapped) return key;
  }
  return search_token<S, WC>(win, h, c, W, MIN, wmask, lane);
}

// The inner loop of the dense parse for one window column (1-byte symbols
// with W <= 256, 2-byte ones with W <= 128), written out: it extends an open
// token position by position until no offset matches or n reaches steps.
// In: live (the token's live bits), n (positions matched past the first),
// steps, qa (LDS byte address of the dword holding the next position), ph
// (that position's byte within the dword), wbase (this lane's window dword
// offset from the compared position's dword). Out: live, n (unchanged
// meaning), z (differs bits of the last compared position, valid if the
// token died, i.e. n < steps). The dword group's kK positions are unrolled
// with constant shifts and selectors; the loads complete inside the block.
template <int S>
__device__ __forceinline__ void extend_run(uint32_t& live, uint32_t& n, uint32_t& z, uint32_t steps,
                                           uint32_t qa, uint32_t ph, uint32_t wbase) {
  uint32_t a, b, x, t0, t1, wa, xa;
  if constexpr (S == 1) {
    const uint32_t s1 = 0x01010101u, s2 = 0x02020202u, s3 = 0x03030303u;
#define GPULZ_STEP1(K, SEL)                                   \
  "s_cmp_eq_u32 %[n], %[steps]\n\t"                           \
  "s_cbranch_scc1 .Lend%=\n\t"                                \
  "v_perm_b32 %[t0], %[x], %[x], " SEL "\n\t"                 \
  "v_alignbyte_b32 %[t1], %[b], %[a], " #K "\n\t"             \
  "v_xor_b32 %[t1], %[t1], %[t0]\n\t"                         \
  "v_and_b32 %[t0], 0x7f7f7f7f, %[t1]\n\t"                    \
  "v_add_u32 %[t0], 0x7f7f7f7f, %[t0]\n\t"                    \
  "v_or_b32 %[z], %[t0], %[t1]\n\t"                           \
  "v_bfi_b32 %[t0], %[z], 0, %[live]\n\t"                     \
  "v_cmp_ne_u32 vcc, 0, %[t0]\n\t"                            \
  "s_cbranch_vccz .Lend%=\n\t"                                \
  "v_mov_b32 %[live], %[t0]\n\t"                              \
  "s_add_u32 %[n], %[n], 1\n\t"
    asm volatile(
        "v_add_u32 %[wa], %[qa], %[wbase]\n\t"
        "v_mov_b32 %[xa], %[qa]\n\t"
        "ds_read_b32 %[a], %[wa]\n\t"
        "ds_read_b32 %[b], %[wa] offset:4\n\t"
        "ds_read_b32 %[x], %[xa]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "s_cmp_eq_u32 %[ph], 1\n\t"
        "s_cbranch_scc1 .Lp1%=\n\t"
        "s_cmp_eq_u32 %[ph], 2\n\t"
        "s_cbranch_scc1 .Lp2%=\n\t"
        "s_cmp_eq_u32 %[ph], 3\n\t"
        "s_cbranch_scc1 .Lp3%=\n"
        ".Lp0%=:\n\t"
        GPULZ_STEP1(0, "0")
        "\n.Lp1%=:\n\t"
        GPULZ_STEP1(1, "%[s1]")
        "\n.Lp2%=:\n\t"
        GPULZ_STEP1(2, "%[s2]")
        "\n.Lp3%=:\n\t"
        GPULZ_STEP1(3, "%[s3]")
        "v_add_u32 %[wa], 4, %[wa]\n\t"
        "v_add_u32 %[xa], 4, %[xa]\n\t"
        "ds_read_b32 %[a], %[wa]\n\t"
        "ds_read_b32 %[b], %[wa] offset:4\n\t"
        "ds_read_b32 %[x], %[xa]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "s_branch .Lp0%=\n"
        ".Lend%=:"
        : [live] "+v"(live), [n] "+s"(n), [z] "=&v"(z), [a] "=&v"(a), [b] "=&v"(b), [x] "=&v"(x),
          [t0] "=&v"(t0), [t1] "=&v"(t1), [wa] "=&v"(wa), [xa] "=&v"(xa)
        : [steps] "s"(steps), [qa] "s"(qa), [ph] "s"(ph), [wbase] "v"(wbase), [s1] "s"(s1),
          [s2] "s"(s2), [s3] "s"(s3)
        : "vcc", "scc", "memory");
#undef GPULZ_STEP1
  } else {
    const uint32_t s0 = 0x01000100u, s2 = 0x03020302u, ones = 0x00010001u;
#define GPULZ_STEP2(K, SEL)                                   \
  "s_cmp_eq_u32 %[n], %[steps]\n\t"                           \
  "s_cbranch_scc1 .Lend%=\n\t"                                \
  "v_perm_b32 %[t0], %[x], %[x], " SEL "\n\t"                 \
  "v_alignbyte_b32 %[t1], %[b], %[a], " #K "\n\t"             \
  "v_xor_b32 %[t1], %[t1], %[t0]\n\t"                         \
  "v_pk_min_u16 %[z], %[t1], %[ones]\n\t"                     \
  "v_bfi_b32 %[t0], %[z], 0, %[live]\n\t"                     \
  "v_cmp_ne_u32 vcc, 0, %[t0]\n\t"                            \
  "s_cbranch_vccz .Lend%=\n\t"                                \
  "v_mov_b32 %[live], %[t0]\n\t"                              \
  "s_add_u32 %[n], %[n], 1\n\t"
    asm volatile(
        "v_add_u32 %[wa], %[qa], %[wbase]\n\t"
        "v_mov_b32 %[xa], %[qa]\n\t"
        "ds_read_b32 %[a], %[wa]\n\t"
        "ds_read_b32 %[b], %[wa] offset:4\n\t"
        "ds_read_b32 %[x], %[xa]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "s_cmp_eq_u32 %[ph], 2\n\t"
        "s_cbranch_scc1 .Lp2%=\n"
        ".Lp0%=:\n\t"
        GPULZ_STEP2(0, "%[s0]")
        "\n.Lp2%=:\n\t"
        GPULZ_STEP2(2, "%[s2]")
        "v_add_u32 %[wa], 4, %[wa]\n\t"
        "v_add_u32 %[xa], 4, %[xa]\n\t"
        "ds_read_b32 %[a], %[wa]\n\t"
        "ds_read_b32 %[b], %[wa] offset:4\n\t"
        "ds_read_b32 %[x], %[xa]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "s_branch .Lp0%=\n"
        ".Lend%=:"
        : [live] "+v"(live), [n] "+s"(n), [z] "=&v"(z), [a] "=&v"(a), [b] "=&v"(b), [x] "=&v"(x),
          [t0] "=&v"(t0), [t1] "=&v"(t1), [wa] "=&v"(wa), [xa] "=&v"(xa)
        : [steps] "s"(steps), [qa] "s"(qa), [ph] "s"(ph), [wbase] "v"(wbase), [s0] "s"(s0),
          [s2] "s"(s2), [ones] "s"(ones)
        : "vcc", "scc", "memory");
#undef GPULZ_STEP2
  }
}

// Greedy parse of a dense chunk of c symbols (1- and 2-byte symbols,
// MIN <= 2) from position h0, taking tokens that start before hend (the
// last one may run past hend, up to c): [0, c) for the whole chunk, a
// segment for the split parse. Every position is compared once with its
// window (StreamMatch's packed layout). A token open at h with t positions matched either
// survives position h + t (some offset still matches), or ends there: a
// pointer (t, largest survivor) if t >= MIN, else a literal at h; either
// way the next token starts at h + t (MIN <= 2), whose compare is the one
// just made. A token also ends at min(255, c - h) positions. A token that
// the cap L <= d decides (see StreamMatch) is redone by the capped
// per-column search, and the parse continues from its end. Each compare
// reads its window dwords from LDS at dword alignment.
//
// Token descriptors are collected one per lane in dlo; flush(dlo) takes
// each full group of 64. Returns the number of tokens left in dlo.
template <int S, int WC, typename Flush>
__device__ __forceinline__ uint32_t parse_dense(const uint8_t* stage, uint32_t h0, uint32_t hend,
                                                uint32_t c, uint32_t W, uint32_t MIN,
                                                const uint64_t (&wmask64)[WC], uint32_t lane,
                                                uint32_t& dlo, Flush&& flush) {
  using T = typename SymType<S>::T;
  using SM = StreamMatchFor<S, WC>;
  constexpr int NC = stream_cols(S, WC);
  const T* win = reinterpret_cast<const T*>(stage);
  const uint32_t* st = reinterpret_cast<const uint32_t*>(stage);
  uint32_t wm[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) wm[k] = SM::mask_le(k, W, lane);

  uint32_t nb = 0, lo = dlo;
  // Per-lane byte offsets (from the stage) of the window dwords of column j,
  // relative to the dword of the compared position.
  int32_t woff[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) woff[j] = -4 * (int32_t)(64 * j + lane + 1);
  // z = differs bits of position vq, a copy of the position in a vector
  // register: its address and shift arithmetic run on the vector unit, which
  // has issue slots to spare, instead of the scalar unit, which the parse's
  // control flow keeps busy.
#define GPULZ_DENSE_COMPARE(vq)                                                            \
  do {                                                                                     \
    const uint32_t qb_ = S * (vq);                                                         \
    const uint32_t sh_ = qb_ & 3u;                                                         \
    const uint8_t* w_ = stage + (qb_ & ~3u);                                               \
    const uint32_t xc_ = *reinterpret_cast<const uint32_t*>(w_);                           \
    const uint32_t sel_ = __builtin_amdgcn_perm(sh_, sh_, 0u) + (S == 1 ? 0u : 0x01000100u); \
    const uint32_t xr_ = __builtin_amdgcn_perm(xc_, xc_, sel_);                            \
    _Pragma("unroll") for (int j_ = 0; j_ < NC; ++j_) {                                    \
      const uint32_t* p_ = reinterpret_cast<const uint32_t*>(w_ + woff[j_]);               \
      z[j_] = differs<S>(__builtin_amdgcn_alignbyte(p_[1], p_[0], sh_), xr_);              \
    }                                                                                      \
  } while (0)
#define GPULZ_DENSE_REC(val)    \
  do {                          \
    if (lane == nb) lo = (val); \
    if (++nb == 64) {           \
      flush(lo);                \
      nb = 0;                   \
    }                           \
  } while (0)

  // LDS byte address of the stage (the window dwords the inner loop reads):
  // the low 32 bits of the generic address (the shared aperture starts on a
  // 4 GiB boundary)
  const uint32_t stage_lds = (uint32_t)(uintptr_t)stage;
  uint32_t z[NC];
  bool have_z = false;  // z holds position h's compare already
  // wave-uniform bounds (a caller may derive them from the wave index)
  uint32_t h = __builtin_amdgcn_readfirstlane(h0);
  hend = __builtin_amdgcn_readfirstlane(hend);
  uint32_t vq;  // next position to compare, in a vector register
  asm volatile("v_mov_b32 %0, %1" : "=v"(vq) : "s"(h));
  // From each group-aligned token start the group loop (dense_groups) takes
  // over, until a flush, a capped token (redone here first, then the group
  // loop again) or the chunk's last groups (finished here).
  constexpr uint32_t kPh = 4 / S;  // positions per dword
  constexpr uint32_t kGp = kDenseGroupPositions<S>;  // positions per group of the loop
  bool fast_ok = true, skip_fast = false;
  uint32_t hi = 0;
  const uint32_t dk = (4 / S) * lane + 4 / S;  // largest offset of this lane in column 0
  while (h < hend) {
    if (fast_ok && !skip_fast && (h & (kPh - 1)) == 0 && h + kGp < hend) {
      uint32_t q = h, hh = h, t = 0, tlim = 0, code;
      uint32_t lv[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) lv[j] = 0;
      for (;;) {
        nb = __builtin_amdgcn_readfirstlane(nb);  // uniform (the compiler cannot tell)
        code = dense_groups<S, NC>(q, hh, t, tlim, nb, lv, lo, hi, c, hend, W, MIN, stage_lds,
                                   (uint32_t)woff[0], dk, wm, SM::P::kLive);
        if (code != kDenseFlush) break;
        flush(lo);
        lo = hi;
        nb -= 64;
        if (q + kGp >= hend) {
          code = kDenseTail;
          break;
        }
      }
      if (nb >= 64) {
        flush(lo);
        lo = hi;
        nb -= 64;
      }
      if (code == kDenseCapped) {
        h = hh;
        skip_fast = true;
      } else {
        h = t ? hh : q;
        fast_ok = false;
      }
      have_z = false;
      asm volatile("v_mov_b32 %0, %1" : "=v"(vq) : "s"(h));
      continue;
    }
    skip_fast = false;
    if (!have_z) {
      GPULZ_DENSE_COMPARE(vq);
      vq += 1;
    }
    uint32_t live[NC];
    if (h < W) {
#pragma unroll
      for (int j = 0; j < NC; ++j) live[j] = wm[j] & SM::mask_le(j, h, lane) & ~z[j];
    } else {
#pragma unroll
      for (int j = 0; j < NC; ++j) live[j] = wm[j] & ~z[j];
    }
    if (!SM::any(live)) {
      GPULZ_DENSE_REC(h << 1);  // a literal
      have_z = false;
      ++h;
      continue;
    }
    // extend through h + 1 .. h + steps while some offset still matches
    const uint32_t steps = min(kMaxMatch, c - h) - 1;
    uint32_t n = 0;
    if constexpr (NC == 1) {
      const uint32_t qb = S * (h + 1);
      extend_run<S>(live[0], n, z[0], steps, stage_lds + (qb & ~3u), qb & 3u, (uint32_t)woff[0]);
      have_z = n < steps;  // then z holds the compare of h + 1 + n: the next token's start
      vq = h + 2 + n - (have_z ? 0u : 1u);
    } else {
      have_z = false;
      for (;;) {
        if (n == steps) break;
        GPULZ_DENSE_COMPARE(vq);
        vq += 1;
        uint32_t nl[NC];
#pragma unroll
        for (int j = 0; j < NC; ++j) nl[j] = live[j] & ~z[j];
        if (!SM::any(nl)) {
          have_z = true;  // the compare of h + 1 + n: the next token's start
          break;
        }
#pragma unroll
        for (int j = 0; j < NC; ++j) live[j] = nl[j];
        ++n;
      }
    }
    uint32_t t = n + 1;
    if (t < MIN) {
      GPULZ_DENSE_REC(h << 1);
    } else {
      // the largest live offset: the highest lane with a live bit, its
      // lowest live part (each lane works out its own, one lane is read)
      uint32_t dl = 0;
      int col = -1;
#pragma unroll
      for (int j = NC - 1; j >= 0; --j) {
        if (col < 0 && ballot(live[j] != 0) != 0) col = j;
      }
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        if (j == col) {
          dl = (uint32_t)(j * SM::P::kPerCol + SM::P::K * lane + SM::P::K) -
               (uint32_t)__builtin_ctz(live[j] | 0x80000000u) / (8 * S);
        }
      }
      const uint64_t b = ballot(live[col] != 0);
      const uint32_t d = readlane(dl, 63u - (uint32_t)__builtin_clzll(b));
      if (d >= t) {
        GPULZ_DENSE_REC(1u | (t << 1) | ((d & 0xFFu) << 9));
      } else {
        // periodic run: the capped search decides, then resume at its end
        const uint32_t key = search_token<S, WC>(win, h, c, W, MIN, wmask64, lane);
        GPULZ_DENSE_REC(key ? 1u | ((key >> 9) << 1) | ((key & 0xFFu) << 9) : h << 1);
        t = key ? key >> 9 : 1u;
        asm volatile("v_mov_b32 %0, %1" : "=v"(vq) : "s"(h + t));
        have_z = false;
      }
    }
    h += t;
  }
#undef GPULZ_DENSE_COMPARE
#undef GPULZ_DENSE_REC
  dlo = lo;
  return nb;
}

// ---- single-pass output: record offsets by decoupled look-back -------------
//
// A chunk's record offset is the sum of the record sizes before it (the
// global prefix sum of section 3.2.2). Instead of a separate scan and a
// compaction pass over scratch copies of the records (Kernels II and III of
// section 3.3), each chunk publishes its size as soon as its parse ends, adds
// up its predecessors' published sizes, and writes its table entry and
// record once, at the final offset.

__device__ __forceinline__ void desc_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t desc_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Polls of one look-back before it gives up (about half a second).
constexpr uint32_t kLookbackPolls = 1u << 22;
constexpr uint32_t kNoGroup = 0xFFFFFFFFu;

// One wavefront, all lanes: publishes chunk i's record bytes `agg`, sums the
// record bytes of chunks 0..i-1 from their descriptors, 64 per round, back to
// the nearest inclusive prefix, publishes chunk i's inclusive prefix and
// returns the exclusive one (the record's offset past the table). Chunk ids
// follow the order of an atomic ticket taken when a workgroup starts, so
// every predecessor belongs to a running or finished workgroup, which
// publishes its size right after its own parse: every wait ends. As a guard
// a wait of more than kLookbackPolls polls gives up; the chunk then
// publishes and returns kDescValue ("failed"), and its successors pass it on.
__device__ inline uint64_t lookback(uint64_t* desc, uint64_t i, uint64_t agg) {
  const uint32_t lane = lane_id();
  if (i == 0) {
    if (lane == 0) desc_store(desc, kDescPrefix | agg);
    return 0;
  }
  if (lane == 0) desc_store(desc + i, kDescAgg | agg);
  uint64_t excl = 0;
  uint64_t j = i;  // chunks [0, j) not yet summed
  uint32_t polls = 0;
  bool failed = false;
  for (;;) {
    // lane l reads chunk j - 1 - l; lanes past chunk 0 read an empty prefix
    const uint64_t v = lane < j ? desc_load(desc + (j - 1 - lane)) : kDescPrefix;
    const uint32_t st = (uint32_t)(v >> 62);
    const uint64_t ready = ballot(st != 0);
    const uint64_t pref = ballot(st == 2);
    // lanes 0 .. run-1 are all published
    const uint32_t run = ready == ~0ull ? 64u : (uint32_t)__builtin_ctzll(~ready);
    const uint64_t pm = pref & (run == 64u ? ~0ull : ((1ull << run) - 1ull));
    if (pm) {
      const uint32_t pl = (uint32_t)__builtin_ctzll(pm);
      // single-chunk sizes (lanes below pl) are far below 2^32 each
      excl += readlane(wave_incl_scan(lane < pl ? (uint32_t)v : 0u), 63);
      const uint64_t pv = ((uint64_t)readlane((uint32_t)(v >> 32), pl) << 32 |
                           readlane((uint32_t)v, pl)) & kDescValue;
      failed = pv == kDescValue;
      excl += pv;
      break;
    }
    if (run) {
      excl += readlane(wave_incl_scan(lane < run ? (uint32_t)v : 0u), 63);
      j -= run;
      polls = 0;
      continue;
    }
    if (++polls > kLookbackPolls) {
      failed = true;
      break;
    }
    __builtin_amdgcn_s_sleep(4);
  }
  if (failed) excl = kDescValue;
  if (lane == 0) desc_store(desc + i, kDescPrefix | (failed ? kDescValue : excl + agg));
  return excl;
}

// The stream's last chunk, one wavefront after its look-back: the stream
// size, the status (OK, OUT_OF_SPACE, or the internal error of a failed
// look-back) and, if the stream fits, the header.
__device__ inline void finish_stream(const ChunkJob& job, uint64_t excl, uint64_t agg) {
  const uint32_t lane = lane_id();
  if (excl == kDescValue) {
    if (lane == 0) {
      *job.out_bytes = 0;
      *job.status = kInternal;
    }
    return;
  }
  const uint64_t total = kHeaderBytes + 8 * job.N + excl + agg;
  const bool fits = total <= job.capacity;
  if (lane == 0) {
    *job.out_bytes = total;
    *job.status = fits ? kOk : kOutOfSpace;
  }
  if (fits && lane < kHeaderBytes)
    job.out[lane] = stream::header_byte(lane, job.nbytes, job.S, job.C, job.W, job.MIN, job.policy,
                                        job.N, total, job.in + job.nbytes / job.S * job.S);
}

// Parse-side handling of a finished group of up to 64 tokens. Two-pass
// path: every group goes into the scratch slot. Single-pass path: groups
// before the chunk's first pointer are all literals, whose payload is the
// staged chunk itself, so nothing is written for them; from the first group
// with a pointer (g0) on, groups go into the slot as before.
template <int S, bool kSinglePass>
__device__ __forceinline__ void emit_group(uint32_t cnt, uint32_t desc, uint32_t g,
                                           const typename SymType<S>::T* win, uint8_t* slot,
                                           uint64_t flag_area, uint32_t& pay, uint32_t& g0) {
  if constexpr (kSinglePass) {
    if (g0 == kNoGroup) {
      if (ballot(lane_id() < cnt && (desc & 1u)) == 0) {
        pay += S * cnt;
        return;
      }
      g0 = g;
      // flag words are copied out of the slot from an even group on, so
      // that the copy starts 16-byte aligned: zero the one before an odd g0
      if ((g & 1u) && lane_id() == 0) *reinterpret_cast<uint64_t*>(slot + 8u * (g - 1)) = 0;
    }
  }
  encode_group<S>(cnt, desc, g, win, slot, flag_area, pay);
}

// One wavefront: the table entry and, if it ends within the capacity, the
// record of chunk job.i at offset excl past the table. Flag bytes of groups
// before g0 are zero and the rest come from the slot; payload bytes before
// group g0 (64 S per group, all literals) come from the staged chunk in LDS,
// the rest from the slot. No byte at or past the capacity is written.
template <int S>
__device__ inline void write_record(const ChunkJob& job, uint64_t excl, uint32_t F, uint32_t P,
                                    uint32_t g0, const uint8_t* stage) {
  const uint32_t lane = lane_id();
  const uint64_t te = kHeaderBytes + 8 * job.i;
  if (lane == 0 && te + 8 <= job.capacity)
    *reinterpret_cast<uint64_t*>(job.out + te) = (uint64_t)F | ((uint64_t)P << 32);
  const uint64_t base = kHeaderBytes + 8 * job.N;
  if (excl == kDescValue || base + excl + F + P > job.capacity) return;
  uint8_t* rec = job.out + base + excl;
  if (g0 != kNoGroup) {
    // the slot was written by this wavefront's lanes: complete those stores
    // and drop any cached copy before reading it back
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  const uint64_t ge = 8ull * (g0 & ~1u);
  const uint32_t fz = (uint32_t)min<uint64_t>(F, ge);
  stream::fill_zero(rec, fz, lane, 64);
  if (F > fz) stream::copy_bytes(rec + fz, job.slot + fz, F - fz, lane, 64);
  const uint32_t pz = (uint32_t)min<uint64_t>(P, 64ull * S * g0);
  stream::copy_bytes(rec + F, stage, pz, lane, 64);
  if (P > pz) stream::copy_bytes(rec + F + pz, job.slot + job.flag_area + pz, P - pz, lane, 64);
}

// encode_group writing straight into the final record `rec` (F flag bytes,
// then the payload): the group's flag bytes are stored one per lane, and only
// those below F (the payload follows them).
template <int S>
__device__ __forceinline__ void encode_group_out(uint32_t cnt, uint32_t desc, uint32_t group,
                                                 const typename SymType<S>::T* win, uint8_t* rec,
                                                 uint32_t F, uint32_t pay) {
  using T = typename SymType<S>::T;
  const uint32_t lane = lane_id();
  const bool valid = lane < cnt;
  const bool is_ptr = valid && (desc & 1u);
  const uint64_t pm = ballot(is_ptr);
  const uint64_t lm = ballot(valid && !(desc & 1u));
  const uint32_t off = pay + S * mbcnt(lm) + 2u * mbcnt(pm);
  uint8_t* dst = rec + F + off;
  if (is_ptr) {
    dst[0] = (uint8_t)(desc >> 1);
    dst[1] = (uint8_t)(desc >> 9);
  } else if (valid) {
    T v = win[desc >> 1];
#pragma unroll
    for (int b = 0; b < S; ++b) dst[b] = (uint8_t)((uint64_t)v >> (8 * b));
  }
  if (lane < 8 && 8u * group + lane < F) rec[8u * group + lane] = (uint8_t)(pm >> (8u * lane));
}

// Sparse chunks in workgroups of several waves: the exact search at a
// candidate depends on its position only, not on the parse, so the waves
// run the searches of all candidates before the parse, each over its share
// of the bitmap words, into the candidate list (positions in order, one
// sub-list per wave). All waves call this after the hit bitmap is complete;
// it returns, uniformly over the workgroup, whether every sub-list fit (else
// the parse searches as it goes). Candidates the parse later jumps over are
// searched for nothing, which is why this is for sparse chunks only.
template <int S, int WC>
__device__ bool build_list(const uint8_t* stage, const uint32_t* hits, uint32_t nhw,
                           bool sampled, const ChunkJob& job, const uint64_t (&wmask)[WC],
                           uint32_t* list, uint32_t wave, uint32_t nwaves) {
  using T = typename SymType<S>::T;
  const uint32_t lane = lane_id();
  const uint32_t c = job.c;
  uint32_t* lpos = list + wave * kListPerWave;
  uint32_t* lkey = list + kEncodeWaves * kListPerWave + wave * kListPerWave;
  uint32_t* cnt = list + 2 * kEncodeWaves * kListPerWave;
  const uint32_t nwords = (c + 31) / 32;
  const uint32_t w0 = wave * nwords / nwaves, w1 = (wave + 1) * nwords / nwaves;
  uint32_t n = 0;
  bool over = false;
  for (uint32_t wb = w0; wb < w1; wb += 64) {
    const uint32_t gw = wb + lane;
    uint32_t word = gw < w1 ? cand_word(hits, gw, nhw, sampled) : 0u;
    if (gw * 32u + 32u > c) word &= gw * 32u >= c ? 0u : (1u << (c - gw * 32u)) - 1u;
    const uint32_t pc = (uint32_t)__popc(word);
    const uint32_t incl = wave_incl_scan(pc);
    const uint32_t tot = readlane(incl, 63);
    if (n + tot > kListPerWave) {
      over = true;
      break;
    }
    uint32_t o = n + incl - pc;
    while (word) {
      lpos[o++] = gw * 32u + (uint32_t)__ffs(word) - 1u;
      word &= word - 1u;
    }
    n += tot;
  }
  wave_sync();
  if (lane == 0) cnt[wave] = over ? ~0u : n;
  if (!over) {
    const T* win = reinterpret_cast<const T*>(stage);
    StreamMatchFor<S, WC> sm;
    sm.init(stage, job.W, lane);
    for (uint32_t i = 0; i < n; ++i) {
      const uint32_t h = __builtin_amdgcn_readfirstlane(lpos[i]);
      const uint32_t key = find_token<S, WC>(sm, win, h, c, job.W, job.MIN, wmask, lane);
      if (lane == 0) lkey[i] = key;
    }
  }
  __syncthreads();
  bool ok = true;
  for (uint32_t w = 0; w < nwaves; ++w) ok &= cnt[w] != ~0u;
  return ok;
}

// Encodes one chunk. Every wave of the workgroup stages the chunk and builds
// the hit bitmap; waves other than 0 return after that, wave 0 parses and
// encodes.
//   two-pass path (kSinglePass false): the record goes to the chunk's
//     scratch slot and {F, P} to job.sizes, for a later scan and compaction;
//   single-pass path: groups from the first pointer on go to the slot, then
//     wave 0 takes the record offset from the look-back and writes the table
//     entry and the record into the stream (and the header, size and status
//     if this is the stream's last chunk).
template <int S, int WC, bool kSinglePass = false>
__device__ void encode_chunk(const ChunkJob& job, uint8_t* lds) {
  using T = typename SymType<S>::T;
  constexpr int V = Geo<S>::V;
  constexpr uint32_t kBlock = Geo<S>::kBlock;
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = lane_id();
  const uint32_t wave = tid >> 6;
  const uint32_t nwaves = blockDim.x >> 6;
  const uint32_t c = job.c;
  uint8_t* stage = lds + pad_bytes<S, WC>();
  uint32_t* hits = reinterpret_cast<uint32_t*>(stage + chunk_lds_bytes(job.C, S));
  const uint32_t nhw = (uint32_t)hit_words(job.C, S);

  // ---- stage: HBM -> LDS with 16-byte loads
  stage_chunk<S>(job, stage);
  for (uint32_t k = tid; k < nhw; k += blockDim.x) hits[k] = 0;
  __syncthreads();

  // ---- hits: all waves, one block of 64 * V positions at a time. With
  // MIN >= 2 only even positions are tested: a pointer (length >= MIN)
  // starting at p covers an even position p' in {p, p + 1}, and p' matches
  // at the pointer's offset, which is at most min(W, p'). So p can start a
  // pointer only if p or p + 1 is an even hit; the parse widens the bitmap
  // accordingly (candidates are a superset of pointer starts, and every
  // candidate still gets the exact search).
  //
  // Dense chunks (streaming search, one wave per chunk): the streaming
  // search compares every position it passes anyway, at a fixed cost per
  // position, while the per-candidate search costs several times that, so
  // the bitmap only pays where candidates are rare. If at least 1/4 of the
  // tested positions of the first block are hits, the rest of the bitmap is
  // not built and every position is a candidate.
  const bool sampled = job.MIN >= 2;
  bool dense = false;
  {
    const uint4* w4 = reinterpret_cast<const uint4*>(stage);
    const uint32_t nblocks = (c + kBlock - 1) / kBlock;
    uint32_t b0 = wave;
    if constexpr (kStreamSearch<S>) {
      if (nwaves == 1 && nblocks > 1) {
        if (sampled) hit_block<S, true, 2>(w4, 0, job.W, hits);
        else hit_block<S, true, 1>(w4, 0, job.W, hits);
        wave_sync();
        constexpr uint32_t kWords = kBlock / 32;
        const uint32_t cnt = lane < kWords ? (uint32_t)__popc(hits[lane]) : 0u;
        const uint32_t tested = sampled ? kBlock / 2 : kBlock;
        dense = 4 * readlane(wave_incl_scan(cnt), 63) >= tested;
        b0 = dense ? nblocks : 1;
      }
    }
    build_hits<S, WC>(stage, b0, nblocks, nwaves, job.W, c, sampled, hits);
  }
  __syncthreads();
  const T* win = reinterpret_cast<const T*>(stage);
  uint64_t wmask[WC];
#pragma unroll
  for (int col = 0; col < WC; ++col) wmask[col] = ballot(64u * col + lane + 1u <= job.W);
  // the candidate list is taken for 4- and 8-byte symbols (1- and 2-byte
  // chunks with sparse candidates are rare and keep the search in the parse)
  uint32_t* list = hits + nhw;
  bool listed = false;
  if constexpr (S >= 4)
    listed = nwaves > 1 && build_list<S, WC>(stage, hits, nhw, sampled, job, wmask, list, wave,
                                             nwaves);
  if (wave != 0) return;

  // ---- parse + encode: wave 0

  uint8_t* slot = job.slot;
  uint32_t ntok = 0, pay = 0, desc = 0, g0 = kNoGroup;
  uint32_t p = 0;
  if constexpr (kStreamSearch<S>) {
    if (dense && job.MIN <= 2) {
      const uint32_t rest = parse_dense<S, WC>(stage, 0, c, c, job.W, job.MIN, wmask, lane,
                                               desc, [&](uint32_t d64) {
        emit_group<S, kSinglePass>(64, d64, ntok >> 6, win, slot, job.flag_area, pay, g0);
        ntok += 64;
      });
      ntok += rest;
      p = c;
    }
  }
  CandCursor cc;
  ListCursor lc;
  if (listed) lc.init(list, nwaves);
  else cc.init(hits, nhw, sampled);
  StreamMatchFor<S, WC> sm;
  sm.init(stage, job.W, lane);
  while (p < c) {
    uint32_t lkey = 0;
    const uint32_t h = listed ? lc.next(p, c, lkey) : cc.next(p, c, hits, nhw, sampled);
    // literals for [p, h); on the single-pass path, whole all-literal groups
    // before the first pointer are only counted
    if constexpr (kSinglePass) {
      if (g0 == kNoGroup && (ntok & 63u) == 0 && h - p >= 64) {
        const uint32_t k = (h - p) / 64;
        ntok += 64 * k;
        p += 64 * k;
        pay += 64 * S * k;
      }
    }
    while (p < h) {
      const uint32_t sl = ntok & 63u;
      const uint32_t take = min(h - p, 64u - sl);
      if (lane >= sl && lane < sl + take) desc = (p + lane - sl) << 1;
      ntok += take;
      p += take;
      if ((ntok & 63u) == 0)
        emit_group<S, kSinglePass>(64, desc, (ntok >> 6) - 1, win, slot, job.flag_area, pay, g0);
    }
    if (h >= c) break;

    const uint32_t key =
        listed ? lkey : find_token<S, WC>(sm, win, h, c, job.W, job.MIN, wmask, lane);
    uint32_t val;
    if (key) {
      val = 1u | ((key >> 9) << 1) | ((key & 0xFFu) << 9);
      p = h + (key >> 9);
    } else {
      val = h << 1;
      p = h + 1;
    }
    if (lane == (ntok & 63u)) desc = val;
    ++ntok;
    if ((ntok & 63u) == 0)
      emit_group<S, kSinglePass>(64, desc, (ntok >> 6) - 1, win, slot, job.flag_area, pay, g0);
  }
  if (ntok & 63u)
    emit_group<S, kSinglePass>(ntok & 63u, desc, ntok >> 6, win, slot, job.flag_area, pay, g0);
  const uint32_t F = (ntok + 7) / 8;
  if constexpr (kSinglePass) {
    const uint64_t excl = lookback(job.desc, job.i, (uint64_t)F + pay);
    if (job.i + 1 == job.N) finish_stream(job, excl, (uint64_t)F + pay);
    write_record<S>(job, excl, F, pay, g0, stage);
  } else {
    if (lane == 0) {
      job.sizes[0] = F;
      job.sizes[1] = pay;
    }
  }
}

// ---- the same parse with the chunk split across waves ---------------------

constexpr uint32_t kSpecWaves = 16;      // waves of the split-parse encoder
constexpr uint32_t kSpecMaxSyms = 4096;  // chunks it takes (16-bit positions)

__host__ __device__ constexpr uint64_t spec_bitmap_words(uint32_t C) { return (C + 31) / 32 + 2; }
// LDS: [pad | chunk | hit bitmap | token starts | pointer starts | the same
// two for the extensions | (L, d) per position | prefix counts of the token
// and pointer bitmaps | segment ends | meeting points]
template <int S, int WC>
__host__ __device__ constexpr uint64_t spec_lds_bytes(uint32_t C) {
  return encode_lds(C, S, WC, 1) + 4 * 4 * spec_bitmap_words(C) + align_up(2ull * C, 16) +
         2 * 4 * (spec_bitmap_words(C) + 1) + 2 * 4 * kSpecWaves;
}

// Sets (or clears) bits [a, b) of an LDS bitmap; all lanes of the wave.
__device__ __forceinline__ void bits_range(uint32_t* bm, uint32_t a, uint32_t b, bool set) {
  if (a >= b) return;
  const uint32_t w0 = a >> 5, w1 = (b - 1) >> 5;
  for (uint32_t w = w0 + lane_id(); w <= w1; w += 64) {
    uint32_t m = ~0u;
    if (w == w0) m &= ~0u << (a & 31u);
    if (w == w1) m &= ~0u >> (31u - ((b - 1) & 31u));
    if (set) atomicOr(&bm[w], m);
    else atomicAnd(&bm[w], ~m);
  }
}

// Encodes one chunk like encode_chunk's single-pass path (the same stream),
// with the greedy parse split across the workgroup's waves for latency: wave w parses its
// segment [w seg, (w + 1) seg) as if a token started at its first position,
// recording token starts, pointer starts and (L, d) per pointer. The greedy
// parse is deterministic, so once the true parse reaches a position where a
// segment's parse has a token start, the two agree from there on. Each wave
// then extends its parse into the next segment until it lands on one of that
// segment's starts, and wave 0 joins the segments: where the true parse leaves
// a segment at that segment's own end, the extension is spliced in; otherwise
// wave 0 walks the boundary token by token until the parses meet. Every wave
// then encodes 64-token groups independently, straight into the record at
// the offset the look-back gives: a token's position comes from prefix counts
// of the token bitmap, a group's payload offset from the pointers before it.
template <int S, int WC>
__device__ void encode_chunk_spec(const ChunkJob& job, uint8_t* lds) {
  using T = typename SymType<S>::T;
  constexpr uint32_t kBlock = Geo<S>::kBlock;
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = lane_id();
  const uint32_t wave = tid >> 6;
  const uint32_t nwaves = blockDim.x >> 6;
  const uint32_t c = job.c;
  uint8_t* stage = lds + pad_bytes<S, WC>();
  uint32_t* hits = reinterpret_cast<uint32_t*>(stage + chunk_lds_bytes(job.C, S));
  const uint32_t nhw = (uint32_t)hit_words(job.C, S);
  const uint32_t tw = (uint32_t)spec_bitmap_words(job.C);
  uint32_t* tok = hits + nhw;
  uint32_t* ptr = tok + tw;
  uint32_t* xtok = ptr + tw;  // extension parses
  uint32_t* xptr = xtok + tw;
  uint16_t* tinfo = reinterpret_cast<uint16_t*>(xptr + tw);
  uint32_t* pc_tok = reinterpret_cast<uint32_t*>(tinfo + align_up(job.C, 8));
  uint32_t* pc_ptr = pc_tok + tw + 1;
  uint32_t* ends = pc_ptr + tw + 1;
  uint32_t* meet = ends + kSpecWaves;

  stage_chunk<S>(job, stage);
  for (uint32_t k = tid; k < nhw; k += blockDim.x) hits[k] = 0;
  for (uint32_t k = tid; k < 4 * tw; k += blockDim.x) tok[k] = 0;
  __syncthreads();
  const bool sampled = job.MIN >= 2;
  const uint32_t nblocks = (c + kBlock - 1) / kBlock;
  if constexpr (Geo<S>::R == 1) {
    // fewer blocks than waves: the waves of one block split its window
    // offsets (steps [kb, ke) each) and OR their hits into the bitmap
    constexpr uint32_t V = Geo<S>::V;
    const uint32_t nsplit = min(8u, max(1u, nwaves / max(1u, nblocks)));
    const uint32_t kmax = job.W / V + (job.W % V ? 1u : 0u);
    const uint4* w4 = reinterpret_cast<const uint4*>(stage);
    for (uint32_t u = wave; u < nblocks * nsplit; u += nwaves) {
      const uint32_t b = u / nsplit, part = u % nsplit;
      const uint32_t kb = 1 + part * kmax / nsplit, ke = 1 + (part + 1) * kmax / nsplit;
      if (kb >= ke) continue;
      const uint32_t base = b * kBlock;
      if (sampled) {
        if (base >= job.W) hit_block<S, false, 2>(w4, base, job.W, hits, kb, ke);
        else hit_block<S, true, 2>(w4, base, job.W, hits, kb, ke);
      } else {
        if (base >= job.W) hit_block<S, false, 1>(w4, base, job.W, hits, kb, ke);
        else hit_block<S, true, 1>(w4, base, job.W, hits, kb, ke);
      }
    }
  } else {
    build_hits<S, WC>(stage, wave, nblocks, nwaves, job.W, c, sampled, hits);
  }
  __syncthreads();
  // match-dense chunks (1- and 2-byte symbols, MIN <= 2): at least 1/4 of the
  // tested positions hit; their segments take the streaming parse
  bool dense = false;
  if constexpr (kStreamSearch<S>) {
    if (job.MIN <= 2) {
      if (wave == 0) {
        uint32_t cnt = 0;
        for (uint32_t k = lane; k < (c + 31) / 32; k += 64) {
          uint32_t wd = hits[k];
          if (32 * k + 32 > c) wd &= (1u << (c - 32 * k)) - 1u;
          cnt += (uint32_t)__popc(wd);
        }
        cnt = readlane(wave_incl_scan(cnt), 63);
        const uint32_t tested = sampled ? (c + 1) / 2 : c;
        if (lane == 0) pc_tok[0] = 4 * cnt >= tested;
      }
      __syncthreads();
      dense = pc_tok[0] != 0;
    }
  }

  const T* win = reinterpret_cast<const T*>(stage);
  uint64_t wmask[WC];
#pragma unroll
  for (int col = 0; col < WC; ++col) wmask[col] = ballot(64u * col + lane + 1u <= job.W);
  const uint32_t seg = (c + nwaves - 1) / nwaves;
  StreamMatchFor<S, WC> sm;
  sm.init(stage, job.W, lane);

  // ---- each wave: the greedy parse of its own segment
  if constexpr (kStreamSearch<S>) {
    if (dense) {
      // the streaming parse of the segment; each group of token descriptors
      // becomes token and pointer bits and (L, d) at the tokens' positions
      // (a token's position: the segment start plus the lengths before it)
      const uint32_t s0 = min(c, wave * seg), s1 = min(c, s0 + seg);
      uint32_t gpos = s0, dlo = 0;
      auto mark = [&](uint32_t d, uint32_t cnt) {
        const bool v = lane < cnt;
        const bool isp = v && (d & 1u);
        const uint32_t len = !v ? 0u : (isp ? (d >> 1) & 0xFFu : 1u);
        const uint32_t incl = wave_incl_scan(len);
        const uint32_t pos = gpos + incl - len;
        if (v) atomicOr(&tok[pos >> 5], 1u << (pos & 31u));
        if (isp) {
          atomicOr(&ptr[pos >> 5], 1u << (pos & 31u));
          tinfo[pos] = (uint16_t)((((d >> 1) & 0xFFu) << 8) | ((d >> 9) & 0xFFu));
        }
        gpos += readlane(incl, 63);
      };
      const uint32_t rest = parse_dense<S, WC>(stage, s0, s1, c, job.W, job.MIN, wmask, lane, dlo,
                                               [&](uint32_t d64) { mark(d64, 64); });
      mark(dlo, rest);
      if (lane == 0) ends[wave] = gpos;
    }
  }
  if (!dense) {
    const uint32_t s0 = min(c, wave * seg), s1 = min(c, s0 + seg);
    uint32_t p = s0;
    CandCursor cc;
    cc.init(hits, nhw, sampled);
    while (p < s1) {
      const uint32_t h = cc.next(p, c, hits, nhw, sampled);
      if (h > p) {  // literals up to the next candidate
        const uint32_t e = min(h, s1);
        bits_range(tok, p, e, true);
        p = e;
        continue;
      }
      const uint32_t key = find_token<S, WC>(sm, win, p, c, job.W, job.MIN, wmask, lane);
      if (lane == 0) {
        atomicOr(&tok[p >> 5], 1u << (p & 31u));
        if (key) {
          atomicOr(&ptr[p >> 5], 1u << (p & 31u));
          tinfo[p] = (uint16_t)((key >> 9) << 8 | (key & 0xFFu));
        }
      }
      p += key ? key >> 9 : 1u;
    }
    if (lane == 0) ends[wave] = p;
  }
  __syncthreads();

  // ---- each wave: extend its parse into the next segment until it lands on
  // a start of that segment's own parse (recorded in the extension bitmaps;
  // the (L, d) of a position does not depend on which parse reached it)
  if (wave + 1 < nwaves && (wave + 1) * seg < c) {
    const uint32_t n0 = (wave + 1) * seg, n1 = min(c, n0 + seg);
    uint32_t q = ends[wave];
    CandCursor cc;
    cc.init(hits, nhw, sampled);
    while (q < n1 && !((tok[q >> 5] >> (q & 31u)) & 1u)) {
      const uint32_t h = cc.next(q, c, hits, nhw, sampled);
      uint32_t key = 0;
      if (h == q) key = find_token<S, WC>(sm, win, q, c, job.W, job.MIN, wmask, lane);
      if (lane == 0) {
        atomicOr(&xtok[q >> 5], 1u << (q & 31u));
        if (key) {
          atomicOr(&xptr[q >> 5], 1u << (q & 31u));
          tinfo[q] = (uint16_t)((key >> 9) << 8 | (key & 0xFFu));
        }
      }
      q += key ? key >> 9 : 1u;
    }
    if (lane == 0) meet[wave] = q;
  }
  __syncthreads();

  // ---- wave 0: join the segments. Where the true parse leaves segment w - 1
  // at that segment's own end, wave w - 1's extension is its continuation:
  // splice it in over [w seg, meeting point). Otherwise walk the boundary
  // token by token (dropping segment w's starts it covers) until it lands on
  // one of segment w's starts.
  if (wave == 0) {
    uint32_t q = ends[0];
    CandCursor cc;
    cc.init(hits, nhw, sampled);
    for (uint32_t w = 1; w < nwaves; ++w) {
      const uint32_t s0 = w * seg;
      if (s0 >= c) break;
      const uint32_t s1 = min(c, s0 + seg);
      if (q == ends[w - 1]) {
        const uint32_t m = meet[w - 1], e = min(m, s1);
        if (s0 < e) {
          const uint32_t w0 = s0 >> 5, w1 = (e - 1) >> 5;
          for (uint32_t k = w0 + lane; k <= w1; k += 64) {
            uint32_t msk = ~0u;
            if (k == w0) msk &= ~0u << (s0 & 31u);
            if (k == w1) msk &= ~0u >> (31u - ((e - 1) & 31u));
            tok[k] = (tok[k] & ~msk) | (xtok[k] & msk);
            ptr[k] = (ptr[k] & ~msk) | (xptr[k] & msk);
          }
        }
        wave_sync();
        q = m < s1 ? ends[w] : m;
        continue;
      }
      // segment w's starts before q lie inside tokens of the true parse
      bits_range(tok, s0, min(q, s1), false);
      bits_range(ptr, s0, min(q, s1), false);
      wave_sync();
      while (q < s1 && !((tok[q >> 5] >> (q & 31u)) & 1u)) {
        const uint32_t h = cc.next(q, c, hits, nhw, sampled);
        uint32_t key = 0;
        if (h == q) key = find_token<S, WC>(sm, win, q, c, job.W, job.MIN, wmask, lane);
        const uint32_t L = key ? key >> 9 : 1u;
        if (lane == 0) {
          atomicOr(&tok[q >> 5], 1u << (q & 31u));
          if (key) {
            atomicOr(&ptr[q >> 5], 1u << (q & 31u));
            tinfo[q] = (uint16_t)((key >> 9) << 8 | (key & 0xFFu));
          }
        }
        wave_sync();
        bits_range(tok, q + 1, min(q + L, s1), false);
        bits_range(ptr, q + 1, min(q + L, s1), false);
        wave_sync();
        q += L;
      }
      if (q < s1) q = ends[w];  // met segment w's parse: it is the true one from here
    }
  }
  __syncthreads();

  // ---- prefix counts of both bitmaps (wave 0), then the groups (all waves)
  const uint32_t nbw = (c + 31) / 32;
  if (wave == 0) {
    uint32_t run_t = 0, run_p = 0;
    for (uint32_t base = 0; base < nbw; base += 64) {
      const uint32_t w = base + lane;
      const uint32_t ct = w < nbw ? (uint32_t)__popc(tok[w]) : 0u;
      const uint32_t cp = w < nbw ? (uint32_t)__popc(ptr[w]) : 0u;
      const uint32_t it = wave_incl_scan(ct), ip = wave_incl_scan(cp);
      if (w < nbw) {
        pc_tok[w] = run_t + it - ct;
        pc_ptr[w] = run_p + ip - cp;
      }
      run_t += readlane(it, 63);
      run_p += readlane(ip, 63);
    }
    if (lane == 0) {
      pc_tok[nbw] = run_t;
      pc_ptr[nbw] = run_p;
    }
  }
  __syncthreads();
  const uint32_t ntok = pc_tok[nbw], nptr = pc_ptr[nbw];
  const uint32_t F = (ntok + 7) / 8, P = S * (ntok - nptr) + 2 * nptr;
  // ---- record offset (wave 0: look-back), then every wave writes its
  // groups straight into the record (the join's `ends` words are free now)
  if (wave == 0) {
    const uint64_t excl = lookback(job.desc, job.i, (uint64_t)F + P);
    if (job.i + 1 == job.N) finish_stream(job, excl, (uint64_t)F + P);
    const uint64_t te = kHeaderBytes + 8 * job.i;
    if (lane == 0) {
      if (te + 8 <= job.capacity)
        *reinterpret_cast<uint64_t*>(job.out + te) = (uint64_t)F | ((uint64_t)P << 32);
      ends[0] = (uint32_t)excl;
      ends[1] = (uint32_t)(excl >> 32);
    }
  }
  __syncthreads();
  const uint64_t excl = (uint64_t)ends[0] | ((uint64_t)ends[1] << 32);
  const uint64_t rec_off = kHeaderBytes + 8 * job.N + excl;
  if (excl == kDescValue || rec_off + F + P > job.capacity) return;
  uint8_t* rec = job.out + rec_off;
  const uint32_t groups = (ntok + 63) / 64;
  for (uint32_t g = wave; g < groups; g += nwaves) {
    const uint32_t r = 64 * g + lane;  // this lane's token rank
    uint32_t p = 0;
    if (r < ntok) {
      // the word holding it: the last word whose prefix count is <= r
      uint32_t lo = 0, hi = nbw - 1;
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) / 2;
        if (pc_tok[mid] <= r) lo = mid;
        else hi = mid - 1;
      }
      uint32_t m = tok[lo], k = r - pc_tok[lo], bit = 0;
#pragma unroll
      for (uint32_t width = 16; width >= 1; width >>= 1) {
        const uint32_t lowc = (uint32_t)__popc(m & ((1u << width) - 1u));
        if (k >= lowc) {
          k -= lowc;
          m >>= width;
          bit += width;
        }
      }
      p = 32 * lo + bit;
    }
    uint32_t desc = p << 1;
    if (r < ntok && ((ptr[p >> 5] >> (p & 31u)) & 1u)) {
      const uint32_t ti = tinfo[p];
      desc = 1u | ((ti >> 8) << 1) | ((ti & 0xFFu) << 9);
    }
    // payload before the group: S per literal and 2 per pointer among its
    // first 64 g tokens
    const uint32_t p0 = readlane(p, 0);
    const uint32_t before_ptr = pc_ptr[p0 >> 5] + (uint32_t)__popc(ptr[p0 >> 5] & ((1u << (p0 & 31u)) - 1u));
    const uint32_t pay = S * (64 * g - before_ptr) + 2 * before_ptr;
    encode_group_out<S>(min(64u, ntok - 64 * g), desc, g, win, rec, F, pay);
  }
}

// ---- match policy 1: the paper's single window pass ----------------------

// LDS of one policy-1 chunk encoder: chunk | lengths (u8) | offsets - 1 (u8)
// | candidate bitmap.
__host__ __device__ constexpr uint64_t scan_lds_bytes(uint32_t C, uint32_t S) {
  return chunk_lds_bytes(C, S) + 2 * align_up(C, 16) + 4 * hit_words(C, S);
}

// Encodes one chunk with match policy 1 (section 3.3.2, matching steps 1-4,
// Kernel I): every position gets the result of its own single pass over
// the window, one position per lane (the walk takes min(W, p) steps at
// every position, so the lanes stay in step), stored as a length / offset
// table; positions whose length reaches MIN form the candidate bitmap. Wave
// 0 then parses greedily as on the exact path, taking each pointer from the
// table. Per position: a window pointer w walks once from the oldest slot
// toward p and a look-ahead pointer b from p; equal symbols extend the
// open run (its offset is p - w at its first symbol); at a mismatch, or
// once the run has 255 symbols, the run replaces the best one if strictly
// longer, b returns to p, and w moves on; the walk ends when w reaches p or
// b the chunk end, and the open run is compared once more.
template <int S>
__device__ void encode_chunk_scan(const ChunkJob& job, uint8_t* lds) {
  using T = typename SymType<S>::T;
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = lane_id();
  const uint32_t wave = tid >> 6;
  const uint32_t nwaves = blockDim.x >> 6;
  const uint32_t c = job.c;
  uint8_t* stage = lds;
  uint8_t* Ltab = stage + chunk_lds_bytes(job.C, S);
  uint8_t* Dtab = Ltab + align_up(job.C, 16);
  uint32_t* hits = reinterpret_cast<uint32_t*>(Dtab + align_up(job.C, 16));
  const uint32_t nhw = (uint32_t)hit_words(job.C, S);

  stage_chunk<S>(job, stage);
  for (uint32_t k = tid; k < nhw; k += blockDim.x) hits[k] = 0;
  __syncthreads();
  const T* win = reinterpret_cast<const T*>(stage);

  // ---- per-position walks, 64 consecutive positions per wave
  for (uint32_t base = 64 * wave; base < c; base += 64 * nwaves) {
    const uint32_t p = base + lane;
    uint32_t bestL = 0, bestd = 0;
    if (p < c) {
      uint32_t w = p > job.W ? p - job.W : 0, b = p, len = 0, off = 0;
      while (w < p && b < c) {
        const bool eq = (len < kMaxMatch) & (win[b] == win[w]);
        off = (eq & (len == 0)) ? p - w : off;
        const bool better = !eq & (len > bestL);
        bestL = better ? len : bestL;
        bestd = better ? off : bestd;
        len = eq ? len + 1 : 0u;
        b = eq ? b + 1 : p;
        ++w;
      }
      if (len > bestL) {
        bestL = len;
        bestd = off;
      }
      Ltab[p] = (uint8_t)bestL;
      Dtab[p] = (uint8_t)(bestd - 1);
    }
    const uint64_t m = ballot(p < c && bestL >= job.MIN);
    if (lane == 0) {
      hits[base >> 5] = (uint32_t)m;
      hits[(base >> 5) + 1] = (uint32_t)(m >> 32);
    }
  }
  __syncthreads();
  if (wave != 0) return;

  // ---- greedy parse + encode (wave 0): candidates are exactly the
  // positions whose walk found a run of at least MIN symbols; groups from the
  // first pointer on go to the slot, then the record goes out at the offset
  // the look-back gives (as encode_chunk's single-pass path)
  uint8_t* slot = job.slot;
  uint32_t ntok = 0, pay = 0, desc = 0, g0 = kNoGroup;
  uint32_t p = 0;
  CandCursor cc;
  cc.init(hits, nhw, false);
  while (p < c) {
    const uint32_t h = cc.next(p, c, hits, nhw, false);
    if (g0 == kNoGroup && (ntok & 63u) == 0 && h - p >= 64) {
      const uint32_t k = (h - p) / 64;
      ntok += 64 * k;
      p += 64 * k;
      pay += 64 * S * k;
    }
    while (p < h) {
      const uint32_t sl = ntok & 63u;
      const uint32_t take = min(h - p, 64u - sl);
      if (lane >= sl && lane < sl + take) desc = (p + lane - sl) << 1;
      ntok += take;
      p += take;
      if ((ntok & 63u) == 0)
        emit_group<S, true>(64, desc, (ntok >> 6) - 1, win, slot, job.flag_area, pay, g0);
    }
    if (h >= c) break;
    const uint32_t L = Ltab[h], d = (uint32_t)Dtab[h] + 1u;
    if (lane == (ntok & 63u)) desc = 1u | (L << 1) | ((d & 0xFFu) << 9);
    ++ntok;
    if ((ntok & 63u) == 0)
      emit_group<S, true>(64, desc, (ntok >> 6) - 1, win, slot, job.flag_area, pay, g0);
    p = h + L;
  }
  if (ntok & 63u) emit_group<S, true>(ntok & 63u, desc, ntok >> 6, win, slot, job.flag_area, pay, g0);
  const uint32_t F = (ntok + 7) / 8;
  const uint64_t excl = lookback(job.desc, job.i, (uint64_t)F + pay);
  if (job.i + 1 == job.N) finish_stream(job, excl, (uint64_t)F + pay);
  write_record<S>(job, excl, F, pay, g0, stage);
}

template <int S, int WC>
__host__ __device__ constexpr size_t lds_bytes(uint32_t C, uint32_t waves) {
  return encode_lds(C, S, WC, waves);
}

}  // namespace enc
}  // namespace gpulz
