// Entropy stage after LZSS (gpuLZ section 4.5 pairs LZSS with a Huffman
// coder): byte Huffman coding in chunks that decode in parallel. The rules of
// the code and of the stream are in huff_internal.h and gpulz.h.
//
// Compression, five launches on one stream, no host round trip:
//   hist_kernel    per-workgroup byte histograms (32 bank-padded LDS
//                  sub-histograms, 16-byte loads);
//   build_kernel   one workgroup: sums the histograms, sorts (weight,
//                  symbol) keys, runs Huffman's merge with two queues (sorted
//                  leaves, internal nodes in creation order), limits the
//                  lengths, assigns canonical codes, writes the code lengths;
//   size_kernel    one wave per chunk: code bits of the chunk;
//   scan_kernel    one workgroup: record offsets and the header;
//   encode_kernel  one wave per chunk: bit offsets by a wave scan, codes
//                  ORed into LDS words, the record written once.
// Decompression:
//   dec_prepare_kernel  one workgroup: checks the header and the code,
//                       builds the lookup tables, scans the record sizes;
//   decode_kernel       one lane per 128-symbol sub-block (32 lanes per
//                       chunk): code words staged in LDS, a two-level
//                       lookup table in LDS, symbols staged in LDS and
//                       written out in consecutive 4-byte stores.
#include "huff_internal.h"
#include "stream_device.h"
#include "wave.h"

namespace gpulz {
namespace huff {
namespace {

__device__ inline uint64_t input_size(const EncArgs& a) { return a.d_n ? *a.d_n : a.max_n; }

__device__ inline uint32_t byte_of(const uint4& q, uint32_t b) {
  const uint32_t w = b < 8 ? (b < 4 ? q.x : q.y) : (b < 12 ? q.z : q.w);
  return (w >> (8 * (b & 3))) & 0xFFu;
}

// ---- compression -----------------------------------------------------------

// 32 sub-histograms per workgroup, one per lane of a half-wave (lanes l and
// l + 32 share one), each padded by a word so that the copies of one byte
// value fall in different LDS banks: a skewed input (most bytes equal) then
// costs two-way same-address atomics instead of 64-way ones.
constexpr uint32_t kHistCopies = 32;
constexpr uint32_t kHistStride = 257;

__global__ __launch_bounds__(256) void hist_kernel(EncArgs a) {
  __shared__ uint32_t h[kHistCopies * kHistStride];
  const uint32_t tid = threadIdx.x;
  for (uint32_t k = tid; k < kHistCopies * kHistStride; k += 256) h[k] = 0;
  __syncthreads();
  uint32_t* mine = h + (tid & (kHistCopies - 1)) * kHistStride;
  const uint64_t n = input_size(a);
  if (n <= a.max_n) {
    const uint64_t words = (n + 15) / 16;
    const uint64_t per = (words + gridDim.x - 1) / gridDim.x;
    const uint64_t w0 = (uint64_t)blockIdx.x * per;
    const uint64_t w1 = w0 + per < words ? w0 + per : words;
    const uint4* in4 = reinterpret_cast<const uint4*>(a.in);
    const uint64_t wfull = n / 16;  // whole 16-byte words
    uint64_t w = w0 + tid;
    // four loads in flight per thread, then their 64 bytes counted
    for (; w + 3 * 256 < w1 && w + 3 * 256 < wfull; w += 4 * 256) {
      uint4 q[4];
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u) q[u] = in4[w + u * 256];
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u)
#pragma unroll
        for (uint32_t b = 0; b < 16; ++b) atomicAdd(&mine[byte_of(q[u], b)], 1u);
    }
    for (; w < w1; w += 256) {
      if (16 * w + 16 <= n) {
        const uint4 q = in4[w];
#pragma unroll
        for (uint32_t b = 0; b < 16; ++b) atomicAdd(&mine[byte_of(q, b)], 1u);
      } else {
        for (uint64_t b = 16 * w; b < n; ++b) atomicAdd(&mine[a.in[b]], 1u);
      }
    }
  }
  __syncthreads();
  uint32_t sum = 0;
#pragma unroll 8
  for (uint32_t c = 0; c < kHistCopies; ++c) sum += h[c * kHistStride + tid];
  a.partial[(uint64_t)blockIdx.x * 256 + tid] = sum;
}

struct BuildLds {
  uint64_t w[256];    // weight by symbol (0 = absent)
  uint64_t tmp[256];  // unsorted keys
  uint64_t key[256];  // weight << 8 | symbol, ascending; absent symbols last
  uint64_t iw[256];   // internal node weights in creation order
  uint16_t parent[512];
  uint16_t anc[256], dist[256];  // pointer jumping over internal nodes
  uint8_t len[256];
  uint32_t count[16], next[16];
  uint64_t total;       // sum of the weights
  uint32_t present, deepest, internal;
};

// Huffman's merge with two queues: sorted leaves, and internal nodes in
// creation order (their weights never decrease). A leaf wins a tie (its index
// is smaller). The four front candidates are read together, so each join
// costs one LDS round trip. W is uint32_t when the weights sum below 2^31
// (cheaper compares; used below 2^31 so that no weight equals the 32-bit
// infinity), else uint64_t. Returns the number of internal nodes.
template <typename W>
__device__ uint32_t merge(BuildLds& sm, uint32_t m) {
  const W kInf = (W)~0ull;
  uint32_t li = 0, kf = 0, kc = 0;
  for (uint32_t s = 0; s + 1 < m; ++s) {
    const W l0 = li < m ? (W)(sm.key[li] >> 8) : kInf;
    const W l1 = li + 1 < m ? (W)(sm.key[li + 1] >> 8) : kInf;
    const W i0 = kf < kc ? (W)sm.iw[kf] : kInf;
    const W i1 = kf + 1 < kc ? (W)sm.iw[kf + 1] : kInf;
    uint32_t na, nb;
    W wa, wb;
    if (l0 <= i0) {
      na = li;
      wa = l0;
      if (l1 <= i0) {
        nb = li + 1;
        wb = l1;
        li += 2;
      } else {
        nb = 256 + kf;
        wb = i0;
        li += 1;
        kf += 1;
      }
    } else {
      na = 256 + kf;
      wa = i0;
      if (l0 <= i1) {
        nb = li;
        wb = l0;
        li += 1;
        kf += 1;
      } else {
        nb = 256 + kf + 1;
        wb = i1;
        kf += 2;
      }
    }
    sm.iw[kc] = (uint64_t)wa + wb;
    sm.parent[na] = (uint16_t)(256 + kc);
    sm.parent[nb] = (uint16_t)(256 + kc);
    ++kc;
  }
  return kc;
}

__global__ __launch_bounds__(1024) void build_kernel(EncArgs a) {
  __shared__ BuildLds sm;
  const uint32_t tid = threadIdx.x;
  if (input_size(a) > a.max_n) return;
  if (tid < 256) sm.w[tid] = 0;
  if (tid == 0) sm.present = 0;
  __syncthreads();
  {
    // partial histograms: 64 column groups of 4 bins x 16 row groups, 16-byte
    // loads, several in flight per thread
    const uint32_t cg = tid & 63u;
    uint64_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    const uint4* p4 = reinterpret_cast<const uint4*>(a.partial);
#pragma unroll 8
    for (uint32_t r = tid >> 6; r < a.hist_blocks; r += 16) {
      const uint4 v = p4[(uint64_t)r * 64 + cg];
      s0 += v.x;
      s1 += v.y;
      s2 += v.z;
      s3 += v.w;
    }
    atomicAdd(reinterpret_cast<unsigned long long*>(&sm.w[4 * cg]), (unsigned long long)s0);
    atomicAdd(reinterpret_cast<unsigned long long*>(&sm.w[4 * cg + 1]), (unsigned long long)s1);
    atomicAdd(reinterpret_cast<unsigned long long*>(&sm.w[4 * cg + 2]), (unsigned long long)s2);
    atomicAdd(reinterpret_cast<unsigned long long*>(&sm.w[4 * cg + 3]), (unsigned long long)s3);
  }
  __syncthreads();
  if (tid < 256 && sm.w[tid]) atomicAdd(&sm.present, 1u);
  __syncthreads();
  const uint32_t m = sm.present;
  // weights are at most 2^40, so 41 halvings make them all 1 and the tree at
  // most 8 deep: the cap never binds for a correct build, it only guarantees
  // that the loop ends
  uint32_t rounds = 0;
  for (;; ++rounds) {
    // sort by rank: keys are distinct (absent symbols get distinct keys
    // above every present one)
    if (tid == 0) sm.total = 0;
    if (tid < 256) {
      sm.tmp[tid] = sm.w[tid] ? (sm.w[tid] << 8 | tid) : (~0ull << 8 | tid);
      sm.len[tid] = 0;
    }
    __syncthreads();
    if (tid < 256 && sm.w[tid]) atomicAdd(reinterpret_cast<unsigned long long*>(&sm.total),
                                          (unsigned long long)sm.w[tid]);
    if (tid < 256) {
      const uint64_t k = sm.tmp[tid];
      uint32_t r = 0;
      for (uint32_t j = 0; j < 256; ++j) r += sm.tmp[j] < k;
      sm.key[r] = k;
    }
    __syncthreads();
    if (tid == 0) {
      uint32_t kc = 0;
      if (m == 1) {
        sm.len[sm.key[0] & 255u] = 1;
      } else if (m > 1) {
        // 32-bit weights while every weight stays below the 32-bit infinity
        kc = sm.total >> 31 ? merge<uint64_t>(sm, m) : merge<uint32_t>(sm, m);
      }
      sm.internal = kc;
      sm.deepest = m == 1 ? 1u : 0u;
    }
    __syncthreads();
    // depths of the internal nodes by pointer jumping (8 rounds cover 255)
    const uint32_t kc = sm.internal;
    if (tid < kc) {
      const bool root = tid + 1 == kc;
      sm.anc[tid] = (uint16_t)(root ? tid : sm.parent[256 + tid] - 256u);
      sm.dist[tid] = root ? 0 : 1;
    }
    __syncthreads();
    for (uint32_t round = 0; round < 8; ++round) {
      uint32_t d = 0, na = 0;
      if (tid < kc) {
        const uint32_t up = sm.anc[tid];
        d = sm.dist[tid] + sm.dist[up];
        na = sm.anc[up];
      }
      __syncthreads();
      if (tid < kc) {
        sm.dist[tid] = (uint16_t)d;
        sm.anc[tid] = (uint16_t)na;
      }
      __syncthreads();
    }
    if (kc && tid < m) {
      const uint32_t d = sm.dist[sm.parent[tid] - 256u] + 1u;
      sm.len[sm.key[tid] & 255u] = (uint8_t)d;
      atomicMax(&sm.deepest, d);
    }
    __syncthreads();
    if (sm.deepest <= kLimit) break;
    if (rounds == kMaxLimitRounds) {
      if (tid == 0) a.codes[256] = 1;  // reported by scan_kernel
      return;
    }
    if (tid < 256) sm.w[tid] = (sm.w[tid] + 1) / 2;
    __syncthreads();
  }
  // canonical codes
  if (tid < 16) sm.count[tid] = 0;
  __syncthreads();
  if (tid < 256 && sm.len[tid]) atomicAdd(&sm.count[sm.len[tid]], 1u);
  __syncthreads();
  if (tid == 0) {
    uint32_t c = 0;
    sm.next[0] = 0;
    for (uint32_t l = 1; l <= kLimit; ++l) {
      c = (c + (l > 1 ? sm.count[l - 1] : 0u)) << 1;
      sm.next[l] = c;
    }
  }
  __syncthreads();
  if (tid < 256) {
    const uint32_t l = sm.len[tid];
    uint32_t code = 0;
    if (l) {
      uint32_t r = 0;
      for (uint32_t t = 0; t < tid; ++t) r += sm.len[t] == l;
      code = sm.next[l] + r;
    }
    a.codes[tid] = l << 16 | code;
  }
  if (tid < 128) a.out[64 + tid] = (uint8_t)(sm.len[2 * tid] | sm.len[2 * tid + 1] << 4);
  if (tid == 0) a.codes[256] = 0;
}

__global__ __launch_bounds__(256) void size_kernel(EncArgs a) {
  __shared__ uint32_t L[256];
  const uint64_t n = input_size(a);
  if (n > a.max_n || a.codes[256] != 0) return;
  const uint64_t N = chunks(n);
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  L[tid] = a.codes[tid] >> 16;
  __syncthreads();
  const uint64_t i = (uint64_t)blockIdx.x * 4 + (tid >> 6);
  if (i >= N) return;
  const uint64_t first = i * kChunk;
  const uint32_t c = (uint32_t)(n - first < kChunk ? n - first : kChunk);
  uint32_t bits = 0;
  if (c == kChunk) {
    const uint4* in4 = reinterpret_cast<const uint4*>(a.in + first) + 4 * lane;
#pragma unroll
    for (uint32_t v = 0; v < 4; ++v) {
      const uint4 q = in4[v];
#pragma unroll
      for (uint32_t b = 0; b < 16; ++b) bits += L[byte_of(q, b)];
    }
  } else {
    for (uint32_t b = 64 * lane; b < c && b < 64 * lane + 64; ++b) bits += L[a.in[first + b]];
  }
  bits = readlane(wave_incl_scan(bits), 63);
  if (lane == 0) {
    const uint32_t nsub = (c + kSub - 1) / kSub;
    a.sizes[2 * i] = offsets_bytes(nsub);
    a.sizes[2 * i + 1] = 4 * ((bits + 31) / 32);
    reinterpret_cast<uint32_t*>(a.out + kPre)[i] = bits;
  }
}

__device__ inline uint8_t header_byte(uint32_t b, uint64_t n, uint64_t N, uint64_t total) {
  switch (b) {
    case 0: return 'G';
    case 1: return 'L';
    case 2: return 'H';
    case 3: return '1';
    case 4: return 1;  // version
    case 6: return (uint8_t)kLimit;
    default: break;
  }
  if (b >= 8 && b < 12) return (uint8_t)(kChunk >> (8 * (b - 8)));
  if (b >= 12 && b < 16) return (uint8_t)(kSub >> (8 * (b - 12)));
  if (b >= 16 && b < 24) return (uint8_t)(n >> (8 * (b - 16)));
  if (b >= 24 && b < 32) return (uint8_t)(N >> (8 * (b - 24)));
  if (b >= 32 && b < 40) return (uint8_t)(total >> (8 * (b - 32)));
  return 0;
}

__global__ __launch_bounds__(1024) void scan_kernel(EncArgs a) {
  __shared__ uint64_t scratch[1024 / 64 + 1];
  const uint64_t n = input_size(a);
  const uint32_t tid = threadIdx.x;
  if (n > a.max_n || a.codes[256] != 0) {
    if (tid == 0) {
      *a.out_bytes = 0;
      *a.status = kInvalidArg;
    }
    return;
  }
  const uint64_t N = chunks(n);
  const uint64_t sum = stream::scan_record_sizes<16>(a.sizes, N, a.offs, scratch);
  const uint64_t total = kPre + 4 * N + sum;
  if (tid == 0) {
    a.offs[N] = sum;
    *a.out_bytes = total;
    *a.status = kOk;
  }
  if (tid < 64) a.out[tid] = header_byte(tid, n, N, total);
}

// One wave per chunk, four chunks per workgroup. Lane l codes the chunk's
// bytes [64 l, 64 l + 64): its bit count, a wave prefix sum (DPP) for its bit
// offset, then its codes ORed into the wave's LDS words through a 64-bit
// accumulator (only the first and last word of a lane's range are shared
// with a neighbour). Sub-block k starts at lane 2k's offset.
constexpr uint32_t kEncWaves = 4;

struct EncWaveLds {
  uint32_t words[kMaxWords];
  uint32_t offs32[kSubs / 2 + 1];
};

__global__ __launch_bounds__(64 * kEncWaves) void encode_kernel(EncArgs a) {
  __shared__ uint32_t code[256];
  __shared__ EncWaveLds wl[kEncWaves];
  const uint64_t n = input_size(a);
  if (n > a.max_n || a.codes[256] != 0) return;
  const uint64_t N = chunks(n);
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  code[tid] = a.codes[tid];
  __syncthreads();
  const uint64_t i = (uint64_t)blockIdx.x * kEncWaves + wave;
  if (i >= N) return;
  EncWaveLds& w = wl[wave];
  const uint64_t first = i * kChunk;
  const uint32_t c = (uint32_t)(n - first < kChunk ? n - first : kChunk);
  const uint32_t nsub = (c + kSub - 1) / kSub;
  // this lane's 64 bytes
  const uint32_t j0 = 64 * lane;
  const uint32_t cnt = j0 < c ? (c - j0 < 64 ? c - j0 : 64) : 0;
  uint4 q[4];
  if (cnt == 64) {
    const uint4* in4 = reinterpret_cast<const uint4*>(a.in + first + j0);
#pragma unroll
    for (uint32_t v = 0; v < 4; ++v) q[v] = in4[v];
  } else {
    uint32_t t[16];
#pragma unroll
    for (uint32_t v = 0; v < 16; ++v) t[v] = 0;
#pragma unroll
    for (uint32_t b = 0; b < 64; ++b)
      if (b < cnt) t[b >> 2] |= (uint32_t)a.in[first + j0 + b] << (8 * (b & 3));
#pragma unroll
    for (uint32_t v = 0; v < 4; ++v) q[v] = make_uint4(t[4 * v], t[4 * v + 1], t[4 * v + 2], t[4 * v + 3]);
  }
  uint32_t mybits = 0;
#pragma unroll
  for (uint32_t b = 0; b < 64; ++b) mybits += b < cnt ? code[byte_of(q[b >> 4], b & 15u)] >> 16 : 0u;
  const uint32_t incl = wave_incl_scan(mybits);
  const uint32_t off = incl - mybits;
  const uint32_t total = readlane(incl, 63);
  uint16_t* offs16 = reinterpret_cast<uint16_t*>(w.offs32);
  if ((lane & 1u) == 0 && j0 < c) offs16[lane >> 1] = (uint16_t)off;  // sub-block lane / 2
  if (lane == 0 && (nsub & 1u)) offs16[nsub] = 0;
  const uint32_t nwords = (total + 31) / 32;
  for (uint32_t k = lane; k < nwords; k += 64) w.words[k] = 0;
  wave_sync();
  if (cnt) {
    uint64_t acc = 0;
    uint32_t used = off & 31u, wi = off >> 5;
#pragma unroll
    for (uint32_t b = 0; b < 64; ++b) {
      if (b < cnt) {
        const uint32_t e = code[byte_of(q[b >> 4], b & 15u)];
        const uint32_t l = e >> 16;
        acc |= (uint64_t)(e & 0xFFFFu) << (64 - used - l);
        used += l;
        if (used >= 32) {
          atomicOr(&w.words[wi++], (uint32_t)(acc >> 32));
          acc <<= 32;
          used -= 32;
        }
      }
    }
    if (used) atomicOr(&w.words[wi], (uint32_t)(acc >> 32));
  }
  wave_sync();
  const uint32_t ow = offsets_bytes(nsub) / 4;
  uint32_t* rec = reinterpret_cast<uint32_t*>(a.out + kPre + 4 * N + a.offs[i]);
  for (uint32_t k = lane; k < ow + nwords; k += 64) rec[k] = k < ow ? w.offs32[k] : w.words[k - ow];
}

// ---- decompression ---------------------------------------------------------

__device__ inline uint64_t get_le(const uint8_t* p, int bytes) {
  uint64_t v = 0;
  for (int k = bytes - 1; k >= 0; --k) v = v << 8 | p[k];
  return v;
}

struct PrepLds {
  DecTables t;
  uint8_t len[256];
  uint32_t kraft, present, bad;
  uint64_t scratch[1024 / 64 + 1];
};

__global__ __launch_bounds__(1024) void dec_prepare_kernel(DecArgs a) {
  __shared__ PrepLds sm;
  const uint32_t tid = threadIdx.x;
  DecTables& T = sm.t;
  if (tid == 0) {
    const uint8_t* h = a.in;
    bool ok = a.in_bytes >= kPre && h[0] == 'G' && h[1] == 'L' && h[2] == 'H' && h[3] == '1' &&
              get_le(h + 4, 2) == 1 && h[6] == kLimit && h[7] == 0 && get_le(h + 8, 4) == kChunk &&
              get_le(h + 12, 4) == kSub;
    for (uint32_t b = 40; ok && b < 64; ++b) ok = h[b] == 0;
    if (ok) {
      T.n = get_le(h + 16, 8);
      T.N = get_le(h + 24, 8);
      ok = get_le(h + 32, 8) == a.in_bytes && T.N == chunks(T.n) && T.N <= (a.in_bytes - kPre) / 4;
    }
    T.status = ok ? kOk : kCorrupt;
    sm.kraft = 0;
    sm.present = 0;
    sm.bad = 0;
  }
  if (tid < 16) T.count[tid] = 0;
  __syncthreads();
  if (T.status == kOk && tid < 256) {
    const uint32_t l = (a.in[64 + tid / 2] >> (4 * (tid & 1u))) & 15u;
    sm.len[tid] = (uint8_t)l;
    if (l) {
      atomicAdd(&sm.present, 1u);
      atomicAdd(&T.count[l], 1u);
      atomicAdd(&sm.kraft, 1u << (kLimit - l));
    }
  }
  __syncthreads();
  if (tid == 0 && T.status == kOk) {
    const bool code_ok = T.n == 0 ? sm.present == 0
                                  : (sm.present == 1 ? T.count[1] == 1 : sm.kraft == (1u << kLimit));
    if (!code_ok) T.status = kCorrupt;
    uint32_t c = 0, r = 0;
    for (uint32_t l = 1; l <= kLimit; ++l) {
      c = (c + (l > 1 ? T.count[l - 1] : 0u)) << 1;
      T.first[l] = c;
      T.rank0[l] = r;
      r += T.count[l];
    }
    T.first[0] = T.rank0[0] = 0;
  }
  __syncthreads();
  if (T.status != kOk) {
    if (tid == 0) {
      *a.tab = T;
      *a.out_bytes = 0;
      *a.status = kCorrupt;
    }
    return;
  }
  if (tid < 256 && sm.len[tid]) {
    const uint32_t l = sm.len[tid];
    uint32_t r = 0;
    for (uint32_t t = 0; t < tid; ++t) r += sm.len[t] == l;
    T.by_rank[T.rank0[l] + r] = (uint8_t)tid;
  }
  __syncthreads();
  // two-level table, every entry decoded on its own thread: an 11-bit prefix
  // holds the code of length <= 11 it starts with; prefixes from first(12) / 2
  // on (where the codes longer than 11 bits begin, being the last codes) point
  // to 16-entry subtables over the next 4 bits; anything else matches no code
  const uint32_t p0 = T.first[kLutBits + 1] >> 1;
  for (uint32_t k = tid; k < (1u << kLutBits); k += 1024) {
    uint32_t e = 0;
    for (uint32_t l = 1; l <= kLutBits; ++l) {
      const uint32_t d = (k >> (kLutBits - l)) - T.first[l];
      if (d < T.count[l]) {
        e = l << 8 | T.by_rank[T.rank0[l] + d];
        break;
      }
    }
    if (e == 0 && k >= p0 && k - p0 < kMaxSubtables) e = 0x8000u | (k - p0);
    T.lut[k] = (uint16_t)e;
  }
  for (uint32_t k = tid; k < kMaxSubtables * 16; k += 1024) {
    const uint32_t prefix = p0 + k / 16;
    uint32_t e = 0;
    if (prefix < (1u << kLutBits)) {
      const uint32_t v = prefix << 4 | (k & 15u);  // 15-bit window
      for (uint32_t l = kLutBits + 1; l <= kLimit; ++l) {
        const uint32_t d = (v >> (kLimit - l)) - T.first[l];
        if (d < T.count[l]) {
          e = l << 8 | T.by_rank[T.rank0[l] + d];
          break;
        }
      }
    }
    T.lut2[k] = (uint16_t)e;
  }
  // record sizes from the table of code bits: 8 entries per thread per
  // tile, read with 16-byte loads before any size is written (the table
  // starts 16-byte aligned; sizes is 256-byte aligned)
  const uint32_t* bits_tab = reinterpret_cast<const uint32_t*>(a.in + kPre);
  for (uint64_t base = 0; base < T.N; base += 8 * 1024) {
    const uint64_t i0 = base + 8 * (uint64_t)tid;
    if (i0 >= T.N) continue;
    uint32_t bits[8];
    if (i0 + 8 <= T.N) {
      const uint4 lo = reinterpret_cast<const uint4*>(bits_tab + i0)[0];
      const uint4 hi = reinterpret_cast<const uint4*>(bits_tab + i0)[1];
      bits[0] = lo.x, bits[1] = lo.y, bits[2] = lo.z, bits[3] = lo.w;
      bits[4] = hi.x, bits[5] = hi.y, bits[6] = hi.z, bits[7] = hi.w;
    } else {
#pragma unroll
      for (uint32_t k = 0; k < 8; ++k) bits[k] = i0 + k < T.N ? bits_tab[i0 + k] : 0u;
    }
    uint32_t sz[16];
    bool bad = false;
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) {
      const uint64_t i = i0 + k;
      const uint32_t c = i < T.N ? (uint32_t)(T.n - i * kChunk < kChunk ? T.n - i * kChunk : kChunk) : 0u;
      bad = bad || bits[k] > kLimit * c;
      sz[2 * k] = i < T.N ? offsets_bytes((c + kSub - 1) / kSub) : 0u;
      sz[2 * k + 1] = 4 * ((bits[k] + 31) / 32);
    }
    if (bad) sm.bad = 1;
    if (i0 + 8 <= T.N) {
      uint4* dst = reinterpret_cast<uint4*>(a.sizes + 2 * i0);
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) dst[q] = make_uint4(sz[4 * q], sz[4 * q + 1], sz[4 * q + 2], sz[4 * q + 3]);
    } else {
#pragma unroll
      for (uint32_t k = 0; k < 8; ++k)
        if (i0 + k < T.N) {
          a.sizes[2 * (i0 + k)] = sz[2 * k];
          a.sizes[2 * (i0 + k) + 1] = sz[2 * k + 1];
        }
    }
  }
  __syncthreads();
  const uint64_t sum = stream::scan_record_sizes<16>(a.sizes, T.N, a.offs, sm.scratch);
  if (tid == 0) {
    if (sm.bad || kPre + 4 * T.N + sum != a.in_bytes) {
      T.status = kCorrupt;
      *a.out_bytes = 0;
    } else {
      T.status = T.n > a.capacity ? kOutOfSpace : kOk;
      *a.out_bytes = T.n;
    }
    *a.status = T.status;
  }
  __syncthreads();
  // publish the tables
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&T);
  uint32_t* dst = reinterpret_cast<uint32_t*>(a.tab);
  for (uint32_t k = tid; k < sizeof(DecTables) / 4; k += 1024) dst[k] = src[k];
}

constexpr uint32_t kDecWaves = 4;                  // waves per decode workgroup
constexpr uint32_t kInStageWords = 1024;           // code words staged per chunk (8 bits/symbol)
constexpr uint32_t kStageSub = kSub + 4;           // LDS bytes per decoded sub-block (bank padding)
constexpr uint32_t kStageChunk = kSubs * kStageSub + 4;
constexpr uint32_t kDecodeBlocks = 256 * 2;

struct DecWaveLds {
  uint32_t in[2][kInStageWords];       // code words of the wave's two chunks
  uint32_t out[2][kStageChunk / 4];    // their decoded bytes
};

struct DecLds {
  uint16_t lut[1u << kLutBits];
  uint16_t lut2[kMaxSubtables * 16];
  DecWaveLds w[kDecWaves];
};

struct DecCode {
  const uint16_t* lut;
  const uint16_t* lut2;
};

// Decodes the `cnt` symbols of one sub-block starting at bit `start` of the
// chunk's code words `wds` (nwords >= 1 of them) into `out32`; returns the
// bit position after them, or ~0u if one of them matches no code. Every lane
// runs all 128 steps, so the loop is uniform across the wave: steps past
// `cnt` decode whatever bits follow and are ignored (they only write into
// this sub-block's own stage slot). Word reads are clamped to the last word
// instead of branching: bits past a sub-block's end never decide whether it
// ends exactly at its end bit. The bit buffer is refilled once per pair of
// symbols (after a refill it holds at least 32 bits; two codes take at most
// 30). Codes of up to 11 bits take one table read, longer ones a second one.
template <typename WordPtr>
__device__ __forceinline__ uint32_t decode_sub(const DecCode& dc, WordPtr wds, uint32_t nwords,
                                               uint32_t start, uint32_t cnt, uint32_t* out32) {
  const uint32_t last = nwords - 1;
  uint32_t wi = start >> 5;
  const uint32_t w0 = wds[wi < last ? wi : last], w1 = wds[wi + 1 < last ? wi + 1 : last];
  wi += 2;
  uint64_t buf = ((uint64_t)w0 << 32 | w1) << (start & 31u);
  uint32_t avail = 64 - (start & 31u), p = start, p_end = start;
  bool bad = false;
  for (uint32_t j = 0; j < kSub; j += 4) {
    uint32_t acc = 0;
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u) {
      if ((u & 1u) == 0) {
        const uint32_t w = wds[wi < last ? wi : last];
        const bool take = avail < 32;
        buf |= take ? (uint64_t)w << (32 - avail) : 0ull;
        wi += take ? 1u : 0u;
        avail += take ? 32u : 0u;
      }
      const uint32_t peek = (uint32_t)(buf >> (64 - kLimit));
      uint32_t e = dc.lut[peek >> (kLimit - kLutBits)];
      if (e & 0x8000u) e = dc.lut2[(e & 0x7FFFu) * 16 + (peek & 15u)];
      uint32_t l = e >> 8;
      const uint32_t sym = e & 0xFFu;
      if (l == 0) bad = bad || j + u < cnt;
      l = l ? l : 1u;
      buf <<= l;
      avail -= l;
      p += l;
      p_end = j + u + 1 == cnt ? p : p_end;
      acc |= sym << (8 * u);
    }
    out32[j >> 2] = acc;
  }
  return bad ? ~0u : p_end;
}

// Each wave takes two chunks at a time (32 lanes each, one lane per
// 128-symbol sub-block): it stages the chunks' code words in LDS with
// coalesced loads, decodes every sub-block from LDS into an LDS stage, and
// writes the chunks out with consecutive 4-byte stores. Only the wave
// synchronises; a chunk with more than 4 KiB of code words (above 8 bits per
// symbol) is decoded from global memory instead.
__global__ __launch_bounds__(64 * kDecWaves) void decode_kernel(DecArgs a) {
  __shared__ DecLds sm;
  const DecTables* T = a.tab;
  if (T->status != kOk) return;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint64_t n = T->n, N = T->N;
  for (uint32_t k = tid; k < (1u << kLutBits); k += 64 * kDecWaves) sm.lut[k] = T->lut[k];
  for (uint32_t k = tid; k < kMaxSubtables * 16; k += 64 * kDecWaves) sm.lut2[k] = T->lut2[k];
  DecCode dc;
  dc.lut = sm.lut;
  dc.lut2 = sm.lut2;
  __syncthreads();
  const uint32_t* bits_tab = reinterpret_cast<const uint32_t*>(a.in + kPre);
  const uint64_t rec_base = kPre + 4 * N;
  DecWaveLds& w = sm.w[wave];
  const uint32_t half = lane >> 5, k = lane & 31u;
  uint8_t* out8 = reinterpret_cast<uint8_t*>(w.out[half]);
  bool bad = false;
  for (uint64_t g = (uint64_t)blockIdx.x * kDecWaves + wave; 2 * g < N; g += (uint64_t)gridDim.x * kDecWaves) {
    const uint64_t i = 2 * g + half;
    const bool live = i < N;
    uint32_t c = 0, nsub = 0, bits = 0, nwords = 0;
    const uint8_t* rec = nullptr;
    const uint32_t* wds = nullptr;
    if (live) {
      c = (uint32_t)(n - i * kChunk < kChunk ? n - i * kChunk : kChunk);
      nsub = (c + kSub - 1) / kSub;
      rec = a.in + rec_base + a.offs[i];
      bits = bits_tab[i];
      nwords = (bits + 31) / 32;
      wds = reinterpret_cast<const uint32_t*>(rec + offsets_bytes(nsub));
    }
    const bool staged = nwords <= kInStageWords;
    if (live && staged)
      for (uint32_t q = k; q < nwords; q += 32) w.in[half][q] = wds[q];
    wave_sync();
    if (live && k < nsub) {
      const uint16_t* o16 = reinterpret_cast<const uint16_t*>(rec);
      const uint32_t start = o16[k];
      const uint32_t end = k + 1 < nsub ? o16[k + 1] : bits;
      const uint32_t cnt = k + 1 < nsub ? kSub : c - kSub * k;
      bool ok = !((k == 0 && start != 0) || end > bits || start > end || bits == 0);
      if (k + 1 == nsub && (nsub & 1u) && o16[nsub] != 0) ok = false;
      if (ok && k + 1 == nsub && (bits & 31u) && (wds[nwords - 1] << (bits & 31u)) != 0) ok = false;
      if (ok) {
        uint32_t* out32 = reinterpret_cast<uint32_t*>(out8 + k * kStageSub);
        const uint32_t p = staged ? decode_sub(dc, (const uint32_t*)w.in[half], nwords, start, cnt, out32)
                                  : decode_sub(dc, wds, nwords, start, cnt, out32);
        ok = p == end;
      }
      bad = bad || !ok;
    }
    wave_sync();
    if (live) {
      uint8_t* dst = a.out + i * kChunk;
      for (uint32_t p = 4 * k; p < c; p += 4 * 32) {
        const uint32_t v = *reinterpret_cast<const uint32_t*>(out8 + (p / kSub) * kStageSub + p % kSub);
        if (p + 4 <= c) {
          *reinterpret_cast<uint32_t*>(dst + p) = v;
        } else {
          for (uint32_t b = 0; p + b < c; ++b) dst[p + b] = (uint8_t)(v >> (8 * b));
        }
      }
    }
    wave_sync();
  }
  if (bad) atomicExch(a.status, kCorrupt);
}

}  // namespace

hipError_t launch_compress(const EncArgs& a, hipStream_t s) {
  const uint64_t N = chunks(a.max_n);
  hipLaunchKernelGGL(hist_kernel, dim3(a.hist_blocks), dim3(256), 0, s, a);
  hipLaunchKernelGGL(build_kernel, dim3(1), dim3(1024), 0, s, a);
  if (N) hipLaunchKernelGGL(size_kernel, dim3((uint32_t)((N + 3) / 4)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, a);
  if (N) hipLaunchKernelGGL(encode_kernel, dim3((uint32_t)((N + kEncWaves - 1) / kEncWaves)),
                           dim3(64 * kEncWaves), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_decompress(const DecArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(dec_prepare_kernel, dim3(1), dim3(1024), 0, s, a);
  hipLaunchKernelGGL(decode_kernel, dim3(kDecodeBlocks), dim3(64 * kDecWaves), 0, s, a);
  return hipGetLastError();
}

}  // namespace huff
}  // namespace gpulz
