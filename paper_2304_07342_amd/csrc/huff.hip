// Entropy stage after LZSS (gpuLZ section 4.5 pairs LZSS with a Huffman
// coder): byte Huffman coding in chunks that decode in parallel. The rules of
// the code and of the stream are in huff_internal.h and gpulz.h.
//
// Compression, five launches on one stream, no host round trip:
//   hist_kernel    per-workgroup byte histograms (one LDS sub-histogram per
//                  wave, 16-byte loads);
//   build_kernel   one workgroup: sums the histograms, sorts (weight,
//                  symbol) keys, runs Huffman's merge with two queues (sorted
//                  leaves, internal nodes in creation order), limits the
//                  lengths, assigns canonical codes, writes the code lengths;
//   size_kernel    one wave per chunk: code bits of the chunk;
//   scan_kernel    one workgroup: record offsets and the header;
//   encode_kernel  one workgroup per chunk: bit offsets by a block scan,
//                  codes ORed into LDS words, the record written once.
// Decompression:
//   dec_prepare_kernel  one workgroup: checks the header and the code,
//                       builds the lookup tables, scans the record sizes;
//   decode_kernel       one lane per 128-symbol sub-block (32 lanes per
//                       chunk), an 11-bit lookup table in LDS, symbols staged
//                       in LDS and written out in 4-byte stores.
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

__global__ __launch_bounds__(256) void hist_kernel(EncArgs a) {
  __shared__ uint32_t h[4][256];
  const uint32_t tid = threadIdx.x, wid = tid >> 6;
  for (uint32_t k = tid; k < 4 * 256; k += 256) (&h[0][0])[k] = 0;
  __syncthreads();
  const uint64_t n = input_size(a);
  if (n <= a.max_n) {
    const uint64_t words = (n + 15) / 16;
    const uint64_t per = (words + gridDim.x - 1) / gridDim.x;
    const uint64_t w0 = (uint64_t)blockIdx.x * per;
    const uint64_t w1 = w0 + per < words ? w0 + per : words;
    const uint4* in4 = reinterpret_cast<const uint4*>(a.in);
    for (uint64_t w = w0 + tid; w < w1; w += 256) {
      if (16 * w + 16 <= n) {
        const uint4 q = in4[w];
#pragma unroll
        for (uint32_t b = 0; b < 16; ++b) atomicAdd(&h[wid][byte_of(q, b)], 1u);
      } else {
        for (uint64_t b = 16 * w; b < n; ++b) atomicAdd(&h[wid][a.in[b]], 1u);
      }
    }
  }
  __syncthreads();
  a.partial[(uint64_t)blockIdx.x * 256 + tid] = h[0][tid] + h[1][tid] + h[2][tid] + h[3][tid];
}

struct BuildLds {
  uint64_t part[4][256];
  uint64_t w[256];    // weight by symbol (0 = absent)
  uint64_t key[256];  // weight << 8 | symbol, sorted; absent = all ones
  uint64_t iw[256];   // internal node weights in creation order
  uint16_t parent[512];
  uint8_t depth[256];  // internal node depths
  uint8_t len[256];
  uint32_t count[16], next[16];
  uint32_t present, deepest;
};

__global__ __launch_bounds__(1024) void build_kernel(EncArgs a) {
  __shared__ BuildLds sm;
  const uint32_t tid = threadIdx.x;
  if (input_size(a) > a.max_n) return;
  {
    const uint32_t col = tid & 255u, q = tid >> 8;
    uint64_t f = 0;
    for (uint32_t r = q; r < a.hist_blocks; r += 4) f += a.partial[(uint64_t)r * 256 + col];
    sm.part[q][col] = f;
  }
  if (tid == 0) sm.present = 0;
  __syncthreads();
  if (tid < 256) {
    sm.w[tid] = sm.part[0][tid] + sm.part[1][tid] + sm.part[2][tid] + sm.part[3][tid];
    if (sm.w[tid]) atomicAdd(&sm.present, 1u);
  }
  __syncthreads();
  const uint32_t m = sm.present;
  for (;;) {
    if (tid < 256) {
      sm.key[tid] = sm.w[tid] ? (sm.w[tid] << 8 | tid) : ~0ull;
      sm.len[tid] = 0;
    }
    __syncthreads();
    // bitonic sort, ascending
    for (uint32_t k = 2; k <= 256; k <<= 1) {
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
        if (tid < 128) {
          const uint32_t i = (tid / j) * (2 * j) + (tid % j), p = i + j;
          const uint64_t x = sm.key[i], y = sm.key[p];
          if ((x > y) == ((i & k) == 0)) {
            sm.key[i] = y;
            sm.key[p] = x;
          }
        }
        __syncthreads();
      }
    }
    if (tid == 0) {
      uint32_t deepest = 0;
      if (m == 1) {
        sm.len[sm.key[0] & 255u] = 1;
        deepest = 1;
      } else if (m > 1) {
        // Huffman's merge: the next node is the front leaf unless the front
        // internal node is strictly lighter (a leaf wins ties: its index is
        // smaller); internal nodes are made in nondecreasing weight order
        uint32_t li = 0, kf = 0, kc = 0;
        for (uint32_t s = 0; s + 1 < m; ++s) {
          uint32_t node[2];
          uint64_t wt[2];
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            if (li < m && (kf == kc || (sm.key[li] >> 8) <= sm.iw[kf])) {
              wt[t] = sm.key[li] >> 8;
              node[t] = li++;
            } else {
              wt[t] = sm.iw[kf];
              node[t] = 256 + kf++;
            }
          }
          sm.iw[kc] = wt[0] + wt[1];
          sm.parent[node[0]] = (uint16_t)(256 + kc);
          sm.parent[node[1]] = (uint16_t)(256 + kc);
          ++kc;
        }
        // depths: every node's parent is made after it
        sm.depth[kc - 1] = 0;
        for (int k = (int)kc - 2; k >= 0; --k) sm.depth[k] = sm.depth[sm.parent[256 + k] - 256] + 1;
        for (uint32_t j = 0; j < m; ++j) {
          const uint32_t d = sm.depth[sm.parent[j] - 256] + 1u;
          sm.len[sm.key[j] & 255u] = (uint8_t)d;
          deepest = d > deepest ? d : deepest;
        }
      }
      sm.deepest = deepest;
    }
    __syncthreads();
    if (sm.deepest <= kLimit) break;
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
}

__global__ __launch_bounds__(256) void size_kernel(EncArgs a) {
  __shared__ uint32_t L[256];
  const uint64_t n = input_size(a);
  if (n > a.max_n) return;
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
  if (n > a.max_n) {
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

__global__ __launch_bounds__(256) void encode_kernel(EncArgs a) {
  __shared__ uint32_t code[256];
  __shared__ uint32_t words[kMaxWords];
  __shared__ uint32_t offs32[kSubs / 2 + 1];
  __shared__ uint32_t scratch[8];
  const uint64_t n = input_size(a);
  if (n > a.max_n) return;
  const uint64_t N = chunks(n);
  const uint64_t i = blockIdx.x;
  if (i >= N) return;
  const uint32_t tid = threadIdx.x;
  code[tid] = a.codes[tid];
  const uint64_t first = i * kChunk;
  const uint32_t c = (uint32_t)(n - first < kChunk ? n - first : kChunk);
  const uint32_t nsub = (c + kSub - 1) / kSub;
  // this thread's 16 symbols
  const uint32_t j0 = 16 * tid;
  const uint32_t cnt = j0 < c ? (c - j0 < 16 ? c - j0 : 16) : 0;
  uint4 q = make_uint4(0, 0, 0, 0);
  if (cnt == 16) {
    q = reinterpret_cast<const uint4*>(a.in + first)[tid];
  } else {
    uint32_t v[4] = {0, 0, 0, 0};
    for (uint32_t b = 0; b < cnt; ++b) v[b >> 2] |= (uint32_t)a.in[first + j0 + b] << (8 * (b & 3));
    q = make_uint4(v[0], v[1], v[2], v[3]);
  }
  __syncthreads();
  uint32_t mybits = 0;
#pragma unroll
  for (uint32_t b = 0; b < 16; ++b) mybits += b < cnt ? code[byte_of(q, b)] >> 16 : 0u;
  // block-wide exclusive scan of the bit counts
  const uint32_t lane = tid & 63u, wid = tid >> 6;
  const uint32_t incl = wave_incl_scan(mybits);
  if (lane == 63) scratch[wid] = incl;
  __syncthreads();
  uint32_t before = 0, total = 0;
#pragma unroll
  for (uint32_t w = 0; w < 4; ++w) {
    before += w < wid ? scratch[w] : 0u;
    total += scratch[w];
  }
  const uint32_t off = before + incl - mybits;
  uint16_t* offs16 = reinterpret_cast<uint16_t*>(offs32);
  if ((tid & 7u) == 0 && j0 < c) offs16[tid >> 3] = (uint16_t)off;  // sub-block tid / 8 starts here
  if (tid == 0 && (nsub & 1u)) offs16[nsub] = 0;
  const uint32_t nwords = (total + 31) / 32;
  for (uint32_t k = tid; k < nwords; k += 256) words[k] = 0;
  __syncthreads();
  // codes into the words: a 64-bit accumulator whose top `used` bits are
  // taken; full top words are ORed into LDS (only the first and last word
  // of a thread's range are shared with a neighbour)
  if (cnt) {
    uint64_t acc = 0;
    uint32_t used = off & 31u, wi = off >> 5;
    for (uint32_t b = 0; b < cnt; ++b) {
      const uint32_t e = code[byte_of(q, b)];
      const uint32_t l = e >> 16;
      acc |= (uint64_t)(e & 0xFFFFu) << (64 - used - l);
      used += l;
      if (used >= 32) {
        atomicOr(&words[wi++], (uint32_t)(acc >> 32));
        acc <<= 32;
        used -= 32;
      }
    }
    if (used) atomicOr(&words[wi], (uint32_t)(acc >> 32));
  }
  __syncthreads();
  const uint32_t ow = offsets_bytes(nsub) / 4;
  uint32_t* rec = reinterpret_cast<uint32_t*>(a.out + kPre + 4 * N + a.offs[i]);
  for (uint32_t k = tid; k < ow + nwords; k += 256) rec[k] = k < ow ? offs32[k] : words[k - ow];
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
  for (uint32_t k = tid; k < (1u << kLutBits); k += 1024) T.lut[k] = 0;
  __syncthreads();
  if (tid < 256 && sm.len[tid]) {
    const uint32_t l = sm.len[tid];
    uint32_t r = 0;
    for (uint32_t t = 0; t < tid; ++t) r += sm.len[t] == l;
    T.by_rank[T.rank0[l] + r] = (uint8_t)tid;
    if (l <= kLutBits) {
      const uint32_t base = (T.first[l] + r) << (kLutBits - l);
      for (uint32_t k = 0; k < (1u << (kLutBits - l)); ++k) T.lut[base + k] = (uint16_t)(l << 8 | tid);
    }
  }
  // record sizes from the table of code bits
  const uint32_t* bits_tab = reinterpret_cast<const uint32_t*>(a.in + kPre);
  for (uint64_t i = tid; i < T.N; i += 1024) {
    const uint32_t c = (uint32_t)(T.n - i * kChunk < kChunk ? T.n - i * kChunk : kChunk);
    const uint32_t bits = bits_tab[i];
    if (bits > kLimit * c) sm.bad = 1;
    a.sizes[2 * i] = offsets_bytes((c + kSub - 1) / kSub);
    a.sizes[2 * i + 1] = 4 * ((bits + 31) / 32);
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

constexpr uint32_t kGroupChunks = 8;                  // chunks per decode workgroup (2 per wave)
constexpr uint32_t kStageSub = kSub + 4;              // LDS bytes per sub-block (bank padding)
constexpr uint32_t kStageChunk = kSubs * kStageSub + 4;
constexpr uint32_t kDecodeBlocks = 256 * 4;

struct DecLds {
  uint16_t lut[1u << kLutBits];
  uint32_t first[16], count[16], rank0[16];
  uint8_t by_rank[256];
  uint32_t stage[kGroupChunks * kStageChunk / 4];
};

__global__ __launch_bounds__(256) void decode_kernel(DecArgs a) {
  __shared__ DecLds sm;
  const DecTables* T = a.tab;
  if (T->status != kOk) return;
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint64_t n = T->n, N = T->N;
  for (uint32_t k = tid; k < (1u << kLutBits); k += 256) sm.lut[k] = T->lut[k];
  if (tid < 16) {
    sm.first[tid] = T->first[tid];
    sm.count[tid] = T->count[tid];
    sm.rank0[tid] = T->rank0[tid];
  }
  sm.by_rank[tid] = T->by_rank[tid];
  __syncthreads();
  const uint32_t* bits_tab = reinterpret_cast<const uint32_t*>(a.in + kPre);
  const uint64_t rec_base = kPre + 4 * N;
  uint8_t* stage8 = reinterpret_cast<uint8_t*>(sm.stage);
  for (uint64_t g = blockIdx.x; g * kGroupChunks < N; g += gridDim.x) {
    const uint32_t slot = 2 * (tid >> 6) + (lane >> 5);
    const uint32_t k = lane & 31u;
    const uint64_t i = g * kGroupChunks + slot;
    bool bad = false;
    if (i < N) {
      const uint32_t c = (uint32_t)(n - i * kChunk < kChunk ? n - i * kChunk : kChunk);
      const uint32_t nsub = (c + kSub - 1) / kSub;
      if (k < nsub) {
        const uint8_t* rec = a.in + rec_base + a.offs[i];
        const uint16_t* o16 = reinterpret_cast<const uint16_t*>(rec);
        const uint32_t bits = bits_tab[i];
        const uint32_t nwords = (bits + 31) / 32;
        const uint32_t* wds = reinterpret_cast<const uint32_t*>(rec + offsets_bytes(nsub));
        const uint32_t start = o16[k];
        const uint32_t end = k + 1 < nsub ? o16[k + 1] : bits;
        const uint32_t cnt = k + 1 < nsub ? kSub : c - kSub * k;
        if ((k == 0 && start != 0) || end > bits || start > end) bad = true;
        if (k + 1 == nsub && (nsub & 1u) && o16[nsub] != 0) bad = true;
        if (k + 1 == nsub && (bits & 31u) && (wds[nwords - 1] << (bits & 31u)) != 0) bad = true;
        if (!bad) {
          uint32_t wi = start >> 5;
          const uint32_t w0 = wi < nwords ? wds[wi] : 0u, w1 = wi + 1 < nwords ? wds[wi + 1] : 0u;
          uint64_t buf = ((uint64_t)w0 << 32 | w1) << (start & 31u);
          uint32_t avail = 64 - (start & 31u), p = start;
          wi += 2;
          uint32_t acc = 0;
          uint32_t* out32 = reinterpret_cast<uint32_t*>(stage8 + slot * kStageChunk + k * kStageSub);
          for (uint32_t j = 0; j < cnt; ++j) {
            if (avail < 32) {
              buf |= (uint64_t)(wi < nwords ? wds[wi] : 0u) << (32 - avail);
              ++wi;
              avail += 32;
            }
            const uint32_t peek = (uint32_t)(buf >> (64 - kLimit));
            const uint32_t e = sm.lut[peek >> (kLimit - kLutBits)];
            uint32_t l = e >> 8, s = e & 0xFFu;
            if (l == 0) {
              uint32_t v = 0;
              for (l = kLutBits + 1; l <= kLimit; ++l) {
                v = peek >> (kLimit - l);
                if (v - sm.first[l] < sm.count[l]) break;
              }
              if (l > kLimit) {
                bad = true;
                break;
              }
              s = sm.by_rank[sm.rank0[l] + v - sm.first[l]];
            }
            buf <<= l;
            avail -= l;
            p += l;
            acc |= s << (8 * (j & 3u));
            if ((j & 3u) == 3u) {
              out32[j >> 2] = acc;
              acc = 0;
            }
          }
          if (!bad && (cnt & 3u)) out32[cnt >> 2] = acc;
          if (p != end) bad = true;
        }
      }
    }
    __syncthreads();
    // staged chunks to the output, 4 bytes per store
    for (uint32_t q = tid; q < kGroupChunks * kChunk / 4; q += 256) {
      const uint32_t s = q / (kChunk / 4), p = 4 * (q % (kChunk / 4));
      const uint64_t ci = g * kGroupChunks + s;
      if (ci >= N) break;
      const uint32_t c = (uint32_t)(n - ci * kChunk < kChunk ? n - ci * kChunk : kChunk);
      if (p >= c) continue;
      const uint32_t v =
          *reinterpret_cast<const uint32_t*>(stage8 + s * kStageChunk + (p / kSub) * kStageSub + p % kSub);
      uint8_t* dst = a.out + ci * kChunk + p;
      if (p + 4 <= c) {
        *reinterpret_cast<uint32_t*>(dst) = v;
      } else {
        for (uint32_t b = 0; p + b < c; ++b) dst[b] = (uint8_t)(v >> (8 * b));
      }
    }
    if (bad) atomicExch(a.status, kCorrupt);
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_compress(const EncArgs& a, hipStream_t s) {
  const uint64_t N = chunks(a.max_n);
  hipLaunchKernelGGL(hist_kernel, dim3(a.hist_blocks), dim3(256), 0, s, a);
  hipLaunchKernelGGL(build_kernel, dim3(1), dim3(1024), 0, s, a);
  if (N) hipLaunchKernelGGL(size_kernel, dim3((uint32_t)((N + 3) / 4)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, a);
  if (N) hipLaunchKernelGGL(encode_kernel, dim3((uint32_t)N), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_decompress(const DecArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(dec_prepare_kernel, dim3(1), dim3(1024), 0, s, a);
  hipLaunchKernelGGL(decode_kernel, dim3(kDecodeBlocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace huff
}  // namespace gpulz
