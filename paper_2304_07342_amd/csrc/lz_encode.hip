// Chunk encoder: one wavefront per chunk.
//
// Steps, following gpuLZ (Zhang et al., ICS'23):
//   stage   the chunk is copied HBM -> LDS with 16-byte loads; window and
//           look-ahead live in the same LDS array (section 3.3.2, unified
//           shared buffer);
//   match   exact longest match at each token start: the 64 lanes of the
//           wave hold 64 window offsets each (up to 256 offsets in 4
//           columns); one v_cmp per column compares the coding symbol with
//           the symbol d back and the resulting 64-bit mask is the set of
//           offsets still matching. Extending the match ANDs the mask with
//           the comparison at the next look-ahead symbol and drops offsets
//           shorter than the current length (a match never exceeds its
//           offset, section 3.3.2). The length is the number of steps before
//           the mask empties; the offset is the highest set bit (ties go to
//           the largest offset);
//   parse   greedy: pointer if length >= min_match, else one literal
//           (section 2.2 basic steps; section 3.3.2 encoding step). Only
//           token starts are searched: positions covered by a pointer are
//           never matched, unlike the paper's per-symbol matching;
//   encode  every 64 tokens the wave encodes them in parallel, one token per
//           lane: the flag byte group is the ballot of the pointer lanes and
//           each lane's payload offset is S * (literal lanes below it) +
//           2 * (pointer lanes below it), computed with mbcnt (the local
//           prefix sum of section 3.2.2, over per-token sizes).
// The record goes to a per-chunk scratch slot; the chunk's flag and payload
// sizes go to `sizes` for the global prefix sum.
#include "gpulz_internal.h"
#include "wave.h"

namespace gpulz {
namespace {

// Bytes of LDS before the chunk's first symbol: the window may look up to
// 64 * WC symbols before position 0 (those offsets are masked out).
template <int S, int WC>
__host__ __device__ constexpr uint32_t pad_bytes() {
  return (uint32_t)align_up(64u * WC * S, 16);
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

template <int S, int WC>
__global__ __launch_bounds__(64) void encode_kernel(EncodeArgs a) {
  using T = typename SymType<S>::T;
  extern __shared__ __align__(16) uint8_t lds[];
  const uint32_t lane = lane_id();
  const uint64_t chunk = blockIdx.x;
  const uint64_t cs = chunk * a.C;
  const uint32_t c = (uint32_t)min<uint64_t>(a.C, a.m - cs);

  // ---- stage: HBM -> LDS, 16-byte words; the chunk keeps its address
  // alignment modulo 16 so that whole words can be copied.
  const uint64_t src_begin = cs * S;
  const uint64_t src_al = src_begin & ~(uint64_t)15;
  const uint32_t head = (uint32_t)(src_begin - src_al);
  const uint32_t nwords = (uint32_t)((head + (uint64_t)c * S + 15) / 16);
  uint8_t* stage = lds + pad_bytes<S, WC>();
  for (uint32_t k = lane; k < nwords; k += 64) {
    const uint64_t g = src_al + 16ull * k;
    if (g + 16 <= a.nbytes) {
      *reinterpret_cast<uint4*>(stage + 16 * k) = *reinterpret_cast<const uint4*>(a.in + g);
    } else {
      for (uint32_t b = 0; b < 16 && g + b < a.nbytes; ++b) stage[16 * k + b] = a.in[g + b];
    }
  }
  const T* win = reinterpret_cast<const T*>(stage + head);
  __syncthreads();

  uint64_t wmask[WC];
#pragma unroll
  for (int col = 0; col < WC; ++col) wmask[col] = ballot(64u * col + lane + 1u <= a.W);

  uint8_t* slot = a.slots + chunk * a.slot_bytes;
  uint32_t ntok = 0, pay = 0, desc = 0;
  uint32_t p = 0;
  while (p < c) {
    // step 0: which window offsets d <= min(W, p) hold the coding symbol
    const T x = win[p];
    uint64_t A[WC];
    uint64_t any = 0;
#pragma unroll
    for (int col = 0; col < WC; ++col) {
      const uint32_t d = 64u * col + lane + 1u;
      A[col] = ballot((d <= p) & (win[(int)p - (int)d] == x)) & wmask[col];
      any |= A[col];
    }
    uint32_t L = 0;
    if (any) {
      // extend while some offset keeps matching; offsets d <= L drop out
      L = 1;
      const uint32_t lim = min(kMaxMatch, c - p);
      while (L < lim) {
        const uint32_t q = p + L;
        const T xq = win[q];
        uint64_t B[WC];
        uint64_t anyb = 0;
#pragma unroll
        for (int col = 0; col < WC; ++col) {
          const uint32_t d = 64u * col + lane + 1u;
          B[col] = A[col] & ballot((d > L) & (win[(int)q - (int)d] == xq));
          anyb |= B[col];
        }
        if (!anyb) break;
#pragma unroll
        for (int col = 0; col < WC; ++col) A[col] = B[col];
        ++L;
      }
    }
    uint32_t val;
    if (L >= a.MIN) {
      uint32_t d = 0;
#pragma unroll
      for (int col = WC - 1; col >= 0; --col) {
        if (d == 0 && A[col]) d = 64u * col + 64u - (uint32_t)__clzll(A[col]);
      }
      val = 1u | (L << 1) | ((d & 0xFFu) << 9);
      p += L;
    } else {
      val = p << 1;
      p += 1;
    }
    if (lane == (ntok & 63u)) desc = val;
    ++ntok;
    if ((ntok & 63u) == 0) encode_group<S>(64, desc, (ntok >> 6) - 1, win, slot, a.flag_area, pay);
  }
  if (ntok & 63u) encode_group<S>(ntok & 63u, desc, ntok >> 6, win, slot, a.flag_area, pay);
  if (lane == 0) {
    a.sizes[2 * chunk] = (ntok + 7) / 8;
    a.sizes[2 * chunk + 1] = pay;
  }
}

template <int S, int WC>
hipError_t launch_sw(const EncodeArgs& a, uint64_t N, hipStream_t s) {
  const size_t lds = pad_bytes<S, WC>() + align_up((uint64_t)a.C * S + 32, 16);
  hipLaunchKernelGGL((encode_kernel<S, WC>), dim3((uint32_t)N), dim3(64), lds, s, a);
  return hipGetLastError();
}

template <int S>
hipError_t launch_s(const EncodeArgs& a, uint64_t N, hipStream_t s) {
  switch ((a.W + 63) / 64) {
    case 1: return launch_sw<S, 1>(a, N, s);
    case 2: return launch_sw<S, 2>(a, N, s);
    case 3: return launch_sw<S, 3>(a, N, s);
    default: return launch_sw<S, 4>(a, N, s);
  }
}

}  // namespace

size_t encode_lds_bytes(uint32_t C, uint32_t S, uint32_t W) {
  const uint32_t wc = (W + 63) / 64;
  return align_up(64ull * wc * S, 16) + align_up((uint64_t)C * S + 32, 16);
}

hipError_t launch_encode(const EncodeArgs& a, uint32_t S, uint64_t N, hipStream_t s) {
  if (N == 0) return hipSuccess;
  switch (S) {
    case 1: return launch_s<1>(a, N, s);
    case 2: return launch_s<2>(a, N, s);
    case 4: return launch_s<4>(a, N, s);
    default: return launch_s<8>(a, N, s);
  }
}

}  // namespace gpulz
