// Pairwise intersection over a set store (section 4.2 algorithms on the
// layouts of section 4.3).
//
// A group of G lanes (4, 16 or 64) takes one pair (A, B).  The group walks
// the two segment lists in block order, all lanes reading the same headers,
// and for each pair of overlapping segments restricted to the blocks both
// cover it spreads the work over its lanes:
//   bitset & bitset  AND of the overlapping words, popcount;
//   uint & bitset    each member of the uint run tests its bit;
//   uint & uint      when the longer run is more than 32 times the shorter,
//                    a binary search of each member of the shorter (the
//                    galloping regime); otherwise a merge of LDS windows of
//                    both runs (tiled_count).
// A run restricted to blocks [lo, hi] is found by binary searches on the
// block of its members, done only when the run reaches outside [lo, hi].
#include <hip/hip_runtime.h>

#include "eh_internal.h"

namespace eh {
namespace {

constexpr uint32_t kPairWPB = 4;        // waves per block
constexpr uint64_t kGallopRatio = 32;   // longer / shorter above which uint & uint searches
constexpr uint32_t kWinPerLane = 4;     // members per lane in an LDS window of the uint merge

struct PairArgs {
  const uint32_t* seg_off;
  const uint4* seg;
  const uint32_t* vals;
  const uint32_t* words;
  const uint32_t* pairs;
  uint32_t* counts;
  unsigned long long* total;
  unsigned long long* bad;
  uint64_t n_pairs;
  uint32_t n_sets;
  uint32_t bl;   // log2 block size in ids
  uint32_t wpb;  // words per block
};

// first k in [k0, k1) with (v[k] >> bl) >= b, k1 if none
__device__ __forceinline__ uint32_t lower_block(const uint32_t* __restrict__ v, uint32_t k0,
                                                uint32_t k1, uint32_t b, uint32_t bl) {
  while (k0 < k1) {
    const uint32_t mid = k0 + ((k1 - k0) >> 1);
    if ((v[mid] >> bl) < b) k0 = mid + 1;
    else k1 = mid;
  }
  return k0;
}

// first k in [0, n) with v[k] >= x, n if none
__device__ __forceinline__ uint32_t lower_value(const uint32_t* __restrict__ v, uint32_t n,
                                                uint32_t x) {
  uint32_t k0 = 0, k1 = n;
  while (k0 < k1) {
    const uint32_t mid = k0 + ((k1 - k0) >> 1);
    if (v[mid] < x) k0 = mid + 1;
    else k1 = mid;
  }
  return k0;
}

// Orders the wave's LDS accesses before and after this point.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// |S & L| for sorted runs S (na >= 1) and L (nb >= 1) by a group of G lanes:
// windows of kWinPerLane G members of each run are staged in LDS (tS, tL) with
// coalesced loads and merged window by window, as a two-pointer merge over
// the windows' value ranges: the window that ends first advances (both when
// they end together).  When two windows overlap in value, each member of
// the S window within the L window's range is searched there.  A member of
// S matches at most one member of L, and the two windows holding them
// overlap and are visited together once, so each match is counted once.
// dst[0 .. n) = src[0 .. n), n <= kWinPerLane G, by a group of G lanes: every
// load is issued before the first store, so a window costs one round trip
template <uint32_t G>
__device__ __forceinline__ void copy_window(uint32_t* dst, const uint32_t* __restrict__ src,
                                            uint32_t n, uint32_t gl) {
  uint32_t v[kWinPerLane];
#pragma unroll
  for (uint32_t i = 0; i < kWinPerLane; ++i) {
    const uint32_t k = gl + i * G;
    v[i] = k < n ? src[k] : 0u;
  }
#pragma unroll
  for (uint32_t i = 0; i < kWinPerLane; ++i) {
    const uint32_t k = gl + i * G;
    if (k < n) dst[k] = v[i];
  }
}

template <uint32_t G>
__device__ __forceinline__ uint32_t tiled_count(const uint32_t* __restrict__ S, uint32_t na,
                                                const uint32_t* __restrict__ L, uint32_t nb,
                                                uint32_t* tS, uint32_t* tL, uint32_t gl) {
  constexpr uint32_t T = kWinPerLane * G;
  uint32_t cnt = 0, s0 = 0, l0 = 0;
  uint32_t tn = min(T, na), cn = min(T, nb);
  copy_window<G>(tS, S, tn, gl);
  copy_window<G>(tL, L, cn, gl);
  wave_sync();
  for (;;) {
    const uint32_t s_first = tS[0], s_last = tS[tn - 1];
    const uint32_t l_first = tL[0], l_last = tL[cn - 1];
    if (s_first <= l_last && l_first <= s_last) {
      for (uint32_t k = gl; k < tn; k += G) {
        const uint32_t x = tS[k];
        if (x < l_first || x > l_last) continue;
        uint32_t lo = 0, len = cn;
        while (len > 0) {
          const uint32_t half = len >> 1;
          if (tL[lo + half] < x) {
            lo += half + 1;
            len -= half + 1;
          } else {
            len = half;
          }
        }
        cnt += tL[lo] == x ? 1u : 0u;  // lo < cn: x <= l_last
      }
    }
    const bool next_s = s_last <= l_last, next_l = l_last <= s_last;
    wave_sync();
    if (next_s) {
      s0 += T;
      if (s0 >= na) break;
      tn = min(T, na - s0);
      copy_window<G>(tS, S + s0, tn, gl);
    }
    if (next_l) {
      l0 += T;
      if (l0 >= nb) break;
      cn = min(T, nb - l0);
      copy_window<G>(tL, L + l0, cn, gl);
    }
    wave_sync();
  }
  wave_sync();
  return cnt;
}

// positions in vals of the members of uint run r that lie in blocks [lo, hi]
__device__ __forceinline__ uint2 run_members(const PairArgs& a, const uint4& r, uint32_t lo,
                                             uint32_t hi) {
  uint32_t k0 = r.z, k1 = r.z + (r.w & kMaxIndex);
  if (r.x < lo) k0 = lower_block(a.vals, k0, k1, lo, a.bl);
  // hi < 2^(32 - bl), so hi + 1 does not wrap
  if (r.y > hi) k1 = lower_block(a.vals, k0, k1, hi + 1, a.bl);
  return uint2{k0, k1};
}

template <uint32_t G>
__device__ __forceinline__ uint32_t segment_pair(const PairArgs& a, const uint4& A, const uint4& B,
                                                 uint32_t lo, uint32_t hi, uint32_t gl,
                                                 uint32_t* tS, uint32_t* tL) {
  const bool a_bits = (A.w & kHiBit) != 0, b_bits = (B.w & kHiBit) != 0;
  uint32_t cnt = 0;
  if (a_bits && b_bits) {
    // word w of the id space is word w - first block * wpb of a run
    const uint32_t w0 = lo * a.wpb, w1 = (hi + 1) * a.wpb;
    const uint32_t* __restrict__ wa = a.words + A.z;
    const uint32_t* __restrict__ wb = a.words + B.z;
    const uint32_t da = A.x * a.wpb, db = B.x * a.wpb;
    for (uint32_t w = w0 + gl; w < w1; w += G) cnt += __popc(wa[w - da] & wb[w - db]);
    return cnt;
  }
  if (a_bits || b_bits) {
    const uint4& U = a_bits ? B : A;
    const uint4& W = a_bits ? A : B;
    const uint2 r = run_members(a, U, lo, hi);
    const uint32_t* __restrict__ wv = a.words + W.z;
    const uint32_t dw = W.x * a.wpb;
    for (uint32_t k = r.x + gl; k < r.y; k += G) {
      const uint32_t x = a.vals[k];
      cnt += (wv[(x >> 5) - dw] >> (x & 31)) & 1u;
    }
    return cnt;
  }
  uint2 ra = run_members(a, A, lo, hi), rb = run_members(a, B, lo, hi);
  uint32_t na = ra.y - ra.x, nb = rb.y - rb.x;
  if (na == 0 || nb == 0) return 0;
  if (na > nb) {
    const uint2 t = ra;
    ra = rb;
    rb = t;
    const uint32_t tn = na;
    na = nb;
    nb = tn;
  }
  const uint32_t* __restrict__ S = a.vals + ra.x;
  const uint32_t* __restrict__ L = a.vals + rb.x;
  if (uint64_t(nb) > kGallopRatio * na) {
    for (uint32_t k = gl; k < na; k += G) {
      const uint32_t x = S[k];
      const uint32_t p = lower_value(L, nb, x);
      cnt += (p < nb && L[p] == x) ? 1u : 0u;
    }
    return cnt;
  }
  return tiled_count<G>(S, na, L, nb, tS, tL, gl);
}

template <uint32_t G>
__global__ __launch_bounds__(kPairWPB * 64) __attribute__((amdgpu_waves_per_eu(8)))
void k_intersect_pairs(PairArgs a) {
  constexpr uint32_t kGroups = kPairWPB * 64 / G;  // groups per block
  // LDS windows of the uint & uint merge, per group
  __shared__ uint32_t s_win[kGroups][2][kWinPerLane * G];
  const uint32_t lane = threadIdx.x & 63u, gl = threadIdx.x % G;
  uint32_t* tS = s_win[threadIdx.x / G][0];
  uint32_t* tL = s_win[threadIdx.x / G][1];
  const uint64_t stride = uint64_t(gridDim.x) * kGroups;
  unsigned long long tot = 0;
  bool bad = false;
  for (uint64_t p = uint64_t(blockIdx.x) * kGroups + threadIdx.x / G; p < a.n_pairs; p += stride) {
    const uint32_t s = a.pairs[2 * p], t = a.pairs[2 * p + 1];
    uint32_t cnt = 0;
    if (s >= a.n_sets || t >= a.n_sets) {
      bad = true;
    } else {
      uint32_t i = a.seg_off[s], j = a.seg_off[t];
      const uint32_t i1 = a.seg_off[s + 1], j1 = a.seg_off[t + 1];
      if (i < i1 && j < j1) {
        uint4 A = a.seg[i], B = a.seg[j];
        for (;;) {
          const uint32_t lo = max(A.x, B.x), hi = min(A.y, B.y);
          if (lo <= hi) cnt += segment_pair<G>(a, A, B, lo, hi, gl, tS, tL);
          // advance the run that ends first (both when they end together)
          const bool next_a = A.y <= B.y, next_b = B.y <= A.y;
          if (next_a) {
            if (++i == i1) break;
            A = a.seg[i];
          }
          if (next_b) {
            if (++j == j1) break;
            B = a.seg[j];
          }
        }
      }
    }
    // every lane of the group is here for the same p
    for (uint32_t o = G / 2; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, G);
    if (gl == 0) {
      if (a.counts) a.counts[p] = cnt;
      tot += cnt;
    }
  }
  // one atomic per block: waves that finish together would queue on the
  // total's address
  __shared__ unsigned long long s_part[kPairWPB];
  for (uint32_t o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
  if (lane == 0) s_part[threadIdx.x >> 6] = tot;
  const bool any_bad = __ballot(bad) != 0ull;
  if (a.bad && any_bad && lane == 0) atomicOr(a.bad, 1ull);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long sum = 0;
    for (uint32_t w = 0; w < kPairWPB; ++w) sum += s_part[w];
    if (sum) atomicAdd(a.total, sum);
  }
}

}  // namespace

eh_status launch_intersect_pairs(Ctx* c, hipStream_t s, const Sets& st, uint64_t n_pairs,
                                 const uint32_t* pairs, uint32_t* counts, uint32_t lanes,
                                 unsigned long long* total, unsigned long long* bad) {
  if (n_pairs == 0) return EH_OK;
  PairArgs a;
  a.seg_off = static_cast<const uint32_t*>(st.seg_off.p);
  a.seg = static_cast<const uint4*>(st.seg.p);
  a.vals = static_cast<const uint32_t*>(st.vals.p);
  a.words = static_cast<const uint32_t*>(st.words.p);
  a.pairs = pairs;
  a.counts = counts;
  a.total = total;
  a.bad = bad;
  a.n_pairs = n_pairs;
  a.n_sets = st.info.n_sets;
  a.bl = st.info.block_log;
  a.wpb = 1u << (a.bl - 5);
  const uint64_t groups = uint64_t(kPairWPB) * 64 / lanes;
  const uint64_t want = (n_pairs + groups - 1) / groups;
  const uint32_t grid = uint32_t(std::min<uint64_t>(want, uint64_t(c->n_cu) * 16));
  const dim3 blk(kPairWPB * 64);
  if (lanes == 4)
    hipLaunchKernelGGL(k_intersect_pairs<4>, dim3(grid), blk, 0, s, a);
  else if (lanes == 16)
    hipLaunchKernelGGL(k_intersect_pairs<16>, dim3(grid), blk, 0, s, a);
  else
    hipLaunchKernelGGL(k_intersect_pairs<64>, dim3(grid), blk, 0, s, a);
  return hip_check(c, hipGetLastError(), "pairwise set intersection launch");
}

}  // namespace eh
