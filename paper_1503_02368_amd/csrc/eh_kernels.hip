// gfx950 kernels for the set intersections of Generic-Join (paper section 2.1,
// Algorithm 1) on the degree-pruned trie, with COUNT(*) aggregation.
//
// Triangle:  T = sum over oriented edges (u,v) of |N+(u) & N+(v)|
// 4-clique:  K = sum over (u,v) of sum over w in S of |S & N+(w)|,
//            S = N+(u) & N+(v)   (the loop nest of section 3.3 extended by
//            one attribute; one GHD node, section 5.3)
//
// Two kernel families consume the same work items {s, idx[lbeg..+llen), tag}:
//
// * Staged ("k_*_staged"): one wave per item.  The staged set is written
//   into the wave's LDS region once, as a bitset over [min, max] when that
//   range fits (the bitset layout of section 4.1 with one block of the set's
//   range, as the set optimizer of section 4.4 builds it), else as a bitset
//   over its top window plus a searched prefix (a two-block composite,
//   section 4.3).  The streamed sets are concatenated into one flat index
//   space that the 64 lanes walk: long sets lane-strided, each lane moving a
//   cursor along the batch's length prefix; short sets in contiguous runs
//   per lane, each found by one binary search of the prefix.  Short and long
//   lists alike keep every lane busy.  Each streamed element is tested
//   against the staged set: a bit probe (uint & bitset, section 4.2), or,
//   when the streamed set is stored as a bitset with fewer words than
//   elements, a 32-bit word AND + popcount (bitset & bitset), or a binary
//   search of the composite's prefix (galloping).  Small items can be
//   grouped: up to four share a wave, their staged sets interleaved in one
//   bitmap and their streamed sets in one walk.
//
// * Pairwise ("k_tri_pairwise"): a group of G lanes per pair (s, t) reading
//   both sets from HBM, dispatching per pair on the layouts and sizes as in
//   section 4.2: bitset & bitset by word AND + popcount over the overlapping
//   words; uint & bitset by probing each uint value; uint & uint by a
//   partitioned merge when the sizes are within a factor gamma (32 in the
//   paper) and by binary search of the shorter list's values in the longer
//   one otherwise.
//
// Counts accumulate per lane in registers and leave a wave through one
// reduction and one 64-bit atomic per output slot change.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>
#include <unordered_map>

#include "eh_internal.h"

// Scratch of the allocation-free counting entry point (eh_count_add_noalloc):
// the work cursors of the cursor schedules, then one accumulator, in device
// memory the library holds from load until the process ends (one copy per
// GPU).  Host code must not pass this name to a kernel: on the host it is a
// stand-in, not a device address; eh::noalloc_scratch_init looks up each
// device's address once.
static __device__ __align__(256) unsigned long long scratch[eh::kNoAllocScratchBytes / 8];

namespace eh {
namespace {

constexpr int kWave = 64;
constexpr int kSeg = 64;  // streamed sets per flat batch

struct DevArgs {
  const Item* items;
  uint64_t n_items;
  const uint32_t* idx;
  const uint4* sdesc;  // per item {begin, length, min, max} of the staged set, or null
  const uint2* rec;    // per in-edge streamed segment {start, length | word offset << 16}, or null
  const uint2* vdesc;
  const uint32_t* col;
  const uint4* bsdesc;
  const uint32_t* bsw;
  unsigned long long* acc;
  uint32_t tag_base;
  unsigned long long* per_root;
  const uint32_t* vert;
  uint32_t* cursor;
  uint32_t use_bitsets;
  uint32_t dynamic;
  uint32_t algo;
  float gamma;
  uint32_t stage_words;  // <= the kernel's region size
  uint32_t xcds;
  uint32_t grab;
  uint32_t deg_lo, deg_hi;  // 4-clique: items with deg_lo < d+(u) <= deg_hi
  uint32_t search_below;    // segments shorter on average: the walk binary-searches
  const uint4* gsub;        // grouped items' members, or null
  uint32_t symmetric;       // the trie holds both directions of every edge
  uint32_t reverse;         // items taken from the last to the first
  uint32_t* k4s;            // 4-cliques: per-wave S lists in HBM (the HBM-list instance)
  uint32_t k4s_stride;      //   words per wave's list
  const uint4* roots;       // 4-cliques over induced neighbourhoods: root records
  uint64_t n_roots;
};

DevArgs to_dev(const LaunchArgs& a) {
  DevArgs d;
  d.items = a.items;
  d.n_items = a.n_items;
  d.idx = a.idx;
  d.sdesc = a.sdesc;
  d.rec = a.rec;
  d.vdesc = a.vdesc;
  d.col = a.col;
  d.bsdesc = a.bsdesc;
  d.bsw = a.bsw;
  d.acc = a.acc;
  d.tag_base = a.tag_base;
  d.per_root = a.per_root;
  d.vert = a.vert;
  d.cursor = a.cursor;
  d.use_bitsets = a.use_bitsets;
  d.dynamic = a.dynamic;
  d.algo = a.algo;
  d.gamma = a.gamma;
  d.stage_words = a.stage_words;
  d.xcds = a.xcds;
  d.grab = a.grab;
  d.deg_lo = a.deg_lo;
  d.deg_hi = a.deg_hi;
  d.search_below = a.search_below;
  d.gsub = a.gsub;
  d.symmetric = a.symmetric;
  d.reverse = a.reverse;
  d.k4s = a.k4s;
  d.k4s_stride = a.k4s_stride;
  d.roots = a.roots;
  d.n_roots = a.n_roots;
  return d;
}

// Orders the wave's LDS accesses before and after this point.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t uniform(uint32_t x) {
  return __builtin_amdgcn_readfirstlane(x);
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, uint32_t lane) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, kWave);
    if (lane >= uint32_t(o)) v += t;
  }
  return v;
}

// first index in a[0..n) with a[i] >= x
__device__ __forceinline__ uint32_t lower_bound_lds(const uint32_t* a, uint32_t n, uint32_t x) {
  uint32_t lo = 0, len = n;
  while (len > 0) {
    const uint32_t half = len >> 1;
    if (a[lo + half] < x) { lo += half + 1; len -= half + 1; }
    else len = half;
  }
  return lo;
}

__device__ __forceinline__ uint32_t lower_bound_glb(const uint32_t* __restrict__ a, uint32_t n,
                                                    uint32_t x) {
  uint32_t lo = 0, len = n;
  while (len > 0) {
    const uint32_t half = len >> 1;
    if (a[lo + half] < x) { lo += half + 1; len -= half + 1; }
    else len = half;
  }
  return lo;
}

// Work-item iteration.  Schedules (DevArgs.dynamic):
//  0 interleaved: item i to wave i mod W;
//  1 one atomic cursor (work stealing, one item per fetch);
//  2 blocked: wave w takes one contiguous range of items, so consecutive
//    items of one graph or request share a wave;
//  3 partitioned interleave: the items are cut into P contiguous ranges, one
//    per L2 domain (XCD; blocks are dealt to the P domains round-robin), and
//    each range is interleaved over the waves of its domain, so the sets a
//    window of items reads are fetched into one L2 instead of all P;
//  4 partitioned cursors: as 3, but each range has its own atomic cursor,
//    waves take `grab` consecutive items per fetch (the window of items in
//    flight stays tight, so it stays in L2), and a wave whose range is used
//    up moves on to the next range (work stealing across domains).
//  5 snake: wave w of W takes positions w, 2W-1-w, 2W+w, 4W-1-w, ...; over
//    items sorted by decreasing estimated cost (the plan sorts them for this
//    schedule) every wave's sum of costs stays close to the mean, with no
//    atomics.
// P = DevArgs.xcds (0: 8, the XCD count of MI355X).  Cursors are
// kCursorWords words apart, one per partition, zeroed before the launch.
struct ItemIter {
  uint64_t i, step, end;
  uint32_t mode;
  bool rev;
  uint32_t* cursor;
  uint64_t n;
  uint32_t part, parts, left, grab;
  __device__ ItemIter(const DevArgs& a, uint32_t wpb) {
    mode = a.dynamic;
    rev = a.reverse != 0;
    cursor = a.cursor;
    end = a.n_items;
    n = a.n_items;
    if (mode == 1) {
      step = 0;
      i = fetch();
      return;
    }
    if (mode == 5) {
      // position k*W + w (k even) or k*W + W-1-w (k odd): the steps from one
      // to the next alternate between 2(W-w)-1 and 2w+1, which sum to 2W
      const uint32_t w = blockIdx.x * wpb + (threadIdx.x >> 6), W = gridDim.x * wpb;
      i = w;
      step = 2ull * (W - w) - 1;
      left = 2u * W;
      return;
    }
    if (mode == 3 || mode == 4) {
      parts = a.xcds ? a.xcds : 8u;
      const uint32_t nb = gridDim.x;
      if (mode == 3 && nb % parts != 0) parts = 1;  // every range needs waves
      part = blockIdx.x % parts;
      if (mode == 3) {
        const uint64_t nwp = uint64_t(nb / parts) * wpb;
        i = range_lo(part) + uint64_t(blockIdx.x / parts) * wpb + (threadIdx.x >> 6);
        end = range_lo(part + 1);
        step = nwp;
      } else {
        grab = a.grab;
        left = parts;
        refill();
      }
      return;
    }
    // Blocks are dealt round-robin to the L2 domains (XCDs): block b runs on
    // domain b % x.  Renumbering them so each domain holds a contiguous range
    // of logical blocks gives each domain a contiguous slice of every window
    // of items, whose streamed sets overlap, instead of every x-th block.
    uint32_t b = blockIdx.x;
    const uint32_t x = a.xcds, nb = gridDim.x;
    if (x > 1 && nb % x == 0) b = (b % x) * (nb / x) + b / x;
    const uint64_t w = uint64_t(b) * wpb + (threadIdx.x >> 6);
    const uint64_t nw = uint64_t(gridDim.x) * wpb;
    if (a.dynamic == 2) {
      const uint64_t per = (a.n_items + nw - 1) / nw;
      i = w * per;
      end = i + per < a.n_items ? i + per : a.n_items;
      step = 1;
    } else {
      i = w;
      step = nw;
    }
  }
  __device__ bool more() const { return i < end; }
  // The item the current position stands for: under `reverse`, position i
  // takes item n - 1 - i, so the schedule deals the items last first.
  __device__ uint64_t idx() const { return rev ? n - 1 - i : i; }
  __device__ uint64_t range_lo(uint32_t p) const { return n * p / parts; }
  __device__ uint64_t fetch() {
    uint32_t v = 0;
    if ((threadIdx.x & 63) == 0) v = atomicAdd(cursor, 1u);
    return uniform(__shfl(v, 0, kWave));
  }
  // Takes the next `grab` items of the current range, else moves on; every
  // range is tried at most once after it is found used up, so this ends.
  __device__ void refill() {
    while (left) {
      uint32_t v = 0;
      if ((threadIdx.x & 63) == 0) v = atomicAdd(cursor + part * kCursorWords, grab);
      v = uniform(__shfl(v, 0, kWave));
      const uint64_t s = range_lo(part) + v, hi = range_lo(part + 1);
      if (s < hi) {
        i = s;
        end = s + grab < hi ? s + grab : hi;
        return;
      }
      part = part + 1 == parts ? 0u : part + 1;
      --left;
    }
    i = end = 0;
  }
  __device__ void next() {
    if (mode == 5) {
      i += step;
      step = left - step;
    } else if (mode == 1) i = fetch();
    else if (mode == 4) { if (++i >= end) refill(); }
    else i += step;
  }
};

// Adds a wave's per-lane counts to acc[tag - tag_base] (one atomic per wave).
__device__ __forceinline__ void flush_tag(const DevArgs& a, unsigned long long& acc, uint32_t tag,
                                          uint32_t lane) {
  const unsigned long long s = wave_sum(acc);
  if (lane == 0 && s) atomicAdd(&a.acc[tag - a.tag_base], s);
  acc = 0;
}

// ---------------------------------------------------------------------------
// Staged set: state shared by the triangle and 4-clique kernels
// ---------------------------------------------------------------------------

// How a set is held on chip.
//  Bitmap:    one bitset over [base, base + 32 cap) covering the whole set
//             (the bitset layout of section 4.1, block = the set's range).
//  Composite: the set's range is too wide: the bitset covers the top window
//             [base, hi] and the plen members below base (a sorted prefix of
//             the set) are searched, in the wave's prefix list when at most
//             kPrefixCap long, else in HBM -- a two-block instance of the
//             block-level composite layout of section 4.3, dense block on top
//             because degree order puts the dense hub neighbourhoods there.
//  List:      a sorted list of len ids in R, searched (4-clique level 2).
//  Empty:     nothing.
//  Group:     the sets of K small items at once, interleaved: bit
//             (x - base) K + k marks x as a member of set k (K = 2^glog);
//             each streamed set is tested against its own item's set.
enum : uint32_t { kModeBitmap = 0, kModeComposite = 1, kModeList = 2, kModeEmpty = 3,
                  kModeGroup = 4 };
constexpr int kPrefixCap = 128;

struct Staged {
  uint32_t beg, len, lo, hi, base, plen, mode;
  uint32_t glog, glim;  // group mode: log2 K, and the offsets x - base that fit
  uint32_t x0;  // per lane: member number `lane` of the set (lane < len), kept to clear R
  // composite mode: the set's own bitset in HBM (position of its first word in
  // the list buffer, first id covered), gw = kNoBitset if it has none
  uint32_t gw, gb;
  // composite mode: when not null, the sorted prefix is gp[0 .. plen) in HBM
  // (a 4-clique S list kept there) instead of Lp / the set's own members
  const uint32_t* gp;
};

// Loads the set col[beg .. beg+len) with known min lo and max hi into region
// R (RW words) and prefix list Lp, and returns how it is held.
template <int RW>
__device__ __forceinline__ Staged stage_extent(const DevArgs& a, uint32_t beg, uint32_t len,
                                               uint32_t lo, uint32_t hi, uint32_t* R, uint32_t* Lp,
                                               uint32_t lane) {
  Staged st;
  st.beg = beg;
  st.len = len;
  st.plen = 0;
  st.x0 = 0;
  st.gw = kNoBitset;
  st.gb = 0;
  st.glog = 0;
  st.glim = 0;
  st.gp = nullptr;
  if (st.len == 0) { st.mode = kModeEmpty; st.lo = st.hi = st.base = 0; return st; }
  st.lo = lo;
  st.hi = hi;
  const uint32_t cap = (a.stage_words && a.stage_words < uint32_t(RW)) ? a.stage_words : uint32_t(RW);
  const uint32_t lo_al = lo & ~31u;
  if (hi - lo_al < cap * 32u) {
    st.mode = kModeBitmap;
    st.base = lo_al;
  } else {
    // top window: hi - base < 32 cap, base a multiple of 32, base > lo
    st.mode = kModeComposite;
    st.base = (hi + 1u - cap * 32u + 31u) & ~31u;
  }
  uint32_t below = 0;
  for (uint32_t k0 = 0; k0 < st.len; k0 += kWave) {
    const uint32_t k = k0 + lane;
    bool low = false;
    if (k < st.len) {
      const uint32_t x = a.col[st.beg + k];
      if (k0 == 0) st.x0 = x;
      low = x < st.base;
      if (!low) {
        const uint32_t d = x - st.base;
        atomicOr(&R[d >> 5], 1u << (d & 31));
      } else if (k < uint32_t(kPrefixCap)) {
        Lp[k] = x;
      }
    }
    below += uint32_t(__popcll(__ballot(low)));
  }
  st.plen = below;
  wave_sync();
  return st;
}

// Loads N+(s), looking up its extent.
template <int RW>
__device__ __forceinline__ Staged stage_set(const DevArgs& a, uint32_t s, uint32_t* R,
                                            uint32_t* Lp, uint32_t lane) {
  const uint2 sd = a.vdesc[s];
  const uint32_t beg = uniform(sd.x), len = uniform(sd.y & kMaxIndex);
  if (len == 0) return stage_extent<RW>(a, beg, 0, 0, 0, R, Lp, lane);
  Staged st = stage_extent<RW>(a, beg, len, uniform(a.col[beg]), uniform(a.col[beg + len - 1]), R,
                               Lp, lane);
  // a composite set that also has the bitset layout answers its prefix with
  // one word of that bitset instead of a search
  if (st.mode == kModeComposite && a.use_bitsets && (sd.y & kHiBit)) {
    const uint4 bd = a.bsdesc[s];
    st.gw = uniform(bd.x);
    st.gb = uniform(bd.y);
  }
  return st;
}

// Returns region R to all-zero after stage_extent (the prefix list needs no
// clearing: only its first plen entries are ever read).
template <int RW>
__device__ __forceinline__ void unstage_set(const DevArgs& a, const Staged& st, uint32_t* R,
                                            uint32_t lane) {
  wave_sync();
  if (st.mode == kModeBitmap || st.mode == kModeComposite) {
    if (st.len <= uint32_t(kWave)) {
      // the members are still in registers (the prefix lies below base)
      if (lane < st.len && st.x0 >= st.base) R[(st.x0 - st.base) >> 5] = 0;
    } else {
      for (uint32_t k = st.plen + lane; k < st.len; k += kWave)
        R[(a.col[st.beg + k] - st.base) >> 5] = 0;
    }
  }
  wave_sync();
}

// Membership of x in the composite set's prefix (below the window).
__device__ __forceinline__ uint32_t prefix_has(const DevArgs& a, const Staged& st,
                                               const uint32_t* Lp, uint32_t x) {
  if (x < st.lo || x >= st.base) return 0u;
  if (st.gw != kNoBitset) {
    // st.gb <= lo <= x < base <= hi: inside the bitset's words
    const uint32_t d = x - st.gb;
    return (a.bsw[st.gw + (d >> 5)] >> (d & 31)) & 1u;
  }
  if (st.gp) {
    const uint32_t p = lower_bound_glb(st.gp, st.plen, x);
    return (p < st.plen && st.gp[p] == x) ? 1u : 0u;
  }
  if (st.plen <= uint32_t(kPrefixCap)) {
    const uint32_t p = lower_bound_lds(Lp, st.plen, x);
    return (p < st.plen && Lp[p] == x) ? 1u : 0u;
  }
  const uint32_t* L = a.col + st.beg;
  const uint32_t p = lower_bound_glb(L, st.plen, x);
  return (p < st.plen && L[p] == x) ? 1u : 0u;
}

// Membership of x in the staged set: a bit probe (uint & bitset, section
// 4.2), else a search of the prefix or of the list (galloping regime).
template <int RW>
__device__ __forceinline__ uint32_t staged_has(const DevArgs& a, const Staged& st,
                                               const uint32_t* R, const uint32_t* Lp, uint32_t x) {
  if (st.mode == kModeList) {
    if (x < st.lo || x > st.hi) return 0u;
    const uint32_t p = lower_bound_lds(R, st.len, x);
    return R[p] == x ? 1u : 0u;
  }
  if (st.mode == kModeEmpty) return 0u;
  const uint32_t d = x - st.base;
  if (d < uint32_t(RW) * 32u) return (R[d >> 5] >> (d & 31)) & 1u;
  return st.mode == kModeComposite ? prefix_has(a, st, Lp, x) : 0u;
}

// Segment table of one flat batch: P = prefix of lengths (kSeg+1), and per
// segment {start in the list buffer, word delta (kNoWords: not words)}, read
// together as one 64-bit LDS load.  Starts use all 32 bits.
struct SegTab {
  uint32_t* P;
  uint2* S;
};

// One streamed segment: start in the list buffer (col, then bitset words),
// length, and for bitset words the offset of its first word from the staged
// bitmap's (kNoWords for members).
constexpr int32_t kNoWords = INT32_MIN;
struct Seg {
  uint32_t sb, len;
  int32_t sm;
};

// When a streamed set may be read as bitset words against the staged set:
// the staged set has a bitmap, and no word can hold a member of a composite
// set's searched prefix (every word starts at or above the window base).
struct WordRule {
  bool ok;        // use_bitsets and the staged set has a bitmap
  uint32_t base;  // bitmap base id
  uint32_t wmin;  // lowest id a streamed word may start at (0 for a plain bitmap)
};

__device__ __forceinline__ WordRule word_rule(const DevArgs& a, const Staged& st) {
  WordRule r;
  r.ok = a.use_bitsets && (st.mode == kModeBitmap || st.mode == kModeComposite);
  r.base = st.base;
  r.wmin = st.mode == kModeComposite ? st.base : 0u;
  return r;
}

// The whole set N+(t), as elements or, when fewer, as bitset words.  kEager:
// when words may be used, the set's bitset descriptor is loaded beside its
// extent instead of after it (one round trip to memory per batch of sets, for
// two more registers).
template <bool kEager = false>
__device__ __forceinline__ Seg seg_full(const DevArgs& a, uint32_t t, const WordRule& wr) {
  const uint2 td = a.vdesc[t];
  uint4 bd{0, 0, 0, 0};
  if (kEager && wr.ok) bd = a.bsdesc[t];  // wr.ok implies a bitset table
  const uint32_t tl = td.y & kMaxIndex;
  Seg g{td.x, tl, kNoWords};
  if (wr.ok && (td.y & kHiBit)) {
    if (!kEager) bd = a.bsdesc[t];
    if (bd.z < tl && bd.y >= wr.wmin) {
      g.sb = bd.x;
      g.len = bd.z;
      g.sm = int32_t(bd.y >> 5) - int32_t(wr.base >> 5);
    }
  }
  return g;
}

// Publishes one segment per lane into the table and returns the flat length.
__device__ __forceinline__ uint32_t publish_segments(const SegTab& T, const Seg& g, uint32_t lane) {
  const uint32_t incl = wave_incl_scan(g.len, lane);
  wave_sync();  // previous batch's readers are done
  T.P[lane + 1] = incl;
  if (lane == 0) T.P[0] = 0;
  T.S[lane] = uint2{g.sb, uint32_t(g.sm)};
  wave_sync();
  return uniform(__shfl(incl, kWave - 1, kWave));
}

// Per-lane cursor over the segment table: for a flat index f it yields the
// element's position in the list buffer (col followed by all bitset words)
// and, for bitset words, the word's index in the staged bitmap.  Segment
// bases are kept relative to f so each element costs one add.
// kRaw (grouped items): wbase is the segment's stored value itself, the index
// of the item whose set the segment is tested against.
template <bool kRaw = false>
struct SegCursor {
  uint32_t j, nxt, base, wbase;
  bool bits;
  __device__ __forceinline__ SegCursor() {}
  __device__ __forceinline__ explicit SegCursor(const SegTab& T) {
    j = 0;
    nxt = T.P[1];
    const uint2 sg = T.S[0];
    base = sg.x;
    wbase = sg.y;
    bits = !kRaw && sg.y != uint32_t(kNoWords);
  }
  __device__ __forceinline__ void seek(const SegTab& T, uint32_t f) {
    while (nxt <= f) {
      const uint32_t start = nxt;
      ++j;
      nxt = T.P[j + 1];
      const uint2 sg = T.S[j];
      base = sg.x - start;
      wbase = kRaw ? sg.y : sg.y - start;
      bits = !kRaw && sg.y != uint32_t(kNoWords);
    }
  }
  // seek for walks with no bitset words: only the element position is kept
  __device__ __forceinline__ void seek_base(const SegTab& T, uint32_t f) {
    while (nxt <= f) {
      const uint32_t start = nxt;
      ++j;
      nxt = T.P[j + 1];
      base = T.S[j].x - start;
    }
  }
  // Places the cursor on the segment of f by a branch-free binary search of
  // the prefix table (P[0] = 0 <= f < E, and entries past the last segment
  // equal E): six LDS reads.
  __device__ __forceinline__ void find(const SegTab& T, uint32_t f) {
    uint32_t p = 0, start = 0;
#pragma unroll
    for (uint32_t s = uint32_t(kSeg) / 2; s >= 1; s >>= 1) {
      const uint32_t q = T.P[p + s];
      if (q <= f) {
        p += s;
        start = q;
      }
    }
    j = p;
    nxt = T.P[p + 1];
    const uint2 sg = T.S[p];
    base = sg.x - start;
    wbase = kRaw ? sg.y : sg.y - start;
    bits = !kRaw && sg.y != uint32_t(kNoWords);
  }
};

// Walks flat indices lane, lane+64, ... < E of the segment table and counts
// the elements found in the staged set.  Against a staged bitmap every
// element costs the same: a uint value x tests bit x - base, a bitset word
// is ANDed with the bitmap word it overlaps, both as popc(R[w] & mask).  A
// composite set's members below its window are found by searching its prefix.
// Group mode counts x when bit (x - base) K + k is set, k the segment's item.
// kElems: no segment of the batch is bitset words (every element a member).
template <int RW, int U, bool kComposite, bool kGroup = false, bool kElems = false>
__device__ __forceinline__ uint32_t flat_probe_bits(const DevArgs& a, const SegTab& T, uint32_t E,
                                                    const Staged& st, const uint32_t* R,
                                                    const uint32_t* Lp, uint32_t lane) {
  const uint32_t* __restrict__ L = a.col;
  uint32_t cnt = 0;
  SegCursor<kGroup> c(T);
  const uint32_t base = st.base;
  for (uint32_t f0 = 0; f0 < E; f0 += kWave * U) {
    uint32_t val[U], key[U];
    bool ok[U], bits[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t f = f0 + uint32_t(u) * kWave + lane;
      ok[u] = f < E;
      val[u] = 0;
      key[u] = 0;
      bits[u] = false;
      if (ok[u]) {
        c.seek(T, f);
        val[u] = L[c.base + f];
        key[u] = kGroup ? c.wbase : c.wbase + f;
        bits[u] = c.bits;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t d = val[u] - base;
      if (kGroup) {
        const uint32_t pos = (d << st.glog) + key[u];
        if (ok[u] && d < st.glim) cnt += (R[pos >> 5] >> (pos & 31)) & 1u;
        continue;
      }
      if (kElems) {
        if (ok[u] && (d >> 5) < uint32_t(RW)) cnt += (R[d >> 5] >> (d & 31)) & 1u;
        else if (kComposite && ok[u]) cnt += prefix_has(a, st, Lp, val[u]);
        continue;
      }
      const uint32_t w = bits[u] ? key[u] : (d >> 5);
      const uint32_t m = bits[u] ? val[u] : (1u << (d & 31));
      if (ok[u] && w < uint32_t(RW)) cnt += __popc(R[w] & m);
      else if (kComposite && ok[u] && !bits[u]) cnt += prefix_has(a, st, Lp, val[u]);
    }
  }
  return cnt;
}

// The same count for short streamed sets, where one step of 64 would cross
// several of them: lane l takes the contiguous flat range [l per, (l+1) per)
// with per = ceil(E / 64), finds the set of its first element by a binary
// search of the length prefix and walks on from there, so a set boundary
// costs one cursor step instead of a search per element.
template <int RW, int U, bool kComposite, bool kGroup = false, bool kElems = false>
__device__ __forceinline__ uint32_t flat_probe_bits_blocked(const DevArgs& a, const SegTab& T,
                                                            uint32_t E, const Staged& st,
                                                            const uint32_t* R, const uint32_t* Lp,
                                                            uint32_t lane) {
  const uint32_t* __restrict__ L = a.col;
  const uint32_t per = (E + kWave - 1) / kWave;
  const uint32_t f_beg = lane * per;
  const uint32_t f_end = min(f_beg + per, E);
  uint32_t cnt = 0;
  if (f_beg >= f_end) return 0u;
  SegCursor<kGroup> c;
  c.find(T, f_beg);
  const uint32_t base = st.base;
  for (uint32_t f0 = f_beg; f0 < f_end; f0 += U) {
    uint32_t val[U], key[U];
    bool ok[U], bits[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t f = f0 + uint32_t(u);
      ok[u] = f < f_end;
      val[u] = 0;
      key[u] = 0;
      bits[u] = false;
      if (ok[u]) {
        c.seek(T, f);
        val[u] = L[c.base + f];
        key[u] = kGroup ? c.wbase : c.wbase + f;
        bits[u] = c.bits;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t d = val[u] - base;
      if (kGroup) {
        const uint32_t pos = (d << st.glog) + key[u];
        if (ok[u] && d < st.glim) cnt += (R[pos >> 5] >> (pos & 31)) & 1u;
        continue;
      }
      if (kElems) {
        if (ok[u] && (d >> 5) < uint32_t(RW)) cnt += (R[d >> 5] >> (d & 31)) & 1u;
        else if (kComposite && ok[u]) cnt += prefix_has(a, st, Lp, val[u]);
        continue;
      }
      const uint32_t w = bits[u] ? key[u] : (d >> 5);
      const uint32_t m = bits[u] ? val[u] : (1u << (d & 31));
      if (ok[u] && w < uint32_t(RW)) cnt += __popc(R[w] & m);
      else if (kComposite && ok[u] && !bits[u]) cnt += prefix_has(a, st, Lp, val[u]);
    }
  }
  return cnt;
}

// nseg: segments in the table.  When they average fewer than search_below
// elements, lanes take contiguous ranges (flat_probe_bits_blocked).
// elems: no segment of the batch is bitset words (wave-uniform).
template <int RW, int U>
__device__ __forceinline__ uint32_t flat_probe(const DevArgs& a, const SegTab& T, uint32_t E,
                                               uint32_t nseg, const Staged& st, const uint32_t* R,
                                               const uint32_t* Lp, uint32_t lane,
                                               bool elems = false) {
  const bool search = E < nseg * a.search_below;
  if (st.mode == kModeGroup)
    return search ? flat_probe_bits_blocked<RW, U, false, true>(a, T, E, st, R, Lp, lane)
                  : flat_probe_bits<RW, U, false, true>(a, T, E, st, R, Lp, lane);
  if (st.mode == kModeBitmap) {
    if (elems)
      return search ? flat_probe_bits_blocked<RW, U, false, false, true>(a, T, E, st, R, Lp, lane)
                    : flat_probe_bits<RW, U, false, false, true>(a, T, E, st, R, Lp, lane);
    return search ? flat_probe_bits_blocked<RW, U, false>(a, T, E, st, R, Lp, lane)
                  : flat_probe_bits<RW, U, false>(a, T, E, st, R, Lp, lane);
  }
  if (st.mode == kModeComposite) {
    // (the eight-element instance would spill with a fourth walk variant)
    if (U <= 4 && elems)
      return search ? flat_probe_bits_blocked<RW, U, true, false, true>(a, T, E, st, R, Lp, lane)
                    : flat_probe_bits<RW, U, true, false, true>(a, T, E, st, R, Lp, lane);
    return search ? flat_probe_bits_blocked<RW, U, true>(a, T, E, st, R, Lp, lane)
                  : flat_probe_bits<RW, U, true>(a, T, E, st, R, Lp, lane);
  }
  const uint32_t* __restrict__ L = a.col;
  uint32_t cnt = 0;
  SegCursor c(T);
  // list: uint elements only, searched
  for (uint32_t f0 = 0; f0 < E; f0 += kWave * U) {
    uint32_t val[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t f = f0 + uint32_t(u) * kWave + lane;
      ok[u] = f < E;
      val[u] = 0;
      if (ok[u]) {
        c.seek(T, f);
        val[u] = L[c.base + f];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (ok[u]) cnt += staged_has<RW>(a, st, R, Lp, val[u]);
  }
  return cnt;
}

// The Lollipop count's walk: as flat_probe_bits over a bitmap or composite
// staged set, and each element found also adds the weight W[j] of its
// segment j (the degree of the streamed set's vertex) to wsum.
template <int RW, int U>
__device__ __forceinline__ uint32_t flat_probe_weighted(const DevArgs& a, const SegTab& T,
                                                        const uint32_t* W, uint32_t E,
                                                        const Staged& st, const uint32_t* R,
                                                        const uint32_t* Lp, uint32_t lane,
                                                        unsigned long long& wsum) {
  const uint32_t* __restrict__ L = a.col;
  const bool comp = st.mode == kModeComposite;
  uint32_t cnt = 0;
  SegCursor<false> c(T);
  for (uint32_t f0 = 0; f0 < E; f0 += kWave * U) {
    uint32_t val[U], key[U], wt[U];
    bool ok[U], bits[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t f = f0 + uint32_t(u) * kWave + lane;
      ok[u] = f < E;
      val[u] = key[u] = wt[u] = 0;
      bits[u] = false;
      if (ok[u]) {
        c.seek(T, f);
        val[u] = L[c.base + f];
        key[u] = c.wbase + f;
        bits[u] = c.bits;
        wt[u] = W[c.j];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t d = val[u] - st.base;
      const uint32_t w = bits[u] ? key[u] : (d >> 5);
      const uint32_t m = bits[u] ? val[u] : (1u << (d & 31));
      uint32_t h = 0;
      if (ok[u] && w < uint32_t(RW)) h = __popc(R[w] & m);
      else if (comp && ok[u] && !bits[u]) h = prefix_has(a, st, Lp, val[u]);
      cnt += h;
      wsum += static_cast<unsigned long long>(h) * wt[u];
    }
  }
  return cnt;
}

// ---------------------------------------------------------------------------
// Triangles, staged: a group of K small items in one pass
// ---------------------------------------------------------------------------

// Counts a grouped item: members gsub[gi .. gi+K) ({first record, records,
// first staged member in col, staged members}), nrec records and descriptor
// sd = {bitmap base, log2 of the interleave, staged members, max member} in
// all.  Lane m < members stages one member of one set, lane r < nrec loads
// one record; the sets share the region interleaved and the streamed sets of
// all K items share one flat walk.  At most 4 members, 64 staged members and
// 64 records (the plan guarantees it).
template <int RW, int U>
__device__ __forceinline__ uint32_t grouped_item(const DevArgs& a, const SegTab& T, uint32_t* R,
                                                 const uint32_t* Lp, uint32_t gi, uint32_t K,
                                                 uint32_t nrec, const uint4& sd, uint32_t lane) {
  const uint32_t base = uniform(sd.x), glog = uniform(sd.y), nmem = uniform(sd.z);
  uint4 gs{0, 0, 0, 0};
  if (lane < K) gs = a.gsub[gi + lane];
  // lanes at or past K hold zeros, so the prefix sums stop growing there
  const uint32_t rb0 = __builtin_amdgcn_readlane(gs.x, 0), rb1 = __builtin_amdgcn_readlane(gs.x, 1);
  const uint32_t rb2 = __builtin_amdgcn_readlane(gs.x, 2), rb3 = __builtin_amdgcn_readlane(gs.x, 3);
  const uint32_t q1 = __builtin_amdgcn_readlane(gs.y, 0);
  const uint32_t q2 = q1 + __builtin_amdgcn_readlane(gs.y, 1);
  const uint32_t q3 = q2 + __builtin_amdgcn_readlane(gs.y, 2);
  const uint32_t mb0 = __builtin_amdgcn_readlane(gs.z, 0), mb1 = __builtin_amdgcn_readlane(gs.z, 1);
  const uint32_t mb2 = __builtin_amdgcn_readlane(gs.z, 2), mb3 = __builtin_amdgcn_readlane(gs.z, 3);
  const uint32_t p1 = __builtin_amdgcn_readlane(gs.w, 0);
  const uint32_t p2 = p1 + __builtin_amdgcn_readlane(gs.w, 1);
  const uint32_t p3 = p2 + __builtin_amdgcn_readlane(gs.w, 2);
  // records: lane r holds record r - q_k of item k
  Seg g{0, 0, 0};  // kRaw: sm is the item index
  if (lane < nrec) {
    const uint32_t k = uint32_t(lane >= q1) + uint32_t(lane >= q2) + uint32_t(lane >= q3);
    const uint32_t qk = k == 0 ? 0u : k == 1 ? q1 : k == 2 ? q2 : q3;
    const uint32_t bk = k == 0 ? rb0 : k == 1 ? rb1 : k == 2 ? rb2 : rb3;
    const uint2 r = a.rec[bk + lane - qk];
    g = Seg{r.x, r.y & 0xFFFFu, int32_t(k)};
  }
  // staging: lane m holds member m - p_k of set k, at bit (x - base) K + k
  uint32_t pos = 0;
  if (lane < nmem) {
    const uint32_t k = uint32_t(lane >= p1) + uint32_t(lane >= p2) + uint32_t(lane >= p3);
    const uint32_t pk = k == 0 ? 0u : k == 1 ? p1 : k == 2 ? p2 : p3;
    const uint32_t bk = k == 0 ? mb0 : k == 1 ? mb1 : k == 2 ? mb2 : mb3;
    const uint32_t x = a.col[bk + lane - pk];
    pos = ((x - base) << glog) + k;
    atomicOr(&R[pos >> 5], 1u << (pos & 31));
  }
  const uint32_t E = publish_segments(T, g, lane);  // also orders the staging
  Staged st;
  st.beg = st.len = st.lo = st.hi = st.plen = st.x0 = st.gb = 0;
  st.gw = kNoBitset;
  st.gp = nullptr;
  st.mode = kModeGroup;
  st.base = base;
  st.glog = glog;
  st.glim = (uint32_t(RW) * 32u) >> glog;
  const uint32_t cnt = flat_probe<RW, U>(a, T, E, nrec, st, R, Lp, lane);
  wave_sync();
  if (lane < nmem) R[pos >> 5] = 0;
  wave_sync();
  return cnt;
}

// ---------------------------------------------------------------------------
// Triangles, staged
// ---------------------------------------------------------------------------

// kLollipop: the symmetric relation's Lollipop count over each undirected
// edge once (kStageHalf plans, no grouped items): an edge {x, u} with c common
// neighbours adds c (|N(x)| + |N(u)|) -- u's part per item, x's per element
// found, weighted by its segment's degree.
template <int WPB, int RW, int U, bool kLollipop = false>
__device__ __forceinline__ void tri_staged(const DevArgs& a) {
  __shared__ uint32_t s_region[WPB][RW];
  __shared__ uint32_t s_pre[WPB][kSeg + 1];
  __shared__ uint2 s_seg[WPB][kSeg];
  __shared__ uint32_t s_pref[WPB][kPrefixCap];
  __shared__ uint32_t s_wt[kLollipop ? WPB : 1][kLollipop ? kSeg : 1];
  const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
  uint32_t* R = s_region[wid];
  uint32_t* Lp = s_pref[wid];
  const SegTab T{s_pre[wid], s_seg[wid]};
  for (uint32_t k = lane; k < uint32_t(RW); k += kWave) R[k] = 0;
  wave_sync();
  unsigned long long acc = 0;
  uint32_t cur_tag = 0;
  bool have_tag = false;
  ItemIter it(a, WPB);
  // the next item (and its staged-set descriptor) is loaded one item ahead
  Item nitem{0, 0, 0, 0};
  uint4 nsd{0, 0, 0, 0};
  if (it.more()) {
    nitem = a.items[it.idx()];
    if (a.sdesc) nsd = a.sdesc[it.idx()];
  }
  while (it.more()) {
    const Item item = nitem;
    const uint4 sd = nsd;
    it.next();
    if (it.more()) {
      nitem = a.items[it.idx()];
      if (a.sdesc) nsd = a.sdesc[it.idx()];
    }
    const uint32_t s = uniform(item.s), lbeg = uniform(item.lbeg), llen = uniform(item.llen);
    const uint32_t tag = uniform(item.tag);
    if (have_tag && tag != cur_tag) flush_tag(a, acc, cur_tag, lane);
    cur_tag = tag;
    have_tag = true;
    if (a.gsub && (s & kHiBit)) {
      acc += grouped_item<RW, U>(a, T, R, Lp, s & kMaxIndex, lbeg, llen, sd, lane);
      continue;
    }
    // the first batch of segment records is loaded beside the staged set
    uint2 r0{0, 0};
    if (a.rec && lane < min(uint32_t(kSeg), llen)) r0 = a.rec[lbeg + lane];
    const Staged st = a.sdesc ? stage_extent<RW>(a, uniform(sd.x), uniform(sd.y), uniform(sd.z),
                                                 uniform(sd.w), R, Lp, lane)
                              : stage_set<RW>(a, s, R, Lp, lane);
    if (st.len == 0) continue;
    const WordRule wr = word_rule(a, st);
    uint32_t cnt = 0;
    for (uint32_t b0 = 0; b0 < llen; b0 += kSeg) {
      const uint32_t nseg = min(uint32_t(kSeg), llen - b0);
      Seg g{0, 0, kNoWords};
      uint32_t wt = 0;
      if (lane < nseg) {
        if (a.rec) {
          // resolved at plan time: one load per streamed set
          const uint2 r = b0 == 0 ? r0 : a.rec[lbeg + b0 + lane];
          g = Seg{r.x, r.y & 0xFFFFu, (r.y & kHiBit) ? int32_t((r.y >> 16) & 0x7FFFu) : kNoWords};
        } else {
          const uint32_t t = a.idx[lbeg + b0 + lane];
          g = seg_full(a, t, wr);
          if (kLollipop) wt = a.vdesc[t].y & kMaxIndex;
        }
      }
      // a batch with no bitset words takes the element-only walk
      const bool elems = __ballot(lane < nseg && g.sm != kNoWords) == 0;
      const uint32_t E = publish_segments(T, g, lane);
      if constexpr (kLollipop) {
        // the previous batch's readers finished before publish_segments
        s_wt[wid][lane] = wt;
        wave_sync();
        cnt += flat_probe_weighted<RW, U>(a, T, s_wt[wid], E, st, R, Lp, lane, acc);
      } else {
        cnt += flat_probe<RW, U>(a, T, E, nseg, st, R, Lp, lane, elems);
      }
    }
    if constexpr (kLollipop) acc += static_cast<unsigned long long>(cnt) * st.len;
    else acc += cnt;
    if (a.per_root) {
      const unsigned long long tot = wave_sum((unsigned long long)cnt);
      if (lane == 0 && tot) atomicAdd(&a.per_root[a.vert[s]], tot);
    }
    unstage_set<RW>(a, st, R, lane);
  }
  if (have_tag) flush_tag(a, acc, cur_tag, lane);
}

// At least 6 waves per SIMD: the LDS budget allows 7 blocks of 4 waves per CU.
template <int WPB, int RW, int U>
__global__ __launch_bounds__(WPB * kWave) __attribute__((amdgpu_waves_per_eu(6)))
void k_tri_staged(DevArgs a) {
  tri_staged<WPB, RW, U>(a);
}

// Half-size staged region and two streamed elements in flight per lane: it
// fits 64 VGPRs and 13 KB of LDS per block, so 8 waves per SIMD.  Many small
// items are latency-bound, and more waves hide more of it.
template <int WPB, int RW, int U>
__global__ __launch_bounds__(WPB * kWave) __attribute__((amdgpu_waves_per_eu(8)))
void k_tri_staged_lean(DevArgs a) {
  tri_staged<WPB, RW, U>(a);
}

template <int WPB, int RW, int U>
__global__ __launch_bounds__(WPB * kWave) __attribute__((amdgpu_waves_per_eu(6)))
void k_lollipop_staged(DevArgs a) {
  tri_staged<WPB, RW, U, true>(a);
}

// ---------------------------------------------------------------------------
// 4-cliques, staged: N+(u) in region A; per v, S = N+(u) & N+(v) is written
// in order to list S and (bitmap mode) to bitmap B; level 2 streams N+(w)
// for w in S against B (or searches the list S).
// ---------------------------------------------------------------------------

// SCAP > 0: S is an LDS list of SCAP entries.  SCAP == 0: S lives in HBM, in
// wave w's list a.k4s[w k4s_stride ..] (roots whose out-degree exceeds any
// LDS list); S's members below the staged window are then searched there.
template <int WPB, int RW, int SCAP, int U>
__global__ __launch_bounds__(WPB * kWave) void k_k4_staged(DevArgs a) {
  constexpr bool kGlb = SCAP == 0;
  __shared__ uint32_t s_A[WPB][RW];
  __shared__ uint32_t s_B[WPB][RW];
  __shared__ uint32_t s_S[WPB][kGlb ? 1 : SCAP];
  __shared__ uint32_t s_pre[WPB][kSeg + 1];
  __shared__ uint2 s_seg[WPB][kSeg];
  __shared__ uint32_t s_pref[WPB][kPrefixCap];
  const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
  uint32_t* A = s_A[wid];
  uint32_t* B = s_B[wid];
  uint32_t* S = kGlb ? a.k4s + size_t(blockIdx.x * WPB + wid) * a.k4s_stride : s_S[wid];
  uint32_t* Lp = s_pref[wid];
  const SegTab T{s_pre[wid], s_seg[wid]};
  for (uint32_t k = lane; k < uint32_t(RW); k += kWave) { A[k] = 0; B[k] = 0; }
  wave_sync();
  const unsigned long long lt_mask = (1ull << lane) - 1ull;
  unsigned long long acc = 0;
  uint32_t cur_tag = 0;
  bool have_tag = false;
  for (ItemIter it(a, WPB); it.more(); it.next()) {
    const Item item = a.items[it.idx()];
    const uint32_t u = uniform(item.s), lbeg = uniform(item.lbeg), llen = uniform(item.llen);
    const uint32_t tag = uniform(item.tag);
    if (have_tag && tag != cur_tag) flush_tag(a, acc, cur_tag, lane);
    cur_tag = tag;
    have_tag = true;
    // |S| <= d+(u): a launch of this instance takes only the items whose S
    // fits its list (the others go to an instance with a longer one)
    const uint32_t du = uniform(a.vdesc[u].y & kMaxIndex);
    if (du <= a.deg_lo || du > a.deg_hi) continue;
    const Staged su = stage_set<RW>(a, u, A, Lp, lane);
    if (su.len == 0) continue;
    const bool su_bits = su.mode == kModeBitmap || su.mode == kModeComposite;
    uint32_t cnt = 0;
    for (uint32_t q = 0; q < llen; ++q) {
      // S lies in N+(v) and, on pruned data, in the part of N+(u) after v:
      // with fewer than two members in either, no 4-clique extends (u, v)
      // (nor, for the second, any later v).  The unpruned relation has no
      // such order: S may hold members of N(u) before v.
      if (!a.symmetric && su.beg + su.len - (lbeg + q) - 1 < 2) break;
      const uint32_t v = uniform(a.idx[lbeg + q]);
      const uint2 vd = a.vdesc[v];
      const uint32_t vb = uniform(vd.x), vl = uniform(vd.y & kMaxIndex);
      if (vl < 2) continue;
      // level 1: S = N+(u) & N+(v), compacted in ascending order; members at
      // or above the window base also go into bitmap B (same base as A)
      uint32_t ns = 0, nlow = 0;
      for (uint32_t k0 = 0; k0 < vl; k0 += kWave) {
        const uint32_t k = k0 + lane;
        uint32_t x = 0, hit = 0;
        if (k < vl) {
          x = a.col[vb + k];
          hit = staged_has<RW>(a, su, A, Lp, x);
        }
        const unsigned long long m = __ballot(hit);
        if (hit) {
          S[ns + __popcll(m & lt_mask)] = x;
          if (su_bits && x >= su.base) {
            const uint32_t d = x - su.base;
            atomicOr(&B[d >> 5], 1u << (d & 31));
          }
        }
        nlow += uint32_t(__popcll(__ballot(hit && x < su.base)));
        ns += uint32_t(__popcll(m));
      }
      if (kGlb) __threadfence_block();  // the list's stores before its loads
      wave_sync();
      if (ns >= 2) {
        // level 2: sum over w in S of |S & N+(w)|, against bitmap B when it
        // holds all of S; else (LDS list) by searching the sorted list S, or
        // (HBM list) B for members in the window and a search of S's prefix
        // below it
        Staged ss;
        ss.beg = 0;
        ss.len = ns;
        ss.lo = S[0];
        ss.hi = S[ns - 1];
        ss.plen = 0;
        ss.x0 = ss.gb = 0;
        ss.gw = kNoBitset;
        ss.gp = nullptr;
        ss.base = su.base;
        ss.glog = ss.glim = 0;
        if (kGlb) {
          ss.mode = nlow ? kModeComposite : kModeBitmap;
          ss.plen = nlow;
          ss.gp = S;
        } else {
          ss.mode = (su_bits && nlow == 0) ? kModeBitmap : kModeList;
        }
        const uint32_t* probe = ss.mode == kModeList ? S : B;
        const WordRule wr = word_rule(a, ss);
        for (uint32_t b0 = 0; b0 < ns; b0 += kSeg) {
          const uint32_t nseg = min(uint32_t(kSeg), ns - b0);
          Seg g{0, 0, kNoWords};
          if (lane < nseg) g = seg_full<true>(a, S[b0 + lane], wr);
          const uint32_t E = publish_segments(T, g, lane);
          // bitmap bounds are B's (RW words); the list S is searched by length
          cnt += flat_probe<RW, U>(a, T, E, nseg, ss, probe, Lp, lane);
        }
      }
      wave_sync();
      if (su_bits)
        for (uint32_t i = nlow + lane; i < ns; i += kWave) B[(S[i] - su.base) >> 5] = 0;
      wave_sync();
    }
    acc += cnt;
    if (a.per_root) {
      const unsigned long long tot = wave_sum((unsigned long long)cnt);
      if (lane == 0 && tot) atomicAdd(&a.per_root[a.vert[u]], tot);
    }
    unstage_set<RW>(a, su, A, lane);
  }
  if (have_tag) flush_tag(a, acc, cur_tag, lane);
}

// ---------------------------------------------------------------------------
// 4-cliques over a root's induced out-neighbourhood
// ---------------------------------------------------------------------------

// For a root u with N+(u) = {v_0 < ... < v_{d-1}}, row i holds
// T_i = N+(v_i) & N+(u) as a bitset over local ids (v_j is bit j): the join's
// second-level set for (u, v_i), in the bitset layout over the root's own
// domain.  The third level's sets are then T_i & T_j for j in T_i (bits of
// T_j all lie above j), counted by word AND and popcount in LDS (section
// 4.2's bitset-bitset intersection), so each N+(v) is read once per root
// instead of once per triangle it closes.
// N+(u) is held as a composite set (section 4.3): a bitmap of nw <= RW words
// from wb (the top window, or all of N+(u)) and the plen members below wb
// (the first plen of the sorted list), which a streamed element below the
// window is searched in.  A member's local id is its index in the list:
// below the window, the search's result; in it, plen plus the members in the
// words below and below it in its word.  The plan resolves per root
// {position of N+(u), d | plen << 10 | nw << 20, first segment record, wb}
// and per row the streamed part of N+(v_i) as a segment record, so a root
// costs one dependent load before its members and records arrive.  Blocks
// of WPB waves take the roots, each with 3 <= d <= DMAX.
// kItems (rooted requests of a server): the roots are the work items a.items
// (root s, request slot tag), each count added to a.acc[tag - tag_base]; the
// window, plen and the streamed sets are found from the trie on the fly
// (elements beyond max N+(u) and words outside the window simply miss).
template <int WPB, int RW, int DMAX, int U, bool kItems>
__global__ __launch_bounds__(WPB * kWave) void k_k4_local(DevArgs a) {
  constexpr uint32_t W = DMAX / 32;       // words per row
  // row stride: rows start in different banks; rows of more than 4 words
  // start on 8-byte boundaries, so that the third level reads word pairs
  constexpr uint32_t RS = W <= 4 ? W + 1 : W + 2;
  constexpr uint32_t NT = WPB * kWave;
  __shared__ uint32_t s_a[RW];            // the window's bitmap
  __shared__ uint16_t s_p[RW];            // members in the window's words below
  __shared__ uint32_t s_u[DMAX];          // N+(u), sorted
  __shared__ __align__(16) uint32_t s_m[DMAX * RS];  // rows T_i
  __shared__ uint32_t s_pre[WPB][kSeg + 1];
  __shared__ uint2 s_seg[WPB][kSeg];
  __shared__ uint32_t s_plen;
  // third level of rows of more than 4 words: pairs per row, scanned, and
  // the waves' sums
  __shared__ uint32_t s_pc[W > 4 ? DMAX : 1];
  __shared__ uint32_t s_wt[WPB];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
  const SegTab T{s_pre[wid], s_seg[wid]};
  const uint32_t* __restrict__ L = a.col;
  for (uint32_t k = tid; k < uint32_t(RW); k += NT) s_a[k] = 0;
  for (uint32_t k = tid; k < DMAX * RS; k += NT) s_m[k] = 0;
  if (tid == 0) s_plen = 0;
  __syncthreads();
  unsigned long long acc = 0;
  // roots come by decreasing estimated cost.  The class of out-degree <= 64
  // (many roots per block) deals them boustrophedon: block b takes b, 2G-1-b,
  // 2G+b, 4G-1-b, ... (G blocks), so that every block's share costs about the
  // same.  The other classes' blocks hold one or two roots each and start as
  // the CUs free up beside the other classes, so they take the next root from
  // a cursor when done with one (the costliest first)
  constexpr bool kGrab = DMAX > 64 && !kItems;
  __shared__ uint32_t s_root;
  const uint64_t G = gridDim.x;
  const uint64_t n_roots = kItems ? a.n_items : a.n_roots;
  for (uint64_t k = 0;; ++k) {
    uint64_t r;
    if (kGrab) {
      if (tid == 0) s_root = atomicAdd(a.cursor, 1u);
      __syncthreads();
      r = s_root;
    } else {
      r = k * G + ((k & 1) ? G - 1 - blockIdx.x : blockIdx.x);
    }
    if (r >= n_roots) break;
    uint32_t beg, d, plen, nw, roff = 0, wb, tag = 0;
    uint2 rc0{0, 0};
    if constexpr (kItems) {
      const Item it = a.items[r];
      tag = it.tag;
      const uint2 ud = a.vdesc[it.s];
      beg = ud.x;
      d = ud.y & kMaxIndex;
      const uint32_t lo = L[beg], hi = L[beg + d - 1];
      // window base: a multiple of 32 with hi - wb < 32 RW, as low as possible
      wb = hi - (lo & ~31u) < uint32_t(RW) * 32u ? (lo & ~31u)
                                                 : ((hi + 1u - uint32_t(RW) * 32u + 31u) & ~31u);
      nw = ((hi - wb) >> 5) + 1;
      for (uint32_t k = tid; k < d; k += NT) {
        const uint32_t x = L[beg + k];
        s_u[k] = x;
        if (x >= wb) {
          atomicOr(&s_a[(x - wb) >> 5], 1u << ((x - wb) & 31));
          if (k == 0 || L[beg + k - 1] < wb) s_plen = k;
        }
      }
      __syncthreads();
      plen = s_plen;
    } else {
      const uint4 rr = a.roots[r];
      beg = rr.x;
      d = rr.y & 1023u;
      plen = (rr.y >> 10) & 1023u;
      nw = rr.y >> 20;
      roff = rr.z;
      wb = rr.w;
      // the wave's first batch of segment records is loaded beside the members
      if (wid + WPB * lane + 1 < d) rc0 = a.rec[roff + wid + WPB * lane];
      for (uint32_t k = tid; k < d; k += NT) {
        const uint32_t x = L[beg + k];
        s_u[k] = x;
        if (k >= plen) atomicOr(&s_a[(x - wb) >> 5], 1u << ((x - wb) & 31));
      }
      __syncthreads();
    }
    if (wid == 0) {
      // s_p[w]: window members in words [0, w), lane l summing a run of words
      const uint32_t per = (nw + kWave - 1) / kWave, w0 = lane * per, w1 = min(w0 + per, nw);
      uint32_t sum = 0;
      for (uint32_t w = w0; w < w1; ++w) sum += __popc(s_a[w]);
      uint32_t run = wave_incl_scan(sum, lane) - sum;
      for (uint32_t w = w0; w < w1; ++w) {
        s_p[w] = uint16_t(run);
        run += __popc(s_a[w]);
      }
    }
    __syncthreads();
    // rows T_0 .. T_{d-2} (v_{d-1} has no later member in N+(u)), 64 rows per
    // flat batch; wave w takes rows w, w + WPB, w + 2 WPB, ..., so that the
    // waves' shares of a root cost about the same
    for (uint32_t b0 = 0; b0 + wid + 1 < d; b0 += NT) {
      const uint32_t rb = b0 + wid;  // row of the batch's segment j: rb + WPB j
      const uint32_t nseg = min(uint32_t(kSeg), (d - 1 - rb + WPB - 1) / WPB);
      Seg g{0, 0, kNoWords};
      if (lane < nseg) {
        const uint32_t row = rb + WPB * lane;
        if constexpr (kItems) {
          // a row below the window streams words only from a bitset inside it
          const WordRule wr{a.use_bitsets != 0, wb, row < plen ? wb : 0u};
          g = seg_full<true>(a, s_u[row], wr);
        } else {
          const uint2 rc = b0 == 0 ? rc0 : a.rec[roff + row];
          g = Seg{rc.x, rc.y & 0x3FFFFFu,
                  (rc.y & kHiBit) ? int32_t((rc.y >> 22) & 0x1FFu) : kNoWords};
        }
      }
      const uint32_t E = publish_segments(T, g, lane);
      // an element x tests bit x - wb; a bitset word (key: its index from
      // wb's word) is ANDed whole; an element below the window is searched
      // an element's segment, packed to save registers: its row (bits 0-9),
      // whether it is a bitset word (bit 10) and, for a word, its index from
      // wb's word (bits 16-31; 0xFFFF when outside the window)
      constexpr uint32_t kNone = 0xFFFFFFFFu;
      auto pack = [&](const SegCursor<false>& c, uint32_t f) {
        const uint32_t key = c.wbase + f;
        return (rb + WPB * c.j) | (c.bits ? (1u << 10) : 0u) | ((key < nw ? key : 0xFFFFu) << 16);
      };
      auto take = [&](uint32_t val, uint32_t info) {
        const bool bits = (info >> 10) & 1u;
        const uint32_t row = info & 1023u;
        const uint32_t dx = val - wb;
        const uint32_t w = bits ? (info >> 16) : (dx >> 5);
        uint32_t m = 0;
        if (w < nw) m = s_a[w] & (bits ? val : (1u << (dx & 31)));
        uint32_t* R = s_m + row * RS;
        while (m) {
          const uint32_t b = uint32_t(__builtin_ctz(m));
          m &= m - 1u;
          const uint32_t j = plen + s_p[w] + __popc(s_a[w] & ((1u << b) - 1u));
          atomicOr(&R[j >> 5], 1u << (j & 31));
        }
        if (plen && !bits && val < wb) {
          const uint32_t j = lower_bound_lds(s_u, plen, val);
          if (j < plen && s_u[j] == val) atomicOr(&R[j >> 5], 1u << (j & 31));
        }
      };
      // a batch with no bitset words takes element-only walks
      const bool elems = __ballot(lane < nseg && g.sm != kNoWords) == 0;
      auto take_elem = [&](uint32_t val, uint32_t row) {
        const uint32_t dx = val - wb;
        uint32_t* R = s_m + row * RS;
        if ((dx >> 5) < nw) {
          const uint32_t aw = s_a[dx >> 5];
          if ((aw >> (dx & 31)) & 1u) {
            const uint32_t j = plen + s_p[dx >> 5] + __popc(aw & ((1u << (dx & 31)) - 1u));
            atomicOr(&R[j >> 5], 1u << (j & 31));
          }
        } else if (plen && val < wb) {
          const uint32_t j = lower_bound_lds(s_u, plen, val);
          if (j < plen && s_u[j] == val) atomicOr(&R[j >> 5], 1u << (j & 31));
        }
      };
      const bool blocked = E < nseg * a.search_below;
      // the walk, instantiated for element-only batches (kE) and for batches
      // with bitset words
      auto walk = [&](auto kE) {
        constexpr bool kElemsOnly = decltype(kE)::value;
        auto seek = [&](SegCursor<false>& c, uint32_t f) {
          if constexpr (kElemsOnly) c.seek_base(T, f);
          else c.seek(T, f);
        };
        auto tag_of = [&](const SegCursor<false>& c, uint32_t f) {
          if constexpr (kElemsOnly) return rb + WPB * c.j;
          else return pack(c, f);
        };
        auto use = [&](uint32_t v, uint32_t info) {
          if constexpr (kElemsOnly) take_elem(v, info);
          else take(v, info);
        };
        if (blocked) {
          // short sets: lane l walks the contiguous flat range [l per, (l+1) per)
          const uint32_t per = (E + kWave - 1) / kWave;
          const uint32_t f_beg = lane * per, f_end = min(f_beg + per, E);
          if (f_beg < f_end) {
            SegCursor<false> c;
            c.find(T, f_beg);
            for (uint32_t f0 = f_beg; f0 < f_end; f0 += U) {
              uint32_t val[U], info[U];
#pragma unroll
              for (int q = 0; q < U; ++q) {
                const uint32_t f = f0 + uint32_t(q);
                val[q] = 0;
                info[q] = kNone;
                if (f < f_end) {
                  seek(c, f);
                  val[q] = L[c.base + f];
                  info[q] = tag_of(c, f);
                }
              }
#pragma unroll
              for (int q = 0; q < U; ++q)
                if (info[q] != kNone) use(val[q], info[q]);
            }
          }
        } else {
          SegCursor<false> c(T);
          for (uint32_t f0 = 0; f0 < E; f0 += kWave * U) {
            uint32_t val[U], info[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
              const uint32_t f = f0 + uint32_t(q) * kWave + lane;
              val[q] = 0;
              info[q] = kNone;
              if (f < E) {
                seek(c, f);
                val[q] = L[c.base + f];
                info[q] = tag_of(c, f);
              }
            }
#pragma unroll
            for (int q = 0; q < U; ++q)
              if (info[q] != kNone) use(val[q], info[q]);
          }
        }
      };
      if (elems)
        walk(std::true_type{});
      else
        walk(std::false_type{});
    }
    __syncthreads();
    // sum over rows i <= d-3 (a pair needs two later members) and members j
    // of T_i of |T_i & T_j|; T_j's bits lie above j, so only the words from
    // j's on are ANDed
    uint32_t cnt = 0;
    const uint32_t wd = (d + 31) >> 5;  // words that can hold a member
    if constexpr (W <= 4) {
      // short rows: one row per lane, T_i in registers
      for (uint32_t i = wid * kWave + lane; i + 2 < d; i += NT) {
        const uint32_t* Ti = s_m + i * RS;
        uint32_t t[W];
#pragma unroll
        for (uint32_t w = 0; w < W; ++w) t[w] = Ti[w];
#pragma unroll
        for (uint32_t w = 0; w < W; ++w) {
          uint32_t bm = t[w];
          while (bm) {
            const uint32_t j = w * 32u + uint32_t(__builtin_ctz(bm));
            bm &= bm - 1u;
            const uint32_t* Tj = s_m + j * RS;
#pragma unroll
            for (uint32_t v = w; v < W; ++v) cnt += __popc(t[v] & Tj[v]);
          }
        }
      }
    } else {
      // longer rows: the pairs (i, j), j in T_i, taken in row order, are
      // dealt to the block's lanes in equal contiguous shares, so that no
      // lane waits on a longer row; s_pc[i] = pairs in the rows below i
      uint32_t pc = 0;
      if (tid + 2 < d)
        for (uint32_t w = (tid + 1) >> 5; w < wd; ++w) pc += __popc(s_m[tid * RS + w]);
      const uint32_t incl = wave_incl_scan(pc, lane);
      if (lane == kWave - 1) s_wt[wid] = incl;
      __syncthreads();
      uint32_t before = 0, total = 0;
#pragma unroll
      for (uint32_t k = 0; k < uint32_t(WPB); ++k) {
        before += k < wid ? s_wt[k] : 0u;
        total += s_wt[k];
      }
      if (tid + 2 < d) s_pc[tid] = before + incl - pc;
      __syncthreads();
      const uint32_t f0 = uint32_t(uint64_t(total) * tid / NT);
      const uint32_t f1 = uint32_t(uint64_t(total) * (tid + 1) / NT);
      if (f0 < f1) {
        // the pair f0: its row (the last with s_pc[i] <= f0), word and bit
        uint32_t i = 0;
        for (uint32_t n = d - 2; n > 1;) {
          const uint32_t h = n >> 1;
          if (s_pc[i + h] <= f0) i += h;
          n -= h;
        }
        const uint32_t* Ti = s_m + i * RS;
        uint32_t k = f0 - s_pc[i], w = (i + 1) >> 5, bm = Ti[w];
        while (k >= uint32_t(__popc(bm))) {
          k -= uint32_t(__popc(bm));
          bm = Ti[++w];
        }
        for (; k; --k) bm &= bm - 1u;
        for (uint32_t f = f0; f < f1; ++f) {
          while (bm == 0 && i + 2 < d) {
            if (++w >= wd) {
              ++i;
              Ti += RS;
              w = (i + 1) >> 5;
            }
            bm = Ti[w];
          }
          const uint32_t j = w * 32u + uint32_t(__builtin_ctz(bm));
          bm &= bm - 1u;
          // word pairs from the pair holding j's word (T_j's words below
          // j's are zero, and so are both rows' words from wd on)
          const uint2* Ti2 = reinterpret_cast<const uint2*>(Ti);
          const uint2* Tj2 = reinterpret_cast<const uint2*>(s_m + j * RS);
          for (uint32_t v = w >> 1; v < (wd + 1) >> 1; ++v) {
            const uint2 x = Ti2[v], y = Tj2[v];
            cnt += __popc(x.x & y.x) + __popc(x.y & y.y);
          }
        }
      }
    }
    if constexpr (kItems) {
      const unsigned long long tot = wave_sum((unsigned long long)cnt);
      if (lane == 0 && tot) atomicAdd(&a.acc[tag - a.tag_base], tot);
    } else {
      acc += cnt;
    }
    __syncthreads();
    for (uint32_t k = tid; k < d * RS; k += NT) s_m[k] = 0;
    for (uint32_t k = plen + tid; k < d; k += NT) s_a[(s_u[k] - wb) >> 5] = 0;
    if (kItems && tid == 0) s_plen = 0;
    __syncthreads();
  }
  if constexpr (!kItems) {
    const unsigned long long tot = wave_sum(acc);
    if (lane == 0 && tot) atomicAdd(&a.acc[0], tot);
  }
}

// ---------------------------------------------------------------------------
// Triangles, pairwise (both sets from HBM), G lanes per pair
// ---------------------------------------------------------------------------

template <int G>
__device__ __forceinline__ uint32_t pair_count(const DevArgs& a, uint32_t s, uint32_t t,
                                               uint32_t gl) {
  const uint2 sd = a.vdesc[s], td = a.vdesc[t];
  uint32_t sl = sd.y & kMaxIndex, tl = td.y & kMaxIndex;
  if (sl == 0 || tl == 0) return 0;
  const bool sbs = a.use_bitsets && (sd.y & kHiBit);
  const bool tbs = a.use_bitsets && (td.y & kHiBit);
  uint32_t cnt = 0;
  if (sbs && tbs) {
    // bitset & bitset: AND the overlapping 32-bit words, popcount
    const uint4 bs = a.bsdesc[s], bt = a.bsdesc[t];
    const uint32_t w0 = max(bs.y, bt.y) >> 5;
    const uint32_t e_s = (bs.y >> 5) + bs.z, e_t = (bt.y >> 5) + bt.z;
    const uint32_t w1 = min(e_s, e_t);
    for (uint32_t w = w0 + gl; w < w1; w += G)
      cnt += __popc(a.bsw[bs.x + (w - (bs.y >> 5))] & a.bsw[bt.x + (w - (bt.y >> 5))]);
    return cnt;
  }
  if (sbs || tbs) {
    // uint & bitset: probe each uint value in the bitset
    const uint4 b = a.bsdesc[sbs ? s : t];
    const uint32_t ub = sbs ? td.x : sd.x, ul = sbs ? tl : sl;
    for (uint32_t k = gl; k < ul; k += G) {
      const uint32_t d = a.col[ub + k] - b.y;
      if (d < b.z * 32u) cnt += (a.bsw[b.x + (d >> 5)] >> (d & 31)) & 1u;
    }
    return cnt;
  }
  // uint & uint: A shorter, B longer
  const uint32_t* Ap = a.col + (sl <= tl ? sd.x : td.x);
  const uint32_t* Bp = a.col + (sl <= tl ? td.x : sd.x);
  const uint32_t na = min(sl, tl), nb = max(sl, tl);
  const bool search = a.algo == EH_ALGO_SEARCH ||
                      (a.algo == EH_ALGO_AUTO && float(nb) > a.gamma * float(na));
  if (search) {
    // galloping regime: each value of the shorter list searched in the longer
    for (uint32_t k = gl; k < na; k += G) {
      const uint32_t x = Ap[k];
      const uint32_t p = lower_bound_glb(Bp, nb, x);
      cnt += (p < nb && Bp[p] == x) ? 1u : 0u;
    }
    return cnt;
  }
  // partitioned merge: lane gl owns A[a0, a1) and merges it with B from
  // lower_bound(B, A[a0]); every match is found by exactly one lane
  const uint32_t chunk = (na + G - 1) / G;
  const uint32_t a0 = gl * chunk, a1 = min(a0 + chunk, na);
  if (a0 >= a1) return 0;
  uint32_t i = a0, j = lower_bound_glb(Bp, nb, Ap[a0]);
  uint32_t x = Ap[i];
  uint32_t y = j < nb ? Bp[j] : 0u;
  while (i < a1 && j < nb) {
    if (x < y) { if (++i < a1) x = Ap[i]; }
    else if (x > y) { if (++j < nb) y = Bp[j]; }
    else {
      ++cnt;
      if (++i < a1) x = Ap[i];
      if (++j < nb) y = Bp[j];
    }
  }
  return cnt;
}

template <int WPB, int G>
__global__ __launch_bounds__(WPB * kWave) void k_tri_pairwise(DevArgs a) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t grp = lane / G, gl = lane % G;
  constexpr uint32_t kGroups = kWave / G;
  unsigned long long acc = 0;
  uint32_t cur_tag = 0;
  bool have_tag = false;
  for (ItemIter it(a, WPB); it.more(); it.next()) {
    const Item item = a.items[it.idx()];
    const uint32_t s = uniform(item.s), lbeg = uniform(item.lbeg), llen = uniform(item.llen);
    const uint32_t tag = uniform(item.tag);
    if (have_tag && tag != cur_tag) flush_tag(a, acc, cur_tag, lane);
    cur_tag = tag;
    have_tag = true;
    uint32_t cnt = 0;
    for (uint32_t q = grp; q < llen; q += kGroups) cnt += pair_count<G>(a, s, a.idx[lbeg + q], gl);
    acc += cnt;
    if (a.per_root) {
      const unsigned long long tot = wave_sum((unsigned long long)cnt);
      if (lane == 0 && tot) atomicAdd(&a.per_root[a.vert[s]], tot);
    }
  }
  if (have_tag) flush_tag(a, acc, cur_tag, lane);
}

__global__ void k_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += uint64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

// Copies pieces {first source item, first destination item, items, 0} of
// work items: one block per piece, its lanes striding over the piece.
__global__ void k_gather_items(const Item* __restrict__ src, const uint4* __restrict__ pieces,
                               uint32_t n_pieces, Item* __restrict__ dst) {
  for (uint32_t p = blockIdx.x; p < n_pieces; p += gridDim.x) {
    const uint4 pc = pieces[p];
    for (uint32_t k = threadIdx.x; k < pc.z; k += blockDim.x) dst[pc.y + k] = src[pc.x + k];
  }
}

__global__ void k_scatter_roots(const unsigned long long* by_rank, const uint32_t* vert,
                                unsigned long long* by_id, uint32_t n) {
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
    by_id[vert[r]] = by_rank[r];
}

constexpr int kTriWPB = 4;
constexpr int kTriRW = int(kStageWords);  // 32768-bit staging range, or 1024-entry list
constexpr int kTriU = 8;
constexpr int kK4WPB = 2;
constexpr int kK4RW = int(kStageWords);
constexpr int kK4U = 2;
constexpr int kPairWPB = 4;

uint32_t grid_for(Ctx* c, uint64_t n_items, uint32_t wpb, uint32_t waves_per_cu) {
  uint64_t want = (uint64_t(c->n_cu) * std::max<uint32_t>(waves_per_cu, wpb) + wpb - 1) / wpb;
  const uint64_t need = (n_items + wpb - 1) / wpb;
  if (want > need) want = need;
  // a multiple of the L2-domain count keeps the block renumbering a bijection
  const uint64_t x = (c->tune.dynamic == 3 && !c->tune.xcds) ? 8 : c->tune.xcds;
  if (x > 1 && want > x) want -= want % x;
  if (want < 1) want = 1;
  return uint32_t(std::min<uint64_t>(want, 1u << 20));
}

}  // namespace

// Device address of `scratch` on the current device, looked up once per
// device (the first context created on it) and kept for the process.
eh_status noalloc_scratch_init(Ctx* c) {
  static std::mutex mu;
  static std::unordered_map<int, void*> by_device;
  std::lock_guard<std::mutex> lk(mu);
  auto it = by_device.find(c->device);
  if (it == by_device.end()) {
    void* p = nullptr;
    const eh_status st = hip_check(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
                                   "hipGetSymbolAddress(scratch)");
    if (st != EH_OK) return st;
    if (!p) {
      c->err = "hipGetSymbolAddress(scratch) returned a null address";
      return EH_EHIP;
    }
    it = by_device.emplace(c->device, p).first;
  }
  c->noalloc_scratch = it->second;
  return EH_OK;
}

eh_status launch_fill_u64(Ctx* c, hipStream_t s, unsigned long long* p, uint64_t n,
                          unsigned long long v) {
  if (n == 0) return EH_OK;
  const uint32_t blocks = uint32_t(std::min<uint64_t>((n + 255) / 256, 4096));
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks), dim3(256), 0, s, p, n, v);
  return hip_check(c, hipGetLastError(), "fill kernel launch");
}

eh_status launch_gather_items(Ctx* c, hipStream_t s, const Item* src, const uint4* pieces,
                              uint32_t n_pieces, Item* dst) {
  if (n_pieces == 0) return EH_OK;
  hipLaunchKernelGGL(k_gather_items, dim3(std::min<uint32_t>(n_pieces, 4096)), dim3(256), 0, s, src,
                     pieces, n_pieces, dst);
  return hip_check(c, hipGetLastError(), "gather kernel launch");
}

eh_status launch_scatter_roots(Ctx* c, hipStream_t s, const unsigned long long* by_rank,
                               const uint32_t* vert, unsigned long long* by_id, uint32_t n) {
  if (n == 0) return EH_OK;
  const uint32_t blocks = std::min<uint32_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_scatter_roots, dim3(blocks), dim3(256), 0, s, by_rank, vert, by_id, n);
  return hip_check(c, hipGetLastError(), "scatter kernel launch");
}

// Zeroes the work cursors of schedules 1 and 4 ahead of a launch.
eh_status reset_cursors(Ctx* c, hipStream_t s, const LaunchArgs& la) {
  if (la.dynamic != 1 && la.dynamic != 4) return EH_OK;
  return launch_fill_u64(c, s, reinterpret_cast<unsigned long long*>(la.cursor),
                         uint64_t(kCursorWords) * kMaxParts / 2, 0);
}

eh_status launch_triangles(Ctx* c, hipStream_t s, const LaunchArgs& la, uint32_t kernel,
                           uint32_t waves_per_cu) {
  if (la.n_items == 0) return EH_OK;
  const DevArgs a = to_dev(la);
  if (eh_status st = reset_cursors(c, s, la); st != EH_OK) return st;
  if (kernel == EH_KERNEL_PAIRWISE) {
    uint32_t g = la.group_lanes;
    if (g == 0) g = la.dmax >= 256 ? 64 : la.dmax >= 64 ? 16 : 4;
    const uint32_t grid = grid_for(c, la.n_items, kPairWPB, waves_per_cu);
    const dim3 blk(kPairWPB * kWave);
    switch (g) {
      case 4: hipLaunchKernelGGL((k_tri_pairwise<kPairWPB, 4>), dim3(grid), blk, 0, s, a); break;
      case 8: hipLaunchKernelGGL((k_tri_pairwise<kPairWPB, 8>), dim3(grid), blk, 0, s, a); break;
      case 16: hipLaunchKernelGGL((k_tri_pairwise<kPairWPB, 16>), dim3(grid), blk, 0, s, a); break;
      case 32: hipLaunchKernelGGL((k_tri_pairwise<kPairWPB, 32>), dim3(grid), blk, 0, s, a); break;
      case 64: hipLaunchKernelGGL((k_tri_pairwise<kPairWPB, 64>), dim3(grid), blk, 0, s, a); break;
      default:
        c->err = "group_lanes must be 4, 8, 16, 32 or 64";
        return EH_EINVAL;
    }
    return hip_check(c, hipGetLastError(), "pairwise triangle kernel launch");
  }
  const uint32_t grid = grid_for(c, la.n_items, kTriWPB, waves_per_cu);
  if (la.stage_words > 0 && la.stage_words <= uint32_t(kTriRW) / 2)
    hipLaunchKernelGGL((k_tri_staged_lean<kTriWPB, kTriRW / 2, 2>), dim3(grid),
                       dim3(kTriWPB * kWave), 0, s, a);
  else if (la.unroll == 4)
    hipLaunchKernelGGL((k_tri_staged<kTriWPB, kTriRW, 4>), dim3(grid), dim3(kTriWPB * kWave), 0, s,
                       a);
  else
    hipLaunchKernelGGL((k_tri_staged<kTriWPB, kTriRW, kTriU>), dim3(grid), dim3(kTriWPB * kWave), 0,
                       s, a);
  return hip_check(c, hipGetLastError(), "staged triangle kernel launch");
}

eh_status launch_lollipop(Ctx* c, hipStream_t s, const LaunchArgs& la, uint32_t waves_per_cu) {
  if (la.n_items == 0) return EH_OK;
  if (la.rec || la.gsub || la.sdesc || !la.symmetric) {
    c->err = "the Lollipop launch takes a symmetric trie's edge-once plan";
    return EH_EINVAL;
  }
  if (eh_status st = reset_cursors(c, s, la); st != EH_OK) return st;
  const uint32_t grid = grid_for(c, la.n_items, kTriWPB, waves_per_cu);
  hipLaunchKernelGGL((k_lollipop_staged<kTriWPB, kTriRW, 4>), dim3(grid),
                     dim3(kTriWPB * kWave), 0, s, to_dev(la));
  return hip_check(c, hipGetLastError(), "Lollipop kernel launch");
}

eh_status launch_4cliques_local_items(Ctx* c, hipStream_t s, const LaunchArgs& la, int k) {
  if (la.n_items == 0) return EH_OK;
  static constexpr uint32_t kPerCu[kK4LocalClasses] = {32, 28, 9, 3};
  const DevArgs d = to_dev(la);
  const uint32_t grid = uint32_t(std::min<uint64_t>(la.n_items, uint64_t(c->n_cu) * kPerCu[k]));
  constexpr int RW = int(kK4LocalWords);
  if (k == 0)
    hipLaunchKernelGGL((k_k4_local<1, RW / 2, 64, 8, true>), dim3(grid), dim3(kWave), 0, s, d);
  else if (k == 1)
    hipLaunchKernelGGL((k_k4_local<1, RW / 2, 128, 8, true>), dim3(grid), dim3(kWave), 0, s, d);
  else if (k == 2)
    hipLaunchKernelGGL((k_k4_local<4, RW, 256, 8, true>), dim3(grid), dim3(4 * kWave), 0, s, d);
  else
    hipLaunchKernelGGL((k_k4_local<8, RW, 512, 8, true>), dim3(grid), dim3(8 * kWave), 0, s, d);
  return hip_check(c, hipGetLastError(), "induced-neighbourhood 4-clique launch (items)");
}

eh_status launch_4cliques_local(Ctx* c, hipStream_t s, const LaunchArgs& la,
                               const uint64_t n[kK4LocalClasses]) {
  // one wave per root at out-degree <= 64 and <= 128 (a 256-word window),
  // four at <= 256 and eight at <= 512.  Blocks per CU: a class alone fills
  // the CUs as the LDS allows; classes side by side take smaller grids, whose
  // blocks the CUs hold together (R-MAT s18 4-cliques: 0.61 ms against
  // 0.65 ms with the full grids)
  static constexpr uint32_t kAlone[kK4LocalClasses] = {32, 28, 9, 3};
  static constexpr uint32_t kShared[kK4LocalClasses] = {16, 16, 6, 3};
  const int present = (n[0] != 0) + (n[1] != 0) + (n[2] != 0) + (n[3] != 0);
  const uint32_t* kPerCu = present > 1 ? kShared : kAlone;
  // the classes run side by side: the first on s, each other on a side
  // stream of the context forked from s before the first launch, joined
  // back into s at the end
  if (n[1] || n[2] || n[3]) {
    // the cursors of the classes that take roots from one start at zero
    if (!la.root_cursors) {
      c->err = "the 4-clique root classes above out-degree 64 need their cursors";
      return EH_EINVAL;
    }
    if (eh_status st = launch_fill_u64(c, s, reinterpret_cast<unsigned long long*>(la.root_cursors),
                                       uint64_t(kCursorWords) * kK4LocalClasses / 2, 0);
        st != EH_OK)
      return st;
  }
  if (n[1] || n[2] || n[3])
    if (eh_status st = hip_check(c, hipEventRecord(c->fork, s), "fork event"); st != EH_OK)
      return st;
  uint64_t off = 0;
  for (int k = 0; k < int(kK4LocalClasses); ++k) {
    if (n[k] == 0) continue;
    DevArgs d = to_dev(la);
    d.roots = la.roots + off;
    d.n_roots = n[k];
    d.cursor = la.root_cursors ? la.root_cursors + uint64_t(k) * kCursorWords : nullptr;
    off += n[k];
    hipStream_t ks = s;
    if (k > 0) {
      ks = c->side[k - 1];
      if (eh_status st = hip_check(c, hipStreamWaitEvent(ks, c->fork, 0), "fork wait");
          st != EH_OK)
        return st;
    }
    const uint32_t grid = uint32_t(std::min<uint64_t>(n[k], uint64_t(c->n_cu) * kPerCu[k]));
    constexpr int RW = int(kK4LocalWords);
    static_assert(RW / 2 == int(k4_local_window(0)) && RW / 2 == int(k4_local_window(1)) &&
                  RW == int(k4_local_window(2)) && RW == int(k4_local_window(3)),
                  "the planner's windows are the kernels'");
    if (k == 0)
      hipLaunchKernelGGL((k_k4_local<1, RW / 2, 64, 8, false>), dim3(grid), dim3(kWave), 0, ks, d);
    else if (k == 1)
      hipLaunchKernelGGL((k_k4_local<1, RW / 2, 128, 8, false>), dim3(grid), dim3(kWave), 0, ks, d);
    else if (k == 2)
      hipLaunchKernelGGL((k_k4_local<4, RW, 256, 8, false>), dim3(grid), dim3(4 * kWave), 0, ks, d);
    else
      hipLaunchKernelGGL((k_k4_local<8, RW, 512, 8, false>), dim3(grid), dim3(8 * kWave), 0, ks, d);
    eh_status st = hip_check(c, hipGetLastError(), "induced-neighbourhood 4-clique launch");
    if (st == EH_OK && k > 0) {
      st = hip_check(c, hipEventRecord(c->join[k - 1], ks), "join event");
      if (st == EH_OK) st = hip_check(c, hipStreamWaitEvent(s, c->join[k - 1], 0), "join wait");
    }
    if (st != EH_OK) return st;
  }
  return EH_OK;
}

eh_status launch_4cliques(Ctx* c, hipStream_t s, const LaunchArgs& la, uint32_t /*kernel*/,
                          uint32_t waves_per_cu) {
  if (la.n_items == 0) return EH_OK;
  const uint32_t grid = grid_for(c, la.n_items, kK4WPB, waves_per_cu);
  const dim3 blk(kK4WPB * kWave);
  // S = N+(u) & N+(v) has at most d+(u) members.  Items with d+(u) <= 512
  // run in an instance with a 512-entry S list (and, for stage_words in
  // (0, 512], a half-size staged region): less LDS, more waves per CU.  Only
  // when some item's d+(u) exceeds 512 does a second launch, over the same
  // items, take those with an S list sized for the largest out-degree up to
  // kK4ListMax, and only when some exceeds that does a third take them with
  // S in HBM (per-wave lists the caller provides).
  const uint32_t bound = la.item_dmax ? la.item_dmax : la.dmax;
  if (bound > kK4ListMax && (!la.k4s || la.k4s_stride < bound || la.k4s_waves < kK4WPB)) {
    c->err = "4-clique roots of out-degree above " + std::to_string(kK4ListMax) +
             " need per-wave S lists in HBM of at least " + std::to_string(bound) +
             " entries, which this launch was not given";
    return EH_EOVERFLOW;
  }
  const bool half = la.stage_words > 0 && la.stage_words <= kK4RW / 2;
  LaunchArgs light = la;
  light.deg_lo = 0;
  light.deg_hi = 512;
  const DevArgs al = to_dev(light);
  eh_status st = reset_cursors(c, s, la);
  if (st != EH_OK) return st;
  if (half)
    hipLaunchKernelGGL((k_k4_staged<kK4WPB, kK4RW / 2, 512, kK4U>), dim3(grid), blk, 0, s, al);
  else
    hipLaunchKernelGGL((k_k4_staged<kK4WPB, kK4RW, 512, kK4U>), dim3(grid), blk, 0, s, al);
  st = hip_check(c, hipGetLastError(), "staged 4-clique kernel launch");
  if (st != EH_OK || bound <= 512) return st;
  LaunchArgs heavy = la;
  heavy.deg_lo = 512;
  heavy.deg_hi = kK4ListMax;
  const DevArgs ah = to_dev(heavy);
  if ((st = reset_cursors(c, s, la)) != EH_OK) return st;
  if (bound <= 1024)
    hipLaunchKernelGGL((k_k4_staged<kK4WPB, kK4RW, 1024, kK4U>), dim3(grid), blk, 0, s, ah);
  else
    hipLaunchKernelGGL((k_k4_staged<kK4WPB, kK4RW, 2048, kK4U>), dim3(grid), blk, 0, s, ah);
  st = hip_check(c, hipGetLastError(), "staged 4-clique kernel launch (high out-degree)");
  if (st != EH_OK || bound <= kK4ListMax) return st;
  // S in HBM: one list per wave, so the grid is exactly the lists' waves
  LaunchArgs hub = la;
  hub.deg_lo = kK4ListMax;
  hub.deg_hi = 0xFFFFFFFFu;
  const DevArgs ahub = to_dev(hub);
  if ((st = reset_cursors(c, s, la)) != EH_OK) return st;
  hipLaunchKernelGGL((k_k4_staged<kK4WPB, kK4RW, 0, kK4U>), dim3(la.k4s_waves / kK4WPB), blk, 0, s,
                     ahub);
  return hip_check(c, hipGetLastError(), "staged 4-clique kernel launch (S lists in HBM)");
}

eh_status prepare_k4_lists(Ctx* c, const HostTrie& h, const Item* items, uint64_t n_items,
                           DevBuf& buf, uint32_t& waves, uint32_t& stride) {
  uint64_t heavy = 0;
  uint32_t dmax = 0;
  for (uint64_t i = 0; i < n_items; ++i) {
    const uint32_t d = h.row[items[i].s + 1] - h.row[items[i].s];
    if (d > kK4ListMax) {
      ++heavy;
      dmax = std::max(dmax, d);
    }
  }
  if (!heavy) return EH_OK;
  uint64_t w = std::min<uint64_t>(uint64_t(c->n_cu) * 4, heavy);
  w = (w + kK4WPB - 1) / kK4WPB * kK4WPB;
  if (buf.p && stride >= dmax && waves >= w) return EH_OK;
  dev_free(c, buf);
  waves = stride = 0;
  const eh_status st = dev_alloc(c, buf, sizeof(uint32_t) * size_t(dmax) * w);
  if (st != EH_OK) return st;
  waves = uint32_t(w);
  stride = dmax;
  return EH_OK;
}

}  // namespace eh
