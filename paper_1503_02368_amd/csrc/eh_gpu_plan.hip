// Work-item plan for target staging, built on the GPU from the trie's device
// arrays.  It follows the host planner (get_plan) rule for rule, so both give
// the same items, descriptors, grouped members and segment records:
//
//   1. transpose: a radix sort of (target << 32 | position) keys orders the
//      in-edges by target, then by source (positions grow with the source);
//   2. items: per target v, the in-edges are cut greedily into items of about
//      chunk_work streamed elements, each item charged |N+(v)| for staging
//      (count, scan, write);
//   3. grouping: per graph, consecutive small whole-vertex items share a wave
//      under the host's limits (count, scan, write);
//   4. records: per in-edge, the streamed part of N+(u) above v, as elements
//      or as bitset words clipped to the staged bitmap's window.
#include <cstring>
#include <hip/hip_runtime.h>
#include <rocprim/rocprim.hpp>

#include <algorithm>
#include <vector>

#include "eh_internal.h"

namespace eh {
namespace {

constexpr uint32_t kB = 256;

uint32_t grid_of(uint64_t n) {
  return uint32_t(std::max<uint64_t>(1, std::min<uint64_t>((n + kB - 1) / kB, 1u << 16)));
}
__device__ inline uint64_t gtid() { return uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; }
__device__ inline uint64_t gstride() { return uint64_t(gridDim.x) * blockDim.x; }

__global__ void __launch_bounds__(kB) k_fill_u32_plan(uint32_t* __restrict__ p, uint64_t n,
                                                      uint32_t v) {
  for (uint64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}

__global__ void __launch_bounds__(kB) k_fill_u8_plan(uint8_t* __restrict__ p, uint64_t n) {
  for (uint64_t i = gtid(); i < n; i += gstride()) p[i] = 0;
}

struct TrieView {
  const uint2* vdesc;   // {row begin, out-degree | kHiBit if bitset}
  const uint32_t* col;  // members, then words
  const uint4* bsdesc;  // {first word, base, words, 0}, or null
  uint32_t n;
};

__device__ inline uint32_t outdeg(const TrieView& t, uint32_t v) {
  return t.vdesc[v].y & kMaxIndex;
}

// Streamed elements of the part of N+(u) above v = col[e] (the host's suffix_len).
__device__ inline uint32_t suffix_len(const TrieView& t, uint32_t u, uint32_t e, bool ub) {
  const uint2 du = t.vdesc[u];
  const uint32_t len = du.x + (du.y & kMaxIndex) - e - 1;
  if (ub && len && (du.y & kHiBit)) {
    const uint4 b = t.bsdesc[u];
    const uint32_t w0 = (t.col[e] + 1 - b.y) >> 5;
    const uint32_t nw = w0 < b.z ? b.z - w0 : 0;
    if (nw < len) return nw;
  }
  return len;
}

__global__ void __launch_bounds__(kB) k_sources(TrieView t, uint32_t* __restrict__ src) {
  for (uint64_t u = gtid(); u < t.n; u += gstride()) {
    const uint2 d = t.vdesc[u];
    for (uint32_t e = d.x; e < d.x + (d.y & kMaxIndex); ++e) src[e] = uint32_t(u);
  }
}

__global__ void __launch_bounds__(kB) k_target_keys(TrieView t, uint64_t m,
                                                    unsigned long long* __restrict__ key) {
  for (uint64_t e = gtid(); e < m; e += gstride())
    key[e] = (static_cast<unsigned long long>(t.col[e]) << 32) | e;
}

// tin[k] = {u, e} of the k-th in-edge; trow[v] = first in-edge of v.
__global__ void __launch_bounds__(kB) k_in_edges(const unsigned long long* __restrict__ key,
                                                 uint64_t m, const uint32_t* __restrict__ src,
                                                 uint2* __restrict__ tin) {
  for (uint64_t k = gtid(); k < m; k += gstride()) {
    const uint32_t e = uint32_t(key[k]);
    tin[k] = make_uint2(src[e], e);
  }
}

__global__ void __launch_bounds__(kB) k_in_rows(const unsigned long long* __restrict__ key,
                                                uint64_t m, uint32_t n,
                                                uint32_t* __restrict__ trow) {
  for (uint64_t r = gtid(); r <= n; r += gstride()) {
    const unsigned long long want = static_cast<unsigned long long>(r) << 32;
    uint64_t lo = 0, hi = m;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (key[mid] < want) lo = mid + 1;
      else hi = mid;
    }
    trow[r] = uint32_t(lo);
  }
}

__device__ inline uint32_t graph_of(const uint32_t* vbase, uint32_t n_graphs, uint32_t v) {
  uint32_t lo = 0, hi = n_graphs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (vbase[mid] <= v) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Work of each in-edge for item cutting: its streamed elements plus 2.
__global__ void __launch_bounds__(kB) k_in_edge_costs(TrieView t, const uint2* __restrict__ tin,
                                                      uint64_t m, uint32_t ub,
                                                      uint32_t* __restrict__ cost) {
  for (uint64_t k = gtid(); k < m; k += gstride())
    cost[k] = suffix_len(t, tin[k].x, tin[k].y, ub != 0) + 2;
}

// Greedy cut of v's in-edges (the host's split_items): an item starting at
// in-edge i, charged |N+(v)| for staging, ends after the first in-edge at
// which its work reaches chunk.  Costs are positive, so with Q the inclusive
// prefix of the costs that end is a lower bound on Q: one binary search per
// item instead of a walk.  With `out` null it only counts the items.
__device__ inline uint32_t cut_items(const TrieView& t, const unsigned long long* Q,
                                     const uint32_t* trow, uint32_t v, uint32_t chunk,
                                     uint32_t tag, Item* out) {
  const uint32_t dv = outdeg(t, v);
  const uint32_t lb = trow[v], len = trow[v + 1] - lb;
  if (dv == 0 || len == 0) return 0;
  uint32_t n = 0, i = 0;
  while (i < len) {
    uint32_t j;
    if (dv >= chunk) {
      j = i + 1;  // the first in-edge already reaches chunk
    } else {
      // smallest k in [lb+i, lb+len) with Q[k] - Q[lb+i-1] >= chunk - dv
      const unsigned long long before = lb + i > 0 ? Q[lb + i - 1] : 0ull;
      const unsigned long long want = before + (chunk - dv);
      uint32_t lo = lb + i, hi = lb + len;
      while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (Q[mid] < want) lo = mid + 1;
        else hi = mid;
      }
      j = lo < lb + len ? lo - lb + 1 : len;
    }
    if (out) out[n] = Item{v, lb + i, j - i, tag};
    ++n;
    i = j;
  }
  return n;
}

__global__ void __launch_bounds__(kB) k_count_items(TrieView t,
                                                    const unsigned long long* __restrict__ Q,
                                                    const uint32_t* __restrict__ trow,
                                                    uint32_t chunk, uint32_t* __restrict__ cnt) {
  for (uint64_t v = gtid(); v <= t.n; v += gstride())
    cnt[v] = v < t.n ? cut_items(t, Q, trow, uint32_t(v), chunk, 0, nullptr) : 0u;
}

__global__ void __launch_bounds__(kB) k_write_items(TrieView t,
                                                    const unsigned long long* __restrict__ Q,
                                                    const uint32_t* __restrict__ trow,
                                                    uint32_t chunk,
                                                    const unsigned long long* __restrict__ ioff,
                                                    const uint32_t* __restrict__ vbase,
                                                    uint32_t n_graphs, Item* __restrict__ items,
                                                    uint32_t* __restrict__ dmax) {
  uint32_t mx = 0;
  for (uint64_t v = gtid(); v < t.n; v += gstride()) {
    if (ioff[v + 1] == ioff[v]) continue;
    const uint32_t tag = n_graphs > 1 ? graph_of(vbase, n_graphs, uint32_t(v)) : 0u;
    cut_items(t, Q, trow, uint32_t(v), chunk, tag, items + ioff[v]);
    mx = max(mx, outdeg(t, uint32_t(v)));
  }
  // one atomic per wave
  for (int o = 32; o; o >>= 1) mx = max(mx, uint32_t(__shfl_xor(int(mx), o)));
  if ((threadIdx.x & 63u) == 0 && mx) atomicMax(dmax, mx);
}

// Graph g's items start at the first item whose vertex is at or above vbase[g].
__global__ void __launch_bounds__(kB) k_graph_offsets(const Item* __restrict__ items,
                                                      uint64_t n_items,
                                                      const uint32_t* __restrict__ vbase,
                                                      uint32_t n_graphs,
                                                      unsigned long long* __restrict__ goff) {
  for (uint64_t g = gtid(); g <= n_graphs; g += gstride()) {
    uint64_t lo = 0, hi = n_items;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (items[mid].s < vbase[g]) lo = mid + 1;
      else hi = mid;
    }
    goff[g] = lo;
  }
}

// Staged-set descriptor of a single vertex's item: {begin, length, min, max}.
__device__ inline uint4 single_desc(const TrieView& t, uint32_t v) {
  const uint2 d = t.vdesc[v];
  const uint32_t len = d.y & kMaxIndex;
  return make_uint4(d.x, len, t.col[d.x], t.col[d.x + len - 1]);
}

__global__ void __launch_bounds__(kB) k_single_descs(TrieView t, const Item* __restrict__ items,
                                                     uint64_t n_items, uint4* __restrict__ sd) {
  for (uint64_t i = gtid(); i < n_items; i += gstride()) sd[i] = single_desc(t, items[i].s);
}

// Per item, what the grouping pass reads: {|N+(v)| | 2^31 if the item holds
// all of v's in-edges, min N+(v), max N+(v), in-edges of the item}.
__global__ void __launch_bounds__(kB) k_item_info(TrieView t, const Item* __restrict__ items,
                                                  uint64_t n_items,
                                                  const uint32_t* __restrict__ trow,
                                                  uint4* __restrict__ info) {
  for (uint64_t i = gtid(); i < n_items; i += gstride()) {
    const Item it = items[i];
    const uint2 d = t.vdesc[it.s];
    const uint32_t dv = d.y & kMaxIndex;
    const bool whole = it.lbeg == trow[it.s] && it.llen == trow[it.s + 1] - trow[it.s];
    info[i] = make_uint4(dv | (whole ? kHiBit : 0u), t.col[d.x], t.col[d.x + dv - 1], it.llen);
  }
}

// One graph's grouping pass (the host's rule) over the item facts, read
// contiguously: with the outputs null it only counts output items and grouped
// members.
__device__ inline void group_graph(const TrieView& t, const Item* items, const uint4* info,
                                   uint64_t i0, uint64_t i1, uint32_t group, uint32_t cap,
                                   uint64_t* n_out, uint64_t* n_mem, Item* out, uint4* sd,
                                   uint4* gsub, uint64_t gsub_base, uint8_t* grouped) {
  uint64_t no = 0, nm = 0;
  for (uint64_t i = i0; i < i1;) {
    // the facts of the at most 4 items a group can span, loaded together
    uint4 fa[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) fa[q] = i + q < i1 ? info[i + q] : make_uint4(0, 0, 0, 0);
    const uint4 f0 = fa[0];
    uint64_t j = i + 1;
    if (f0.x & kHiBit) {
      uint32_t base = f0.y, top = f0.z;
      uint32_t recs = f0.w, mem = f0.x & kMaxIndex;
      while (j < i1 && j - i < group && (fa[j - i].x & kHiBit)) {
        const uint4 f = fa[j - i];
        const uint32_t dv = f.x & kMaxIndex;
        const uint32_t nb = min(base, f.y);
        const uint32_t nt = max(top, f.z);
        const uint64_t kk = (j - i + 1) <= 2 ? 2 : 4;
        if (recs + f.w > 64 || mem + dv > 64 || (uint64_t(nt) - nb + 1) * kk > uint64_t(cap) * 32)
          break;
        base = nb;
        top = nt;
        recs += f.w;
        mem += dv;
        ++j;
      }
      if (j - i > 1) {
        const uint32_t cnt = uint32_t(j - i);
        if (out) {
          out[no] = Item{uint32_t((gsub_base + nm)) | kHiBit, cnt, recs, items[i].tag};
          sd[no] = make_uint4(base, cnt <= 2 ? 1u : 2u, mem, top);
          for (uint64_t q = i; q < j; ++q) {
            const uint32_t v = items[q].s;
            const uint2 d = t.vdesc[v];
            grouped[v] = 1;
            gsub[nm + (q - i)] = make_uint4(items[q].lbeg, items[q].llen, d.x, d.y & kMaxIndex);
          }
        }
        ++no;
        nm += j - i;
        i = j;
        continue;
      }
    }
    if (out) {
      out[no] = items[i];
      sd[no] = single_desc(t, items[i].s);
    }
    ++no;
    i = i + 1;
  }
  *n_out = no;
  *n_mem = nm;
}

// Grouping runs over chunks of at most kGroupChunk consecutive items of one
// graph (a group never spans two chunks), so that a large graph's items are
// grouped by many threads.  nch[g]: graph g's chunks (the entry past the last
// graph 0, for the scan's total).
constexpr uint32_t kGroupChunk = 256;

__global__ void __launch_bounds__(kB) k_chunk_counts(const unsigned long long* __restrict__ goff,
                                                     uint32_t n_graphs,
                                                     unsigned long long* __restrict__ nch) {
  for (uint64_t g = gtid(); g <= n_graphs; g += gstride())
    nch[g] = g < n_graphs ? (goff[g + 1] - goff[g] + kGroupChunk - 1) / kGroupChunk : 0;
}

// cb[c]: the first item of chunk c (choff: the chunk scan); cb[n_chunks] = end.
__global__ void __launch_bounds__(kB) k_chunk_bounds(const unsigned long long* __restrict__ goff,
                                                     const unsigned long long* __restrict__ choff,
                                                     uint32_t n_graphs,
                                                     unsigned long long* __restrict__ cb) {
  for (uint64_t g = gtid(); g <= n_graphs; g += gstride()) {
    if (g == n_graphs) {
      cb[choff[g]] = goff[g];
      continue;
    }
    for (uint64_t c = choff[g]; c < choff[g + 1]; ++c)
      cb[c] = goff[g] + (c - choff[g]) * kGroupChunk;
  }
}

// Per graph, the first output item: the output offset of its first chunk.
__global__ void __launch_bounds__(kB) k_graph_out(const unsigned long long* __restrict__ choff,
                                                  const unsigned long long* __restrict__ o_off,
                                                  uint32_t n_graphs,
                                                  unsigned long long* __restrict__ g_out) {
  for (uint64_t g = gtid(); g <= n_graphs; g += gstride()) g_out[g] = o_off[choff[g]];
}

__global__ void __launch_bounds__(kB) k_group_count(TrieView t, const Item* __restrict__ items,
                                                    const uint4* __restrict__ info,
                                                    const unsigned long long* __restrict__ cb,
                                                    uint64_t n_chunks, uint32_t group, uint32_t cap,
                                                    unsigned long long* __restrict__ n_out,
                                                    unsigned long long* __restrict__ n_mem) {
  for (uint64_t c = gtid(); c <= n_chunks; c += gstride()) {
    uint64_t no = 0, nm = 0;
    if (c < n_chunks)
      group_graph(t, items, info, cb[c], cb[c + 1], group, cap, &no, &nm, nullptr, nullptr,
                  nullptr, 0, nullptr);
    n_out[c] = no;
    n_mem[c] = nm;
  }
}

__global__ void __launch_bounds__(kB) k_group_write(TrieView t, const Item* __restrict__ items,
                                                    const uint4* __restrict__ info,
                                                    const unsigned long long* __restrict__ cb,
                                                    uint64_t n_chunks, uint32_t group, uint32_t cap,
                                                    const unsigned long long* __restrict__ o_off,
                                                    const unsigned long long* __restrict__ m_off,
                                                    Item* __restrict__ out, uint4* __restrict__ sd,
                                                    uint4* __restrict__ gsub,
                                                    uint8_t* __restrict__ grouped) {
  for (uint64_t c = gtid(); c < n_chunks; c += gstride()) {
    uint64_t no = 0, nm = 0;
    group_graph(t, items, info, cb[c], cb[c + 1], group, cap, &no, &nm, out + o_off[c],
                sd + o_off[c], gsub + m_off[c], m_off[c], grouped);
  }
}

// The host's segment record per in-edge k (target v = col[e]): {start,
// length | word offset << 16 | kHiBit for words}; *wide flags a length beyond
// 16 bits or an offset beyond 15.
__global__ void __launch_bounds__(kB) k_records(TrieView t, const unsigned long long* __restrict__ key,
                                                const uint2* __restrict__ tin, uint64_t m,
                                                const uint8_t* __restrict__ grouped, uint32_t ub,
                                                uint32_t cap, uint2* __restrict__ rec,
                                                uint32_t* __restrict__ wide) {
  for (uint64_t k = gtid(); k < m; k += gstride()) {
    const uint32_t v = uint32_t(key[k] >> 32);
    const uint32_t u = tin[k].x, e = tin[k].y;
    const uint2 du = t.vdesc[u], dv = t.vdesc[v];
    const uint32_t len = du.x + (du.y & kMaxIndex) - e - 1;
    uint32_t sb = e + 1, n = len, sm = 0, wf = 0;
    const uint32_t lv = dv.y & kMaxIndex;
    if (ub && len && !grouped[v] && (du.y & kHiBit) && lv > 0) {
      const uint32_t lo_al = t.col[dv.x] & ~31u, hi = t.col[dv.x + lv - 1];
      if (hi - lo_al < cap * 32u) {
        const uint4 b = t.bsdesc[u];
        const uint32_t w0 = (v + 1 - b.y) >> 5;
        const int64_t nw = w0 < b.z ? int64_t(b.z - w0) : 0;
        const int64_t off = int64_t((b.y >> 5) + w0) - int64_t(lo_al >> 5);
        const int64_t first = off < 0 ? -off : 0;
        const int64_t last = min(nw, int64_t(cap) - off);
        const int64_t words = last > first ? last - first : 0;
        if (words < int64_t(len)) {
          sb = b.x + w0 + uint32_t(first);
          n = uint32_t(words);
          sm = words ? uint32_t(off + first) : 0u;
          wf = kHiBit;
        }
      }
    }
    if (n > 0xFFFFu || sm > 0x7FFFu) {
      atomicOr(wide, 1u);
      continue;
    }
    rec[k] = make_uint2(sb, n | (sm << 16) | wf);
  }
}

template <class T>
T* ptr(DevBuf& b) {
  return static_cast<T*>(b.p);
}

}  // namespace

namespace {

// Estimated cost of each work item, in the planners' units (streamed
// elements plus 2 per streamed set, plus the held set's members), as the key
// (~cost << 32 | item) whose ascending sort puts the costliest items first.
// Target staging reads the records (grouped items: their members' records);
// source staging the streamed vertices' out-degrees, and for 4-cliques the
// second level's estimate min(d+(u), d+(v)) * 24 per streamed vertex.
__global__ void __launch_bounds__(kB) k_item_cost_keys(TrieView t, const Item* __restrict__ items,
                                                       uint64_t n_items,
                                                       const uint4* __restrict__ sdesc,
                                                       const uint2* __restrict__ rec,
                                                       const uint4* __restrict__ gsub,
                                                       uint32_t target, uint32_t k4,
                                                       unsigned long long* __restrict__ key) {
  for (uint64_t i = gtid(); i < n_items; i += gstride()) {
    const Item it = items[i];
    uint64_t cost = 0;
    if (target) {
      if (gsub && (it.s & kHiBit)) {
        const uint32_t gi = it.s & kMaxIndex;
        for (uint32_t k = 0; k < it.lbeg; ++k) {
          const uint4 g = gsub[gi + k];
          cost += g.w;
          for (uint32_t r = 0; r < g.y; ++r) cost += (rec[g.x + r].y & 0xFFFFu) + 2;
        }
      } else {
        if (sdesc) cost += sdesc[i].y;
        for (uint32_t r = 0; r < it.llen; ++r) cost += (rec[it.lbeg + r].y & 0xFFFFu) + 2;
      }
    } else {
      const uint32_t du = outdeg(t, it.s);
      cost = du;
      for (uint32_t q = 0; q < it.llen; ++q) {
        const uint32_t dv = outdeg(t, t.col[it.lbeg + q]);
        cost += uint64_t(dv) + 2 + (k4 ? uint64_t(min(du, dv)) * 24 : 0);
      }
    }
    const uint32_t c32 = cost > 0xFFFFFFFFull ? 0xFFFFFFFFu : uint32_t(cost);
    key[i] = (uint64_t(~c32) << 32) | uint64_t(i);
  }
}

__global__ void __launch_bounds__(kB) k_permute_items(const unsigned long long* __restrict__ key,
                                                      uint64_t n_items, const Item* __restrict__ in,
                                                      const uint4* __restrict__ sd_in,
                                                      Item* __restrict__ out,
                                                      uint4* __restrict__ sd_out) {
  for (uint64_t j = gtid(); j < n_items; j += gstride()) {
    const uint32_t i = uint32_t(key[j] & 0xFFFFFFFFull);
    out[j] = in[i];
    if (sd_in) sd_out[j] = sd_in[i];
  }
}

}  // namespace

eh_status device_plan_balance(Ctx* c, Trie& tr, Plan& plan) {
  const uint64_t n = plan.n_items;
  if (n < 2) return EH_OK;
  if (n > 0xFFFFFFFFull) {
    c->err = "too many work items to sort by cost";
    return EH_EOVERFLOW;
  }
  const HostTrie& h = tr.host;
  hipStream_t s = c->stream;
  TrieView tv{static_cast<const uint2*>(tr.vdesc.p), static_cast<const uint32_t*>(tr.col.p),
              h.n_bs ? static_cast<const uint4*>(tr.bsdesc.p) : nullptr, h.n};
  const bool target = plan.staging == EH_STAGE_TARGET && plan.pattern == EH_TRIANGLE;
  DevBuf key_a, key_b, tmp, items2, sd2;
  auto cleanup = [&]() {
    dev_free(c, key_a);
    dev_free(c, key_b);
    dev_free(c, tmp);
    dev_free(c, items2);
    dev_free(c, sd2);
  };
  auto chk = [&](hipError_t e, const char* what) { return hip_check(c, e, what); };
  eh_status st;
  if ((st = dev_alloc(c, key_a, 8 * n)) != EH_OK || (st = dev_alloc(c, key_b, 8 * n)) != EH_OK ||
      (st = dev_alloc(c, items2, sizeof(Item) * n)) != EH_OK ||
      (plan.sdesc.p && (st = dev_alloc(c, sd2, sizeof(uint4) * n)) != EH_OK)) {
    cleanup();
    return st;
  }
  rocprim::double_buffer<unsigned long long> db(static_cast<unsigned long long*>(key_a.p),
                                                static_cast<unsigned long long*>(key_b.p));
  size_t tb = 0;
  if ((st = chk(rocprim::radix_sort_keys(nullptr, tb, db, size_t(n), 0, 64, s),
                "balance sort size")) != EH_OK ||
      (st = dev_alloc(c, tmp, tb)) != EH_OK) {
    cleanup();
    return st;
  }
  hipLaunchKernelGGL(k_item_cost_keys, dim3(grid_of(n)), dim3(kB), 0, s, tv,
                     static_cast<const Item*>(plan.items.p), n,
                     target ? static_cast<const uint4*>(plan.sdesc.p) : nullptr,
                     target ? static_cast<const uint2*>(plan.rec.p) : nullptr,
                     target && plan.group > 1 ? static_cast<const uint4*>(plan.gsub.p) : nullptr,
                     target ? 1u : 0u, plan.pattern == EH_4CLIQUE ? 1u : 0u,
                     static_cast<unsigned long long*>(key_a.p));
  tb = tmp.bytes;
  if ((st = chk(rocprim::radix_sort_keys(tmp.p, tb, db, size_t(n), 0, 64, s), "balance sort")) !=
      EH_OK) {
    cleanup();
    return st;
  }
  hipLaunchKernelGGL(k_permute_items, dim3(grid_of(n)), dim3(kB), 0, s, db.current(), n,
                     static_cast<const Item*>(plan.items.p),
                     static_cast<const uint4*>(plan.sdesc.p), static_cast<Item*>(items2.p),
                     static_cast<uint4*>(sd2.p));
  if ((st = chk(hipGetLastError(), "balance kernels")) != EH_OK ||
      (st = chk(hipStreamSynchronize(s), "balance sync")) != EH_OK) {
    cleanup();
    return st;
  }
  std::swap(plan.items, items2);
  if (plan.sdesc.p) std::swap(plan.sdesc, sd2);
  cleanup();
  return EH_OK;
}

eh_status device_plan_target(Ctx* c, Trie& tr, Plan& plan, uint32_t chunk, bool ub, uint32_t cap,
                             uint32_t group) {
  const HostTrie& h = tr.host;
  hipStream_t s = c->stream;
  const uint32_t n = h.n, G = h.n_graphs;
  const uint64_t m = h.m;
  const uint64_t m1 = std::max<uint64_t>(m, 1);
  TrieView tv{static_cast<const uint2*>(tr.vdesc.p), static_cast<const uint32_t*>(tr.col.p),
              h.n_bs ? static_cast<const uint4*>(tr.bsdesc.p) : nullptr, n};
  DevBuf src, key_a, key_b, tin, trow, cnt, ioff, items, vbase, goff, small, tmp;
  DevBuf n_out, n_mem, o_off, m_off, grouped, cost, info, qsum, nch, choff, cbnd, g_out, tmp_big;
  Scratch sc(c);
  eh_status st;
  auto chk = [&](hipError_t e, const char* what) { return hip_check(c, e, what); };
  if ((st = sc.get(src, 4 * m1)) != EH_OK || (st = sc.get(key_a, 8 * m1)) != EH_OK ||
      (st = sc.get(key_b, 8 * m1)) != EH_OK || (st = sc.get(tin, 8 * m1)) != EH_OK ||
      (st = sc.get(trow, 4ull * (n + 1))) != EH_OK || (st = sc.get(cnt, 4ull * (n + 1))) != EH_OK ||
      (st = sc.get(ioff, 8ull * (n + 1))) != EH_OK || (st = sc.get(vbase, 4ull * (G + 1))) != EH_OK ||
      (st = sc.get(goff, 8ull * (G + 1))) != EH_OK || (st = sc.get(small, 64)) != EH_OK ||
      (st = sc.get(grouped, std::max<uint32_t>(n, 1))) != EH_OK ||
      (st = sc.get(cost, 4 * m1)) != EH_OK || (st = sc.get(qsum, 8 * m1)) != EH_OK)
    return st;
  const unsigned key_bits = 32u + (n > 1 ? 32u - uint32_t(__builtin_clz(n - 1)) : 1u);
  size_t need = 0, b = 0;
  rocprim::double_buffer<unsigned long long> db(ptr<unsigned long long>(key_a),
                                                ptr<unsigned long long>(key_b));
  if ((st = chk(rocprim::radix_sort_keys(nullptr, b, db, size_t(m1), 0, key_bits, s),
                "plan sort size")) != EH_OK)
    return st;
  need = std::max(need, b);
  const uint64_t gcap = uint64_t(G) + 1;
  if ((st = chk(rocprim::exclusive_scan(nullptr, b, ptr<uint32_t>(cnt),
                                        ptr<unsigned long long>(ioff), 0ull, size_t(n) + 1,
                                        rocprim::plus<unsigned long long>(), s),
                "plan scan size")) != EH_OK)
    return st;
  need = std::max(need, b);
  if ((st = chk(rocprim::exclusive_scan(nullptr, b, ptr<unsigned long long>(goff),
                                        ptr<unsigned long long>(goff), 0ull, size_t(gcap),
                                        rocprim::plus<unsigned long long>(), s),
                "plan scan size")) != EH_OK)
    return st;
  need = std::max(need, b);
  if ((st = chk(rocprim::inclusive_scan(nullptr, b, ptr<uint32_t>(cost),
                                        ptr<unsigned long long>(qsum), size_t(m1),
                                        rocprim::plus<unsigned long long>(), s),
                "cost scan size")) != EH_OK)
    return st;
  need = std::max(need, b);
  if ((st = sc.get(tmp, need)) != EH_OK) return st;
  if ((st = chk(hipMemcpyAsync(vbase.p, h.g_vbase.data(), 4ull * (G + 1), hipMemcpyHostToDevice, s),
                "upload graph bases")) != EH_OK)
    return st;
  hipLaunchKernelGGL(k_fill_u32_plan, dim3(1), dim3(kB), 0, s, ptr<uint32_t>(small), uint64_t(16),
                     0u);

  // 1. transpose
  unsigned long long* sorted = ptr<unsigned long long>(key_a);
  if (m) {
    hipLaunchKernelGGL(k_sources, dim3(grid_of(n)), dim3(kB), 0, s, tv, ptr<uint32_t>(src));
    hipLaunchKernelGGL(k_target_keys, dim3(grid_of(m)), dim3(kB), 0, s, tv, m,
                       ptr<unsigned long long>(key_a));
    size_t tb = tmp.bytes;
    if ((st = chk(rocprim::radix_sort_keys(tmp.p, tb, db, size_t(m), 0, key_bits, s),
                  "in-edge sort")) != EH_OK)
      return st;
    sorted = db.current();
    hipLaunchKernelGGL(k_in_edges, dim3(grid_of(m)), dim3(kB), 0, s, sorted, m,
                       ptr<uint32_t>(src), ptr<uint2>(tin));
  }
  hipLaunchKernelGGL(k_in_rows, dim3(grid_of(uint64_t(n) + 1)), dim3(kB), 0, s, sorted, m, n,
                     ptr<uint32_t>(trow));

  // 2. items
  if (m)
    hipLaunchKernelGGL(k_in_edge_costs, dim3(grid_of(m)), dim3(kB), 0, s, tv, ptr<uint2>(tin), m,
                       ub ? 1u : 0u, ptr<uint32_t>(cost));
  if (m) {
    size_t qb = tmp.bytes;
    if ((st = chk(rocprim::inclusive_scan(tmp.p, qb, ptr<uint32_t>(cost),
                                          ptr<unsigned long long>(qsum), size_t(m),
                                          rocprim::plus<unsigned long long>(), s),
                  "cost scan")) != EH_OK)
      return st;
  }
  hipLaunchKernelGGL(k_count_items, dim3(grid_of(uint64_t(n) + 1)), dim3(kB), 0, s, tv,
                     ptr<unsigned long long>(qsum), ptr<uint32_t>(trow), chunk,
                     ptr<uint32_t>(cnt));
  size_t tb = tmp.bytes;
  if ((st = chk(rocprim::exclusive_scan(tmp.p, tb, ptr<uint32_t>(cnt),
                                        ptr<unsigned long long>(ioff), 0ull, size_t(n) + 1,
                                        rocprim::plus<unsigned long long>(), s),
                "item scan")) != EH_OK)
    return st;
  unsigned long long n_items = 0;
  if ((st = chk(hipMemcpyAsync(&n_items, ptr<unsigned long long>(ioff) + n, 8,
                               hipMemcpyDeviceToHost, s), "read item count")) != EH_OK ||
      (st = chk(hipStreamSynchronize(s), "plan sync")) != EH_OK)
    return st;
  if ((st = sc.get(items, sizeof(Item) * std::max<uint64_t>(n_items, 1))) != EH_OK) return st;
  hipLaunchKernelGGL(k_write_items, dim3(grid_of(n)), dim3(kB), 0, s, tv,
                     ptr<unsigned long long>(qsum),
                     ptr<uint32_t>(trow), chunk, ptr<unsigned long long>(ioff),
                     ptr<uint32_t>(vbase), G, ptr<Item>(items), ptr<uint32_t>(small));
  hipLaunchKernelGGL(k_graph_offsets, dim3(grid_of(gcap)), dim3(kB), 0, s, ptr<Item>(items),
                     uint64_t(n_items), ptr<uint32_t>(vbase), G, ptr<unsigned long long>(goff));
  if ((st = chk(hipGetLastError(), "plan kernels")) != EH_OK) return st;

  // 3. grouping (or one descriptor per item)
  uint64_t n_final = n_items, n_members = 0;
  DevBuf out_items, sd, gsub;
  std::vector<unsigned long long> g_off(gcap);
  hipLaunchKernelGGL(k_fill_u8_plan, dim3(grid_of(n)), dim3(kB), 0, s, ptr<uint8_t>(grouped),
                     uint64_t(std::max<uint32_t>(n, 1)));
  if (group > 1) {
    // the graphs' item ranges cut into chunks of at most kGroupChunk items
    if ((st = sc.get(nch, 8 * gcap)) != EH_OK || (st = sc.get(choff, 8 * gcap)) != EH_OK ||
        (st = sc.get(g_out, 8 * gcap)) != EH_OK)
      return st;
    hipLaunchKernelGGL(k_chunk_counts, dim3(grid_of(gcap)), dim3(kB), 0, s,
                       ptr<unsigned long long>(goff), G, ptr<unsigned long long>(nch));
    tb = tmp.bytes;
    if ((st = chk(rocprim::exclusive_scan(tmp.p, tb, ptr<unsigned long long>(nch),
                                          ptr<unsigned long long>(choff), 0ull, size_t(gcap),
                                          rocprim::plus<unsigned long long>(), s),
                  "chunk scan")) != EH_OK)
      return st;
    unsigned long long n_chunks = 0;
    if ((st = chk(hipMemcpyAsync(&n_chunks, ptr<unsigned long long>(choff) + G, 8,
                                 hipMemcpyDeviceToHost, s), "read chunk count")) != EH_OK ||
        (st = chk(hipStreamSynchronize(s), "plan sync")) != EH_OK)
      return st;
    const uint64_t ccap = n_chunks + 1;
    if ((st = sc.get(cbnd, 8 * ccap)) != EH_OK || (st = sc.get(n_out, 8 * ccap)) != EH_OK ||
        (st = sc.get(n_mem, 8 * ccap)) != EH_OK || (st = sc.get(o_off, 8 * ccap)) != EH_OK ||
        (st = sc.get(m_off, 8 * ccap)) != EH_OK ||
        (st = sc.get(info, 16 * std::max<uint64_t>(n_items, 1))) != EH_OK)
      return st;
    // the scans over ccap entries, with scratch of their own when the
    // planner's is too small for them
    DevBuf* stmp = &tmp;
    tb = 0;
    if ((st = chk(rocprim::exclusive_scan(nullptr, tb, ptr<unsigned long long>(n_out),
                                          ptr<unsigned long long>(o_off), 0ull, size_t(ccap),
                                          rocprim::plus<unsigned long long>(), s),
                  "scan size")) != EH_OK)
      return st;
    if (tb > tmp.bytes) {
      if ((st = sc.get(tmp_big, tb)) != EH_OK) return st;
      stmp = &tmp_big;
    }
    hipLaunchKernelGGL(k_chunk_bounds, dim3(grid_of(gcap)), dim3(kB), 0, s,
                       ptr<unsigned long long>(goff), ptr<unsigned long long>(choff), G,
                       ptr<unsigned long long>(cbnd));
    if (n_items)
      hipLaunchKernelGGL(k_item_info, dim3(grid_of(n_items)), dim3(kB), 0, s, tv, ptr<Item>(items),
                         uint64_t(n_items), ptr<uint32_t>(trow), ptr<uint4>(info));
    hipLaunchKernelGGL(k_group_count, dim3(grid_of(ccap)), dim3(kB), 0, s, tv, ptr<Item>(items),
                       ptr<uint4>(info), ptr<unsigned long long>(cbnd), uint64_t(n_chunks), group,
                       cap, ptr<unsigned long long>(n_out), ptr<unsigned long long>(n_mem));
    tb = stmp->bytes;
    if ((st = chk(rocprim::exclusive_scan(stmp->p, tb, ptr<unsigned long long>(n_out),
                                          ptr<unsigned long long>(o_off), 0ull, size_t(ccap),
                                          rocprim::plus<unsigned long long>(), s),
                  "group scan")) != EH_OK)
      return st;
    tb = stmp->bytes;
    if ((st = chk(rocprim::exclusive_scan(stmp->p, tb, ptr<unsigned long long>(n_mem),
                                          ptr<unsigned long long>(m_off), 0ull, size_t(ccap),
                                          rocprim::plus<unsigned long long>(), s),
                  "group scan")) != EH_OK)
      return st;
    unsigned long long tot[2] = {0, 0};
    if ((st = chk(hipMemcpyAsync(&tot[0], ptr<unsigned long long>(o_off) + n_chunks, 8,
                                 hipMemcpyDeviceToHost, s), "read group count")) != EH_OK ||
        (st = chk(hipMemcpyAsync(&tot[1], ptr<unsigned long long>(m_off) + n_chunks, 8,
                                 hipMemcpyDeviceToHost, s), "read member count")) != EH_OK ||
        (st = chk(hipStreamSynchronize(s), "plan sync")) != EH_OK)
      return st;
    n_final = tot[0];
    n_members = tot[1];
    if (n_members > kMaxIndex) {
      c->err = "grouped members exceed 2^31-1";
      return EH_EOVERFLOW;
    }
    if ((st = dev_alloc(c, out_items, sizeof(Item) * std::max<uint64_t>(n_final, 1))) != EH_OK ||
        (st = dev_alloc(c, sd, 16 * std::max<uint64_t>(n_final, 1))) != EH_OK ||
        (st = dev_alloc(c, gsub, 16 * std::max<uint64_t>(n_members, 1))) != EH_OK) {
      dev_free(c, out_items);
      dev_free(c, sd);
      dev_free(c, gsub);
      return st;
    }
    hipLaunchKernelGGL(k_group_write, dim3(grid_of(n_chunks)), dim3(kB), 0, s, tv,
                       ptr<Item>(items), ptr<uint4>(info), ptr<unsigned long long>(cbnd),
                       uint64_t(n_chunks), group, cap, ptr<unsigned long long>(o_off),
                       ptr<unsigned long long>(m_off), ptr<Item>(out_items), ptr<uint4>(sd),
                       ptr<uint4>(gsub), ptr<uint8_t>(grouped));
    hipLaunchKernelGGL(k_graph_out, dim3(grid_of(gcap)), dim3(kB), 0, s,
                       ptr<unsigned long long>(choff), ptr<unsigned long long>(o_off), G,
                       ptr<unsigned long long>(g_out));
    if ((st = chk(hipMemcpyAsync(g_off.data(), g_out.p, 8 * gcap, hipMemcpyDeviceToHost, s),
                  "read graph offsets")) != EH_OK) {
      dev_free(c, out_items);
      dev_free(c, sd);
      dev_free(c, gsub);
      return st;
    }
    g_off[G] = n_final;
  } else {
    // the item list itself is the plan's; only the descriptors are added
    out_items = items;
    items = DevBuf();
    if ((st = dev_alloc(c, sd, 16 * std::max<uint64_t>(n_final, 1))) != EH_OK ||
        (st = dev_alloc(c, gsub, 16)) != EH_OK) {
      dev_free(c, out_items);
      dev_free(c, sd);
      dev_free(c, gsub);
      return st;
    }
    if (n_final)
      hipLaunchKernelGGL(k_single_descs, dim3(grid_of(n_final)), dim3(kB), 0, s, tv,
                         ptr<Item>(out_items), uint64_t(n_final), ptr<uint4>(sd));
    if ((st = chk(hipMemcpyAsync(g_off.data(), goff.p, 8 * gcap, hipMemcpyDeviceToHost, s),
                  "read graph offsets")) != EH_OK) {
      dev_free(c, out_items);
      dev_free(c, sd);
      dev_free(c, gsub);
      return st;
    }
  }

  // 4. records
  DevBuf rec;
  if ((st = dev_alloc(c, rec, 8 * m1)) != EH_OK) {
    dev_free(c, out_items);
    dev_free(c, sd);
    dev_free(c, gsub);
    return st;
  }
  if (m)
    hipLaunchKernelGGL(k_records, dim3(grid_of(m)), dim3(kB), 0, s, tv, sorted, ptr<uint2>(tin), m,
                       ptr<uint8_t>(grouped), ub ? 1u : 0u, cap, ptr<uint2>(rec),
                       ptr<uint32_t>(small) + 1);
  uint32_t flags[2] = {0, 0};
  st = chk(hipGetLastError(), "plan kernels");
  if (st == EH_OK)
    st = chk(hipMemcpyAsync(flags, small.p, 8, hipMemcpyDeviceToHost, s), "read plan flags");
  if (st == EH_OK) st = chk(hipStreamSynchronize(s), "plan sync");
  if (st == EH_OK && flags[1]) {
    c->err = "segment record field beyond 16 bits";
    st = EH_EOVERFLOW;
  }
  if (st != EH_OK) {
    dev_free(c, out_items);
    dev_free(c, sd);
    dev_free(c, gsub);
    dev_free(c, rec);
    return st;
  }
  plan.items = out_items;
  plan.sdesc = sd;
  plan.rec = rec;
  plan.gsub = gsub;
  plan.n_items = n_final;
  plan.item_dmax = flags[0];
  plan.g_item_off.assign(g_off.begin(), g_off.end());
  return EH_OK;
}

namespace {

// Sort key of vertex u for the induced-neighbourhood 4-clique plan: class
// (out-degree <= 64, 128, 256, 512), then decreasing estimated cost
// (d^2 + sum of the out-degrees of N+(u), clamped to 28 bits), then u; all
// ones when u is not such a root.  counts[k] counts class k's roots.
__global__ void __launch_bounds__(kB) k_k4l_keys(TrieView t, unsigned long long* __restrict__ key,
                                                 unsigned long long* __restrict__ counts) {
  constexpr uint64_t kCostMax = (1ull << 28) - 1;
  const uint32_t lane = threadIdx.x & 63u;
  // every lane of a wave takes the same number of turns (the stride is a
  // multiple of 64), so the class counts are summed per wave: one atomic per
  // class and wave instead of one per root
  for (uint64_t u0 = gtid() - lane; u0 < t.n; u0 += gstride()) {
    const uint64_t u = u0 + lane;
    int k = -1;
    if (u < t.n) {
      const uint2 ud = t.vdesc[u];
      const uint32_t d = ud.y & kMaxIndex;
      k = k4_local_class(d);
      if (k < 0) {
        key[u] = ~0ull;
      } else {
        // d <= 512 members of at most 2^31 out-degree each: no overflow
        uint64_t cost = uint64_t(d) * d;
        for (uint32_t e = ud.x; e < ud.x + d; ++e) cost += outdeg(t, t.col[e]);
        cost = cost < kCostMax ? cost : kCostMax;
        key[u] = (uint64_t(k) << 60) | ((kCostMax - cost) << 32) | u;
      }
    }
#pragma unroll
    for (int q = 0; q < int(kK4LocalClasses); ++q) {
      const uint64_t m = __ballot(k == q);
      if (m && lane == uint32_t(__ffsll((unsigned long long)m) - 1))
        atomicAdd(&counts[q], (unsigned long long)__popcll(m));
    }
  }
}

// Rows (d - 1) of each root, in sorted order.
__global__ void __launch_bounds__(kB) k_k4l_rows(TrieView t, const unsigned long long* __restrict__ key,
                                                 uint64_t n_roots, uint32_t* __restrict__ rows) {
  for (uint64_t r = gtid(); r < n_roots; r += gstride())
    rows[r] = outdeg(t, uint32_t(key[r] & 0xFFFFFFFFull)) - 1;
}

__device__ inline uint32_t lower_bound_g(const uint32_t* a, uint32_t n, uint32_t x) {
  uint32_t lo = 0;
  while (n) {
    const uint32_t h = n >> 1;
    if (a[lo + h] < x) { lo += h + 1; n -= h + 1; } else n = h;
  }
  return lo;
}

// One wave per root: the root record {position of N+(u), d | plen << 10 |
// nw << 20, first row record, window base} and, per row i < d - 1, the part
// of N+(v_i) from v_{i+1} up to max N+(u) as elements, or as the bitset's
// words when fewer (only from a bitset starting inside the window), {start,
// length | word offset << 22 | kHiBit for words}.  long_set: a row of 2^22 or
// more members.
__global__ void __launch_bounds__(kB) k_k4l_records(TrieView t, const unsigned long long* __restrict__ key,
                                                    const uint32_t* __restrict__ roff, uint64_t n_roots,
                                                    uint32_t ub, uint4* __restrict__ roots,
                                                    uint2* __restrict__ rec,
                                                    unsigned long long* __restrict__ long_set) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t wave = gtid() >> 6, waves = gstride() >> 6;
  for (uint64_t r = wave; r < n_roots; r += waves) {
    const uint32_t u = uint32_t(key[r] & 0xFFFFFFFFull);
    const int k = int(key[r] >> 60);
    const uint2 ud = t.vdesc[u];
    const uint32_t d = ud.y & kMaxIndex, W = k4_local_window(k);
    const uint32_t* nu = t.col + ud.x;
    const uint32_t lo = nu[0], hi = nu[d - 1];
    const uint32_t wb = hi - (lo & ~31u) < W * 32u ? (lo & ~31u) : ((hi + 1u - W * 32u + 31u) & ~31u);
    const uint32_t plen = lower_bound_g(nu, d, wb);
    const uint32_t nw = ((hi - wb) >> 5) + 1;
    if (lane == 0) roots[r] = make_uint4(ud.x, d | (plen << 10) | (nw << 20), roff[r], wb);
    for (uint32_t i = lane; i + 1 < d; i += 64) {
      const uint32_t v = nu[i];
      const uint2 vd = t.vdesc[v];
      const uint32_t dv = vd.y & kMaxIndex;
      const uint32_t* nv = t.col + vd.x;
      // members from the next member of N+(u) up to hi: T_i only holds
      // members after v_i, and the first of those is v_{i+1}
      uint32_t len = lower_bound_g(nv, dv, hi);
      if (len < dv && nv[len] == hi) ++len;
      const uint32_t from = len ? lower_bound_g(nv, len, nu[i + 1]) : 0u;
      len -= from;
      uint2 g = make_uint2(vd.x + from, len);
      if (ub && len && (vd.y & kHiBit)) {
        const uint4 b = t.bsdesc[v];
        if (b.y >= wb) {
          const uint32_t words = min(b.z, ((hi - b.y) >> 5) + 1);
          if (words < len) g = make_uint2(b.x, words | (((b.y - wb) >> 5) << 22) | kHiBit);
        }
      }
      if (!(g.y & kHiBit) && len >= (1u << 22)) atomicAdd(long_set, 1ull);
      rec[roff[r] + i] = g;
    }
  }
}

}  // namespace

eh_status device_plan_k4_local(Ctx* c, Trie& tr, Plan& plan, bool ub) {
  const HostTrie& h = tr.host;
  const uint32_t n = h.n;
  if (n == 0) return EH_OK;
  hipStream_t s = c->stream;
  TrieView tv{static_cast<const uint2*>(tr.vdesc.p), static_cast<const uint32_t*>(tr.col.p),
              h.n_bs ? static_cast<const uint4*>(tr.bsdesc.p) : nullptr, n};
  auto chk = [&](hipError_t e, const char* what) { return hip_check(c, e, what); };
  Scratch sc(c);
  DevBuf key_a, key_b, small, rows, roff, tmp;
  eh_status st;
  if ((st = sc.get(key_a, 8ull * n)) != EH_OK || (st = sc.get(key_b, 8ull * n)) != EH_OK ||
      (st = sc.get(small, 64)) != EH_OK)
    return st;
  hipLaunchKernelGGL(k_fill_u32_plan, dim3(1), dim3(kB), 0, s, ptr<uint32_t>(small), 16, 0u);
  hipLaunchKernelGGL(k_k4l_keys, dim3(grid_of(n)), dim3(kB), 0, s, tv, ptr<unsigned long long>(key_a),
                     ptr<unsigned long long>(small));
  rocprim::double_buffer<unsigned long long> db(ptr<unsigned long long>(key_a),
                                                ptr<unsigned long long>(key_b));
  size_t tb = 0;
  if ((st = chk(rocprim::radix_sort_keys(nullptr, tb, db, size_t(n), 0, 64, s), "sort size")) !=
      EH_OK)
    return st;
  size_t ts = 0;
  if ((st = chk(rocprim::exclusive_scan(nullptr, ts, ptr<uint32_t>(key_a), ptr<uint32_t>(key_b),
                                        0u, size_t(n), rocprim::plus<uint32_t>(), s),
                "scan size")) != EH_OK)
    return st;
  if ((st = sc.get(tmp, std::max(tb, ts))) != EH_OK) return st;
  tb = tmp.bytes;
  if ((st = chk(rocprim::radix_sort_keys(tmp.p, tb, db, size_t(n), 0, 64, s), "root sort")) !=
      EH_OK)
    return st;
  unsigned long long counts[kK4LocalClasses + 1] = {};
  if ((st = chk(hipMemcpyAsync(counts, small.p, sizeof(counts), hipMemcpyDeviceToHost, s),
                "read root classes")) != EH_OK ||
      (st = chk(hipStreamSynchronize(s), "root sync")) != EH_OK)
    return st;
  uint64_t n_roots = 0;
  for (uint32_t k = 0; k < kK4LocalClasses; ++k) {
    plan.k4l_n[k] = counts[k];
    n_roots += counts[k];
  }
  if (n_roots == 0) return EH_OK;
  const unsigned long long* sorted = db.current();
  if ((st = sc.get(rows, 4 * n_roots)) != EH_OK || (st = sc.get(roff, 4 * n_roots)) != EH_OK)
    return st;
  hipLaunchKernelGGL(k_k4l_rows, dim3(grid_of(n_roots)), dim3(kB), 0, s, tv, sorted, n_roots,
                     ptr<uint32_t>(rows));
  ts = tmp.bytes;
  if ((st = chk(rocprim::exclusive_scan(tmp.p, ts, ptr<uint32_t>(rows), ptr<uint32_t>(roff), 0u,
                                        size_t(n_roots), rocprim::plus<uint32_t>(), s),
                "row scan")) != EH_OK)
    return st;
  uint32_t last[2] = {0, 0};
  if ((st = chk(hipMemcpyAsync(&last[0], ptr<uint32_t>(roff) + n_roots - 1, 4,
                               hipMemcpyDeviceToHost, s), "read rows")) != EH_OK ||
      (st = chk(hipMemcpyAsync(&last[1], ptr<uint32_t>(rows) + n_roots - 1, 4,
                               hipMemcpyDeviceToHost, s), "read rows")) != EH_OK ||
      (st = chk(hipStreamSynchronize(s), "rows sync")) != EH_OK)
    return st;
  const uint64_t n_rec = uint64_t(last[0]) + last[1];
  // the root records, then one work cursor per class (kCursorWords apart)
  if ((st = dev_alloc(c, plan.k4l, sizeof(uint4) * n_roots +
                                       sizeof(uint32_t) * kCursorWords * kK4LocalClasses)) != EH_OK)
    return st;
  if ((st = dev_alloc(c, plan.rec, sizeof(uint2) * std::max<uint64_t>(n_rec, 1))) != EH_OK)
    return st;
  hipLaunchKernelGGL(k_fill_u32_plan, dim3(1), dim3(kB), 0, s, ptr<uint32_t>(small), 16, 0u);
  const uint64_t blocks = std::min<uint64_t>((n_roots + kB / 64 - 1) / (kB / 64), 1u << 16);
  hipLaunchKernelGGL(k_k4l_records, dim3(uint32_t(blocks)), dim3(kB), 0, s, tv, sorted,
                     ptr<uint32_t>(roff), n_roots, ub ? 1u : 0u,
                     static_cast<uint4*>(plan.k4l.p), static_cast<uint2*>(plan.rec.p),
                     ptr<unsigned long long>(small));
  unsigned long long long_set = 0;
  if ((st = chk(hipGetLastError(), "4-clique plan kernels")) != EH_OK ||
      (st = chk(hipMemcpyAsync(&long_set, small.p, 8, hipMemcpyDeviceToHost, s),
                "read plan flag")) != EH_OK ||
      (st = chk(hipStreamSynchronize(s), "plan sync")) != EH_OK)
    return st;
  if (long_set) {
    c->err = "a streamed set of 2^22 or more members in a 4-clique plan";
    return EH_EOVERFLOW;
  }
  return EH_OK;
}

}  // namespace eh
