// Trie construction on the GPU (paper section 2.2: dictionary encoding into
// dense 32-bit ranks, the pruning of section 5.2, and the set layouts of
// sections 4.1 and 4.4), from raw pairs already resident in device memory.
// It produces the same trie as the host build, array for array:
//
//   1. each pair becomes a key min << k | max (k bits per endpoint, k the
//      width of n - 1); self-loops become a sentinel that sorts last;
//   2. radix sort and unique: the simple undirected edge set;
//   3. degrees (atomic counts), then ranks from a stable radix sort of
//      (degree, id) pairs: degree order, reverse degree order or the input
//      ids; for a single graph also the traversal orderings (BFS, hybrid,
//      strong runs), whose label sequences eh_gpu_order.hip computes;
//   4. each edge becomes low rank << k | high rank; a second radix sort gives
//      the oriented CSR (rows found by binary search of the sorted keys);
//   5. per set the density rule picks the bitset layout, a scan places the
//      words, and an atomic OR per member sets its bit.
//
// rocPRIM provides the sorts, unique and scans; every other step is a kernel
// below.  The host copy of the trie, which work-item planning reads, is then
// downloaded.
#include <cstring>
#include <hip/hip_runtime.h>
#include <rocprim/rocprim.hpp>

#include <algorithm>
#include <thread>
#include <vector>

#include "eh_internal.h"

namespace eh {
namespace {

constexpr uint32_t kB = 256;
constexpr unsigned long long kSentinel = ~0ull;

uint32_t grid_of(uint64_t n) {
  return uint32_t(std::max<uint64_t>(1, std::min<uint64_t>((n + kB - 1) / kB, 1u << 16)));
}

__device__ inline uint64_t gtid() { return uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; }
__device__ inline uint64_t gstride() { return uint64_t(gridDim.x) * blockDim.x; }

// Block-wide sum and max (blockDim.x == kB, four waves of 64).
__device__ inline void block_sum_max(unsigned long long& sum, uint32_t& mx) {
  __shared__ unsigned long long s_sum[kB / 64];
  __shared__ uint32_t s_max[kB / 64];
  for (int o = 32; o > 0; o >>= 1) {
    sum += __shfl_xor(sum, o, 64);
    mx = max(mx, uint32_t(__shfl_xor(int(mx), o, 64)));
  }
  const uint32_t w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) {
    s_sum[w] = sum;
    s_max[w] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t i = 1; i < kB / 64; ++i) {
      sum += s_sum[i];
      mx = max(mx, s_max[i]);
    }
  }
}

__global__ void __launch_bounds__(kB) k_pair_keys(const uint32_t* __restrict__ src,
                                                  const uint32_t* __restrict__ dst, uint64_t m,
                                                  uint32_t n, uint32_t kb,
                                                  unsigned long long* __restrict__ key,
                                                  uint32_t* __restrict__ bad) {
  for (uint64_t i = gtid(); i < m; i += gstride()) {
    uint32_t a = src[i], b = dst[i];
    if (a >= n || b >= n) {
      atomicOr(bad, 1u);
      key[i] = kSentinel;
      continue;
    }
    if (a == b) {
      key[i] = kSentinel;
      continue;
    }
    if (a > b) {
      const uint32_t t = a;
      a = b;
      b = t;
    }
    key[i] = (static_cast<unsigned long long>(a) << kb) | b;
  }
}

// Degrees in the simple graph.  Keys are sorted, so equal smaller endpoints
// form runs: the first lane of each run within a wave adds the run's length
// with one atomic (a hub's edges would otherwise serialise on one address).
// Each wave walks 64 consecutive keys per step.
// Batch form of k_pair_keys: pair i belongs to graph g with
// edge_off[g] <= i < edge_off[g + 1]; its local ids become vbase[g] + id.
__global__ void __launch_bounds__(kB) k_batch_pair_keys(const uint32_t* __restrict__ src,
                                                        const uint32_t* __restrict__ dst,
                                                        uint64_t m, uint32_t n_graphs,
                                                        const unsigned long long* __restrict__ eoff,
                                                        const uint32_t* __restrict__ vbase,
                                                        const uint32_t* __restrict__ nv, uint32_t kb,
                                                        unsigned long long* __restrict__ key,
                                                        uint32_t* __restrict__ bad) {
  for (uint64_t i = gtid(); i < m; i += gstride()) {
    uint32_t lo = 0, hi = n_graphs;  // last g with eoff[g] <= i
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (eoff[mid] <= i) lo = mid;
      else hi = mid;
    }
    const uint32_t g = lo;
    uint32_t a = src[i], b = dst[i];
    if (a >= nv[g] || b >= nv[g]) {
      atomicOr(bad, 1u);
      key[i] = kSentinel;
      continue;
    }
    if (a == b) {
      key[i] = kSentinel;
      continue;
    }
    if (a > b) {
      const uint32_t t = a;
      a = b;
      b = t;
    }
    key[i] = (static_cast<unsigned long long>(vbase[g] + a) << kb) | (vbase[g] + b);
  }
}

// Graph of padded vertex v: the last g with vbase[g] <= v (empty graphs skipped).
__device__ inline uint32_t graph_of(const uint32_t* vbase, uint32_t n_graphs, uint32_t v) {
  uint32_t lo = 0, hi = n_graphs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (vbase[mid] <= v) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Rank sort keys of a batch: graph, then degree; a graph's padding vertices
// (the slots that round its rank range up to a multiple of 32) sort last.
__global__ void __launch_bounds__(kB) k_batch_rank_keys(const uint32_t* __restrict__ deg,
                                                        uint32_t n, uint32_t n_graphs,
                                                        const uint32_t* __restrict__ vbase,
                                                        const uint32_t* __restrict__ nv,
                                                        unsigned long long* __restrict__ key,
                                                        uint32_t* __restrict__ ids) {
  for (uint64_t v = gtid(); v < n; v += gstride()) {
    const uint32_t g = graph_of(vbase, n_graphs, uint32_t(v));
    const bool pad = uint32_t(v) - vbase[g] >= nv[g];
    key[v] = (static_cast<unsigned long long>(g) << 32) | (pad ? 0xFFFFFFFFu : deg[v]);
    ids[v] = uint32_t(v);
  }
}

// Ranks of a batch.  seq: vertices sorted by (graph, degree, id), or null for
// the input order.  Graph g's ranks are [vbase[g], vbase[g] + n_g); padding
// keeps rank = id.
__global__ void __launch_bounds__(kB) k_batch_ranks(const uint32_t* __restrict__ seq, uint32_t n,
                                                    uint32_t n_graphs,
                                                    const uint32_t* __restrict__ vbase,
                                                    const uint32_t* __restrict__ nv, uint32_t order,
                                                    uint32_t* __restrict__ rank,
                                                    uint32_t* __restrict__ vert) {
  for (uint64_t p = gtid(); p < n; p += gstride()) {
    const uint32_t v = seq ? seq[p] : uint32_t(p);
    const uint32_t g = graph_of(vbase, n_graphs, v);
    const uint32_t vb = vbase[g], nvg = nv[g];
    uint32_t r;
    if (v - vb >= nvg) r = v;
    else if (order == EH_ORDER_DEGREE) r = uint32_t(p);
    else if (order == EH_ORDER_REV_DEGREE) r = vb + nvg - 1 - (uint32_t(p) - vb);
    else r = vb + nvg - 1 - (v - vb);
    rank[v] = r;
    vert[r] = v;
  }
}

__global__ void __launch_bounds__(kB) k_degrees(const unsigned long long* __restrict__ key,
                                                uint64_t m, uint32_t kb,
                                                uint32_t* __restrict__ deg) {
  const unsigned long long mask = (1ull << kb) - 1;
  const uint32_t lane = threadIdx.x & 63;
  for (uint64_t base = gtid() & ~63ull; base < m; base += gstride()) {
    const uint64_t i = base + lane;
    const bool in = i < m;
    const unsigned long long k = in ? key[i] : 0ull;
    const uint32_t a = in ? uint32_t(k >> kb) : 0xFFFFFFFFu;
    const uint32_t prev = __shfl_up(a, 1, 64);
    const bool head = in && (lane == 0 || prev != a);
    const unsigned long long heads = __ballot(head);
    if (head) {
      const unsigned long long later = lane == 63 ? 0ull : heads >> (lane + 1);
      const uint64_t end = later ? lane + 1 + uint32_t(__builtin_ctzll(later))
                                 : std::min<uint64_t>(64, m - base);
      atomicAdd(&deg[a], uint32_t(end - lane));
    }
    if (in) atomicAdd(&deg[k & mask], 1u);
  }
}

__global__ void __launch_bounds__(kB) k_iota(uint32_t* __restrict__ p, uint32_t n) {
  for (uint64_t i = gtid(); i < n; i += gstride()) p[i] = uint32_t(i);
}

__global__ void __launch_bounds__(kB) k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  for (uint64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}

// seq lists vertices in rank order (reverse = 0) or in label order, ranks
// then counting down from n - 1 (reverse = 1).
__global__ void __launch_bounds__(kB) k_ranks(const uint32_t* __restrict__ seq, uint32_t n,
                                              uint32_t reverse, uint32_t* __restrict__ rank,
                                              uint32_t* __restrict__ vert) {
  for (uint64_t l = gtid(); l < n; l += gstride()) {
    const uint32_t v = seq[l];
    const uint32_t r = reverse ? n - 1 - uint32_t(l) : uint32_t(l);
    rank[v] = r;
    vert[r] = v;
  }
}

// Low rank << k | high rank per edge; a symmetric trie also gets the reverse
// arc at m + i.
__global__ void __launch_bounds__(kB) k_orient(const unsigned long long* __restrict__ key,
                                               uint64_t m, uint32_t kb, uint32_t symmetric,
                                               const uint32_t* __restrict__ rank,
                                               unsigned long long* __restrict__ out) {
  const unsigned long long mask = (1ull << kb) - 1;
  for (uint64_t i = gtid(); i < m; i += gstride()) {
    uint32_t ra = rank[key[i] >> kb], rb = rank[key[i] & mask];
    if (ra > rb) {
      const uint32_t t = ra;
      ra = rb;
      rb = t;
    }
    out[i] = (static_cast<unsigned long long>(ra) << kb) | rb;
    if (symmetric) out[m + i] = (static_cast<unsigned long long>(rb) << kb) | ra;
  }
}

// row[r] = number of oriented edges whose source rank is below r.
__global__ void __launch_bounds__(kB) k_rows(const unsigned long long* __restrict__ key,
                                             uint64_t m, uint32_t n, uint32_t kb,
                                             uint32_t* __restrict__ row) {
  for (uint64_t r = gtid(); r <= n; r += gstride()) {
    const unsigned long long want = static_cast<unsigned long long>(r) << kb;
    uint64_t lo = 0, hi = m;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (key[mid] < want) lo = mid + 1;
      else hi = mid;
    }
    row[r] = uint32_t(lo);
  }
}

// Density rule of section 4.4 per set; stats[0] += bitset sets,
// stats[1] = max out-degree.
__global__ void __launch_bounds__(kB) k_layout(const unsigned long long* __restrict__ key,
                                               const uint32_t* __restrict__ row, uint32_t n,
                                               uint32_t kb, uint32_t layout, float tau,
                                               uint32_t s_min, uint32_t* __restrict__ nw,
                                               uint32_t* __restrict__ base,
                                               unsigned long long* __restrict__ stats) {
  const unsigned long long mask = (1ull << kb) - 1;
  unsigned long long dense_sets = 0;
  uint32_t dmax = 0;
  for (uint64_t u = gtid(); u < uint64_t(n) + 1; u += gstride()) {
    if (u == n) {
      nw[u] = 0;  // the scan's trailing element
      continue;
    }
    const uint32_t b = row[u], e = row[u + 1], len = e - b;
    dmax = max(dmax, len);
    uint32_t words = 0, bs = 0;
    if (len && layout != EH_LAYOUT_UINT) {
      const uint32_t lo = uint32_t(key[b] & mask), hi = uint32_t(key[e - 1] & mask);
      const double range = double(hi) - double(lo) + 1.0;
      const bool dense = layout == EH_LAYOUT_BITSET_ALL ||
                         (len >= s_min && range <= double(tau) * double(len));
      if (dense) {
        bs = lo & ~31u;
        words = ((hi - bs) >> 5) + 1;
        ++dense_sets;
      }
    }
    nw[u] = words;
    base[u] = bs;
  }
  block_sum_max(dense_sets, dmax);
  if (threadIdx.x == 0) {
    if (dense_sets) atomicAdd(&stats[0], dense_sets);
    atomicMax(&stats[1], static_cast<unsigned long long>(dmax));
  }
}

// stats[2] += B_merge = sum over oriented edges (u, v) of 4 (d+(u) + d+(v)).
// target != 0 (pruned tries): stats[3] += the streamed part of B_target, per
// edge u -> v with a non-empty N+(v) an 8-byte record and 4 bytes for each
// member of N+(u) after v (edge i is member i - row[u] of N+(u)).
__global__ void __launch_bounds__(kB) k_bmerge(const unsigned long long* __restrict__ key,
                                               const uint32_t* __restrict__ row, uint64_t m,
                                               uint32_t kb, uint32_t target,
                                               unsigned long long* __restrict__ stats) {
  const unsigned long long mask = (1ull << kb) - 1;
  unsigned long long sum = 0, tsum = 0;
  uint32_t unused = 0;
  for (uint64_t i = gtid(); i < m; i += gstride()) {
    const uint64_t u = key[i] >> kb, v = key[i] & mask;
    const uint32_t dv = row[v + 1] - row[v];
    sum += 4ull * ((row[u + 1] - row[u]) + dv);
    if (target && dv) tsum += 8ull + 4ull * (row[u + 1] - i - 1);
  }
  block_sum_max(sum, unused);
  if (threadIdx.x == 0 && sum) atomicAdd(&stats[2], sum);
  if (!target) return;
  __syncthreads();  // block_sum_max's shared slots are reused
  block_sum_max(tsum, unused);
  if (threadIdx.x == 0 && tsum) atomicAdd(&stats[3], tsum);
}

// stats[3] += the held part of B_target: 32 + 4 d+(r) for each rank r with a
// non-empty out-set and an in-edge (its degree in G exceeds its out-degree).
__global__ void __launch_bounds__(kB) k_btarget_held(const uint32_t* __restrict__ row,
                                                     const uint32_t* __restrict__ deg,
                                                     const uint32_t* __restrict__ vert, uint32_t n,
                                                     unsigned long long* __restrict__ stats) {
  unsigned long long sum = 0;
  uint32_t unused = 0;
  for (uint64_t r = gtid(); r < n; r += gstride()) {
    const uint32_t d = row[r + 1] - row[r];
    if (d && deg[vert[r]] > d) sum += 32ull + 4ull * d;
  }
  block_sum_max(sum, unused);
  if (threadIdx.x == 0 && sum) atomicAdd(&stats[3], sum);
}

// col[i] = the member; a bitset set also gets its bit in the words that
// follow the m members.
__global__ void __launch_bounds__(kB) k_members(const unsigned long long* __restrict__ key,
                                                uint64_t m, uint32_t kb,
                                                const uint32_t* __restrict__ nw,
                                                const uint32_t* __restrict__ base,
                                                const unsigned long long* __restrict__ off,
                                                uint32_t* __restrict__ col) {
  const unsigned long long mask = (1ull << kb) - 1;
  for (uint64_t i = gtid(); i < m; i += gstride()) {
    const uint64_t u = key[i] >> kb;
    const uint32_t x = uint32_t(key[i] & mask);
    col[i] = x;
    if (nw[u]) {
      const uint32_t d = x - base[u];
      atomicOr(&col[m + off[u] + (d >> 5)], 1u << (d & 31));
    }
  }
}

// Vertex and bitset tables the counting kernels read, and the host copy's
// word offsets (kNoBitset for uint-only sets).
__global__ void __launch_bounds__(kB) k_tables(const uint32_t* __restrict__ row,
                                               const uint32_t* __restrict__ nw,
                                               const uint32_t* __restrict__ base,
                                               const unsigned long long* __restrict__ off,
                                               uint32_t n, uint64_t m, uint32_t has_bs,
                                               uint2* __restrict__ vdesc,
                                               uint4* __restrict__ bsdesc,
                                               uint32_t* __restrict__ bs_off) {
  for (uint64_t u = gtid(); u < n; u += gstride()) {
    const uint32_t len = row[u + 1] - row[u];
    const bool bs = nw[u] != 0;
    vdesc[u] = make_uint2(row[u], len | (bs ? kHiBit : 0u));
    if (has_bs)
      bsdesc[u] = make_uint4(bs ? uint32_t(m + off[u]) : 0u, base[u], nw[u], 0u);
    bs_off[u] = bs ? uint32_t(off[u]) : kNoBitset;
  }
}

template <class T>
T* ptr(DevBuf& b) {
  return static_cast<T*>(b.p);
}

eh_status download(Ctx* c, void* dst, const void* src, size_t bytes, const char* what) {
  if (!bytes) return EH_OK;
  return hip_check(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c->stream), what);
}

}  // namespace

eh_status device_build(Ctx* c, const uint32_t* d_src, const uint32_t* d_dst, uint64_t m_raw,
                       uint32_t n, const BuildOpts& opts, Trie& t, const DeviceBatch* batch) {
  hipStream_t s = c->stream;
  if (n == 0 && m_raw) {
    c->err = "edges given for an empty vertex set";
    return EH_EINVAL;
  }
  const uint32_t kb = n > 1 ? 32u - uint32_t(__builtin_clz(n - 1)) : 1u;
  const uint64_t mr = std::max<uint64_t>(m_raw, 1);
  const uint64_t kcap = opts.symmetric ? 2 * mr : mr;  // stored arcs fit 2 m <= 2 m_raw
  const uint32_t n1 = std::max<uint32_t>(n, 1);
  DevBuf keys_a, keys_b, tmp, deg, ids, deg_s, seq, rank, row, nw, base, off, bs_off, stats, cnt;
  DevBuf b_eoff, b_vbase, b_nv, rk_in, rk_out;  // batch only
  Scratch sc(c);
  eh_status st;
  const uint32_t G = batch ? batch->n_graphs : 1u;
  if (batch) {
    if ((st = sc.get(b_eoff, 8ull * (G + 1))) != EH_OK ||
        (st = sc.get(b_vbase, 4ull * (G + 1))) != EH_OK || (st = sc.get(b_nv, 4ull * G)) != EH_OK ||
        (st = sc.get(rk_in, 8ull * n1)) != EH_OK || (st = sc.get(rk_out, 8ull * n1)) != EH_OK)
      return st;
    if ((st = hip_check(c, hipMemcpyAsync(b_eoff.p, batch->edge_off, 8ull * (G + 1),
                                          hipMemcpyHostToDevice, s), "upload edge offsets")) !=
            EH_OK ||
        (st = hip_check(c, hipMemcpyAsync(b_vbase.p, batch->vbase.data(), 4ull * (G + 1),
                                          hipMemcpyHostToDevice, s), "upload graph bases")) !=
            EH_OK ||
        (st = hip_check(c, hipMemcpyAsync(b_nv.p, batch->n_vertices, 4ull * G,
                                          hipMemcpyHostToDevice, s), "upload graph sizes")) !=
            EH_OK ||
        (st = hip_check(c, hipStreamSynchronize(s), "build sync")) != EH_OK)
      return st;
  }
  if ((st = sc.get(keys_a, 8 * kcap)) != EH_OK || (st = sc.get(keys_b, 8 * kcap)) != EH_OK ||
      (st = sc.get(deg, 4ull * n1)) != EH_OK || (st = sc.get(ids, 4ull * n1)) != EH_OK ||
      (st = sc.get(deg_s, 4ull * n1)) != EH_OK || (st = sc.get(seq, 4ull * n1)) != EH_OK ||
      (st = sc.get(rank, 4ull * n1)) != EH_OK || (st = sc.get(row, 4ull * (n + 1))) != EH_OK ||
      (st = sc.get(nw, 4ull * (n + 1))) != EH_OK || (st = sc.get(base, 4ull * n1)) != EH_OK ||
      (st = sc.get(off, 8ull * (n + 1))) != EH_OK || (st = sc.get(bs_off, 4ull * n1)) != EH_OK ||
      (st = sc.get(stats, 64)) != EH_OK || (st = sc.get(cnt, 16)) != EH_OK)
    return st;
  auto* ka = ptr<unsigned long long>(keys_a);
  auto* kbuf = ptr<unsigned long long>(keys_b);
  auto* stat = ptr<unsigned long long>(stats);
  auto* count = ptr<unsigned long long>(cnt);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kB), 0, s, ptr<uint32_t>(stats), uint64_t(16), 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kB), 0, s, ptr<uint32_t>(cnt), uint64_t(4), 0u);

  // rocPRIM scratch: the largest any of the calls below asks for
  size_t need = 0, b = 0;
  const unsigned key_bits = 2 * kb;
  auto chk = [&](hipError_t e, const char* what) { return hip_check(c, e, what); };
  rocprim::double_buffer<unsigned long long> db(ka, kbuf);
  if ((st = chk(rocprim::radix_sort_keys(nullptr, b, db, size_t(kcap), 0, key_bits, s),
                "radix sort size")) != EH_OK)
    return st;
  need = std::max(need, b);
  if ((st = chk(rocprim::unique(nullptr, b, kbuf, ka, count, size_t(mr),
                                rocprim::equal_to<unsigned long long>(), s),
                "unique size")) != EH_OK)
    return st;
  need = std::max(need, b);
  if ((st = chk(rocprim::radix_sort_pairs(nullptr, b, ptr<uint32_t>(deg), ptr<uint32_t>(deg_s),
                                          ptr<uint32_t>(ids), ptr<uint32_t>(seq), size_t(n1), 0,
                                          32, s),
                "pair sort size")) != EH_OK)
    return st;
  need = std::max(need, b);
  if (batch) {
    if ((st = chk(rocprim::radix_sort_pairs(nullptr, b, ptr<unsigned long long>(rk_in),
                                            ptr<unsigned long long>(rk_out), ptr<uint32_t>(ids),
                                            ptr<uint32_t>(seq), size_t(n1), 0, 64, s),
                  "batch rank sort size")) != EH_OK)
      return st;
    need = std::max(need, b);
  }
  if ((st = chk(rocprim::exclusive_scan(nullptr, b, ptr<uint32_t>(nw),
                                        ptr<unsigned long long>(off), 0ull, size_t(n) + 1,
                                        rocprim::plus<unsigned long long>(), s),
                "scan size")) != EH_OK)
    return st;
  need = std::max(need, b);
  if ((st = sc.get(tmp, need)) != EH_OK) return st;
  size_t tmp_bytes = tmp.bytes;

  // 1-2: canonical keys, sorted (in place between the two key buffers), unique
  // into the other buffer: `uniq` holds the edges, `spare` is free
  uint64_t m = 0;
  unsigned long long* uniq = ka;
  unsigned long long* spare = kbuf;
  if (m_raw) {
    if (batch)
      hipLaunchKernelGGL(k_batch_pair_keys, dim3(grid_of(m_raw)), dim3(kB), 0, s, d_src, d_dst,
                         m_raw, G, ptr<unsigned long long>(b_eoff), ptr<uint32_t>(b_vbase),
                         ptr<uint32_t>(b_nv), kb, ka, ptr<uint32_t>(cnt) + 2);
    else
      hipLaunchKernelGGL(k_pair_keys, dim3(grid_of(m_raw)), dim3(kB), 0, s, d_src, d_dst, m_raw,
                         n, kb, ka, ptr<uint32_t>(cnt) + 2);
    if ((st = chk(hipGetLastError(), "pair key kernel")) != EH_OK) return st;
    rocprim::double_buffer<unsigned long long> pairs(ka, kbuf);
    tmp_bytes = tmp.bytes;
    if ((st = chk(rocprim::radix_sort_keys(tmp.p, tmp_bytes, pairs, size_t(m_raw), 0, key_bits,
                                           s),
                  "radix sort of pairs")) != EH_OK)
      return st;
    spare = pairs.current();
    uniq = pairs.alternate();
    tmp_bytes = tmp.bytes;
    if ((st = chk(rocprim::unique(tmp.p, tmp_bytes, spare, uniq, count, size_t(m_raw),
                                  rocprim::equal_to<unsigned long long>(), s),
                  "unique of pairs")) != EH_OK)
      return st;
    unsigned long long h_cnt[2] = {0, 0};
    if ((st = download(c, h_cnt, count, 16, "read unique count")) != EH_OK ||
        (st = chk(hipStreamSynchronize(s), "build sync")) != EH_OK)
      return st;
    if (uint32_t(h_cnt[1])) {
      c->err = batch ? std::string("a vertex id is >= its graph's vertex count")
                     : "a vertex id is >= n = " + std::to_string(n);
      return EH_EINVAL;
    }
    unsigned long long last = 0;
    if (h_cnt[0] &&
        ((st = download(c, &last, uniq + h_cnt[0] - 1, 8, "read last key")) != EH_OK ||
         (st = chk(hipStreamSynchronize(s), "build sync")) != EH_OK))
      return st;
    m = h_cnt[0] - (h_cnt[0] && last == kSentinel ? 1 : 0);
  }
  const uint64_t edges = m;
  if (opts.symmetric) m *= 2;  // from here on, m counts stored arcs
  if (m > kMaxIndex) {
    c->err = "graph has " + std::to_string(m) + " stored edges; at most 2^31-1 supported";
    return EH_EOVERFLOW;
  }

  // 3: degrees and ranks
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_of(n1)), dim3(kB), 0, s, ptr<uint32_t>(deg),
                     uint64_t(n1), 0u);
  if (edges)
    hipLaunchKernelGGL(k_degrees, dim3(grid_of(edges)), dim3(kB), 0, s, uniq, edges, kb,
                       ptr<uint32_t>(deg));
  hipLaunchKernelGGL(k_iota, dim3(grid_of(n1)), dim3(kB), 0, s, ptr<uint32_t>(ids), n1);
  if ((st = dev_alloc(c, t.vert, 4ull * n1)) != EH_OK) return st;
  if (batch) {
    // ranks per graph: a stable sort by (graph, degree) keeps ids ascending
    const uint32_t* order_seq = nullptr;
    if (opts.order != EH_ORDER_INPUT) {
      hipLaunchKernelGGL(k_batch_rank_keys, dim3(grid_of(n1)), dim3(kB), 0, s, ptr<uint32_t>(deg),
                         n, G, ptr<uint32_t>(b_vbase), ptr<uint32_t>(b_nv),
                         ptr<unsigned long long>(rk_in), ptr<uint32_t>(ids));
      const unsigned gbits = 32u + (G > 1 ? 32u - uint32_t(__builtin_clz(G - 1)) : 1u);
      tmp_bytes = tmp.bytes;
      if ((st = chk(rocprim::radix_sort_pairs(tmp.p, tmp_bytes, ptr<unsigned long long>(rk_in),
                                              ptr<unsigned long long>(rk_out), ptr<uint32_t>(ids),
                                              ptr<uint32_t>(seq), size_t(n), 0, gbits, s),
                    "batch degree sort")) != EH_OK)
        return st;
      order_seq = ptr<uint32_t>(seq);
    }
    hipLaunchKernelGGL(k_batch_ranks, dim3(grid_of(n1)), dim3(kB), 0, s, order_seq, n, G,
                       ptr<uint32_t>(b_vbase), ptr<uint32_t>(b_nv), opts.order,
                       ptr<uint32_t>(rank), ptr<uint32_t>(t.vert));
  } else if (opts.order == EH_ORDER_INPUT) {
    hipLaunchKernelGGL(k_ranks, dim3(grid_of(n1)), dim3(kB), 0, s, ptr<uint32_t>(ids), n, 1u,
                       ptr<uint32_t>(rank), ptr<uint32_t>(t.vert));
  } else if (opts.order == EH_ORDER_BFS || opts.order == EH_ORDER_HYBRID ||
             opts.order == EH_ORDER_STRONG_RUNS) {
    // traversal orderings: the label sequence, then rank = n - 1 - label
    if ((st = device_traversal_sequence(c, uniq, edges, kb, n, ptr<uint32_t>(deg), opts.order,
                                        ptr<uint32_t>(seq))) != EH_OK)
      return st;
    hipLaunchKernelGGL(k_ranks, dim3(grid_of(n1)), dim3(kB), 0, s, ptr<uint32_t>(seq), n, 1u,
                       ptr<uint32_t>(rank), ptr<uint32_t>(t.vert));
  } else {
    // stable: equal degrees keep ids ascending
    tmp_bytes = tmp.bytes;
    if ((st = chk(rocprim::radix_sort_pairs(tmp.p, tmp_bytes, ptr<uint32_t>(deg),
                                            ptr<uint32_t>(deg_s), ptr<uint32_t>(ids),
                                            ptr<uint32_t>(seq), size_t(n), 0, 32, s),
                  "degree sort")) != EH_OK)
      return st;
    // degree order: this is rank order; reverse degree order: label order
    hipLaunchKernelGGL(k_ranks, dim3(grid_of(n1)), dim3(kB), 0, s, ptr<uint32_t>(seq), n,
                       opts.order == EH_ORDER_REV_DEGREE ? 1u : 0u, ptr<uint32_t>(rank),
                       ptr<uint32_t>(t.vert));
  }

  // 4: orientation and rows; `ka` then names the sorted oriented edges
  if (m) {
    hipLaunchKernelGGL(k_orient, dim3(grid_of(edges)), dim3(kB), 0, s, uniq, edges, kb,
                       opts.symmetric ? 1u : 0u, ptr<uint32_t>(rank), spare);
    rocprim::double_buffer<unsigned long long> oriented(spare, uniq);
    tmp_bytes = tmp.bytes;
    if ((st = chk(rocprim::radix_sort_keys(tmp.p, tmp_bytes, oriented, size_t(m), 0, key_bits, s),
                  "radix sort of oriented edges")) != EH_OK)
      return st;
    ka = oriented.current();
  }
  hipLaunchKernelGGL(k_rows, dim3(grid_of(uint64_t(n) + 1)), dim3(kB), 0, s, ka, m, n, kb,
                     ptr<uint32_t>(row));

  // 5: layouts, word offsets, members and bits, tables
  hipLaunchKernelGGL(k_layout, dim3(grid_of(uint64_t(n) + 1)), dim3(kB), 0, s, ka,
                     ptr<uint32_t>(row), n, kb, opts.layout, opts.tau, opts.s_min,
                     ptr<uint32_t>(nw), ptr<uint32_t>(base), stat);
  if (m)
    hipLaunchKernelGGL(k_bmerge, dim3(grid_of(m)), dim3(kB), 0, s, ka, ptr<uint32_t>(row), m, kb,
                       opts.symmetric ? 0u : 1u, stat);
  if (n && !opts.symmetric)
    hipLaunchKernelGGL(k_btarget_held, dim3(grid_of(n)), dim3(kB), 0, s, ptr<uint32_t>(row),
                       ptr<uint32_t>(deg), ptr<uint32_t>(t.vert), n, stat);
  tmp_bytes = tmp.bytes;
  if ((st = chk(rocprim::exclusive_scan(tmp.p, tmp_bytes, ptr<uint32_t>(nw),
                                        ptr<unsigned long long>(off), 0ull, size_t(n) + 1,
                                        rocprim::plus<unsigned long long>(), s),
                "word offset scan")) != EH_OK)
    return st;
  if ((st = chk(hipGetLastError(), "build kernels")) != EH_OK) return st;
  unsigned long long h_stat[4] = {0, 0, 0, 0}, W = 0;
  if ((st = download(c, h_stat, stat, 32, "read build statistics")) != EH_OK ||
      (st = download(c, &W, ptr<unsigned long long>(off) + n, 8, "read word count")) != EH_OK ||
      (st = chk(hipStreamSynchronize(s), "build sync")) != EH_OK)
    return st;
  if (m + W > kMaxPosition) {
    c->err = "edges plus bitset words exceed 2^32-2";
    return EH_EOVERFLOW;
  }
  const uint64_t n_bs = h_stat[0];
  if ((st = dev_alloc(c, t.col, 4ull * (m + W))) != EH_OK ||
      (st = dev_alloc(c, t.vdesc, 8ull * n)) != EH_OK ||
      (st = dev_alloc(c, t.bsdesc, 16ull * (n_bs ? n : 0))) != EH_OK)
    return st;
  auto* col = ptr<uint32_t>(t.col);
  if (W)
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_of(W)), dim3(kB), 0, s, col + m, W, 0u);
  if (m)
    hipLaunchKernelGGL(k_members, dim3(grid_of(m)), dim3(kB), 0, s, ka, m, kb, ptr<uint32_t>(nw),
                       ptr<uint32_t>(base), ptr<unsigned long long>(off), col);
  if (n)
    hipLaunchKernelGGL(k_tables, dim3(grid_of(n)), dim3(kB), 0, s, ptr<uint32_t>(row),
                       ptr<uint32_t>(nw), ptr<uint32_t>(base), ptr<unsigned long long>(off), n, m,
                       n_bs ? 1u : 0u, ptr<uint2>(t.vdesc), ptr<uint4>(t.bsdesc),
                       ptr<uint32_t>(bs_off));
  if ((st = chk(hipGetLastError(), "build kernels")) != EH_OK) return st;

  // host copy for work-item planning
  HostTrie& h = t.host;
  h.n = n;
  h.m = m;
  h.dmax = uint32_t(h_stat[1]);
  h.b_merge = h_stat[2];
  h.b_target = h_stat[3];
  h.n_bs = n_bs;
  h.n_graphs = G;
  h.g_vbase = batch ? batch->vbase : std::vector<uint32_t>{0, n};
  h.symmetric = opts.symmetric != 0;
  {
    // sizing a vector zero-fills and first-touches its pages: one thread per
    // array, so the large ones (col) do not wait for the others
    std::thread th[7] = {std::thread([&] { h.rank.resize(n); }),
                         std::thread([&] { h.vert.resize(n); }),
                         std::thread([&] { h.row.resize(size_t(n) + 1); }),
                         std::thread([&] { h.col.resize(m); }),
                         std::thread([&] { h.bs_off.resize(n); }),
                         std::thread([&] { h.bs_base.resize(n); }),
                         std::thread([&] { h.bs_nw.resize(n); })};
    for (auto& x : th) x.join();
  }
  h.n_words = W;  // the words stay in the device list buffer: planning never reads them
  h.words_on_device = true;
  if ((st = download(c, h.rank.data(), rank.p, 4ull * n, "download ranks")) != EH_OK ||
      (st = download(c, h.vert.data(), t.vert.p, 4ull * n, "download ids")) != EH_OK ||
      (st = download(c, h.row.data(), row.p, 4ull * (n + 1), "download rows")) != EH_OK ||
      (st = download(c, h.col.data(), col, 4ull * m, "download columns")) != EH_OK ||
      (st = download(c, h.bs_off.data(), bs_off.p, 4ull * n, "download word offsets")) != EH_OK ||
      (st = download(c, h.bs_base.data(), base.p, 4ull * n, "download bitset bases")) != EH_OK ||
      (st = download(c, h.bs_nw.data(), nw.p, 4ull * n, "download word counts")) != EH_OK ||
      (st = chk(hipStreamSynchronize(s), "build sync")) != EH_OK)
    return st;
  t.device_bytes = t.vdesc.bytes + t.col.bytes + t.bsdesc.bytes + t.vert.bytes;
  return EH_OK;
}

}  // namespace eh
