// Host-side trie construction and work-item planning.
//
// Trie (paper section 2.2): ids are dictionary-encoded to dense 32-bit ranks,
// by default ordered by (degree ascending, id ascending), or by one of the
// other node orderings of appendix A; every undirected edge is kept once,
// directed from lower to higher rank (the pruning of section 5.2), giving a
// two-level trie stored as CSR.  Each non-empty
// neighbour set keeps its uint layout and, when the set optimizer of section
// 4.4 calls it dense, also a bitset layout (section 4.1) with one block
// spanning [min, max]: base = min rounded down to a multiple of 32, words of
// 32 bits.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <thread>

#include "eh_internal.h"

namespace eh {

BuildOpts resolve_opts(const eh_build_opts* o) {
  BuildOpts b;
  if (!o) return b;
  b.layout = o->layout;
  b.tau = o->tau > 0.0f ? o->tau : 256.0f;
  b.s_min = o->s_min ? o->s_min : 1;
  b.order = o->order;
  b.symmetric = o->symmetric ? 1u : 0u;
  return b;
}

namespace {

// LSD radix sort of 64-bit keys on 16-bit digits, skipping constant digits.
void radix_sort_u64(std::vector<uint64_t>& a) {
  const size_t n = a.size();
  if (n < 2) return;
  std::vector<uint64_t> tmp(n);
  std::vector<uint64_t> cnt(1 << 16);
  for (int shift = 0; shift < 64; shift += 16) {
    std::fill(cnt.begin(), cnt.end(), 0);
    for (size_t i = 0; i < n; ++i) cnt[(a[i] >> shift) & 0xFFFF]++;
    bool trivial = false;
    for (uint64_t c : cnt)
      if (c == n) { trivial = true; break; }
    if (trivial) continue;
    uint64_t s = 0;
    for (auto& c : cnt) { uint64_t t = c; c = s; s += t; }
    for (size_t i = 0; i < n; ++i) tmp[cnt[(a[i] >> shift) & 0xFFFF]++] = a[i];
    a.swap(tmp);
  }
}

// Vertices sorted by degree (descending when `desc`), ties by id ascending
// (descending when `ids_desc`): a counting sort on degree.
std::vector<uint32_t> by_degree(const std::vector<uint32_t>& deg, bool desc, bool ids_desc) {
  const uint32_t n = uint32_t(deg.size());
  uint32_t maxd = 0;
  for (uint32_t d : deg) maxd = std::max(maxd, d);
  std::vector<uint32_t> start(size_t(maxd) + 2, 0);
  auto slot = [&](uint32_t d) { return desc ? maxd - d : d; };
  for (uint32_t d : deg) start[slot(d) + 1]++;
  for (size_t d = 1; d < start.size(); ++d) start[d] += start[d - 1];
  std::vector<uint32_t> seq(n);
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t v = ids_desc ? n - 1 - i : i;
    seq[start[slot(deg[v])]++] = v;
  }
  return seq;
}

// Symmetric adjacency of the cleaned pairs (a < b, sorted, unique): row v
// lists v's neighbours in ascending id order.  Filling in pair order gives
// sorted rows: the pairs (a, v), a < v, all precede the pairs (v, b).
void symmetric_rows(uint32_t n, const std::vector<uint64_t>& key,
                    const std::vector<uint32_t>& deg, std::vector<uint64_t>& off,
                    std::vector<uint32_t>& adj) {
  off.assign(size_t(n) + 1, 0);
  for (uint32_t v = 0; v < n; ++v) off[v + 1] = off[v] + deg[v];
  adj.resize(off[n]);
  std::vector<uint64_t> fill(off.begin(), off.end() - 1);
  for (uint64_t k : key) {
    const uint32_t a = uint32_t(k >> 32), b = uint32_t(k & 0xFFFFFFFFu);
    adj[fill[a]++] = b;
    adj[fill[b]++] = a;
  }
}

// Breadth-first labels (appendix A, node ordering): traversals start at the
// unvisited vertex of highest degree (ties: lowest id); neighbours are
// discovered in ascending id order.  Returns the vertices in label order.
std::vector<uint32_t> bfs_sequence(uint32_t n, const std::vector<uint64_t>& off,
                                   const std::vector<uint32_t>& adj,
                                   const std::vector<uint32_t>& deg) {
  std::vector<uint32_t> seq;
  seq.reserve(n);
  std::vector<uint8_t> seen(n, 0);
  for (uint32_t root : by_degree(deg, true, false)) {
    if (seen[root]) continue;
    seen[root] = 1;
    size_t head = seq.size();
    seq.push_back(root);
    while (head < seq.size()) {
      const uint32_t v = seq[head++];
      for (uint64_t e = off[v]; e < off[v + 1]; ++e) {
        const uint32_t w = adj[e];
        if (!seen[w]) { seen[w] = 1; seq.push_back(w); }
      }
    }
  }
  return seq;
}

// Strong runs (appendix A, node ordering): vertices visited by degree
// descending (ties id ascending); a visited vertex takes the next label if it
// has none, then its unlabelled neighbours take the next labels in ascending
// id order.  Returns the vertices in label order.
std::vector<uint32_t> strong_runs_sequence(uint32_t n, const std::vector<uint64_t>& off,
                                           const std::vector<uint32_t>& adj,
                                           const std::vector<uint32_t>& deg) {
  std::vector<uint32_t> seq;
  seq.reserve(n);
  std::vector<uint8_t> seen(n, 0);
  for (uint32_t v : by_degree(deg, true, false)) {
    if (!seen[v]) { seen[v] = 1; seq.push_back(v); }
    for (uint64_t e = off[v]; e < off[v + 1]; ++e) {
      const uint32_t w = adj[e];
      if (!seen[w]) { seen[w] = 1; seq.push_back(w); }
    }
  }
  return seq;
}

// Dictionary encoding (section 2.2) under one of the node orderings of
// appendix A.  `seq` lists the vertices in the order the ordering hands out
// labels; the paper keeps each edge from the larger label to the smaller, so
// rank = n - 1 - label with edges directed from lower to higher rank keeps
// the same edges and the same gaps inside every set.
void rank_vertices(uint32_t order, uint32_t n, const std::vector<uint64_t>& key,
                   const std::vector<uint32_t>& deg, std::vector<uint32_t>& rank,
                   std::vector<uint32_t>& vert) {
  std::vector<uint32_t> seq;
  switch (order) {
    case EH_ORDER_REV_DEGREE:
      seq = by_degree(deg, false, false);
      break;
    case EH_ORDER_INPUT:
      seq.resize(n);
      std::iota(seq.begin(), seq.end(), 0u);
      break;
    case EH_ORDER_BFS:
    case EH_ORDER_HYBRID:
    case EH_ORDER_STRONG_RUNS: {
      std::vector<uint64_t> off;
      std::vector<uint32_t> adj;
      symmetric_rows(n, key, deg, off, adj);
      seq = order == EH_ORDER_STRONG_RUNS ? strong_runs_sequence(n, off, adj, deg)
                                          : bfs_sequence(n, off, adj, deg);
      if (order == EH_ORDER_HYBRID) {
        // stable sort of the BFS sequence by degree descending
        std::vector<uint32_t> sorted(n);
        uint32_t maxd = 0;
        for (uint32_t d : deg) maxd = std::max(maxd, d);
        std::vector<uint32_t> start(size_t(maxd) + 2, 0);
        for (uint32_t d : deg) start[maxd - d + 1]++;
        for (size_t d = 1; d < start.size(); ++d) start[d] += start[d - 1];
        for (uint32_t v : seq) sorted[start[maxd - deg[v]]++] = v;
        seq.swap(sorted);
      }
      break;
    }
    default:  // EH_ORDER_DEGREE
      seq = by_degree(deg, true, true);
      break;
  }
  rank.assign(n, 0);
  vert.assign(n, 0);
  for (uint32_t label = 0; label < n; ++label) {
    const uint32_t r = n - 1 - label;
    rank[seq[label]] = r;
    vert[r] = seq[label];
  }
}

// One graph, local ids; output arrays are local (ranks from 0, rows from 0).
eh_status build_one(const uint32_t* src, const uint32_t* dst, uint64_t m_raw, uint32_t n,
                    const BuildOpts& opts, HostTrie& h, std::string& err) {
  for (uint64_t i = 0; i < m_raw; ++i) {
    if (src[i] >= n || dst[i] >= n) {
      err = "vertex id " + std::to_string(std::max(src[i], dst[i])) + " >= n = " +
            std::to_string(n);
      return EH_EINVAL;
    }
  }
  // clean: drop loops, canonical {min, max}, sort, unique
  std::vector<uint64_t> key;
  key.reserve(m_raw);
  for (uint64_t i = 0; i < m_raw; ++i) {
    uint32_t a = src[i], b = dst[i];
    if (a == b) continue;
    if (a > b) std::swap(a, b);
    key.push_back((uint64_t(a) << 32) | b);
  }
  radix_sort_u64(key);
  key.erase(std::unique(key.begin(), key.end()), key.end());
  const uint64_t m = key.size();
  if (m > kMaxIndex) {
    err = "graph has " + std::to_string(m) + " edges; at most 2^31-1 supported";
    return EH_EOVERFLOW;
  }
  h.n = n;
  h.m = m;
  // degree in the simple undirected graph
  std::vector<uint32_t> deg(n, 0);
  for (uint64_t k : key) { deg[k >> 32]++; deg[k & 0xFFFFFFFFu]++; }
  rank_vertices(opts.order, n, key, deg, h.rank, h.vert);
  // orient low rank -> high rank (or keep both directions: the unpruned
  // relation); rows sorted by scattering in target order
  const uint64_t arcs = opts.symmetric ? 2 * m : m;
  if (arcs > kMaxIndex) {
    err = "graph has " + std::to_string(arcs) + " stored edges; at most 2^31-1 supported";
    return EH_EOVERFLOW;
  }
  h.m = arcs;
  h.symmetric = opts.symmetric != 0;
  std::vector<uint32_t> eu(arcs), ev(arcs);
  std::vector<uint32_t> by_v(size_t(n) + 1, 0);
  h.row.assign(size_t(n) + 1, 0);
  for (uint64_t i = 0; i < m; ++i) {
    uint32_t ra = h.rank[key[i] >> 32], rb = h.rank[key[i] & 0xFFFFFFFFu];
    if (ra > rb) std::swap(ra, rb);
    eu[i] = ra;
    ev[i] = rb;
    h.row[ra + 1]++;
    by_v[rb + 1]++;
    if (opts.symmetric) {
      eu[m + i] = rb;
      ev[m + i] = ra;
      h.row[rb + 1]++;
      by_v[ra + 1]++;
    }
  }
  std::vector<uint64_t>().swap(key);
  for (uint32_t r = 0; r < n; ++r) { h.row[r + 1] += h.row[r]; by_v[r + 1] += by_v[r]; }
  std::vector<uint32_t> order(arcs);  // arc ids sorted by target rank
  {
    std::vector<uint32_t> fill(by_v.begin(), by_v.end() - 1);
    for (uint64_t i = 0; i < arcs; ++i) order[fill[ev[i]]++] = uint32_t(i);
  }
  h.col.assign(arcs, 0);
  {
    std::vector<uint32_t> fill(h.row.begin(), h.row.end() - 1);
    for (uint64_t k = 0; k < arcs; ++k) {
      const uint32_t i = order[k];
      h.col[fill[eu[i]]++] = ev[i];
    }
  }
  // statistics: B_merge (both sets of every intersection read once), and
  // B_target (target staging on a pruned trie: N+(v) read once, with a
  // 32-byte item and extent, for each v with a non-empty set and an in-edge;
  // per such in-edge u->v the members of N+(u) after v and an 8-byte record)
  h.dmax = 0;
  h.b_merge = 0;
  h.b_target = 0;
  {
    std::vector<uint8_t> held(opts.symmetric ? 0 : n, 0);
    for (uint32_t u = 0; u < n; ++u) {
      const uint32_t du = h.row[u + 1] - h.row[u];
      h.dmax = std::max(h.dmax, du);
      for (uint32_t e = h.row[u]; e < h.row[u + 1]; ++e) {
        const uint32_t v = h.col[e];
        const uint32_t dv = h.row[v + 1] - h.row[v];
        h.b_merge += 4ull * (du + dv);
        if (!opts.symmetric && dv) {
          held[v] = 1;
          h.b_target += 8ull + 4ull * (h.row[u + 1] - e - 1);
        }
      }
    }
    for (uint32_t v = 0; v < held.size(); ++v)
      if (held[v]) h.b_target += 32ull + 4ull * (h.row[v + 1] - h.row[v]);
  }
  // set layouts
  h.bs_off.assign(n, kNoBitset);
  h.bs_base.assign(n, 0);
  h.bs_nw.assign(n, 0);
  h.bs_words.clear();
  h.n_words = 0;
  h.n_bs = 0;
  if (opts.layout != EH_LAYOUT_UINT) {
    uint64_t words = 0;
    for (uint32_t u = 0; u < n; ++u) {
      const uint32_t len = h.row[u + 1] - h.row[u];
      if (len == 0) continue;
      const uint32_t lo = h.col[h.row[u]], hi = h.col[h.row[u + 1] - 1];
      const double range = double(hi) - double(lo) + 1.0;
      bool dense;
      if (opts.layout == EH_LAYOUT_BITSET_ALL)
        dense = true;
      else
        dense = len >= opts.s_min && range <= double(opts.tau) * double(len);
      if (!dense) continue;
      const uint32_t base = lo & ~31u;
      const uint32_t nw = ((hi - base) >> 5) + 1;
      if (h.m + words + nw > kMaxPosition) {
        err = "edges plus bitset words exceed 2^32-2";
        return EH_EOVERFLOW;
      }
      h.bs_off[u] = uint32_t(words);
      h.bs_base[u] = base;
      h.bs_nw[u] = nw;
      words += nw;
      h.n_bs++;
    }
    h.bs_words.assign(words, 0);
    h.n_words = words;
    for (uint32_t u = 0; u < n; ++u) {
      if (h.bs_off[u] == kNoBitset) continue;
      uint32_t* w = h.bs_words.data() + h.bs_off[u];
      const uint32_t base = h.bs_base[u];
      for (uint32_t e = h.row[u]; e < h.row[u + 1]; ++e) {
        const uint32_t d = h.col[e] - base;
        w[d >> 5] |= 1u << (d & 31);
      }
    }
  }
  h.n_graphs = 1;
  h.g_vbase = {0, n};
  return EH_OK;
}

}  // namespace

eh_status host_build(const uint32_t* src, const uint32_t* dst, uint64_t n_edges, uint32_t n,
                     const BuildOpts& opts, HostTrie& h, std::string& err) {
  if (n == 0 && n_edges > 0) {
    err = "edges given for an empty vertex set";
    return EH_EINVAL;
  }
  return build_one(src, dst, n_edges, n, opts, h, err);
}

eh_status host_build_batch(uint32_t n_graphs, const uint32_t* n_vertices, const uint64_t* edge_off,
                           const uint32_t* src, const uint32_t* dst, const BuildOpts& opts,
                           HostTrie& h, std::string& err) {
  uint64_t total_n = 0;
  for (uint32_t g = 0; g < n_graphs; ++g) {
    total_n += n_vertices[g];
    if (edge_off[g + 1] < edge_off[g]) {
      err = "edge_off is not monotone at graph " + std::to_string(g);
      return EH_EINVAL;
    }
  }
  if (total_n > kMaxIndex) {
    err = "batch has more than 2^31-1 vertices";
    return EH_EOVERFLOW;
  }
  std::vector<HostTrie> parts(n_graphs);
  std::vector<eh_status> st(n_graphs, EH_OK);
  std::vector<std::string> errs(n_graphs);
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::atomic<uint32_t> next{0};
  auto worker = [&]() {
    for (;;) {
      const uint32_t g = next.fetch_add(1);
      if (g >= n_graphs) return;
      const uint64_t a = edge_off[g], b = edge_off[g + 1];
      st[g] = build_one(src + a, dst + a, b - a, n_vertices[g], opts, parts[g], errs[g]);
    }
  };
  std::vector<std::thread> th;
  for (unsigned i = 0; i < nt; ++i) th.emplace_back(worker);
  for (auto& t : th) t.join();
  for (uint32_t g = 0; g < n_graphs; ++g) {
    if (st[g] != EH_OK) {
      err = "graph " + std::to_string(g) + ": " + errs[g];
      return st[g];
    }
  }
  // concatenate: graph g's ranks become vbase[g] + local rank
  uint64_t M = 0, W = 0;
  h = HostTrie();
  h.n_graphs = n_graphs;
  h.symmetric = opts.symmetric != 0;
  h.g_vbase.assign(size_t(n_graphs) + 1, 0);
  // each graph's rank range starts at a multiple of 32 so bitset words of
  // different sets stay aligned to one another; padding ranks are isolated
  uint64_t padded = 0;
  for (uint32_t g = 0; g < n_graphs; ++g) padded += (uint64_t(parts[g].n) + 31) & ~uint64_t(31);
  if (padded > kMaxIndex) {
    err = "batch has more than 2^31-1 vertices";
    return EH_EOVERFLOW;
  }
  for (uint32_t g = 0; g < n_graphs; ++g) {
    h.g_vbase[g + 1] = h.g_vbase[g] + ((parts[g].n + 31u) & ~31u);
    M += parts[g].m;
    W += parts[g].bs_words.size();
  }
  if (M > kMaxIndex || M + W > kMaxPosition) {
    err = "batch exceeds 2^31-1 edges or 2^32-2 edges plus bitset words";
    return EH_EOVERFLOW;
  }
  const uint32_t N = uint32_t(padded);
  h.n = N;
  h.m = M;
  h.rank.resize(N);
  h.vert.resize(N);
  h.row.resize(size_t(N) + 1);
  h.col.resize(M);
  h.bs_off.resize(N);
  h.bs_base.resize(N);
  h.bs_nw.resize(N);
  h.bs_words.resize(W);
  h.n_words = W;
  std::vector<uint64_t> ebase(n_graphs + 1, 0), wbase(n_graphs + 1, 0);
  for (uint32_t g = 0; g < n_graphs; ++g) {
    ebase[g + 1] = ebase[g] + parts[g].m;
    wbase[g + 1] = wbase[g] + parts[g].bs_words.size();
  }
  next = 0;
  auto copier = [&]() {
    for (;;) {
      const uint32_t g = next.fetch_add(1);
      if (g >= n_graphs) return;
      const HostTrie& p = parts[g];
      const uint32_t vb = h.g_vbase[g];
      const uint32_t eb = uint32_t(ebase[g]);
      const uint32_t wb = uint32_t(wbase[g]);
      for (uint32_t v = 0; v < p.n; ++v) {
        h.rank[vb + v] = vb + p.rank[v];
        h.vert[vb + v] = vb + p.vert[v];
        h.row[vb + v] = eb + p.row[v];
        h.bs_off[vb + v] = p.bs_off[v] == kNoBitset ? kNoBitset : wb + p.bs_off[v];
        // vb is a multiple of 32; a set without a bitset keeps base 0
        h.bs_base[vb + v] = p.bs_off[v] == kNoBitset ? 0u : vb + p.bs_base[v];
        h.bs_nw[vb + v] = p.bs_nw[v];
      }
      for (uint32_t v = vb + p.n; v < h.g_vbase[g + 1]; ++v) {
        h.rank[v] = v;
        h.vert[v] = v;
        h.row[v] = eb + uint32_t(p.m);
        h.bs_off[v] = kNoBitset;
        h.bs_base[v] = 0;
        h.bs_nw[v] = 0;
      }
      for (uint64_t e = 0; e < p.m; ++e) h.col[eb + e] = vb + p.col[e];
      std::copy(p.bs_words.begin(), p.bs_words.end(), h.bs_words.begin() + wb);
    }
  };
  th.clear();
  for (unsigned i = 0; i < nt; ++i) th.emplace_back(copier);
  for (auto& t : th) t.join();
  h.row[N] = uint32_t(M);
  h.dmax = 0;
  h.b_merge = 0;
  h.b_target = 0;
  h.n_bs = 0;
  for (uint32_t g = 0; g < n_graphs; ++g) {
    h.dmax = std::max(h.dmax, parts[g].dmax);
    h.b_merge += parts[g].b_merge;
    h.b_target += parts[g].b_target;
    h.n_bs += parts[g].n_bs;
  }
  return EH_OK;
}

// ---- work items -------------------------------------------------------------

namespace {

inline uint32_t out_deg(const HostTrie& h, uint32_t v) { return h.row[v + 1] - h.row[v]; }

// Host threads for planning: up to 16, one below 2^16 elements of work.
unsigned plan_threads(uint64_t work) {
  if (work < (1u << 16)) return 1;
  return std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
}

// Runs f(begin, end, part) over the ranges [b[p], b[p+1]) on one thread each.
// Ranges follow part order, so per-part outputs concatenated in part order
// equal a sequential pass.
template <class F>
void run_parts(const std::vector<uint64_t>& b, F f) {
  const unsigned parts = unsigned(b.size() - 1);
  if (parts == 1) {
    f(b[0], b[1], 0u);
    return;
  }
  std::vector<std::thread> th;
  for (unsigned p = 0; p < parts; ++p) th.emplace_back([&, p]() { f(b[p], b[p + 1], p); });
  for (auto& t : th) t.join();
}

// Equal ranges of [0, n).
std::vector<uint64_t> even_parts(uint64_t n, unsigned parts) {
  std::vector<uint64_t> b(parts + 1);
  for (unsigned p = 0; p <= parts; ++p) b[p] = n * p / parts;
  return b;
}

// Ranges of [0, n) holding about equal shares of the work prefix[x+1] - prefix[x].
template <class T>
std::vector<uint64_t> weighted_parts(const std::vector<T>& prefix, uint64_t n, unsigned parts) {
  std::vector<uint64_t> b(parts + 1, 0);
  const uint64_t total = prefix[n];
  for (unsigned p = 1; p < parts; ++p) {
    const uint64_t want = total * p / parts;
    b[p] = uint64_t(std::lower_bound(prefix.begin(), prefix.begin() + n, T(want)) -
                    prefix.begin());
    b[p] = std::max(b[p], b[p - 1]);
  }
  b[parts] = n;
  return b;
}

// Sources whose out-edges can reach the targets [v0, v1): the vertices of the
// graphs those targets belong to (the graphs of a batch share no edges).
std::pair<uint64_t, uint64_t> source_span(const HostTrie& h, uint64_t v0, uint64_t v1) {
  if (v0 >= v1) return {0, 0};
  const auto& gb = h.g_vbase;
  const size_t ga = size_t(std::upper_bound(gb.begin(), gb.end(), uint32_t(v0)) - gb.begin()) - 1;
  const size_t gz =
      size_t(std::upper_bound(gb.begin(), gb.end(), uint32_t(v1 - 1)) - gb.begin()) - 1;
  return {gb[ga], gb[gz + 1]};
}

template <class F>
void parallel_ranges(uint64_t n, F f) {
  run_parts(even_parts(n, plan_threads(n)), f);
}

// elements the kernel streams for set v: its words when the bitset is shorter
inline uint32_t stream_len(const HostTrie& h, uint32_t v, bool use_bitsets) {
  const uint32_t d = out_deg(h, v);
  if (use_bitsets && h.bs_off[v] != kNoBitset && h.bs_nw[v] < d) return h.bs_nw[v];
  return d;
}

// elements streamed for the part of N+(u) above v = col[e] (target staging)
inline uint32_t suffix_len(const HostTrie& h, uint32_t u, uint32_t e, bool use_bitsets) {
  const uint32_t len = h.row[u + 1] - e - 1;
  if (use_bitsets && len && h.bs_off[u] != kNoBitset) {
    const uint32_t w0 = (h.col[e] + 1 - h.bs_base[u]) >> 5;
    const uint32_t nw = w0 < h.bs_nw[u] ? h.bs_nw[u] - w0 : 0;
    if (nw < len) return nw;
  }
  return len;
}

// Split the streamed list idx[lb .. lb+len) of staged vertex s into items of
// about `chunk` streamed elements each.
template <class CostFn>
void split_items(uint32_t s, uint32_t lb, uint32_t len, uint32_t tag, uint32_t chunk,
                 uint32_t stage_cost, CostFn cost, std::vector<Item>& out) {
  uint32_t i = 0;
  while (i < len) {
    uint64_t acc = stage_cost;
    uint32_t j = i;
    while (j < len) {
      acc += cost(lb + j);
      ++j;
      if (acc >= chunk) break;
    }
    out.push_back(Item{s, lb + i, j - i, tag});
    i = j;
  }
}

}  // namespace

void make_items_source(const HostTrie& h, uint32_t u, uint32_t tag, uint32_t chunk_work,
                       uint32_t pattern, bool use_bitsets, std::vector<Item>& out) {
  const uint32_t du = out_deg(h, u);
  if (du < (pattern == EH_4CLIQUE ? 3u : 2u)) return;
  const uint32_t lb = h.row[u];
  if (pattern == EH_TRIANGLE) {
    // a staged set larger than an item's work (hub lists of a symmetric
    // trie) would be staged again for every streamed set: such items stream
    // at least as much as they stage instead
    const bool wide = du > chunk_work;
    split_items(u, lb, du, tag, wide ? du : chunk_work, wide ? 0 : du,
                [&](uint32_t e) { return uint64_t(stream_len(h, h.col[e], use_bitsets)) + 2; },
                out);
  } else {
    // level 1 streams N+(v); level 2 streams N+(w) for w in S, |S| <= min(du, dv)
    split_items(u, lb, du, tag, chunk_work, du,
                [&](uint32_t e) {
                  const uint32_t dv = out_deg(h, h.col[e]);
                  return uint64_t(dv) + 2 + uint64_t(std::min(du, dv)) * 24;
                },
                out);
  }
}

// Symmetric relation, totals only (kStageHalf): N(u) staged, N(x) streamed
// for the members x of N(u) ranked below u, a prefix of u's sorted row.
void make_items_half(const HostTrie& h, uint32_t u, uint32_t tag, uint32_t chunk_work,
                     bool use_bitsets, std::vector<Item>& out) {
  const uint32_t lb = h.row[u], du = out_deg(h, u);
  const auto first = h.col.begin() + lb;
  const uint32_t below = uint32_t(std::lower_bound(first, first + du, u) - first);
  if (below == 0) return;
  const bool wide = du > chunk_work;  // as in make_items_source
  split_items(u, lb, below, tag, wide ? du : chunk_work, wide ? 0 : du,
              [&](uint32_t e) { return uint64_t(stream_len(h, h.col[e], use_bitsets)) + 2; },
              out);
}

// Out-neighbours per item when only d+(u) is known: each out-neighbour's
// streamed work is taken to be about |N+(u)| (more for the 4-clique's second
// level).  0: u roots no instance (too few out-neighbours).
static uint32_t estimated_slice(uint32_t du, uint32_t chunk_work, uint32_t pattern) {
  if (du < (pattern == EH_4CLIQUE ? 3u : 2u)) return 0;
  const uint64_t per = pattern == EH_4CLIQUE ? uint64_t(du) * 25 + 2 : uint64_t(du) + 2;
  return uint32_t(std::max<uint64_t>(1, chunk_work / per));
}

void make_items_estimated(const HostTrie& h, uint32_t u, uint32_t tag, uint32_t chunk_work,
                          uint32_t pattern, std::vector<Item>& out) {
  const uint32_t du = out_deg(h, u);
  const uint32_t slice = estimated_slice(du, chunk_work, pattern);
  if (slice == 0) return;
  for (uint32_t i = 0; i < du; i += slice)
    out.push_back(Item{u, h.row[u] + i, std::min(slice, du - i), tag});
}

uint64_t count_items_estimated(const HostTrie& h, uint32_t u, uint32_t chunk_work,
                               uint32_t pattern) {
  const uint32_t du = out_deg(h, u);
  const uint32_t slice = estimated_slice(du, chunk_work, pattern);
  return slice ? (uint64_t(du) + slice - 1) / slice : 0;
}

// The snake schedule deals items sorted by decreasing cost; a batch keeps
// each graph's items contiguous (per-graph launches take ranges of them), so
// its plans are not sorted and snake then only changes the dealing order.
void free_plan(Ctx* c, Plan& p) {
  dev_free(c, p.items);
  dev_free(c, p.sdesc);
  dev_free(c, p.rec);
  dev_free(c, p.gsub);
  dev_free(c, p.k4s);
  dev_free(c, p.k4l);
}

// 4-cliques on a pruned single graph: roots that fit the induced-neighbourhood
// kernel are counted there (tuning k4_local).
static bool wants_k4_local(const Tuning& tu, const HostTrie& h, uint32_t pattern) {
  return pattern == EH_4CLIQUE && tu.k4_local && h.n_graphs == 1 && !h.symmetric;
}

static int local_class(const HostTrie& h, uint32_t u) {
  return k4_local_class(h.row[u + 1] - h.row[u]);
}

static bool wants_balance(const Tuning& tu, const HostTrie& h) {
  return tu.dynamic == 5 && h.n_graphs == 1;
}

Plan* find_plan(Ctx* c, Trie* t, uint32_t pattern, uint32_t staging) {
  const Tuning& tu = c->tune;
  const uint32_t chunk = std::max<uint32_t>(tu.chunk_work, 64);
  if (pattern == EH_4CLIQUE) staging = EH_STAGE_SOURCE;
  const uint32_t group = (staging == EH_STAGE_TARGET && pattern == EH_TRIANGLE) ? tu.group : 1u;
  const bool balanced = wants_balance(tu, t->host);
  for (auto& p : t->plans)
    if (p->pattern == pattern && p->staging == staging && p->chunk_work == chunk &&
        p->use_bitsets == tu.use_bitsets && p->stage_words == tu.stage_words &&
        p->group == group && p->balanced == balanced &&
        p->k4_local == wants_k4_local(tu, t->host, pattern))
      return p.get();
  return nullptr;
}

eh_status get_plan(Ctx* c, Trie* t, uint32_t pattern, uint32_t staging, Plan** out) {
  const Tuning& tu = c->tune;
  const uint32_t chunk = std::max<uint32_t>(tu.chunk_work, 64);
  if (pattern == EH_4CLIQUE) staging = EH_STAGE_SOURCE;
  if (Plan* found = find_plan(c, t, pattern, staging)) {
    *out = found;
    return EH_OK;
  }
  const HostTrie& h = t->host;
  std::vector<Item> items;
  auto plan = std::make_unique<Plan>();
  plan->pattern = pattern;
  plan->staging = staging;
  plan->chunk_work = chunk;
  plan->use_bitsets = tu.use_bitsets;
  plan->stage_words = tu.stage_words;
  plan->group = (staging == EH_STAGE_TARGET && pattern == EH_TRIANGLE) ? tu.group : 1u;
  plan->g_item_off.assign(size_t(h.n_graphs) + 1, 0);
  plan->k4_local = wants_k4_local(tu, h, pattern);
  const bool ub = tu.use_bitsets != 0;
  // Target-staged triangle plans are built on the GPU, except grouped plans
  // of a few large graphs (grouping walks each graph's items in one thread
  // there) and when EH_HOST_PLAN is set.
  if (staging == EH_STAGE_TARGET && pattern == EH_TRIANGLE && !std::getenv("EH_HOST_PLAN") &&
      (plan->group <= 1 || h.n_graphs >= 256)) {
    const uint32_t cap = tu.stage_words && tu.stage_words < kStageWords ? tu.stage_words
                                                                         : kStageWords;
    eh_status st = device_plan_target(c, *t, *plan, chunk, ub, cap, plan->group);
    if (st == EH_OK && wants_balance(tu, h)) {
      plan->balanced = true;
      st = device_plan_balance(c, *t, *plan);
    }
    if (st != EH_OK) {
      free_plan(c, *plan);
      return st;
    }
    *out = plan.get();
    t->plans.push_back(std::move(plan));
    return EH_OK;
  }
  if (staging == EH_STAGE_TARGET) {
    if (!t->has_transpose) {
      // in-edges of each v, ascending in u: {u, position of v in N+(u)}.
      // Each thread owns a range of targets and scans, in source order, every
      // edge that can reach them (all of a single graph's, only its own
      // graphs' in a batch), so it writes its targets' in-edges in the
      // sequential order with no shared counters; target ranges hold about
      // equal in-edges.
      const unsigned parts = plan_threads(h.m);
      t->trow.assign(size_t(h.n) + 1, 0);
      run_parts(weighted_parts(h.row, h.n, parts), [&](uint64_t v0, uint64_t v1, unsigned) {
        const auto span = source_span(h, v0, v1);
        for (uint64_t e = h.row[span.first]; e < h.row[span.second]; ++e) {
          const uint32_t v = h.col[e];
          if (v >= v0 && v < v1) t->trow[v + 1]++;
        }
      });
      for (uint32_t v = 0; v < h.n; ++v) t->trow[v + 1] += t->trow[v];
      t->tin.assign(2 * h.m, 0);
      std::vector<uint32_t> fill(t->trow.begin(), t->trow.end() - 1);
      run_parts(weighted_parts(t->trow, h.n, parts), [&](uint64_t v0, uint64_t v1, unsigned) {
        const auto span = source_span(h, v0, v1);
        for (uint64_t u = span.first; u < span.second; ++u)
          for (uint32_t e = h.row[u]; e < h.row[u + 1]; ++e) {
            const uint32_t v = h.col[e];
            if (v < v0 || v >= v1) continue;
            const uint32_t k = fill[v]++;
            t->tin[2 * k] = u;
            t->tin[2 * k + 1] = e;
          }
      });
      t->has_transpose = true;
    }
  }
  {
    // items of each vertex in vertex order: threads take vertex ranges and
    // their lists are joined in range order; graph g's items start at the
    // first item whose vertex is at or above g's first rank
    std::vector<std::vector<Item>> part(16);
    const std::vector<uint32_t>& work = staging == EH_STAGE_TARGET ? t->trow : h.row;
    run_parts(weighted_parts(work, h.n, plan_threads(h.m)), [&](uint64_t x0, uint64_t x1,
                                                                 unsigned p) {
      std::vector<Item>& out = part[p];
      uint32_t g = uint32_t(std::upper_bound(h.g_vbase.begin(), h.g_vbase.end(), uint32_t(x0)) -
                            h.g_vbase.begin()) - 1;
      for (uint64_t x = x0; x < x1; ++x) {
        while (x >= h.g_vbase[g + 1]) ++g;
        const uint32_t tag = h.n_graphs > 1 ? g : 0;
        const uint32_t v = uint32_t(x);
        if (staging == EH_STAGE_TARGET) {
          const uint32_t dv = out_deg(h, v);
          const uint32_t lb = t->trow[v], len = t->trow[v + 1] - t->trow[v];
          if (dv == 0 || len == 0) continue;
          split_items(v, lb, len, tag, chunk, dv,
                      [&](uint32_t k) {
                        return uint64_t(suffix_len(h, t->tin[2 * k], t->tin[2 * k + 1], ub)) + 2;
                      },
                      out);
        } else if (staging == kStageHalf) {
          make_items_half(h, v, tag, chunk, ub, out);
        } else if (!plan->k4_local || local_class(h, v) < 0) {
          make_items_source(h, v, tag, chunk, pattern, ub, out);
        }
      }
    });
    size_t total = 0;
    for (auto& q : part) total += q.size();
    items.reserve(total);
    for (auto& q : part) {
      items.insert(items.end(), q.begin(), q.end());
      std::vector<Item>().swap(q);
    }
    for (uint32_t g = 0; g <= h.n_graphs; ++g)
      plan->g_item_off[g] = uint64_t(
          std::lower_bound(items.begin(), items.end(), h.g_vbase[g],
                           [](const Item& it, uint32_t v) { return it.s < v; }) -
          items.begin());
  }
  for (const Item& it : items) plan->item_dmax = std::max(plan->item_dmax, out_deg(h, it.s));
  eh_status st = EH_OK;
  if (staging == EH_STAGE_TARGET && pattern == EH_TRIANGLE) {
    // Resolve on the host what each wave would otherwise look up through
    // chains of dependent loads: the staged set's extent per item, and per
    // in-edge u->v the streamed part of N+(u) above v (elements, or bitset
    // words when fewer and v's set will be held as a bitmap).  A record is
    // 8 bytes, {start, length | word offset << 16 | kHiBit for words}: a
    // length fits 16 bits because degree order bounds out-degrees by
    // sqrt(2m) < 2^16, and words are clipped to the staged bitmap's window
    // (words outside it cannot match), so the offset is in [0, cap).
    const uint32_t cap = tu.stage_words && tu.stage_words < kStageWords ? tu.stage_words
                                                                         : kStageWords;
    auto staged_lo_al = [&](uint32_t v) { return h.col[h.row[v]] & ~31u; };
    auto bitmap_mode = [&](uint32_t v) {
      const uint32_t lo_al = staged_lo_al(v), hi = h.col[h.row[v + 1] - 1];
      return hi - lo_al < cap * 32u;
    };
    std::vector<uint32_t> sd;   // per item: staged-set extent, or a group's descriptor
    std::vector<uint32_t> gsub; // per grouped member
    std::vector<uint8_t> grouped(h.n, 0);
    if (plan->group > 1) {
      // Consecutive small items of one graph share a wave: up to `group`
      // whole-vertex items whose records and staged members each total at
      // most 64 and whose staged sets fit one bitmap interleaved K ways
      // (bit (x - base) K + k marks x as a member of the k-th set), K the
      // power of two >= the member count.  Their records carry no bitset
      // words (a word does not line up with interleaved bits).
      // Groups never cross graphs: threads take graph ranges holding about
      // equal item counts, and their outputs are joined in graph order (a
      // grouped item's member index is then rebased).
      struct Part {
        std::vector<Item> out;
        std::vector<uint32_t> sd, gsub;
        std::vector<uint64_t> off;  // per graph of the range: first output item
      };
      const std::vector<uint64_t> gparts =
          weighted_parts(plan->g_item_off, h.n_graphs,
                         std::min<unsigned>(plan_threads(items.size()), h.n_graphs));
      std::vector<Part> part(gparts.size() - 1);
      auto whole = [&](const Item& it) {
        return it.lbeg == t->trow[it.s] && it.llen == t->trow[it.s + 1] - t->trow[it.s];
      };
      run_parts(gparts, [&](uint64_t g0, uint64_t g1, unsigned pi) {
        Part& q = part[pi];
        for (uint64_t g = g0; g < g1; ++g) {
          q.off.push_back(q.out.size());
          const uint64_t i1 = plan->g_item_off[g + 1];
          for (uint64_t i = plan->g_item_off[g]; i < i1;) {
            const Item& a0 = items[i];
            uint64_t j = i + 1;
            if (whole(a0)) {
              uint32_t base = h.col[h.row[a0.s]], top = h.col[h.row[a0.s + 1] - 1];
              uint32_t recs = a0.llen, mem = h.row[a0.s + 1] - h.row[a0.s];
              while (j < i1 && j - i < plan->group && whole(items[j])) {
                const uint32_t v = items[j].s;
                const uint32_t nb = std::min(base, h.col[h.row[v]]);
                const uint32_t nt = std::max(top, h.col[h.row[v + 1] - 1]);
                const uint64_t kk = (j - i + 1) <= 2 ? 2 : 4;
                const uint32_t dv = h.row[v + 1] - h.row[v];
                if (recs + items[j].llen > 64 || mem + dv > 64 ||
                    (uint64_t(nt) - nb + 1) * kk > uint64_t(cap) * 32)
                  break;
                base = nb;
                top = nt;
                recs += items[j].llen;
                mem += dv;
                ++j;
              }
              if (j - i > 1) {
                const uint32_t cnt = uint32_t(j - i);
                q.out.push_back(Item{uint32_t(q.gsub.size() / 4) | kHiBit, cnt, recs, a0.tag});
                q.sd.insert(q.sd.end(), {base, cnt <= 2 ? 1u : 2u, mem, top});
                for (uint64_t k = i; k < j; ++k) {
                  const uint32_t v = items[k].s;
                  grouped[v] = 1;
                  q.gsub.insert(q.gsub.end(),
                                {items[k].lbeg, items[k].llen, h.row[v], h.row[v + 1] - h.row[v]});
                }
                i = j;
                continue;
              }
            }
            const uint32_t v = a0.s;
            q.out.push_back(a0);
            q.sd.insert(q.sd.end(), {h.row[v], h.row[v + 1] - h.row[v], h.col[h.row[v]],
                                     h.col[h.row[v + 1] - 1]});
            i = i + 1;
          }
        }
      });
      std::vector<Item> out;
      std::vector<uint64_t> off(h.n_graphs + 1, 0);
      size_t n_out = 0, n_sd = 0, n_gsub = 0;
      for (const Part& q : part) {
        n_out += q.out.size();
        n_sd += q.sd.size();
        n_gsub += q.gsub.size();
      }
      out.reserve(n_out);
      sd.reserve(n_sd);
      gsub.reserve(n_gsub);
      for (size_t pi = 0; pi < part.size(); ++pi) {
        Part& q = part[pi];
        const uint32_t gbase = uint32_t(gsub.size() / 4);
        const uint64_t ibase = out.size();
        for (Item it : q.out) {
          if (it.s & kHiBit) it.s = ((it.s & kMaxIndex) + gbase) | kHiBit;
          out.push_back(it);
        }
        for (size_t k = 0; k < q.off.size(); ++k) off[gparts[pi] + k] = ibase + q.off[k];
        sd.insert(sd.end(), q.sd.begin(), q.sd.end());
        gsub.insert(gsub.end(), q.gsub.begin(), q.gsub.end());
        Part().out.swap(q.out);
      }
      off[h.n_graphs] = out.size();
      items.swap(out);
      plan->g_item_off.swap(off);
    } else {
      for (const Item& it : items) {
        const uint32_t v = it.s;
        sd.insert(sd.end(), {h.row[v], h.row[v + 1] - h.row[v], h.col[h.row[v]],
                             h.col[h.row[v + 1] - 1]});
      }
    }
    if (sd.empty()) sd.assign(4, 0);
    std::vector<uint32_t> rec(2 * std::max<uint64_t>(h.m, 1), 0);
    bool wide = false;
    // per source set, the fields a record reads, packed in one 16-byte entry
    std::vector<uint4> src_info(h.n);
    parallel_ranges(h.n, [&](uint64_t u0, uint64_t u1, unsigned) {
      for (uint64_t u = u0; u < u1; ++u)
        src_info[u] = make_uint4(h.row[u + 1], h.bs_off[u], h.bs_base[u], h.bs_nw[u]);
    });
    // in-edges grouped by target v: v's own values are read once
    run_parts(weighted_parts(t->trow, h.n, plan_threads(h.m)), [&](uint64_t v0, uint64_t v1,
                                                                     unsigned) {
      for (uint64_t vv = v0; vv < v1; ++vv) {
        const uint32_t v = uint32_t(vv);
        const bool words_ok = ub && !grouped[v] && h.row[v + 1] > h.row[v] && bitmap_mode(v);
        const int64_t v_word = words_ok ? int64_t(staged_lo_al(v) >> 5) : 0;
        for (uint32_t k = t->trow[v]; k < t->trow[v + 1]; ++k) {
          const uint32_t u = t->tin[2 * k], e = t->tin[2 * k + 1];
          const uint4 su = src_info[u];  // {row end, word offset, base, words}
          const uint32_t len = su.x - e - 1;
          uint32_t sb = e + 1, n = len, sm = 0, wf = 0;
          if (words_ok && len && su.y != kNoBitset) {
            const uint32_t w0 = (v + 1 - su.z) >> 5;
            const int64_t nw = w0 < su.w ? int64_t(su.w - w0) : 0;
            // the first streamed word's index in the staged bitmap, then the
            // part of the words that overlaps the bitmap [0, cap)
            const int64_t off = int64_t((su.z >> 5) + w0) - v_word;
            const int64_t first = std::max<int64_t>(0, -off);
            const int64_t last = std::min<int64_t>(nw, int64_t(cap) - off);
            const int64_t words = last > first ? last - first : 0;
            if (words < int64_t(len)) {
              sb = uint32_t(h.m) + su.y + w0 + uint32_t(first);
              n = uint32_t(words);
              sm = words ? uint32_t(off + first) : 0u;
              wf = kHiBit;
            }
          }
          if (n > 0xFFFFu || sm > 0x7FFFu) {
            __atomic_store_n(&wide, true, __ATOMIC_RELAXED);
            continue;
          }
          rec[2 * k] = sb;
          rec[2 * k + 1] = n | (sm << 16) | wf;
        }
      }
    });
    if (wide) {
      c->err = "segment record field beyond 16 bits";
      return EH_EOVERFLOW;
    }
    if (gsub.empty()) gsub.assign(4, 0);
    if ((st = dev_alloc(c, plan->sdesc, sizeof(uint32_t) * sd.size())) != EH_OK ||
        (st = dev_alloc(c, plan->rec, sizeof(uint32_t) * rec.size())) != EH_OK ||
        (st = dev_alloc(c, plan->gsub, sizeof(uint32_t) * gsub.size())) != EH_OK ||
        (st = hip_check(c, hipMemcpy(plan->sdesc.p, sd.data(), sizeof(uint32_t) * sd.size(),
                                     hipMemcpyHostToDevice), "upload stage table")) != EH_OK ||
        (st = hip_check(c, hipMemcpy(plan->rec.p, rec.data(), sizeof(uint32_t) * rec.size(),
                                     hipMemcpyHostToDevice), "upload segment records")) != EH_OK ||
        (st = hip_check(c, hipMemcpy(plan->gsub.p, gsub.data(), sizeof(uint32_t) * gsub.size(),
                                     hipMemcpyHostToDevice), "upload grouped members")) != EH_OK) {
      dev_free(c, plan->sdesc);
      dev_free(c, plan->rec);
      dev_free(c, plan->gsub);
      return st;
    }
  }
  if (pattern == EH_4CLIQUE &&
      (st = prepare_k4_lists(c, h, items.data(), items.size(), plan->k4s, plan->k4s_waves,
                             plan->k4s_stride)) != EH_OK)
    return st;
  plan->n_items = items.size();
  if ((st = dev_alloc(c, plan->items, sizeof(Item) * std::max<size_t>(items.size(), 1))) != EH_OK) {
    dev_free(c, plan->k4s);
    return st;
  }
  if (!items.empty())
    if ((st = hip_check(c, hipMemcpy(plan->items.p, items.data(), sizeof(Item) * items.size(),
                                     hipMemcpyHostToDevice), "upload work items")) != EH_OK) {
      dev_free(c, plan->items);
      dev_free(c, plan->k4s);
      return st;
    }
  if (plan->k4_local && (st = device_plan_k4_local(c, *t, *plan, ub)) != EH_OK) {
    free_plan(c, *plan);
    return st;
  }
  if (wants_balance(tu, h)) {
    plan->balanced = true;
    if ((st = device_plan_balance(c, *t, *plan)) != EH_OK) {
      free_plan(c, *plan);
      return st;
    }
  }
  *out = plan.get();
  t->plans.push_back(std::move(plan));
  return EH_OK;
}

}  // namespace eh
