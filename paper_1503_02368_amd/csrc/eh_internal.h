// Internal declarations shared by the host and device halves of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/eh.h"

namespace eh {

constexpr uint32_t kNoBitset = 0xFFFFFFFFu;
constexpr uint32_t kHiBit = 0x80000000u;   // vdesc.y: the set also has a bitset
constexpr uint32_t kMaxIndex = 0x7FFFFFFFu;  // edges (and set sizes) stay below 2^31
// Positions in a trie's list buffer (members, then bitset words) use all 32
// bits; 0xFFFFFFFF is the no-bitset sentinel.
constexpr uint64_t kMaxPosition = 0xFFFFFFFEull;
constexpr uint32_t kStageWords = 1024;        // LDS words per wave for a staged set
// Plan staging beside EH_STAGE_SOURCE / EH_STAGE_TARGET, internal: on a
// symmetric trie, each undirected edge {x, u} (x ranked below u) once, at u:
// N(u) is staged and N(x) streamed for the members of N(u) below u.  It
// counts each triangle 3 times instead of the join's 6 (totals only).
constexpr uint32_t kStageHalf = 3;
constexpr uint32_t kCursorWords = 64;         // uint32 words between work cursors
constexpr uint32_t kMaxParts = 32;           // item partitions (L2 domains) at most
// Allocation-free counting: cursors (kCursorWords * kMaxParts uint32 words)
// then one uint64 accumulator, in a static device array of this many bytes.
constexpr size_t kNoAllocCursorBytes = size_t(kCursorWords) * kMaxParts * sizeof(uint32_t);
constexpr size_t kNoAllocScratchBytes = 16384;
static_assert(kNoAllocCursorBytes + 256 <= kNoAllocScratchBytes, "scratch holds cursors + 1 word");

// One unit of scheduled work: the set N+(s) is held on chip while the sets
// N+(t) of the streamed vertices t = idx[lbeg .. lbeg+llen) are intersected
// with it.  tag selects the output accumulator (graph or request slot).
struct Item {
  uint32_t s;
  uint32_t lbeg;
  uint32_t llen;
  uint32_t tag;
};
static_assert(sizeof(Item) == 16, "Item is one 128-bit load");

// Host half of a trie: rank-space oriented CSR plus set layouts.
struct HostTrie {
  uint32_t n = 0;
  uint64_t m = 0;                    // stored edges (oriented, or both directions)
  uint32_t dmax = 0;                 // max out-degree
  uint64_t b_merge = 0;
  uint64_t b_target = 0;             // reads of target-staged triangle counting (0: symmetric)
  std::vector<uint32_t> rank;        // rank[id]
  std::vector<uint32_t> vert;        // vert[rank] = id
  std::vector<uint32_t> row;         // [n+1]
  std::vector<uint32_t> col;         // [m], rank ids, rows ascending
  std::vector<uint32_t> bs_off;      // [n] word offset or kNoBitset
  std::vector<uint32_t> bs_base;     // [n]
  std::vector<uint32_t> bs_nw;       // [n]
  std::vector<uint32_t> bs_words;    // empty when words_on_device
  uint64_t n_words = 0;              // bitset words in total
  bool words_on_device = false;      // GPU-built: the words live in the device list buffer only
  uint64_t n_bs = 0;
  // batch: graph g owns ranks [g_vbase[g], g_vbase[g+1]) and edges
  // [row[g_vbase[g]], row[g_vbase[g+1]])
  std::vector<uint32_t> g_vbase;     // [G+1]
  uint32_t n_graphs = 1;
  bool symmetric = false;            // both directions of every edge (unpruned relation)
};

struct BuildOpts {
  uint32_t layout = EH_LAYOUT_HYBRID;
  float tau = 256.0f;  // the paper's rule: one 256-bit register per member
  uint32_t s_min = 1;
  uint32_t order = EH_ORDER_DEGREE;
  uint32_t symmetric = 0;
};
BuildOpts resolve_opts(const eh_build_opts* o);

// Builds one graph's trie into h (appending when h already holds graphs:
// batch construction).  Returns EH_OK / EH_EINVAL / EH_EOVERFLOW.
eh_status host_build(const uint32_t* src, const uint32_t* dst, uint64_t n_edges, uint32_t n,
                     const BuildOpts& opts, HostTrie& h, std::string& err);
eh_status host_build_batch(uint32_t n_graphs, const uint32_t* n_vertices, const uint64_t* edge_off,
                           const uint32_t* src, const uint32_t* dst, const BuildOpts& opts,
                           HostTrie& h, std::string& err);

struct Trie;
// A batch for the GPU build: host arrays of the graphs' vertex counts and
// pair offsets, and the padded first rank of each graph (multiples of 32).
struct DeviceBatch {
  uint32_t n_graphs = 0;
  const uint32_t* n_vertices = nullptr;
  const uint64_t* edge_off = nullptr;  // [n_graphs + 1]
  std::vector<uint32_t> vbase;         // [n_graphs + 1]
};
// The same trie built on the GPU from device-resident raw pairs (orderings
// that are sorts: degree, reverse degree, input), with its host copy.
struct Ctx;
eh_status device_build(Ctx* c, const uint32_t* d_src, const uint32_t* d_dst, uint64_t m_raw,
                       uint32_t n, const BuildOpts& opts, Trie& t,
                       const DeviceBatch* batch = nullptr);

struct Tuning {
  uint32_t kernel = EH_KERNEL_STAGED;
  uint32_t staging = EH_STAGE_TARGET;
  uint32_t algo = EH_ALGO_AUTO;
  float gamma = 32.0f;
  uint32_t chunk_work = 4096;
  uint32_t waves_per_cu = 32;
  uint32_t group_lanes = 0;
  uint32_t use_bitsets = 1;
  uint32_t dynamic = 0;
  uint32_t stage_words = 0;
  uint32_t xcds = 0;
  uint32_t unroll = 8;
  uint32_t grab = 8;
  uint32_t search_below = 24;
  uint32_t group = 1;
  uint32_t reverse = 0;
  uint32_t k4_local = 1;
};

struct Ctx;

// Device buffer owned through the context's allocator.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Work-item plan of one (pattern, staging, granularity) on a trie.
struct Plan {
  uint32_t pattern = 0;
  uint32_t staging = 0;
  uint32_t chunk_work = 0;
  uint32_t use_bitsets = 0;
  uint32_t stage_words = 0;
  uint32_t group = 1;                // most per-vertex items in one grouped item
  bool balanced = false;             // items sorted by decreasing estimated cost (schedule 5)
  uint64_t n_items = 0;
  DevBuf items;
  // target staging only: per item {begin, length, min, max} of the staged set,
  // and per in-edge the streamed segment {start | kHiBit for words, length |
  // word offset from the staged bitmap << 16} (uint2)
  DevBuf sdesc;
  DevBuf rec;
  // grouped items: per member {first record, records, first member in col,
  // members}; a grouped item has s = first member entry | kHiBit, lbeg = its
  // member count, llen = its records, and the descriptor {bitmap base, log2
  // of the interleave, members, max member}
  DevBuf gsub;
  std::vector<uint64_t> g_item_off;  // batch: items of graph g are [off[g], off[g+1])
  uint32_t item_dmax = 0;            // max out-degree of an item's source vertex
  // 4-cliques whose root's out-degree exceeds kK4ListMax: S = N+(u) & N+(v)
  // is kept in HBM, one list of k4s_stride words per wave of the launch over
  // those items (k4s_waves waves)
  DevBuf k4s;
  uint32_t k4s_waves = 0;
  uint32_t k4s_stride = 0;
  // 4-cliques over induced neighbourhoods: root records (uint4) of the roots
  // counted by k_k4_local (absent from items), out-degree classes (<= 64,
  // <= 128, <= 256, <= 512) one after another, their segment records in rec
  bool k4_local = false;
  DevBuf k4l;
  uint64_t k4l_n[4] = {0, 0, 0, 0};
};

struct Trie {
  Ctx* ctx = nullptr;
  HostTrie host;
  bool has_transpose = false;
  std::vector<uint32_t> trow;        // [n+1] in-edge offsets
  std::vector<uint32_t> tin;         // [2m] in-edges {u, position of u->v in col}, by v then u
  // device arrays
  DevBuf vdesc;   // uint2 [n]: {row begin, out-degree | kHiBit if bitset}
  DevBuf col;     // uint32 [m + W]: the uint sets, then every bitset's words
  DevBuf bsdesc;  // uint4 [n]: {position of first word in col, base, words, 0}
  DevBuf vert;    // uint32 [n]: rank -> id
  std::vector<std::unique_ptr<Plan>> plans;
  uint64_t device_bytes = 0;
};

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  eh_allocator alloc{};
  bool has_alloc = false;
  Tuning tune;
  std::string err;
  int n_cu = 256;
  // scratch: accumulators and cursor
  DevBuf acc;       // uint64 accumulators
  size_t acc_cap = 0;
  DevBuf cursor;    // uint32 work cursors, kCursorWords apart
  DevBuf half;      // uint64: the half count of a symmetric trie; allocated with the
                    // context and never reallocated, so captured launches stay valid
  uint64_t* pinned = nullptr;  // host staging for results
  size_t pinned_cap = 0;
  void* noalloc_scratch = nullptr;  // this device's static scratch (eh_count_add_noalloc)
  // launches that run side by side with the stream's: streams of the default
  // priority, forked from and joined back into `stream` by events
  static constexpr int kSide = 3;
  hipStream_t side[kSide] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kSide] = {};
};

// Allocation through the context.
eh_status dev_alloc(Ctx* c, DevBuf& b, size_t bytes);
void dev_free(Ctx* c, DevBuf& b);
eh_status hip_check(Ctx* c, hipError_t e, const char* what);
eh_status ensure_acc(Ctx* c, size_t n);

// Device buffers of one call, freed (after the stream drains) when it returns.
struct Scratch {
  Ctx* c;
  std::vector<DevBuf*> bufs;
  explicit Scratch(Ctx* ctx) : c(ctx) {}
  eh_status get(DevBuf& b, size_t bytes) {
    bufs.push_back(&b);
    return dev_alloc(c, b, bytes);
  }
  ~Scratch() {
    (void)hipStreamSynchronize(c->stream);
    for (DevBuf* b : bufs) dev_free(c, *b);
  }
};
eh_status ensure_pinned(Ctx* c, size_t n);

// Work-item construction (host) and the plan cache.
eh_status get_plan(Ctx* c, Trie* t, uint32_t pattern, uint32_t staging, Plan** out);
// The cached plan for the context's current tuning, or null (never builds).
Plan* find_plan(Ctx* c, Trie* t, uint32_t pattern, uint32_t staging);
void make_items_source(const HostTrie& h, uint32_t u, uint32_t tag, uint32_t chunk_work,
                       uint32_t pattern, bool use_bitsets, std::vector<Item>& out);
// Same items cut from out-degrees alone: O(1 + items) per root.
void make_items_estimated(const HostTrie& h, uint32_t u, uint32_t tag, uint32_t chunk_work,
                          uint32_t pattern, std::vector<Item>& out);
// The number of items make_items_estimated makes for u.
uint64_t count_items_estimated(const HostTrie& h, uint32_t u, uint32_t chunk_work,
                               uint32_t pattern);

// Device launches (eh_kernels.hip).  All enqueue on `stream`.
struct LaunchArgs {
  const Item* items = nullptr;
  uint64_t n_items = 0;
  const uint32_t* idx = nullptr;       // streamed vertex list (source staging)
  const uint4* sdesc = nullptr;        // per item staged-set descriptor, or null
  const uint2* rec = nullptr;          // per in-edge segment record, or null
  const uint2* vdesc = nullptr;
  const uint32_t* col = nullptr;
  const uint4* bsdesc = nullptr;
  const uint32_t* bsw = nullptr;       // base of bsdesc positions (= col)
  unsigned long long* acc = nullptr;   // accumulators indexed by item tag
  uint32_t tag_base = 0;               // acc index = tag - tag_base
  unsigned long long* per_root = nullptr;  // optional, source staging only
  const uint32_t* vert = nullptr;
  uint32_t* cursor = nullptr;
  uint32_t use_bitsets = 0;
  uint32_t dynamic = 0;
  uint32_t algo = EH_ALGO_AUTO;
  float gamma = 32.0f;
  uint32_t group_lanes = 0;
  uint32_t dmax = 0;
  uint32_t item_dmax = 0;              // max d+(s) over the launch's items, 0: unknown (dmax)
  uint32_t deg_lo = 0;                 // 4-clique launches take items with
  uint32_t deg_hi = 0xFFFFFFFFu;       //   deg_lo < d+(s) <= deg_hi (set by the launcher)
  uint32_t stage_words = 0;            // 0: kernel maximum
  uint32_t xcds = 0;                   // L2 domains for the static schedule remap
  uint32_t unroll = 8;                 // staged triangle kernel: 4 or 8
  uint32_t grab = 8;                   // schedule 4: items per cursor fetch
  uint32_t search_below = 24;          // average segment length below which the walk searches
  const uint4* gsub = nullptr;         // grouped items' members, or null
  uint32_t symmetric = 0;              // both directions of every edge are stored
  uint32_t reverse = 0;                // items taken from the last to the first
  uint32_t* k4s = nullptr;             // 4-cliques: per-wave S lists in HBM for roots
  uint32_t k4s_stride = 0;             //   of out-degree > kK4ListMax, or null
  uint32_t k4s_waves = 0;
  const uint4* roots = nullptr;        // 4-cliques over induced neighbourhoods: root
  uint64_t n_roots = 0;                //   records (segment records in rec) and the
  uint32_t* root_cursors = nullptr;    //   classes' root cursors, kCursorWords apart
};
eh_status launch_fill_u64(Ctx* c, hipStream_t s, unsigned long long* p, uint64_t n,
                          unsigned long long v);
eh_status launch_triangles(Ctx* c, hipStream_t s, const LaunchArgs& a, uint32_t kernel,
                           uint32_t waves_per_cu);
eh_status launch_4cliques(Ctx* c, hipStream_t s, const LaunchArgs& a, uint32_t kernel,
                          uint32_t waves_per_cu);
// Lollipop COUNT over a symmetric trie's edge-once (kStageHalf) plan: adds
// sum over undirected edges {x, u} of |N(x) & N(u)| (|N(x)| + |N(u)|) to a.acc.
eh_status launch_lollipop(Ctx* c, hipStream_t s, const LaunchArgs& a, uint32_t waves_per_cu);
// dst[piece.y + k] = src[piece.x + k] for k < piece.z, for every piece.
eh_status launch_gather_items(Ctx* c, hipStream_t s, const Item* src, const uint4* pieces,
                              uint32_t n_pieces, Item* dst);
eh_status launch_scatter_roots(Ctx* c, hipStream_t s, const unsigned long long* by_rank,
                               const uint32_t* vert, unsigned long long* by_id, uint32_t n);
// The label sequence (vertices in the order they receive labels) of a
// traversal ordering (EH_ORDER_BFS, _HYBRID, _STRONG_RUNS) of one graph, from
// its m deduplicated edges (min << kb | max) and degrees, into seq (n words).
eh_status device_traversal_sequence(Ctx* c, const unsigned long long* edges, uint64_t m,
                                    uint32_t kb, uint32_t n, const uint32_t* deg, uint32_t order,
                                    uint32_t* seq);
// Frees every device buffer of a plan.
void free_plan(Ctx* c, Plan& p);
// Sorts a built plan's items (and per-item descriptors) by decreasing
// estimated cost, for the snake schedule.
eh_status device_plan_balance(Ctx* c, Trie& t, Plan& plan);
// The target-staging plan of a triangle count built on the GPU from the
// trie's device arrays (items, descriptors, grouped members, records), equal
// to the host planner's.
eh_status device_plan_target(Ctx* c, Trie& t, Plan& plan, uint32_t chunk, bool ub, uint32_t cap,
                             uint32_t group);
// out[0] += f * in[0]
eh_status launch_add_scaled(Ctx* c, hipStream_t s, const unsigned long long* in,
                            unsigned long long f, unsigned long long* out);
// out[0] += sum over ranks r of t_by_id[vert[r]] * |N(r)| (Lollipop COUNT).
eh_status launch_degree_weighted_sum(Ctx* c, hipStream_t s, const unsigned long long* t_by_id,
                                     const uint32_t* vert, const uint2* vdesc, uint32_t n,
                                     unsigned long long* out);
// Largest out-degree whose 4-clique S list the kernel holds in LDS; beyond it
// the lists live in HBM (Plan::k4s).
constexpr uint32_t kK4ListMax = 2048;
// 4-cliques over a root's induced out-neighbourhood (k_k4_local): roots of
// out-degree 3 .. kK4LocalMax, in classes by out-degree (-1: not such a root);
// the membership filter has kK4LocalWords words (half at out-degree <= 128).
constexpr uint32_t kK4LocalMax = 512;
constexpr uint32_t kK4LocalWords = 512;
constexpr uint32_t kK4LocalClasses = 4;
static_assert(Ctx::kSide + 1 >= int(kK4LocalClasses), "a side stream per further class");
constexpr int k4_local_class(uint32_t d) {
  if (d < 3 || d > kK4LocalMax) return -1;
  return d <= 64 ? 0 : d <= 128 ? 1 : d <= 256 ? 2 : 3;
}
// words of the bitmap window of class k
constexpr uint32_t k4_local_window(int k) { return k <= 1 ? kK4LocalWords / 2 : kK4LocalWords; }
// Counts the roots of the root records a.roots (segment records a.rec):
// n[0] of out-degree <= 64, then n[1] <= 128, n[2] <= 256 and n[3] <= 512
// (each in k4_local_class), into a.acc[0].
eh_status launch_4cliques_local(Ctx* c, hipStream_t s, const LaunchArgs& a,
                               const uint64_t n[kK4LocalClasses]);
// Counts the roots of the work items a.items[0 .. n_items) (whole roots of
// class k, any request slots as tags) into a.acc[tag - tag_base].
eh_status launch_4cliques_local_items(Ctx* c, hipStream_t s, const LaunchArgs& a, int k);
// The induced-neighbourhood 4-clique plan of a pruned single-graph trie,
// built on the GPU: plan.k4l (root records, by class and decreasing cost),
// plan.k4l_n and plan.rec (row records).
eh_status device_plan_k4_local(Ctx* c, Trie& tr, Plan& plan, bool ub);
// Sizes and allocates the HBM S lists of a 4-clique launch over `items` when
// a root's out-degree exceeds kK4ListMax (nothing otherwise): one list of
// the largest such out-degree per wave, at most 4 waves per compute unit.
eh_status prepare_k4_lists(Ctx* c, const HostTrie& h, const Item* items, uint64_t n_items,
                           DevBuf& buf, uint32_t& waves, uint32_t& stride);
// Sets c->noalloc_scratch to the current device's static scratch (looked up
// once per device).
eh_status noalloc_scratch_init(Ctx* c);

// Set store (section 4.3): per set, segments {first block, last block, first
// member in vals or first word in words, members | kHiBit for a bitset run}.
struct HostSets {
  uint32_t n_sets = 0;
  uint32_t block_log = 8;
  std::vector<uint32_t> seg_off;  // [n_sets + 1]
  std::vector<uint4> seg;
  std::vector<uint32_t> vals;
  std::vector<uint32_t> words;
  uint64_t n_members = 0;
  uint64_t n_bitset_segs = 0;
  uint64_t bitset_blocks = 0;
};
// The text eh_last_error(NULL) returns (calls made without a context).
void set_no_ctx_error(const std::string& e);
eh_status host_sets_build(uint32_t n_sets, const uint64_t* off, const uint32_t* members,
                          const eh_set_opts* opts, HostSets& h, std::string& err);

struct Sets {
  Ctx* ctx = nullptr;
  eh_sets_info info{};
  DevBuf seg_off, seg, vals, words;
};
// *total += sum over pairs of |A_p & B_p|; counts[p] = |A_p & B_p| when
// counts is not null; *bad |= 1 when a pair names a set >= n_sets and bad is
// not null.  lanes: 4, 16 or 64 per pair.
eh_status launch_intersect_pairs(Ctx* c, hipStream_t s, const Sets& st, uint64_t n_pairs,
                                 const uint32_t* pairs, uint32_t* counts, uint32_t lanes,
                                 unsigned long long* total, unsigned long long* bad);

}  // namespace eh

struct eh_ctx {
  eh::Ctx c;
};
struct eh_trie {
  eh::Trie t;
};
struct eh_host_trie {
  eh::HostTrie h;
};
struct eh_sets {
  eh::Sets s;
};
struct eh_host_sets {
  eh::HostSets h;
};
