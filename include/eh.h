/*
 * eh.h -- C ABI of the MI355X set-intersection engine for triangle and
 * 4-clique counting (EmptyHeaded, Aberger et al., SIGMOD 2016).
 *
 * The engine keeps a graph as a two-level trie (paper section 2.2 "Input
 * Data"): level one is the vertex set, level two the neighbour sets, stored
 * as degree-ordered CSR in HBM.  Each neighbour set has the uint layout
 * (sorted 32-bit ids) and, when the set optimizer of section 4.4 finds it
 * dense, an additional bitset layout (section 4.1, Figure 3) whose single
 * block spans the set's range.  Counting runs Generic-Join (section 2.1,
 * Algorithm 1) for the two patterns of Table 1 that are single-node plans,
 * Triangle and 4-Clique, with COUNT(*) aggregation, on data pruned to one
 * direction per undirected edge with degree-assigned ids (section 5.2).  The
 * work is the set intersections of section 4.2 (uint & uint by merge or
 * galloping, bitset & bitset by word AND, uint & bitset by probing), done by
 * hand-written gfx950 kernels.
 *
 * Conventions shared by every call:
 *   - Vertex ids are uint32 in [0, n).  Input pairs may repeat, appear in both
 *     directions and contain self-loops: loops are dropped and the rest is
 *     read as a simple undirected graph.  An id >= n is EH_EINVAL.
 *   - Counts are exact unsigned 64-bit integers.  A triangle is a 3-vertex
 *     subset with all three edges, a 4-clique a 4-vertex subset with all six.
 *   - rank(v) orders vertices by (degree ascending, id ascending); the root
 *     of a triangle or 4-clique is its vertex of smallest rank.
 *   - Pointers named d_* are device pointers on the context's device; all
 *     others are host pointers.  Input arrays are only read during the call.
 *   - Every call returns an eh_status.  No exception or abort crosses the
 *     ABI.  HIP failures return EH_EHIP with text in eh_last_error().  Host
 *     outputs are written only when the call returns EH_OK.
 *   - Blocking calls return after their result is on the host.  *_async
 *     calls only enqueue work on the context's stream.
 *   - A context is used by one host thread at a time; eh_submit, eh_poll,
 *     eh_wait and eh_server_drain are thread-safe.
 */
#ifndef EH_H_
#define EH_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t eh_status;
enum {
  EH_OK = 0,
  EH_PENDING = 1,     /* eh_poll: request not finished yet */
  EH_EINVAL = -1,     /* bad argument: null pointer, id >= n, bad pattern or range */
  EH_ENOMEM = -2,     /* allocation failed, or a request exceeds the memory budget */
  EH_EHIP = -3,       /* a HIP runtime call failed; see eh_last_error */
  EH_EBUSY = -4,      /* server queue full */
  EH_ENOTFOUND = -5,  /* unknown or already retired ticket */
  EH_EOVERFLOW = -6,  /* size beyond the 32-bit offsets of the trie */
  EH_ESTATE = -7      /* object in the wrong state (e.g. batch call on a single trie) */
};

enum { EH_TRIANGLE = 3, EH_4CLIQUE = 4 };

/* Set layouts (section 4.3 "Tradeoffs"): uint only at relation level, the
 * per-set optimizer (section 4.4), or every non-empty set as a bitset. */
enum { EH_LAYOUT_UINT = 0, EH_LAYOUT_HYBRID = 1, EH_LAYOUT_BITSET_ALL = 2 };

/* Device memory hooks.  alloc returns NULL on failure.  Both may be called
 * from the thread that calls into the context only. */
typedef struct eh_allocator {
  void* (*alloc)(void* self, size_t bytes, void* hip_stream);
  void (*free)(void* self, void* ptr, void* hip_stream);
  void* self;
} eh_allocator;

typedef struct eh_ctx eh_ctx;
typedef struct eh_trie eh_trie;
typedef struct eh_server eh_server;
typedef struct eh_host_trie eh_host_trie;

/* ---- context ------------------------------------------------------------ */

/* device: HIP device ordinal.  hip_stream: a hipStream_t to launch on, or
 * NULL for a stream the context creates.  alloc: NULL for hipMalloc/hipFree.
 * The allocator struct is copied; its `self` must outlive the context. */
eh_status eh_ctx_create(int device, void* hip_stream, const eh_allocator* alloc, eh_ctx** out);
eh_status eh_ctx_destroy(eh_ctx* ctx);
const char* eh_last_error(const eh_ctx* ctx);
const char* eh_status_str(eh_status s);
/* Version of this ABI (major * 10000 + minor * 100 + patch); a caller built
 * against this header checks that the library returns EH_ABI_VERSION. */
#define EH_ABI_VERSION 11000
int32_t eh_abi_version(void);

/* ---- tuning knobs (performance only; counts never depend on them) ------- */

enum { EH_KERNEL_AUTO = 0, EH_KERNEL_STAGED = 1, EH_KERNEL_PAIRWISE = 2 };
enum { EH_STAGE_AUTO = 0, EH_STAGE_SOURCE = 1, EH_STAGE_TARGET = 2 };
enum { EH_ALGO_AUTO = 0, EH_ALGO_MERGE = 1, EH_ALGO_SEARCH = 2 };

typedef struct eh_tuning {
  uint32_t kernel;       /* EH_KERNEL_*: staged (one set held in LDS) or pairwise */
  uint32_t staging;      /* staged kernel, triangle totals: which end of an edge is held;
                            target staging needs out-degrees below 2^16 (always so under
                            degree order) and tries beyond that stage sources.  On a
                            symmetric trie a total is counted over each undirected edge
                            once, at its higher-ranked end (|N(x) & N(u)| is the same for
                            the arcs (x,u) and (u,x)) and doubled, unless this is
                            EH_STAGE_SOURCE, which evaluates every arc */
  uint32_t algo;         /* pairwise uint & uint: EH_ALGO_AUTO applies the gamma rule */
  float gamma;           /* galloping when the longer list exceeds gamma x the shorter
                            (section 4.2 uses 32); <= 0 keeps the current value */
  uint32_t chunk_work;   /* target streamed elements per work item (0: keep) */
  uint32_t waves_per_cu; /* persistent waves per compute unit (0: keep) */
  uint32_t group_lanes;  /* pairwise: lanes per pair, 4..64 power of two; 0: by size bins */
  uint32_t use_bitsets;  /* 1: dense sets are read through their bitset layout */
  uint32_t dynamic;      /* schedule: 0 static interleave (item i to wave i mod waves),
                            1 waves take items from an atomic cursor (work stealing),
                            2 static blocks (each wave one contiguous range of items),
                            3 partitioned interleave (the items cut into xcds contiguous
                              ranges, each interleaved over the waves of one L2 domain),
                            4 partitioned cursors (one atomic cursor per range; waves
                              take `grab` items per fetch and move on to the next range
                              when theirs is used up) */
  uint32_t stage_words;  /* staged kernels: LDS words for a held set (bitset range / 32, or
                            list length), at most 1024; 0 means 1024.  At most 512
                            selects the half-size kernel instances (more waves per CU;
                            for triangles the unroll knob then does not apply) */
  uint32_t xcds;         /* L2 domains blocks are dealt to round-robin (8 on MI355X), at
                            most 32.  Schedules 0 and 2: each domain then takes a
                            contiguous slice of every window of items (0 or 1: no
                            remapping); schedules 3 and 4: the number of item ranges
                            (0: 8) */
  uint32_t unroll;       /* staged triangle kernel: streamed elements in flight per lane,
                            4 (more waves per CU) or 8; 0 means 8 */
  uint32_t grab;         /* schedule 4: consecutive items per cursor fetch, at most 4096;
                            0 means 8 */
  uint32_t search_below; /* staged kernels: when the streamed sets of a batch of 64 average
                            fewer elements than this, each element's set is found by a
                            binary search of the batch's length prefix instead of a walk
                            along it; at most 4096, 0 never searches */
  uint32_t group;        /* staged triangle kernel, target staging: up to this many small
                            consecutive work items of one graph share a wave (1, 2 or 4;
                            0 means 1) */
  uint32_t reverse;      /* 1: waves take the work items from the last to the first (every
                            schedule).  Items follow the held vertex's rank, and under degree
                            order the highest ranks hold the heaviest sets, so they start
                            first instead of forming the launch's tail */
  uint32_t k4_local;     /* 4-cliques on a pruned single-graph trie: 1 counts each root u with
                            3 <= d+(u) <= 512 over its induced out-neighbourhood (rows
                            N+(v) & N+(u) as bitsets over local ids in LDS, the third level
                            as word ANDs); the other roots, and every root when 0, go to the
                            staged S-list kernel.  A context starts with 1 */
} eh_tuning;

eh_status eh_ctx_set_tuning(eh_ctx* ctx, const eh_tuning* t);
eh_status eh_ctx_get_tuning(const eh_ctx* ctx, eh_tuning* out);

/* ---- tries -------------------------------------------------------------- */

/* Node orderings (section 2.2 dictionary encoding; appendix A, node
 * ordering).  An ordering is the sequence in which vertices receive their
 * 32-bit labels; the paper then keeps each undirected edge once, from the
 * larger label to the smaller.  The trie stores rank = n - 1 - label and
 * directs edges from lower to higher rank: the same edges, and the same gaps
 * inside every set.  Ties and traversal details:
 *   DEGREE       degree descending, ties id descending (rank = (degree asc,
 *                id asc)); out-degrees stay below sqrt(2m)
 *   REV_DEGREE   degree ascending, ties id ascending
 *   INPUT        the ids as given (label = id): a caller relabels first for
 *                Random, Shingle or any other external ordering
 *   BFS          breadth-first discovery order; each traversal starts at the
 *                unvisited vertex of highest degree (ties: lowest id), and a
 *                vertex's neighbours are discovered in ascending id order
 *   HYBRID       the BFS labels, then a stable sort by degree descending
 *   STRONG_RUNS  vertices visited by degree descending (ties id ascending);
 *                a visited vertex takes the next label if it has none, then
 *                its unlabelled neighbours take the next labels in ascending
 *                id order
 * Counts do not depend on the ordering; rooted counts (root = the vertex of
 * smallest rank), set layouts and the work do.  Only DEGREE bounds the
 * out-degree, and the 4-clique kernel accepts out-degrees up to 2048. */
enum {
  EH_ORDER_DEGREE = 0,
  EH_ORDER_REV_DEGREE = 1,
  EH_ORDER_INPUT = 2,
  EH_ORDER_BFS = 3,
  EH_ORDER_HYBRID = 4,
  EH_ORDER_STRONG_RUNS = 5
};

/* Set optimizer of section 4.4: a set S becomes a bitset iff |S| >= s_min and
 * (max(S) - min(S) + 1) / |S| <= tau.  The paper's rule is one AVX register
 * (256 bits) per value: tau = 256.  tau <= 0 selects 256; s_min 0 selects 1. */
typedef struct eh_build_opts {
  uint32_t layout;  /* EH_LAYOUT_* */
  float tau;
  uint32_t s_min;
  uint32_t order;   /* EH_ORDER_*; a value above 5 is EH_EINVAL */
  uint32_t symmetric; /* 0: prune (each edge once, low rank -> high rank, section 5.2);
                         1: keep the full undirected adjacency, both directions (the
                         unpruned relation of appendix A, "pruning symmetric queries",
                         on which the paper runs its Lollipop query, section 5.3).  On a
                         symmetric trie the counting calls return the join's output on
                         the unpruned relation: ordered triangles (6 T), ordered 4-cliques
                         (24 K), rooted counts by the first attribute x. */
} eh_build_opts;

typedef struct eh_trie_info {
  uint32_t n;               /* vertices (sum over graphs for a batch) */
  uint32_t n_graphs;        /* 1 for a single graph */
  uint64_t m_plus;          /* oriented edges = unique undirected edges */
  uint64_t n_bitset_sets;   /* sets that also carry the bitset layout */
  uint64_t bitset_words;    /* 32-bit words over all bitsets */
  uint64_t device_bytes;    /* HBM held by the trie */
  uint64_t b_merge;         /* sum over oriented edges (u,v) of 4 (d+(u) + d+(v)) */
  uint32_t max_out_degree;  /* max d+ */
  uint32_t reserved;
  uint64_t b_target;        /* what triangle counting with target staging must read
                               (pruned tries; 0 for a symmetric trie): for each vertex
                               v with a non-empty N+(v) and an in-edge, 4 |N+(v)| + 32
                               (the set, its work item and extent); for each in-edge
                               u -> v of such a v, 4 |N+(u) after v| + 8 (the part of
                               N+(u) above v, which is all that can meet N+(v), and its
                               record).  Summed over the graphs of a batch. */
} eh_trie_info;

/* Builds the trie of one graph on the host (clean, rank, orient, CSR, set
 * layouts; section 2.2 dictionary encoding, section 5.2 pruning) and uploads
 * it.  src/dst: n_edges raw pairs.  opts may be NULL (hybrid layout, tau 256,
 * s_min 1, degree order, pruned). */
eh_status eh_build_trie(eh_ctx* ctx, const uint32_t* src, const uint32_t* dst, uint64_t n_edges,
                        uint32_t n_vertices, const eh_build_opts* opts, eh_trie** out);

/* Many independent graphs in one trie.  Graph g has n_vertices[g] vertices
 * with local ids and the raw pairs src/dst[edge_off[g] .. edge_off[g+1]). */
eh_status eh_build_batch(eh_ctx* ctx, uint32_t n_graphs, const uint32_t* n_vertices,
                         const uint64_t* edge_off, const uint32_t* src, const uint32_t* dst,
                         const eh_build_opts* opts, eh_trie** out);

/* The trie of eh_build_trie, built on the GPU from raw pairs already in
 * device memory (section 2.2 dictionary encoding, section 5.2 pruning,
 * sections 4.1 and 4.4 layouts): the same arrays, pruned or symmetric, and
 * the same host copy (downloaded for work-item planning; the bitset words
 * stay in device memory only).  d_src/d_dst: device arrays of n_edges
 * uint32, read on the context's stream and not kept; the caller keeps them
 * valid until the call returns.  Every node ordering: the sorts (degree,
 * reverse degree, input) and the traversals (BFS, hybrid, strong runs), whose
 * label sequences are computed in parallel (strong runs by each vertex's
 * first visit among itself and its neighbours; BFS level by level over the
 * connected components, a level ordered by (label of the first-visiting
 * parent, id)), equal to the host's sequential ones.  An id >= n is
 * EH_EINVAL; a traversal ordering of 2^31 vertices or more EH_EOVERFLOW.  Scratch device
 * memory of about 16 bytes per raw pair (32 for a symmetric trie) and 40 per
 * vertex, plus the sorts' working space, is freed before it returns. */
eh_status eh_build_trie_device(eh_ctx* ctx, const uint32_t* d_src, const uint32_t* d_dst,
                               uint64_t n_edges, uint32_t n_vertices, const eh_build_opts* opts,
                               eh_trie** out);

/* The batch trie of eh_build_batch, built on the GPU (as
 * eh_build_trie_device): n_vertices and edge_off are host arrays as in
 * eh_build_batch; d_src/d_dst are device arrays of local ids, graph g's pairs
 * at [edge_off[g], edge_off[g+1]).  The orderings that are sorts (degree,
 * reverse degree, input); the traversal orderings are EH_EINVAL for a batch
 * (build it with eh_build_batch).  An id >= its graph's n_vertices is
 * EH_EINVAL. */
eh_status eh_build_batch_device(eh_ctx* ctx, uint32_t n_graphs, const uint32_t* n_vertices,
                                const uint64_t* edge_off, const uint32_t* d_src,
                                const uint32_t* d_dst, const eh_build_opts* opts, eh_trie** out);

eh_status eh_trie_info_get(const eh_trie* trie, eh_trie_info* out);
/* Inspection: the host copy of a built trie, in the layout of
 * eh_host_trie_arrays (rank[n], row[n+1], col[m_plus], bs_off[n],
 * bs_base[n], bs_nw[n], bs_words[bitset_words]; any pointer may be NULL;
 * the caller owns the buffers, sized from eh_trie_info).  A GPU-built trie's
 * words are copied from device memory (after its context's stream drains);
 * EH_EHIP if that copy fails. */
eh_status eh_trie_host_arrays(const eh_trie* trie, uint32_t* rank, uint32_t* row, uint32_t* col,
                              uint32_t* bs_off, uint32_t* bs_base, uint32_t* bs_nw,
                              uint32_t* bs_words);
/* Inspection: the device arrays the counting kernels read, copied to host
 * memory after the context's stream drains (any pointer may be NULL):
 * vdesc[2n] = {first member, out-degree | 2^31 if the set has a bitset} per
 * rank; col[m_plus + bitset_words] = every set's members, then every
 * bitset's words; bsdesc[4n] = {position of the first word in col, first id
 * covered, words, 0} per rank, only when n_bitset_sets > 0; vert[n] = the
 * original id of each rank. */
eh_status eh_trie_device_arrays(eh_ctx* ctx, const eh_trie* trie, uint32_t* vdesc, uint32_t* col,
                                uint32_t* bsdesc, uint32_t* vert);
/* Frees the trie's device memory.  Destroy every server using it first. */
eh_status eh_trie_free(eh_trie* trie);

/* ---- counting ----------------------------------------------------------- */

/* Work-item plans are made on the first count of each (pattern, staging,
 * tuning) and cached in the trie.  Target-staged triangle plans are built on
 * the GPU (transient device memory of about 40 bytes per stored edge); setting
 * EH_HOST_PLAN in the environment builds them on the host instead (the same
 * plans; for tests and comparisons). */

/* Triangle total of a single-graph trie.  d_per_root: NULL, or a device array
 * of n uint64 that receives, per original vertex id, the triangles rooted at
 * it (it is overwritten, not accumulated). */
eh_status eh_count_triangles(eh_ctx* ctx, const eh_trie* trie, uint64_t* total,
                             uint64_t* d_per_root);
/* 4-clique total of a single-graph trie (section 5.3, query K4 on pruned data). */
eh_status eh_count_4cliques(eh_ctx* ctx, const eh_trie* trie, uint64_t* total);
/* COUNT(*) of the Lollipop query of section 5.3,
 *   Lollipop(x,y,z,w) :- R(x,y), S(y,z), T(x,z), U(x,w),
 * evaluated as one Generic-Join over a symmetric trie (the paper runs it on
 * undirected data): for every x, the ordered triangles (x, y, z) times the
 * number of w adjacent to x, i.e. sum over x of t(x) deg(x).  Unless the
 * tuning asks for source staging it is counted over each undirected edge
 * {x, u} once, as |N(x) & N(u)| (deg(x) + deg(u)) summed in one launch of the
 * staged kernel (the edge-once plan of the symmetric triangle total); under
 * source staging t(x) is counted by first attribute over every arc and then
 * weighted, which allocates n uint64 of device scratch per call.  EH_ESTATE
 * on a pruned trie or a batch.  Results above 2^64 - 1 wrap. */
eh_status eh_count_lollipop(eh_ctx* ctx, const eh_trie* trie, uint64_t* total);
/* Enqueue-only forms: the total is written to d_total (one uint64, device)
 * when the stream reaches it.  pattern: EH_TRIANGLE or EH_4CLIQUE. */
eh_status eh_count_async(eh_ctx* ctx, const eh_trie* trie, int pattern, uint64_t* d_total);
/* As eh_count_async, but adds the count to *d_total instead of overwriting
 * it: k calls on a zeroed d_total leave k times the count.  With the static
 * schedules (0, 2, 3) a call is one counting launch; schedules 1 and 4 add
 * a cursor reset before it, and a 4-clique count whose roots include
 * out-degrees above 512 takes a second launch for those.  A total over a
 * symmetric trie (each undirected edge once, doubled) enqueues a fill of the
 * context's half-count word, the counting launch into it, and a kernel adding
 * twice that word to *d_total; the word is allocated with the context and
 * never moved, so a HIP graph captured from these calls stays valid for the
 * context's life. */
eh_status eh_count_add_async(eh_ctx* ctx, const eh_trie* trie, int pattern, uint64_t* d_total);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * eh_count_add_async, but the launches allocate nothing.  Their scratch -- the
 * work cursors of the cursor schedules and, on a symmetric trie, the
 * accumulator of the half count -- lives in a static device array of 16 KiB
 * that the library holds on each GPU until the process ends.  Every call on a
 * GPU shares that GPU's array (the cursors and the accumulator are cleared by
 * a fill kernel on the stream before each use), so calls that overlap on one
 * GPU (two contexts or streams in flight at once) race and must not be made.
 * The work-item plan of (pattern, tuning) must already be cached in the trie
 * by an earlier count with the same tuning (any eh_count_* call on this
 * trie): EH_ESTATE otherwise, as for a batch trie.  EH_EOVERFLOW if the
 * tuning's item partitions need more cursors than the scratch holds (never
 * with the limits of eh_ctx_set_tuning).  d_total: one uint64, device; the
 * count is added to it. */
eh_status eh_count_add_noalloc(eh_ctx* ctx, const eh_trie* trie, int pattern, uint64_t* d_total);

/* Instances whose root is in the set {roots[i]} (original ids; duplicates are
 * ignored): a selection on the first attribute of the join (appendix B.1). */
eh_status eh_count_rooted(eh_ctx* ctx, const eh_trie* trie, int pattern, const uint32_t* roots,
                          uint32_t n_roots, uint64_t* total);

/* Per-graph counts of graphs [first, first+count) of a batch trie, all in one
 * counting launch (see eh_count_add_async for the exceptions).  out_counts:
 * host array of count uint64. */
eh_status eh_count_batch(eh_ctx* ctx, const eh_trie* batch, int pattern, uint32_t first,
                         uint32_t count, uint64_t* out_counts);
/* Enqueue-only batch form; d_out: device array of count uint64. */
eh_status eh_count_batch_async(eh_ctx* ctx, const eh_trie* batch, int pattern, uint32_t first,
                               uint32_t count, uint64_t* d_out);

/* ---- measurement ---------------------------------------------------------- */

/* Streaming-read probe (not part of the method): enqueues one kernel that
 * reads every byte of d_buf once, with 128-bit loads over a grid-stride loop,
 * and XORs a fold of what it read into *d_sink (one uint64, device), so that
 * timing it (events on the context's stream) gives the read bandwidth a plain
 * read-only kernel reaches on this GPU, the practical ceiling beside the
 * nominal HBM peak for the counting kernels' byte models.  d_buf: device
 * memory of `bytes` bytes, 16-byte aligned, bytes a positive multiple of 16
 * (EH_EINVAL otherwise); only read.  blocks_per_cu: blocks of 256 lanes per
 * compute unit, 1..64 (0 means 8).  A buffer larger than the 256 MB
 * last-level cache measures HBM. */
eh_status eh_stream_read(eh_ctx* ctx, const void* d_buf, uint64_t bytes, uint32_t blocks_per_cu,
                         uint64_t* d_sink);

/* ---- serving ------------------------------------------------------------ */

/* A server keeps `resident` in HBM and answers rooted count requests.
 * Worker threads turn each submitted request into work items of 16 bytes
 * (its footprint).  The server owns an HBM arena of hbm_budget_bytes: a
 * progress thread admits expanded requests in arrival order while the next
 * one's items fit a free extent of the arena (first fit) and fewer than
 * max_active are active, uploads them into it, and advances all active
 * requests together in device steps of at most step_items work items, which
 * a gather kernel copies from the arena into the step's item list; a request
 * frees its extent when it completes.  Besides the arena the server holds
 * step_items * 16 bytes for the step's items, 8 bytes per active slot, its
 * work cursors and, for a trie with an out-degree above 2048, the 4-clique
 * S lists (4 per compute unit, each of the largest out-degree).  Zero fields
 * take the defaults in brackets. */
typedef struct eh_server_opts {
  uint64_t hbm_budget_bytes;  /* [2 GiB] size of the arena of admitted work items, at most
                                 64 GiB (EH_EINVAL beyond, or below 16 bytes) */
  uint32_t max_active;        /* [256] */
  uint32_t max_queued;        /* [4096] submitted, not yet admitted */
  uint32_t step_items;        /* [262144] */
  uint32_t policy;            /* which active requests' items fill a step first:
                                 EH_SERVE_FIFO [default] oldest first, or
                                 EH_SERVE_SHORTEST fewest items left first */
} eh_server_opts;

enum { EH_SERVE_FIFO = 0, EH_SERVE_SHORTEST = 1 };

typedef struct eh_req_stats {
  uint64_t t_submit_ns;   /* CLOCK_MONOTONIC times */
  uint64_t t_admit_ns;
  uint64_t t_done_ns;
  uint64_t items;         /* work items the request was split into */
} eh_req_stats;

/* The server uses ctx's device and allocator, a copy of ctx's tuning taken
 * here, and its own stream and work cursors; do not use ctx from another
 * thread while the server lives. */
eh_status eh_server_create(eh_ctx* ctx, const eh_trie* resident, const eh_server_opts* opts,
                           eh_server** out);
/* Copies roots; returns a ticket.  EH_EBUSY when max_queued are waiting,
 * EH_ENOMEM when the request's items alone exceed the arena.  When the budget holds
 * the request with every vertex a root, the roots are only checked and copied
 * here and expanded by a worker; otherwise this call expands them itself so
 * that it can refuse the request. */
eh_status eh_submit(eh_server* srv, int pattern, const uint32_t* roots, uint32_t n_roots,
                    uint64_t* ticket);
/* EH_OK with *count (and stats) once done; the ticket is then retired.
 * EH_PENDING while queued or running; EH_ENOTFOUND for unknown tickets. */
eh_status eh_poll(eh_server* srv, uint64_t ticket, uint64_t* count, eh_req_stats* stats);
/* Blocks until the ticket is done (or timeout_ms passes: EH_PENDING). */
eh_status eh_wait(eh_server* srv, uint64_t ticket, uint32_t timeout_ms, uint64_t* count,
                  eh_req_stats* stats);
/* Completion queue: waits up to timeout_ms until at least one request has
 * finished, then retires up to cap finished requests in completion order,
 * writing tickets[i], counts[i] and (if stats is not NULL) stats[i] for
 * i < *n_out.  *n_out = 0 on timeout.  Requests already retired by eh_poll or
 * eh_wait are skipped. */
eh_status eh_server_drain(eh_server* srv, uint32_t cap, uint32_t timeout_ms, uint64_t* tickets,
                          uint64_t* counts, eh_req_stats* stats, uint32_t* n_out);
/* Finishes admitted work, cancels queued requests, joins the thread. */
eh_status eh_server_destroy(eh_server* srv);

/* ---- set stores and pairwise intersection (section 4.3, "Tradeoffs") ----
 *
 * A set store holds many sorted sets of uint32 ids in one of the layouts the
 * paper compares at its three granularities.  The id domain is cut into
 * fixed blocks of 2^block_log ids (the paper's default block is 256 ids, one
 * AVX register).  Each set is stored as a sequence of segments, ascending and
 * disjoint in blocks; a segment is either a uint run (sorted members, 4 bytes
 * each) or a bitset run (2^block_log / 32 words per block for consecutive
 * blocks).  Adjacent blocks of the same kind share one segment, which stores
 * the same members and words as one header per block would.
 *   EH_SETS_UINT       relation level, uint: one uint run per set;
 *   EH_SETS_SET        set level (section 4.4): one bitset run over every block
 *                      from the set's first to its last if the set is dense by
 *                      the rule of eh_build_opts (|S| >= s_min and
 *                      (max - min + 1) / |S| <= tau), else one uint run;
 *   EH_SETS_BITSET     relation level, bitset (section 4.1, Figure 3): every
 *                      non-empty block as a bitset block, empty blocks omitted;
 *   EH_SETS_COMPOSITE  block level ("composite set"): a block holding at least
 *                      block_min members is a bitset block, the members of the
 *                      other blocks form uint runs.
 * Intersections (section 4.2) walk the two segment lists in block order and,
 * for each overlap, AND words (bitset & bitset), probe words with members
 * (uint & bitset), or merge members, searching the longer run instead when
 * it is more than 32 times the shorter (uint & uint). */
enum { EH_SETS_UINT = 0, EH_SETS_SET = 1, EH_SETS_BITSET = 2, EH_SETS_COMPOSITE = 3 };

typedef struct eh_set_opts {
  uint32_t layout;     /* EH_SETS_*; a value above 3 is EH_EINVAL */
  uint32_t block_log;  /* log2 of the block size in ids, 5..16; 0 selects 8 (256 ids) */
  uint32_t block_min;  /* composite: members that make a block dense; 0 selects
                          2^block_log / 32, the count at which a block's members
                          take as many bytes as its bitset */
  float tau;           /* set level: as eh_build_opts.tau; <= 0 selects 32 */
  uint32_t s_min;      /* set level: as eh_build_opts.s_min; 0 selects 1 */
} eh_set_opts;

typedef struct eh_sets_info {
  uint32_t n_sets;
  uint32_t block_log;
  uint64_t n_members;       /* members over all sets */
  uint64_t n_segments;      /* segments over all sets */
  uint64_t n_bitset_segments;
  uint64_t uint_members;    /* members stored in uint runs */
  uint64_t bitset_blocks;   /* blocks stored as bitsets (empty ones included at set level) */
  uint64_t bitset_words;    /* 32-bit words over all bitset runs */
  uint64_t device_bytes;    /* HBM held by the store (0 for a host store) */
} eh_sets_info;

typedef struct eh_sets eh_sets;
typedef struct eh_host_sets eh_host_sets;

/* Encodes n_sets sets on the host and uploads them.  Set i is
 * members[off[i] .. off[i+1]), strictly ascending (EH_EINVAL otherwise);
 * off has n_sets + 1 entries with off[0] = 0; both arrays are only read
 * during the call.  opts may be NULL (composite, 256-id blocks).  The store
 * owns its device memory (through the context's allocator) until
 * eh_sets_free, and is used with the context that built it only (another
 * context gets EH_EINVAL).  EH_EOVERFLOW when members, words or segments
 * exceed 2^31 - 1; EH_ENOMEM when an allocation fails (nothing is kept). */
eh_status eh_sets_build(eh_ctx* ctx, uint32_t n_sets, const uint64_t* off, const uint32_t* members,
                        const eh_set_opts* opts, eh_sets** out);
eh_status eh_sets_info_get(const eh_sets* sets, eh_sets_info* out);
eh_status eh_sets_free(eh_sets* sets);

/* |A_p & B_p| for the pairs d_pairs[2p], d_pairs[2p+1] (set indices, device
 * array of 2 n_pairs uint32), p < n_pairs < 2^32.  d_counts: NULL, or a
 * device array of n_pairs uint32 that receives each pair's count.  *total:
 * the sum over all pairs.  lanes: lanes per pair, 4, 16 or 64; 0 picks by
 * the store's mean set size.  A pair naming a set >= n_sets counts 0 and
 * makes the call return EH_EINVAL (after the launch has finished). */
eh_status eh_intersect_pairs(eh_ctx* ctx, const eh_sets* sets, uint64_t n_pairs,
                             const uint32_t* d_pairs, uint32_t* d_counts, uint32_t lanes,
                             uint64_t* total);
/* Enqueue-only form: adds the sum to *d_total (one uint64, device).  Pairs
 * naming a set >= n_sets count 0 and are not reported. */
eh_status eh_intersect_pairs_async(eh_ctx* ctx, const eh_sets* sets, uint64_t n_pairs,
                                   const uint32_t* d_pairs, uint32_t* d_counts, uint32_t lanes,
                                   uint64_t* d_total);

/* The host half of eh_sets_build, for checks without a GPU. */
eh_status eh_host_sets_build(uint32_t n_sets, const uint64_t* off, const uint32_t* members,
                             const eh_set_opts* opts, eh_host_sets** out);
eh_status eh_host_sets_info(const eh_host_sets* h, eh_sets_info* out);
/* Copies out (any pointer may be NULL): seg_off[n_sets + 1] (set i owns
 * segments [seg_off[i], seg_off[i+1])); seg[4 n_segments] = per segment
 * {first block, last block, first member in vals or first word in words,
 * members | 2^31 for a bitset run}; vals[uint_members]; words[bitset_words],
 * bit (x mod 32) of word (x / 32 - first block * 2^block_log / 32) of a run
 * holding id x. */
eh_status eh_host_sets_arrays(const eh_host_sets* h, uint32_t* seg_off, uint32_t* seg,
                              uint32_t* vals, uint32_t* words);
eh_status eh_host_sets_free(eh_host_sets* h);

/* ---- host-side trie (no device needed) ----------------------------------- */

/* The host half of eh_build_trie, exposed so the build can be checked
 * without a GPU.  Arrays are owned by the handle. */
eh_status eh_host_trie_build(const uint32_t* src, const uint32_t* dst, uint64_t n_edges,
                             uint32_t n_vertices, const eh_build_opts* opts, eh_host_trie** out);
/* Sizes: n, m_plus, n_bitset_sets, bitset_words, b_merge, max_out_degree. */
eh_status eh_host_trie_info(const eh_host_trie* h, eh_trie_info* out);
/* Copies out (any pointer may be NULL): rank[n] (rank of each id),
 * row[n+1] and col[m_plus] (oriented CSR in rank space),
 * bs_off[n] (word offset of each rank's bitset, 0xFFFFFFFF if none),
 * bs_base[n] (first id covered, a multiple of 32), bs_nw[n] (words),
 * bs_words[bitset_words]. */
eh_status eh_host_trie_arrays(const eh_host_trie* h, uint32_t* rank, uint32_t* row, uint32_t* col,
                              uint32_t* bs_off, uint32_t* bs_base, uint32_t* bs_nw,
                              uint32_t* bs_words);
eh_status eh_host_trie_free(eh_host_trie* h);

#ifdef __cplusplus
}
#endif
#endif /* EH_H_ */
