/*
 * eh_oracle.c -- plain CPU oracle for triangle and 4-clique counting.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call this code:
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load it.  It shares no source with the GPU library.
 *
 * What it computes (all exact, uint64):
 *   Input: n and raw pairs (src[i], dst[i]).  Pairs with src == dst are
 *   dropped, every other pair is read as the undirected edge {src, dst}, and
 *   duplicates collapse, giving a simple undirected graph G = (V, E).
 *   T = number of 3-vertex subsets of V with all three edges in E.
 *   K = number of 4-vertex subsets of V with all six edges in E.
 *   Rooted counts: the root of an instance is its vertex of smallest rank,
 *   where rank orders vertices by (degree in G ascending, id ascending), or
 *   is any permutation given by orc_graph_rerank (a node ordering).
 *
 * How (paper section 2.1, Algorithm 1 "Generic-Join", instantiated for the
 * triangle in section 3.3 "GHD Translation"; pruned input as in section 5.2):
 * each undirected edge is kept once, directed from lower to higher rank
 * (symmetric pruning with degree-assigned ids).  With the attribute order
 * x < y < z (< w) and N+(x) the sorted higher-ranked neighbours of x,
 *   T = sum_x sum_{y in N+(x)} |N+(x) & N+(y)|
 *   K = sum_x sum_{y in N+(x)} sum_{z in S} |S & N+(z)|,  S = N+(x) & N+(y)
 * Every intersection is a two-pointer merge of sorted arrays.
 *
 * Independent cross-checks, with no orientation at all:
 *   sum over {a,b} in E of |N(a) & N(b)|            = 3 T
 *   sum over {a,b} in E of edges(N(a) & N(b))       = 6 K
 *   Generic-Join over the symmetric (unpruned) relation counts ordered
 *   tuples: 3! T and 4! K (appendix A.1.2, pruning symmetric queries).
 *
 * Pairwise set intersection (section 4.2): |A & B| for given pairs of
 * sorted sets, by the same two-pointer merge; the layouts of section 4.3
 * change how a set is stored, never this count.
 *
 * Byte models.  What a list-merge implementation reads (section 4.2: both
 * sets of every intersection read once):
 *   B_merge = sum over oriented edges (x,y) of 4 (|N+(x)| + |N+(y)|)
 *   B_K4    = B_merge + sum over triangles x<y<z of 4 (|S_xy| + |N+(z)|)
 * What an implementation that holds one set of each intersection on chip
 * must read (a model of that design, not of the paper; sizes in bytes):
 *   B_target (triangles, the held set is N+(y) of the middle attribute): for
 *     every y with a non-empty N+(y) and at least one in-edge, N+(y) once
 *     (4 per member) plus 32 for its work descriptor; for every in-edge
 *     x -> y of such a y, the part of N+(x) above y (4 per member: every
 *     member of N+(y) is above y, so nothing below can match) plus an
 *     8-byte descriptor of that part.
 *   B_K4_held (4-cliques, N+(x) held, S_xy kept on chip): the pair (x,y) is
 *     extended only when N+(x) after y and N+(y) both hold two or more
 *     members (a 4-clique needs two more vertices in each); per extended
 *     pair 4 (the id y) + 8 (its set's extent) + 4 |N+(y)|; when |S_xy| >= 2,
 *     per z in S_xy 8 + 4 |N+(z)|; per x with an extended pair 16 + 4 |N+(x)|.
 *     Its element tests are the streamed members: |N+(y)| per extended pair
 *     and |N+(z)| per such z (orc_4cliques_range returns bytes and tests).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct orc_graph {
  uint32_t n;
  uint64_t m;          /* unique undirected edges */
  uint32_t* ea;        /* edge endpoints, ea[i] < eb[i], sorted lexicographically */
  uint32_t* eb;
  uint32_t* deg;       /* degree in G, by original id */
  uint32_t* rank;      /* rank[id] */
  uint32_t* vert;      /* vert[rank] = id */
  uint64_t* off;       /* oriented CSR in rank space: off[n+1] */
  uint32_t* nbr;       /* nbr[m]: higher-ranked neighbours, sorted */
  uint64_t* soff;      /* symmetric CSR by original id (built on demand) */
  uint32_t* snbr;
} orc_graph;

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}
static int cmp_u32(const void* a, const void* b) {
  uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}


void orc_graph_free(orc_graph* g) {
  if (!g) return;
  free(g->ea); free(g->eb); free(g->deg); free(g->rank); free(g->vert);
  free(g->off); free(g->nbr); free(g->soff); free(g->snbr);
  free(g);
}

/* 6: oriented adjacency, lower rank -> higher rank, rows sorted */
static int orient(orc_graph* g) {
  uint32_t n = g->n;
  uint64_t m = g->m;
  memset(g->off, 0, ((size_t)n + 1) * sizeof(uint64_t));
  for (uint64_t i = 0; i < m; ++i) {
    uint32_t ra = g->rank[g->ea[i]], rb = g->rank[g->eb[i]];
    g->off[(ra < rb ? ra : rb) + 1]++;
  }
  for (uint32_t r = 0; r < n; ++r) g->off[r + 1] += g->off[r];
  uint64_t* fill = (uint64_t*)malloc(((size_t)n + 1) * sizeof(uint64_t));
  if (!fill) return 1;
  memcpy(fill, g->off, ((size_t)n + 1) * sizeof(uint64_t));
  for (uint64_t i = 0; i < m; ++i) {
    uint32_t ra = g->rank[g->ea[i]], rb = g->rank[g->eb[i]];
    uint32_t lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
    g->nbr[fill[lo]++] = hi;
  }
  free(fill);
  for (uint32_t r = 0; r < n; ++r)
    qsort(g->nbr + g->off[r], g->off[r + 1] - g->off[r], sizeof(uint32_t), cmp_u32);
  return 0;
}

/* err: 0 ok, 1 id out of range, 2 out of memory */
orc_graph* orc_graph_new(uint32_t n, uint64_t m_raw, const uint32_t* src,
                         const uint32_t* dst, int* err) {
  *err = 0;
  for (uint64_t i = 0; i < m_raw; ++i)
    if (src[i] >= n || dst[i] >= n) { *err = 1; return NULL; }
  orc_graph* g = (orc_graph*)calloc(1, sizeof(orc_graph));
  if (!g) { *err = 2; return NULL; }
  g->n = n;
  /* 1-3: drop loops, canonical {min,max}, sort, unique */
  uint64_t* key = (uint64_t*)malloc((m_raw ? m_raw : 1) * sizeof(uint64_t));
  if (!key) { *err = 2; orc_graph_free(g); return NULL; }
  uint64_t k = 0;
  for (uint64_t i = 0; i < m_raw; ++i) {
    uint32_t a = src[i], b = dst[i];
    if (a == b) continue;
    uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
    key[k++] = ((uint64_t)lo << 32) | hi;
  }
  qsort(key, k, sizeof(uint64_t), cmp_u64);
  uint64_t m = 0;
  for (uint64_t i = 0; i < k; ++i)
    if (m == 0 || key[i] != key[m - 1]) key[m++] = key[i];
  g->m = m;
  g->ea = (uint32_t*)malloc((m ? m : 1) * sizeof(uint32_t));
  g->eb = (uint32_t*)malloc((m ? m : 1) * sizeof(uint32_t));
  g->deg = (uint32_t*)calloc(n ? n : 1, sizeof(uint32_t));
  g->rank = (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t));
  g->vert = (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t));
  g->off = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
  g->nbr = (uint32_t*)malloc((m ? m : 1) * sizeof(uint32_t));
  if (!g->ea || !g->eb || !g->deg || !g->rank || !g->vert || !g->off || !g->nbr) {
    free(key); *err = 2; orc_graph_free(g); return NULL;
  }
  for (uint64_t i = 0; i < m; ++i) {
    g->ea[i] = (uint32_t)(key[i] >> 32);
    g->eb[i] = (uint32_t)(key[i] & 0xffffffffu);
  }
  free(key);
  /* 4: degree in G */
  for (uint64_t i = 0; i < m; ++i) { g->deg[g->ea[i]]++; g->deg[g->eb[i]]++; }
  /* 5: rank by (degree asc, id asc): sort the keys degree * 2^32 + id */
  uint64_t* dk = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
  if (!dk) { *err = 2; orc_graph_free(g); return NULL; }
  for (uint32_t v = 0; v < n; ++v) dk[v] = ((uint64_t)g->deg[v] << 32) | v;
  qsort(dk, n, sizeof(uint64_t), cmp_u64);
  for (uint32_t r = 0; r < n; ++r) g->vert[r] = (uint32_t)(dk[r] & 0xffffffffu);
  free(dk);
  for (uint32_t r = 0; r < n; ++r) g->rank[g->vert[r]] = r;
  if (orient(g)) { *err = 2; orc_graph_free(g); return NULL; }
  return g;
}

/*
 * Replaces the ranking by rank[id] (any permutation of 0..n-1: the node
 * orderings of appendix A, "node ordering") and rebuilds the oriented
 * adjacency.  Counts are the same under every ranking; rooted counts follow
 * the new ranks.  Returns 0 ok, 1 not a permutation, 2 out of memory.
 */
int orc_graph_rerank(orc_graph* g, const uint32_t* rank) {
  uint32_t n = g->n;
  unsigned char* seen = (unsigned char*)calloc(n ? n : 1, 1);
  if (!seen) return 2;
  for (uint32_t v = 0; v < n; ++v) {
    if (rank[v] >= n || seen[rank[v]]) { free(seen); return 1; }
    seen[rank[v]] = 1;
  }
  free(seen);
  for (uint32_t v = 0; v < n; ++v) g->vert[rank[v]] = v;
  memcpy(g->rank, rank, (size_t)n * sizeof(uint32_t));
  return orient(g) ? 2 : 0;
}

uint64_t orc_num_edges(const orc_graph* g) { return g->m; }
uint32_t orc_num_vertices(const orc_graph* g) { return g->n; }

void orc_get_edges(const orc_graph* g, uint32_t* a, uint32_t* b) {
  memcpy(a, g->ea, g->m * sizeof(uint32_t));
  memcpy(b, g->eb, g->m * sizeof(uint32_t));
}
void orc_get_rank(const orc_graph* g, uint32_t* rank) { memcpy(rank, g->rank, g->n * sizeof(uint32_t)); }
void orc_get_degree(const orc_graph* g, uint32_t* deg) { memcpy(deg, g->deg, g->n * sizeof(uint32_t)); }
void orc_get_oriented(const orc_graph* g, uint64_t* off, uint32_t* nbr) {
  memcpy(off, g->off, ((size_t)g->n + 1) * sizeof(uint64_t));
  memcpy(nbr, g->nbr, g->m * sizeof(uint32_t));
}

/* |A & B| for sorted arrays, two-pointer merge */
static uint64_t merge_count(const uint32_t* a, uint64_t na, const uint32_t* b, uint64_t nb) {
  uint64_t i = 0, j = 0, c = 0;
  while (i < na && j < nb) {
    if (a[i] < b[j]) ++i;
    else if (a[i] > b[j]) ++j;
    else { ++c; ++i; ++j; }
  }
  return c;
}

/* A & B written to out (sorted), returns its size */
static uint64_t merge_list(const uint32_t* a, uint64_t na, const uint32_t* b, uint64_t nb,
                           uint32_t* out) {
  uint64_t i = 0, j = 0, c = 0;
  while (i < na && j < nb) {
    if (a[i] < b[j]) ++i;
    else if (a[i] > b[j]) ++j;
    else { out[c++] = a[i]; ++i; ++j; }
  }
  return c;
}

static void add_u64(uint64_t* p, uint64_t v) { __atomic_fetch_add(p, v, __ATOMIC_RELAXED); }

static void set_threads(int threads) {
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#else
  (void)threads;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/*
 * Triangles over outer vertices (ranks) x in [x_begin, x_end).
 *   root_by_id[id]: triangles whose smallest-rank vertex is id (optional)
 *   c3_by_id[id]:   triangles containing id (optional)
 *   bytes:          B_merge over the visited edges (optional)
 *   edges:          oriented edges visited (optional)
 */
uint64_t orc_triangles_range(const orc_graph* g, uint32_t x_begin, uint32_t x_end, int threads,
                             uint64_t* root_by_id, uint64_t* c3_by_id, uint64_t* bytes,
                             uint64_t* edges) {
  set_threads(threads);
  uint64_t total = 0, b = 0, e = 0;
  if (x_end > g->n) x_end = g->n;
  const int64_t xb = x_begin, xe = x_end;
  const int need_list = c3_by_id != NULL;
#pragma omp parallel reduction(+ : total, b, e)
  {
    uint32_t* tmp = NULL;
    if (need_list) {
      uint64_t dmax = 0;
      for (uint32_t r = 0; r < g->n; ++r)
        if (g->off[r + 1] - g->off[r] > dmax) dmax = g->off[r + 1] - g->off[r];
      tmp = (uint32_t*)malloc((dmax ? dmax : 1) * sizeof(uint32_t));
    }
#pragma omp for schedule(dynamic, 64)
    for (int64_t x = xb; x < xe; ++x) {
      const uint32_t* nx = g->nbr + g->off[x];
      const uint64_t dx = g->off[x + 1] - g->off[x];
      uint64_t tx = 0;
      for (uint64_t i = 0; i < dx; ++i) {
        const uint32_t y = nx[i];
        const uint32_t* ny = g->nbr + g->off[y];
        const uint64_t dy = g->off[y + 1] - g->off[y];
        uint64_t c;
        if (need_list) {
          c = merge_list(nx, dx, ny, dy, tmp);
          for (uint64_t t = 0; t < c; ++t) add_u64(&c3_by_id[g->vert[tmp[t]]], 1);
          if (c) add_u64(&c3_by_id[g->vert[y]], c);
        } else {
          c = merge_count(nx, dx, ny, dy);
        }
        tx += c;
        b += 4 * (dx + dy);
      }
      e += dx;
      total += tx;
      if (root_by_id) root_by_id[g->vert[x]] += tx;
      if (c3_by_id && tx) add_u64(&c3_by_id[g->vert[x]], tx);
    }
    free(tmp);
  }
  if (bytes) *bytes = b;
  if (edges) *edges = e;
  return total;
}

uint64_t orc_triangles(const orc_graph* g, int threads, uint64_t* root_by_id, uint64_t* c3_by_id,
                       uint64_t* bytes) {
  return orc_triangles_range(g, 0, g->n, threads, root_by_id, c3_by_id, bytes, NULL);
}

/* 4-cliques over outer vertices x in [x_begin, x_end); same optional outputs */
uint64_t orc_4cliques_range(const orc_graph* g, uint32_t x_begin, uint32_t x_end, int threads,
                            uint64_t* root_by_id, uint64_t* c4_by_id, uint64_t* bytes,
                            uint64_t* edges, uint64_t* held) {
  set_threads(threads);
  uint64_t total = 0, b = 0, e = 0, hb = 0, ht = 0;
  if (x_end > g->n) x_end = g->n;
  const int64_t xb = x_begin, xe = x_end;
  uint64_t dmax = 0;
  for (uint32_t r = 0; r < g->n; ++r)
    if (g->off[r + 1] - g->off[r] > dmax) dmax = g->off[r + 1] - g->off[r];
#pragma omp parallel reduction(+ : total, b, e, hb, ht)
  {
    uint32_t* s = (uint32_t*)malloc((dmax ? dmax : 1) * sizeof(uint32_t));
    uint32_t* t = (uint32_t*)malloc((dmax ? dmax : 1) * sizeof(uint32_t));
#pragma omp for schedule(dynamic, 16)
    for (int64_t x = xb; x < xe; ++x) {
      const uint32_t* nx = g->nbr + g->off[x];
      const uint64_t dx = g->off[x + 1] - g->off[x];
      uint64_t kx = 0;
      int extended = 0;
      for (uint64_t i = 0; i < dx; ++i) {
        const uint32_t y = nx[i];
        const uint32_t* ny = g->nbr + g->off[y];
        const uint64_t dy = g->off[y + 1] - g->off[y];
        const uint64_t ns = merge_list(nx, dx, ny, dy, s);   /* S = N+(x) & N+(y) */
        b += 4 * (dx + dy);
        const int ext = dx - i - 1 >= 2 && dy >= 2;
        if (ext) {
          extended = 1;
          hb += 4 + 8 + 4 * dy;
          ht += dy;
        }
        uint64_t kxy = 0;
        for (uint64_t j = 0; j < ns; ++j) {
          const uint32_t z = s[j];
          const uint32_t* nz = g->nbr + g->off[z];
          const uint64_t dz = g->off[z + 1] - g->off[z];
          b += 4 * (ns + dz);
          if (ext && ns >= 2) {
            hb += 8 + 4 * dz;
            ht += dz;
          }
          if (c4_by_id) {
            const uint64_t c = merge_list(s, ns, nz, dz, t);   /* w in S & N+(z) */
            for (uint64_t q = 0; q < c; ++q) add_u64(&c4_by_id[g->vert[t[q]]], 1);
            if (c) {
              add_u64(&c4_by_id[g->vert[z]], c);
              add_u64(&c4_by_id[g->vert[y]], c);
              add_u64(&c4_by_id[g->vert[x]], c);
            }
            kxy += c;
          } else {
            kxy += merge_count(s, ns, nz, dz);
          }
        }
        kx += kxy;
      }
      if (extended) hb += 16 + 4 * dx;
      e += dx;
      total += kx;
      if (root_by_id) root_by_id[g->vert[x]] += kx;
    }
    free(s);
    free(t);
  }
  if (bytes) *bytes = b;
  if (edges) *edges = e;
  if (held) {
    held[0] = hb;
    held[1] = ht;
  }
  return total;
}

uint64_t orc_4cliques(const orc_graph* g, int threads, uint64_t* root_by_id, uint64_t* c4_by_id,
                      uint64_t* bytes) {
  return orc_4cliques_range(g, 0, g->n, threads, root_by_id, c4_by_id, bytes, NULL, NULL);
}

/*
 * 4-cliques rooted at given vertices: for each distinct original id r in
 * ids[0 .. n_ids), root_by_id[r] = the 4-cliques whose vertex of smallest
 * rank is r, by the same loop nest as orc_4cliques_range with x = rank(r).
 * Entries of ids not listed are left untouched.  Returns the sum over the
 * distinct ids, UINT64_MAX if an id is out of range or memory ran out.
 */
uint64_t orc_4cliques_rooted_at(const orc_graph* g, const uint32_t* ids, uint64_t n_ids,
                                int threads, uint64_t* root_by_id) {
  set_threads(threads);
  for (uint64_t k = 0; k < n_ids; ++k)
    if (ids[k] >= g->n) return UINT64_MAX;
  unsigned char* seen = (unsigned char*)calloc(g->n ? g->n : 1, 1);
  uint32_t* xs = (uint32_t*)malloc((n_ids ? n_ids : 1) * sizeof(uint32_t));
  if (!seen || !xs) {
    free(seen);
    free(xs);
    return UINT64_MAX;
  }
  int64_t nx_roots = 0;
  for (uint64_t k = 0; k < n_ids; ++k)
    if (!seen[ids[k]]) {
      seen[ids[k]] = 1;
      xs[nx_roots++] = g->rank[ids[k]];
    }
  free(seen);
  uint64_t dmax = 0;
  for (uint32_t r = 0; r < g->n; ++r)
    if (g->off[r + 1] - g->off[r] > dmax) dmax = g->off[r + 1] - g->off[r];
  uint64_t total = 0;
  int oom = 0;
#pragma omp parallel reduction(+ : total)
  {
    uint32_t* s = (uint32_t*)malloc((dmax ? dmax : 1) * sizeof(uint32_t));
    if (!s) {
#pragma omp atomic write
      oom = 1;
    }
#pragma omp for schedule(dynamic, 4)
    for (int64_t k = 0; k < nx_roots; ++k) {
      if (!s) continue;
      const uint32_t x = xs[k];
      const uint32_t* nx = g->nbr + g->off[x];
      const uint64_t dx = g->off[x + 1] - g->off[x];
      uint64_t kx = 0;
      for (uint64_t i = 0; i < dx; ++i) {
        const uint32_t y = nx[i];
        const uint64_t ns = merge_list(nx, dx, g->nbr + g->off[y], g->off[y + 1] - g->off[y], s);
        for (uint64_t j = 0; j < ns; ++j) {
          const uint32_t z = s[j];
          kx += merge_count(s, ns, g->nbr + g->off[z], g->off[z + 1] - g->off[z]);
        }
      }
      root_by_id[g->vert[x]] = kx;
      total += kx;
    }
    free(s);
  }
  free(xs);
  return oom ? UINT64_MAX : total;
}

/*
 * The reads of B_target (see the header): the triangle sum taken with the
 * middle attribute y outermost, N+(y) held, and for each in-edge x -> y only
 * N+(x) after y streamed.  out[0] = held sets, out[1] = their members,
 * out[2] = streamed parts (in-edges of held sets), out[3] = streamed members.
 * Returns B_target = 32 out[0] + 4 out[1] + 8 out[2] + 4 out[3].
 */
uint64_t orc_target_reads(const orc_graph* g, uint64_t* out) {
  const uint32_t n = g->n;
  unsigned char* has_in = (unsigned char*)calloc(n ? n : 1, 1);
  if (!has_in) return UINT64_MAX;
  uint64_t parts = 0, streamed = 0;
  for (uint32_t x = 0; x < n; ++x) {
    const uint64_t dx = g->off[x + 1] - g->off[x];
    for (uint64_t i = 0; i < dx; ++i) {
      const uint32_t y = g->nbr[g->off[x] + i];
      if (g->off[y + 1] == g->off[y]) continue;  /* N+(y) empty: nothing to meet */
      has_in[y] = 1;
      parts += 1;
      streamed += dx - i - 1;                    /* members of N+(x) after y */
    }
  }
  uint64_t held = 0, held_members = 0;
  for (uint32_t y = 0; y < n; ++y)
    if (has_in[y]) {
      held += 1;
      held_members += g->off[y + 1] - g->off[y];
    }
  free(has_in);
  if (out) {
    out[0] = held;
    out[1] = held_members;
    out[2] = parts;
    out[3] = streamed;
  }
  return 32 * held + 4 * held_members + 8 * parts + 4 * streamed;
}

/*
 * Many independent graphs: graph i has n_vertices[i] vertices and the raw
 * pairs src/dst[edge_off[i] .. edge_off[i+1]) with local ids.  Graphs are
 * counted in parallel, each by the same definition as orc_triangles on one
 * thread.  Per graph: counts[i] = T, and (optional) b_merge[i], b_target[i].
 * Returns 0, 1 if an id is out of range (that graph's count is then
 * UINT64_MAX), 2 if memory ran out.
 */
int orc_batch_triangles(uint32_t n_graphs, const uint32_t* n_vertices, const uint64_t* edge_off,
                        const uint32_t* src, const uint32_t* dst, int threads, uint64_t* counts,
                        uint64_t* b_merge, uint64_t* b_target) {
  set_threads(threads);
  int status = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < (int64_t)n_graphs; ++i) {
    int err = 0;
    const uint64_t e0 = edge_off[i], e1 = edge_off[i + 1];
    orc_graph* g = orc_graph_new(n_vertices[i], e1 - e0, src + e0, dst + e0, &err);
    if (!g) {
      counts[i] = UINT64_MAX;
#pragma omp critical
      if (err > status) status = err;
      continue;
    }
    uint64_t t = 0, b = 0;
    for (uint32_t x = 0; x < g->n; ++x) {
      const uint32_t* nx = g->nbr + g->off[x];
      const uint64_t dx = g->off[x + 1] - g->off[x];
      for (uint64_t j = 0; j < dx; ++j) {
        const uint32_t y = nx[j];
        const uint64_t dy = g->off[y + 1] - g->off[y];
        t += merge_count(nx, dx, g->nbr + g->off[y], dy);
        b += 4 * (dx + dy);
      }
    }
    counts[i] = t;
    if (b_merge) b_merge[i] = b;
    if (b_target) {
      b_target[i] = orc_target_reads(g, NULL);
      if (b_target[i] == UINT64_MAX) {
#pragma omp critical
        status = 2;
      }
    }
    orc_graph_free(g);
  }
  return status;
}

/* ---- cross-checks without orientation ---------------------------------- */

static int build_symmetric(orc_graph* g) {
  if (g->soff) return 0;
  const uint32_t n = g->n;
  g->soff = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
  g->snbr = (uint32_t*)malloc((g->m > 0 ? 2 * g->m : 1) * sizeof(uint32_t));
  if (!g->soff || !g->snbr) return -1;
  for (uint32_t v = 0; v < n; ++v) g->soff[v + 1] = g->soff[v] + g->deg[v];
  uint64_t* fill = (uint64_t*)malloc(((size_t)n + 1) * sizeof(uint64_t));
  if (!fill) return -1;
  memcpy(fill, g->soff, ((size_t)n + 1) * sizeof(uint64_t));
  for (uint64_t i = 0; i < g->m; ++i) {
    g->snbr[fill[g->ea[i]]++] = g->eb[i];
    g->snbr[fill[g->eb[i]]++] = g->ea[i];
  }
  free(fill);
  for (uint32_t v = 0; v < n; ++v)
    qsort(g->snbr + g->soff[v], g->soff[v + 1] - g->soff[v], sizeof(uint32_t), cmp_u32);
  return 0;
}

/* sum over undirected edges {a,b} of |N(a) & N(b)|  (= 3T) */
uint64_t orc_sym_triangle_sum(orc_graph* g) {
  if (build_symmetric(g)) return UINT64_MAX;
  uint64_t s = 0;
  for (uint64_t i = 0; i < g->m; ++i) {
    const uint32_t a = g->ea[i], b = g->eb[i];
    s += merge_count(g->snbr + g->soff[a], g->soff[a + 1] - g->soff[a],
                     g->snbr + g->soff[b], g->soff[b + 1] - g->soff[b]);
  }
  return s;
}

/* sum over undirected edges {a,b} of the number of edges inside N(a) & N(b)  (= 6K) */
uint64_t orc_sym_4clique_sum(orc_graph* g) {
  if (build_symmetric(g)) return UINT64_MAX;
  uint64_t dmax = 0;
  for (uint32_t v = 0; v < g->n; ++v) if (g->deg[v] > dmax) dmax = g->deg[v];
  uint32_t* c = (uint32_t*)malloc((dmax ? dmax : 1) * sizeof(uint32_t));
  if (!c) return UINT64_MAX;
  uint64_t s = 0;
  for (uint64_t i = 0; i < g->m; ++i) {
    const uint32_t a = g->ea[i], b = g->eb[i];
    const uint64_t nc = merge_list(g->snbr + g->soff[a], g->soff[a + 1] - g->soff[a],
                                   g->snbr + g->soff[b], g->soff[b + 1] - g->soff[b], c);
    /* edges inside C: each counted twice as (p, q) and (q, p) */
    uint64_t twice = 0;
    for (uint64_t j = 0; j < nc; ++j) {
      const uint32_t p = c[j];
      twice += merge_count(c, nc, g->snbr + g->soff[p], g->soff[p + 1] - g->soff[p]);
    }
    s += twice / 2;
  }
  free(c);
  return s;
}

/* Generic-Join on the unpruned symmetric relation: ordered triangle tuples (= 6T) */
uint64_t orc_sym_ordered_triangles(orc_graph* g) {
  if (build_symmetric(g)) return UINT64_MAX;
  uint64_t s = 0;
  for (uint32_t x = 0; x < g->n; ++x) {
    const uint32_t* nx = g->snbr + g->soff[x];
    const uint64_t dx = g->soff[x + 1] - g->soff[x];
    for (uint64_t i = 0; i < dx; ++i) {
      const uint32_t y = nx[i];
      s += merge_count(nx, dx, g->snbr + g->soff[y], g->soff[y + 1] - g->soff[y]);
    }
  }
  return s;
}

/* Generic-Join on the unpruned symmetric relation: ordered 4-clique tuples (= 24K) */
uint64_t orc_sym_ordered_4cliques(orc_graph* g) {
  if (build_symmetric(g)) return UINT64_MAX;
  uint64_t dmax = 0;
  for (uint32_t v = 0; v < g->n; ++v) if (g->deg[v] > dmax) dmax = g->deg[v];
  uint32_t* s1 = (uint32_t*)malloc((dmax ? dmax : 1) * sizeof(uint32_t));
  uint32_t* s2 = (uint32_t*)malloc((dmax ? dmax : 1) * sizeof(uint32_t));
  if (!s1 || !s2) { free(s1); free(s2); return UINT64_MAX; }
  uint64_t s = 0;
  for (uint32_t x = 0; x < g->n; ++x) {
    const uint32_t* nx = g->snbr + g->soff[x];
    const uint64_t dx = g->soff[x + 1] - g->soff[x];
    for (uint64_t i = 0; i < dx; ++i) {
      const uint32_t y = nx[i];
      const uint64_t n1 = merge_list(nx, dx, g->snbr + g->soff[y], g->soff[y + 1] - g->soff[y], s1);
      for (uint64_t j = 0; j < n1; ++j) {
        const uint32_t z = s1[j];
        const uint64_t n2 = merge_list(s1, n1, g->snbr + g->soff[z], g->soff[z + 1] - g->soff[z], s2);
        s += n2;
      }
    }
  }
  free(s1);
  free(s2);
  return s;
}

/*
 * Generic-Join on the unpruned symmetric relation with the first attribute
 * kept: t_by_id[x] = number of ordered triangles (x, y, z), i.e. the sum over
 * y in N(x) of |N(x) & N(y)|.  Returns the total (= 6T).
 */
uint64_t orc_sym_triangles_by_first(orc_graph* g, int threads, uint64_t* t_by_id) {
  if (build_symmetric(g)) return UINT64_MAX;
  set_threads(threads);
  uint64_t s = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : s)
  for (uint32_t x = 0; x < g->n; ++x) {
    const uint32_t* nx = g->snbr + g->soff[x];
    const uint64_t dx = g->soff[x + 1] - g->soff[x];
    uint64_t tx = 0;
    for (uint64_t i = 0; i < dx; ++i) {
      const uint32_t y = nx[i];
      tx += merge_count(nx, dx, g->snbr + g->soff[y], g->soff[y + 1] - g->soff[y]);
    }
    if (t_by_id) t_by_id[x] = tx;
    s += tx;
  }
  return s;
}

/*
 * COUNT(*) of the Lollipop query of section 5.3,
 *   Lollipop(x,y,z,w) :- R(x,y), S(y,z), T(x,z), U(x,w),
 * as one Generic-Join over the unpruned symmetric relation with attribute
 * order x, y, z, w: for x, for y in N(x), for z in N(x) & N(y), for w in N(x)
 * (w is constrained by U alone, so its level adds |N(x)| per (x, y, z)).
 */
uint64_t orc_sym_lollipop(orc_graph* g, int threads) {
  if (build_symmetric(g)) return UINT64_MAX;
  set_threads(threads);
  uint64_t s = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : s)
  for (uint32_t x = 0; x < g->n; ++x) {
    const uint32_t* nx = g->snbr + g->soff[x];
    const uint64_t dx = g->soff[x + 1] - g->soff[x];
    for (uint64_t i = 0; i < dx; ++i) {
      const uint32_t y = nx[i];
      const uint64_t z_count =
          merge_count(nx, dx, g->snbr + g->soff[y], g->soff[y + 1] - g->soff[y]);
      s += z_count * dx;
    }
  }
  return s;
}

/*
 * Pairwise set intersection (section 4.2): out[p] = |A & B| for the sets
 * A = members[off[s] .. off[s+1]) and B = members[off[t] .. off[t+1]) with
 * (s, t) = (pairs[2p], pairs[2p+1]); each set sorted ascending without
 * repeats.  The count does not depend on how a set is laid out (section
 * 4.3), so one definition serves every layout.  Returns the sum, or
 * UINT64_MAX if a pair names a set >= n_sets.
 */
uint64_t orc_pair_intersections(uint32_t n_sets, const uint64_t* off, const uint32_t* members,
                                uint64_t n_pairs, const uint32_t* pairs, int threads,
                                uint64_t* out) {
  for (uint64_t p = 0; p < n_pairs; ++p)
    if (pairs[2 * p] >= n_sets || pairs[2 * p + 1] >= n_sets) return UINT64_MAX;
  set_threads(threads);
  uint64_t s = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : s)
  for (uint64_t p = 0; p < n_pairs; ++p) {
    const uint32_t a = pairs[2 * p], b = pairs[2 * p + 1];
    const uint64_t c = merge_count(members + off[a], off[a + 1] - off[a], members + off[b],
                                   off[b + 1] - off[b]);
    if (out) out[p] = c;
    s += c;
  }
  return s;
}
