// C ABI: contexts, tries, counting entry points, host-trie accessors.
#include <algorithm>
#include <cstring>
#include <new>

#include "eh_internal.h"

namespace eh {

eh_status hip_check(Ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return EH_OK;
  if (c) c->err = std::string(what) + ": " + hipGetErrorString(e);
  return EH_EHIP;
}

eh_status dev_alloc(Ctx* c, DevBuf& b, size_t bytes) {
  b.p = nullptr;
  b.bytes = 0;
  if (bytes == 0) bytes = 8;
  bytes = (bytes + 255) & ~size_t(255);
  void* p = nullptr;
  if (c->has_alloc) {
    p = c->alloc.alloc(c->alloc.self, bytes, c->stream);
    if (!p) {
      c->err = "allocator returned NULL for " + std::to_string(bytes) + " bytes";
      return EH_ENOMEM;
    }
  } else {
    const hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      c->err = "hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e);
      (void)hipGetLastError();
      return EH_ENOMEM;
    }
  }
  b.p = p;
  b.bytes = bytes;
  return EH_OK;
}

void dev_free(Ctx* c, DevBuf& b) {
  if (!b.p) return;
  if (c->has_alloc) c->alloc.free(c->alloc.self, b.p, c->stream);
  else (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

eh_status ensure_acc(Ctx* c, size_t n) {
  if (c->acc_cap >= n && c->acc.p) return EH_OK;
  // the stream may still use the old buffer
  eh_status st = hip_check(c, hipStreamSynchronize(c->stream), "stream sync");
  if (st != EH_OK) return st;
  dev_free(c, c->acc);
  size_t cap = std::max<size_t>(n, 64);
  if ((st = dev_alloc(c, c->acc, cap * sizeof(uint64_t))) != EH_OK) return st;
  c->acc_cap = cap;
  return EH_OK;
}

eh_status ensure_pinned(Ctx* c, size_t n) {
  if (c->pinned_cap >= n && c->pinned) return EH_OK;
  if (c->pinned) (void)hipHostFree(c->pinned);
  c->pinned = nullptr;
  c->pinned_cap = 0;
  size_t cap = std::max<size_t>(n, 64);
  eh_status st = hip_check(c, hipHostMalloc((void**)&c->pinned, cap * sizeof(uint64_t),
                                            hipHostMallocDefault), "hipHostMalloc");
  if (st != EH_OK) { c->pinned = nullptr; return st; }
  c->pinned_cap = cap;
  return EH_OK;
}

namespace {

eh_status upload(Ctx* c, DevBuf& b, const void* src, size_t bytes, const char* what) {
  eh_status st = dev_alloc(c, b, bytes);
  if (st != EH_OK) return st;
  if (bytes)
    if ((st = hip_check(c, hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice), what)) != EH_OK)
      return st;
  return EH_OK;
}

void free_trie_device(Trie& t) {
  Ctx* c = t.ctx;
  for (auto& p : t.plans) free_plan(c, *p);
  t.plans.clear();
  dev_free(c, t.vdesc);
  dev_free(c, t.col);
  dev_free(c, t.bsdesc);
  dev_free(c, t.vert);
  t.device_bytes = 0;
}

// One list buffer holds every set: the uint layout (col, m entries) followed
// by all bitset words, so a kernel reads either through one base pointer.
// bsdesc.x is the absolute position of a set's first word in that buffer.
eh_status upload_trie(Ctx* c, Trie& t) {
  const HostTrie& h = t.host;
  const uint64_t W = h.n_words;
  if (h.m + W > kMaxPosition) {
    c->err = "edges plus bitset words exceed 2^32-2";
    return EH_EOVERFLOW;
  }
  std::vector<uint2> vd(std::max<uint32_t>(h.n, 1));
  std::vector<uint4> bd(std::max<uint32_t>(h.n, 1));
  for (uint32_t v = 0; v < h.n; ++v) {
    const uint32_t len = h.row[v + 1] - h.row[v];
    const bool bs = h.bs_off[v] != kNoBitset;
    vd[v] = make_uint2(h.row[v], len | (bs ? kHiBit : 0u));
    bd[v] = make_uint4(bs ? uint32_t(h.m) + h.bs_off[v] : 0u, h.bs_base[v], h.bs_nw[v], 0u);
  }
  eh_status st;
  if ((st = upload(c, t.vdesc, vd.data(), sizeof(uint2) * h.n, "upload vertex table")) != EH_OK)
    return st;
  if ((st = dev_alloc(c, t.col, sizeof(uint32_t) * (h.m + W))) != EH_OK) return st;
  if (h.m && (st = hip_check(c, hipMemcpy(t.col.p, h.col.data(), sizeof(uint32_t) * h.m,
                                          hipMemcpyHostToDevice), "upload columns")) != EH_OK)
    return st;
  if (W && (st = hip_check(c, hipMemcpy(static_cast<uint32_t*>(t.col.p) + h.m, h.bs_words.data(),
                                        sizeof(uint32_t) * W, hipMemcpyHostToDevice),
                           "upload bitset words")) != EH_OK)
    return st;
  if ((st = upload(c, t.bsdesc, bd.data(), sizeof(uint4) * (h.n_bs ? h.n : 0),
                   "upload bitset table")) != EH_OK)
    return st;
  if ((st = upload(c, t.vert, h.vert.data(), sizeof(uint32_t) * h.n, "upload ids")) != EH_OK)
    return st;
  t.device_bytes = t.vdesc.bytes + t.col.bytes + t.bsdesc.bytes + t.vert.bytes;
  return EH_OK;
}

LaunchArgs base_args(Ctx* c, const Trie& t) {
  LaunchArgs a;
  a.vdesc = static_cast<const uint2*>(t.vdesc.p);
  a.col = static_cast<const uint32_t*>(t.col.p);
  a.bsdesc = static_cast<const uint4*>(t.bsdesc.p);
  a.bsw = static_cast<const uint32_t*>(t.col.p);  // words live after col
  a.vert = static_cast<const uint32_t*>(t.vert.p);
  a.cursor = static_cast<uint32_t*>(c->cursor.p);
  a.use_bitsets = c->tune.use_bitsets && t.host.n_bs > 0;
  a.dynamic = c->tune.dynamic;
  a.algo = c->tune.algo;
  a.gamma = c->tune.gamma;
  a.group_lanes = c->tune.group_lanes;
  a.dmax = t.host.dmax;
  a.stage_words = c->tune.stage_words;
  a.xcds = c->tune.xcds;
  a.unroll = c->tune.unroll;
  a.grab = c->tune.grab;
  a.search_below = c->tune.search_below;
  a.symmetric = t.host.symmetric ? 1u : 0u;
  a.reverse = c->tune.reverse;
  return a;
}

// Enqueues one counting launch over items [i0, i1) of a plan.  cursor: the
// work cursors to use instead of the context's (null: the context's).
// lollipop: the Lollipop launch over an edge-once plan instead of triangles.
eh_status enqueue_count(Ctx* c, Trie& t, Plan* p, uint64_t i0, uint64_t i1,
                        unsigned long long* acc, uint32_t tag_base, unsigned long long* per_root,
                        uint32_t* cursor = nullptr, bool lollipop = false) {
  LaunchArgs a = base_args(c, t);
  if (cursor) a.cursor = cursor;
  a.items = static_cast<const Item*>(p->items.p) + i0;
  a.n_items = i1 - i0;
  a.idx = static_cast<const uint32_t*>(t.col.p);
  if (p->staging == EH_STAGE_TARGET) {
    if (p->sdesc.p) a.sdesc = static_cast<const uint4*>(p->sdesc.p) + i0;
    a.rec = static_cast<const uint2*>(p->rec.p);
    if (p->group > 1) a.gsub = static_cast<const uint4*>(p->gsub.p);
  }
  a.acc = acc;
  a.tag_base = tag_base;
  a.per_root = per_root;
  a.item_dmax = p->item_dmax;
  a.k4s = static_cast<uint32_t*>(p->k4s.p);
  a.k4s_stride = p->k4s_stride;
  a.k4s_waves = p->k4s_waves;
  if (p->pattern == EH_4CLIQUE) {
    if (p->k4l.p) {
      // single-graph plans only: the whole range of items and every root
      LaunchArgs la = a;
      la.roots = static_cast<const uint4*>(p->k4l.p);
      la.root_cursors = reinterpret_cast<uint32_t*>(
          static_cast<uint4*>(p->k4l.p) + (p->k4l_n[0] + p->k4l_n[1] + p->k4l_n[2] + p->k4l_n[3]));
      la.rec = static_cast<const uint2*>(p->rec.p);
      if (eh_status st = launch_4cliques_local(c, c->stream, la, p->k4l_n); st != EH_OK) return st;
    }
    return launch_4cliques(c, c->stream, a, c->tune.kernel, c->tune.waves_per_cu);
  }
  if (lollipop) return launch_lollipop(c, c->stream, a, c->tune.waves_per_cu);
  return launch_triangles(c, c->stream, a, c->tune.kernel, c->tune.waves_per_cu);
}

// Target staging describes each streamed suffix of N+(u) by a 16-bit length,
// which degree order guarantees (out-degrees below sqrt(2m) < 2^16); tries
// built under another node ordering may exceed it and then stage sources.
// Symmetric tries stage sources; a single total (half_ok) is counted with
// each undirected edge once (kStageHalf) unless the tuning asks for source
// staging.
uint32_t tri_staging(const Ctx* c, const Trie& t, bool per_root, bool half_ok = false) {
  if (per_root) return EH_STAGE_SOURCE;
  // suffix streaming relies on orientation (every member of N+(v) exceeds v)
  if (t.host.symmetric)
    return half_ok && c->tune.staging != EH_STAGE_SOURCE ? kStageHalf : EH_STAGE_SOURCE;
  if (c->tune.kernel == EH_KERNEL_PAIRWISE) return EH_STAGE_SOURCE;
  if (t.host.dmax > 0xFFFFu) return EH_STAGE_SOURCE;
  return c->tune.staging == EH_STAGE_SOURCE ? EH_STAGE_SOURCE : EH_STAGE_TARGET;
}


eh_status count_single(Ctx* c, Trie& t, int pattern, unsigned long long* d_total,
                       unsigned long long* d_per_root, bool accumulate = false) {
  if (t.host.n_graphs != 1) {
    c->err = "single-graph count called on a batch trie";
    return EH_ESTATE;
  }
  Plan* p = nullptr;
  const uint32_t staging =
      pattern == EH_TRIANGLE ? tri_staging(c, t, d_per_root != nullptr, true) : EH_STAGE_SOURCE;
  eh_status st = get_plan(c, &t, pattern, staging, &p);
  if (st != EH_OK) return st;
  if (!accumulate && (st = launch_fill_u64(c, c->stream, d_total, 1, 0)) != EH_OK) return st;
  if (d_per_root && (st = launch_fill_u64(c, c->stream, d_per_root, t.host.n, 0)) != EH_OK)
    return st;
  if (staging == kStageHalf) {
    // each undirected edge once: the ordered count is twice the launch's sum
    auto* half = static_cast<unsigned long long*>(c->half.p);
    if ((st = launch_fill_u64(c, c->stream, half, 1, 0)) != EH_OK) return st;
    if ((st = enqueue_count(c, t, p, 0, p->n_items, half, 0, nullptr)) != EH_OK) return st;
    return launch_add_scaled(c, c->stream, half, 2, d_total);
  }
  return enqueue_count(c, t, p, 0, p->n_items, d_total, 0, d_per_root);
}

eh_status read_back(Ctx* c, const unsigned long long* d, uint64_t* out, size_t n) {
  eh_status st = ensure_pinned(c, n);
  if (st != EH_OK) return st;
  if ((st = hip_check(c, hipMemcpyAsync(c->pinned, d, n * sizeof(uint64_t), hipMemcpyDeviceToHost,
                                        c->stream), "copy result")) != EH_OK)
    return st;
  if ((st = hip_check(c, hipStreamSynchronize(c->stream), "stream sync")) != EH_OK) return st;
  std::memcpy(out, c->pinned, n * sizeof(uint64_t));
  return EH_OK;
}

thread_local std::string g_err_no_ctx;

}  // namespace

void set_no_ctx_error(const std::string& e) { g_err_no_ctx = e; }
}  // namespace eh

using namespace eh;

extern "C" {

int32_t eh_abi_version(void) { return EH_ABI_VERSION; }

const char* eh_status_str(eh_status s) {
  switch (s) {
    case EH_OK: return "ok";
    case EH_PENDING: return "pending";
    case EH_EINVAL: return "invalid argument";
    case EH_ENOMEM: return "out of memory";
    case EH_EHIP: return "HIP runtime error";
    case EH_EBUSY: return "busy";
    case EH_ENOTFOUND: return "not found";
    case EH_EOVERFLOW: return "size overflow";
    case EH_ESTATE: return "invalid state";
    default: return "unknown status";
  }
}

const char* eh_last_error(const eh_ctx* ctx) {
  return ctx ? ctx->c.err.c_str() : g_err_no_ctx.c_str();
}

eh_status eh_ctx_create(int device, void* hip_stream, const eh_allocator* alloc, eh_ctx** out) {
  if (!out) return EH_EINVAL;
  *out = nullptr;
  eh_ctx* x = new (std::nothrow) eh_ctx();
  if (!x) return EH_ENOMEM;
  Ctx* c = &x->c;
  c->device = device;
  eh_status st = hip_check(c, hipSetDevice(device), "hipSetDevice");
  if (st == EH_OK) {
    int ncu = 0;
    st = hip_check(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device),
                   "query compute units");
    if (ncu > 0) c->n_cu = ncu;
  }
  if (st == EH_OK) {
    if (hip_stream) {
      c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
      st = hip_check(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking),
                     "hipStreamCreate");
      c->own_stream = st == EH_OK;
    }
  }
  if (st == EH_OK && alloc) {
    if (!alloc->alloc || !alloc->free) {
      c->err = "allocator needs both alloc and free";
      st = EH_EINVAL;
    } else {
      c->alloc = *alloc;
      c->has_alloc = true;
    }
  }
  for (int k = 0; st == EH_OK && k < Ctx::kSide; ++k) {
    st = hip_check(c, hipStreamCreateWithFlags(&c->side[k], hipStreamNonBlocking), "side stream");
    if (st == EH_OK)
      st = hip_check(c, hipEventCreateWithFlags(&c->join[k], hipEventDisableTiming), "join event");
  }
  if (st == EH_OK)
    st = hip_check(c, hipEventCreateWithFlags(&c->fork, hipEventDisableTiming), "fork event");
  // one cursor per item partition, each on its own 256-byte line
  if (st == EH_OK) st = dev_alloc(c, c->cursor, sizeof(uint32_t) * kCursorWords * kMaxParts);
  if (st == EH_OK) st = ensure_acc(c, 64);
  if (st == EH_OK) st = dev_alloc(c, c->half, sizeof(uint64_t));
  if (st == EH_OK) st = noalloc_scratch_init(c);
  if (st != EH_OK) {
    g_err_no_ctx = c->err;
    eh_ctx_destroy(x);
    return st;
  }
  *out = x;
  return EH_OK;
}

eh_status eh_ctx_destroy(eh_ctx* ctx) {
  if (!ctx) return EH_EINVAL;
  Ctx* c = &ctx->c;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  dev_free(c, c->acc);
  dev_free(c, c->cursor);
  dev_free(c, c->half);
  if (c->pinned) (void)hipHostFree(c->pinned);
  for (int k = 0; k < Ctx::kSide; ++k) {
    if (c->side[k]) {
      (void)hipStreamSynchronize(c->side[k]);
      (void)hipStreamDestroy(c->side[k]);
    }
    if (c->join[k]) (void)hipEventDestroy(c->join[k]);
  }
  if (c->fork) (void)hipEventDestroy(c->fork);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete ctx;
  return EH_OK;
}

eh_status eh_ctx_set_tuning(eh_ctx* ctx, const eh_tuning* t) {
  if (!ctx || !t) return EH_EINVAL;
  Tuning& u = ctx->c.tune;
  if (t->kernel > EH_KERNEL_PAIRWISE || t->staging > EH_STAGE_TARGET || t->algo > EH_ALGO_SEARCH) {
    ctx->c.err = "tuning enum out of range";
    return EH_EINVAL;
  }
  if (t->group_lanes && (t->group_lanes < 4 || t->group_lanes > 64 ||
                         (t->group_lanes & (t->group_lanes - 1)))) {
    ctx->c.err = "group_lanes must be 0 or a power of two in [4, 64]";
    return EH_EINVAL;
  }
  if (t->kernel != EH_KERNEL_AUTO) u.kernel = t->kernel;
  if (t->staging != EH_STAGE_AUTO) u.staging = t->staging;
  u.algo = t->algo;
  if (t->gamma > 0.0f) u.gamma = t->gamma;
  if (t->chunk_work) u.chunk_work = t->chunk_work;
  if (t->waves_per_cu) u.waves_per_cu = t->waves_per_cu;
  u.group_lanes = t->group_lanes;
  u.use_bitsets = t->use_bitsets ? 1 : 0;
  if (t->dynamic > 5) {
    ctx->c.err = "dynamic must be 0 (interleaved), 1 (atomic cursor), 2 (blocked), "
                 "3 (partitioned interleave), 4 (partitioned cursors) or 5 (snake)";
    return EH_EINVAL;
  }
  if (t->xcds > kMaxParts) {
    ctx->c.err = "xcds must be at most " + std::to_string(kMaxParts);
    return EH_EINVAL;
  }
  if (t->grab > 4096) {
    ctx->c.err = "grab must be at most 4096";
    return EH_EINVAL;
  }
  u.dynamic = t->dynamic;
  if (t->stage_words > 1024) {
    ctx->c.err = "stage_words must be at most 1024";
    return EH_EINVAL;
  }
  u.stage_words = t->stage_words;
  u.xcds = t->xcds;
  if (t->unroll != 0 && t->unroll != 4 && t->unroll != 8) {
    ctx->c.err = "unroll must be 0, 4 or 8";
    return EH_EINVAL;
  }
  u.unroll = t->unroll ? t->unroll : 8;
  u.grab = t->grab ? t->grab : 8;
  if (t->search_below > 4096) {
    ctx->c.err = "search_below must be at most 4096";
    return EH_EINVAL;
  }
  u.search_below = t->search_below;
  if (t->group > 4 || t->group == 3) {
    ctx->c.err = "group must be 0, 1, 2 or 4";
    return EH_EINVAL;
  }
  u.group = t->group ? t->group : 1;
  if (t->reverse > 1) {
    ctx->c.err = "reverse must be 0 or 1";
    return EH_EINVAL;
  }
  u.reverse = t->reverse;
  if (t->k4_local > 1) {
    ctx->c.err = "k4_local must be 0 or 1";
    return EH_EINVAL;
  }
  u.k4_local = t->k4_local;
  return EH_OK;
}

eh_status eh_ctx_get_tuning(const eh_ctx* ctx, eh_tuning* out) {
  if (!ctx || !out) return EH_EINVAL;
  const Tuning& u = ctx->c.tune;
  out->kernel = u.kernel;
  out->staging = u.staging;
  out->algo = u.algo;
  out->gamma = u.gamma;
  out->chunk_work = u.chunk_work;
  out->waves_per_cu = u.waves_per_cu;
  out->group_lanes = u.group_lanes;
  out->use_bitsets = u.use_bitsets;
  out->dynamic = u.dynamic;
  out->stage_words = u.stage_words;
  out->xcds = u.xcds;
  out->unroll = u.unroll;
  out->grab = u.grab;
  out->search_below = u.search_below;
  out->group = u.group;
  out->reverse = u.reverse;
  out->k4_local = u.k4_local;
  return EH_OK;
}

static eh_status finish_build(eh_ctx* ctx, eh_trie* x, eh_trie** out) {
  Ctx* c = &ctx->c;
  eh_status st = hip_check(c, hipSetDevice(c->device), "hipSetDevice");
  if (st == EH_OK) st = upload_trie(c, x->t);
  if (st != EH_OK) {
    free_trie_device(x->t);
    delete x;
    return st;
  }
  *out = x;
  return EH_OK;
}

eh_status eh_build_trie(eh_ctx* ctx, const uint32_t* src, const uint32_t* dst, uint64_t n_edges,
                        uint32_t n_vertices, const eh_build_opts* opts, eh_trie** out) {
  if (!ctx || !out || (n_edges && (!src || !dst))) return EH_EINVAL;
  *out = nullptr;
  if (opts && (opts->layout > EH_LAYOUT_BITSET_ALL || opts->order > EH_ORDER_STRONG_RUNS)) {
    ctx->c.err = "unknown layout or node ordering";
    return EH_EINVAL;
  }
  eh_trie* x = new (std::nothrow) eh_trie();
  if (!x) return EH_ENOMEM;
  x->t.ctx = &ctx->c;
  eh_status st;
  try {
    st = host_build(src, dst, n_edges, n_vertices, resolve_opts(opts), x->t.host, ctx->c.err);
  } catch (const std::bad_alloc&) {
    ctx->c.err = "host memory exhausted while building the trie";
    st = EH_ENOMEM;
  }
  if (st != EH_OK) {
    delete x;
    return st;
  }
  return finish_build(ctx, x, out);
}

eh_status eh_build_trie_device(eh_ctx* ctx, const uint32_t* d_src, const uint32_t* d_dst,
                               uint64_t n_edges, uint32_t n_vertices, const eh_build_opts* opts,
                               eh_trie** out) {
  if (!ctx || !out || (n_edges && (!d_src || !d_dst))) return EH_EINVAL;
  *out = nullptr;
  if (opts && (opts->layout > EH_LAYOUT_BITSET_ALL || opts->order > EH_ORDER_STRONG_RUNS)) {
    ctx->c.err = "unknown layout or node ordering";
    return EH_EINVAL;
  }
  const BuildOpts o = resolve_opts(opts);
  eh_trie* x = new (std::nothrow) eh_trie();
  if (!x) return EH_ENOMEM;
  x->t.ctx = &ctx->c;
  eh_status st = hip_check(&ctx->c, hipSetDevice(ctx->c.device), "hipSetDevice");
  if (st == EH_OK) {
    try {
      st = device_build(&ctx->c, d_src, d_dst, n_edges, n_vertices, o, x->t);
    } catch (const std::bad_alloc&) {
      ctx->c.err = "host memory exhausted while building the trie";
      st = EH_ENOMEM;
    }
  }
  if (st != EH_OK) {
    (void)hipStreamSynchronize(ctx->c.stream);
    free_trie_device(x->t);
    delete x;
    return st;
  }
  *out = x;
  return EH_OK;
}

eh_status eh_build_batch_device(eh_ctx* ctx, uint32_t n_graphs, const uint32_t* n_vertices,
                                const uint64_t* edge_off, const uint32_t* d_src,
                                const uint32_t* d_dst, const eh_build_opts* opts, eh_trie** out) {
  if (!ctx || !out || !n_vertices || !edge_off || n_graphs == 0) return EH_EINVAL;
  *out = nullptr;
  if (edge_off[n_graphs] > edge_off[0] && (!d_src || !d_dst)) return EH_EINVAL;
  if (opts && (opts->layout > EH_LAYOUT_BITSET_ALL || opts->order > EH_ORDER_STRONG_RUNS)) {
    ctx->c.err = "unknown layout or node ordering";
    return EH_EINVAL;
  }
  const BuildOpts o = resolve_opts(opts);
  if (o.order != EH_ORDER_DEGREE && o.order != EH_ORDER_REV_DEGREE && o.order != EH_ORDER_INPUT) {
    ctx->c.err = "traversal orderings (BFS, hybrid, strong runs) of a batch are built on the host";
    return EH_EINVAL;
  }
  DeviceBatch b;
  b.n_graphs = n_graphs;
  b.n_vertices = n_vertices;
  std::vector<uint64_t> eoff(size_t(n_graphs) + 1);
  b.vbase.assign(size_t(n_graphs) + 1, 0);
  uint64_t padded = 0;
  for (uint32_t g = 0; g < n_graphs; ++g) {
    if (edge_off[g + 1] < edge_off[g]) {
      ctx->c.err = "edge_off is not monotone at graph " + std::to_string(g);
      return EH_EINVAL;
    }
    eoff[g] = edge_off[g] - edge_off[0];
    b.vbase[g] = uint32_t(std::min<uint64_t>(padded, kMaxIndex));
    padded += (uint64_t(n_vertices[g]) + 31) & ~uint64_t(31);
  }
  eoff[n_graphs] = edge_off[n_graphs] - edge_off[0];
  if (padded > kMaxIndex) {
    ctx->c.err = "batch has more than 2^31-1 vertices";
    return EH_EOVERFLOW;
  }
  b.vbase[n_graphs] = uint32_t(padded);
  b.edge_off = eoff.data();
  eh_trie* x = new (std::nothrow) eh_trie();
  if (!x) return EH_ENOMEM;
  x->t.ctx = &ctx->c;
  eh_status st = hip_check(&ctx->c, hipSetDevice(ctx->c.device), "hipSetDevice");
  if (st == EH_OK) {
    try {
      st = device_build(&ctx->c, d_src ? d_src + edge_off[0] : d_src,
                        d_dst ? d_dst + edge_off[0] : d_dst, eoff[n_graphs], uint32_t(padded), o,
                        x->t, &b);
    } catch (const std::bad_alloc&) {
      ctx->c.err = "host memory exhausted while building the batch";
      st = EH_ENOMEM;
    }
  }
  if (st != EH_OK) {
    (void)hipStreamSynchronize(ctx->c.stream);
    free_trie_device(x->t);
    delete x;
    return st;
  }
  *out = x;
  return EH_OK;
}

eh_status eh_trie_host_arrays(const eh_trie* trie, uint32_t* rank, uint32_t* row, uint32_t* col,
                              uint32_t* bs_off, uint32_t* bs_base, uint32_t* bs_nw,
                              uint32_t* bs_words) {
  if (!trie) return EH_EINVAL;
  const HostTrie& h = trie->t.host;
  auto put = [](uint32_t* d, const std::vector<uint32_t>& v) {
    if (d && !v.empty()) std::memcpy(d, v.data(), v.size() * sizeof(uint32_t));
  };
  put(rank, h.rank);
  put(row, h.row);
  put(col, h.col);
  put(bs_off, h.bs_off);
  put(bs_base, h.bs_base);
  put(bs_nw, h.bs_nw);
  if (bs_words && h.words_on_device && h.n_words) {
    // a GPU-built trie keeps its words on the device only
    Ctx* c = trie->t.ctx;
    eh_status st = hip_check(c, hipSetDevice(c->device), "hipSetDevice");
    if (st == EH_OK) st = hip_check(c, hipStreamSynchronize(c->stream), "stream sync");
    if (st == EH_OK)
      st = hip_check(c, hipMemcpy(bs_words, static_cast<const uint32_t*>(trie->t.col.p) + h.m,
                                  sizeof(uint32_t) * h.n_words, hipMemcpyDeviceToHost),
                     "download words");
    return st;
  }
  put(bs_words, h.bs_words);
  return EH_OK;
}

eh_status eh_trie_device_arrays(eh_ctx* ctx, const eh_trie* trie, uint32_t* vdesc, uint32_t* col,
                                uint32_t* bsdesc, uint32_t* vert) {
  if (!ctx || !trie) return EH_EINVAL;
  Ctx* c = &ctx->c;
  const Trie& t = trie->t;
  const HostTrie& h = t.host;
  const uint64_t W = h.n_words;
  eh_status st = hip_check(c, hipSetDevice(c->device), "hipSetDevice");
  if (st != EH_OK) return st;
  if ((st = hip_check(c, hipStreamSynchronize(c->stream), "stream sync")) != EH_OK) return st;
  auto get = [&](uint32_t* d, const DevBuf& b, size_t bytes, const char* what) -> eh_status {
    if (!d || !bytes) return EH_OK;
    return hip_check(c, hipMemcpy(d, b.p, bytes, hipMemcpyDeviceToHost), what);
  };
  if ((st = get(vdesc, t.vdesc, 8ull * h.n, "download vertex table")) != EH_OK ||
      (st = get(col, t.col, 4ull * (h.m + W), "download sets")) != EH_OK ||
      (st = get(bsdesc, t.bsdesc, h.n_bs ? 16ull * h.n : 0, "download bitset table")) != EH_OK ||
      (st = get(vert, t.vert, 4ull * h.n, "download ids")) != EH_OK)
    return st;
  return EH_OK;
}

eh_status eh_build_batch(eh_ctx* ctx, uint32_t n_graphs, const uint32_t* n_vertices,
                         const uint64_t* edge_off, const uint32_t* src, const uint32_t* dst,
                         const eh_build_opts* opts, eh_trie** out) {
  if (!ctx || !out || !n_vertices || !edge_off || n_graphs == 0) return EH_EINVAL;
  if (edge_off[n_graphs] && (!src || !dst)) return EH_EINVAL;
  *out = nullptr;
  if (opts && (opts->layout > EH_LAYOUT_BITSET_ALL || opts->order > EH_ORDER_STRONG_RUNS)) {
    ctx->c.err = "unknown layout or node ordering";
    return EH_EINVAL;
  }
  eh_trie* x = new (std::nothrow) eh_trie();
  if (!x) return EH_ENOMEM;
  x->t.ctx = &ctx->c;
  eh_status st;
  try {
    st = host_build_batch(n_graphs, n_vertices, edge_off, src, dst, resolve_opts(opts), x->t.host,
                          ctx->c.err);
  } catch (const std::bad_alloc&) {
    ctx->c.err = "host memory exhausted while building the batch";
    st = EH_ENOMEM;
  }
  if (st != EH_OK) {
    delete x;
    return st;
  }
  return finish_build(ctx, x, out);
}

static void fill_info(const HostTrie& h, eh_trie_info* out) {
  out->n = h.n;
  out->n_graphs = h.n_graphs;
  out->m_plus = h.m;
  out->n_bitset_sets = h.n_bs;
  out->bitset_words = h.n_words;
  out->device_bytes = 0;
  out->b_merge = h.b_merge;
  out->max_out_degree = h.dmax;
  out->reserved = 0;
  out->b_target = h.b_target;
}

eh_status eh_trie_info_get(const eh_trie* trie, eh_trie_info* out) {
  if (!trie || !out) return EH_EINVAL;
  fill_info(trie->t.host, out);
  out->device_bytes = trie->t.device_bytes;
  return EH_OK;
}

eh_status eh_trie_free(eh_trie* trie) {
  if (!trie) return EH_EINVAL;
  Ctx* c = trie->t.ctx;
  (void)hipStreamSynchronize(c->stream);
  free_trie_device(trie->t);
  delete trie;
  return EH_OK;
}

eh_status eh_count_triangles(eh_ctx* ctx, const eh_trie* trie, uint64_t* total,
                             uint64_t* d_per_root) {
  if (!ctx || !trie || !total) return EH_EINVAL;
  Ctx* c = &ctx->c;
  Trie& t = const_cast<eh_trie*>(trie)->t;
  eh_status st = count_single(c, t, EH_TRIANGLE, static_cast<unsigned long long*>(c->acc.p),
                              reinterpret_cast<unsigned long long*>(d_per_root));
  if (st != EH_OK) return st;
  return read_back(c, static_cast<const unsigned long long*>(c->acc.p), total, 1);
}

eh_status eh_count_4cliques(eh_ctx* ctx, const eh_trie* trie, uint64_t* total) {
  if (!ctx || !trie || !total) return EH_EINVAL;
  Ctx* c = &ctx->c;
  Trie& t = const_cast<eh_trie*>(trie)->t;
  eh_status st =
      count_single(c, t, EH_4CLIQUE, static_cast<unsigned long long*>(c->acc.p), nullptr);
  if (st != EH_OK) return st;
  return read_back(c, static_cast<const unsigned long long*>(c->acc.p), total, 1);
}

eh_status eh_count_lollipop(eh_ctx* ctx, const eh_trie* trie, uint64_t* total) {
  if (!ctx || !trie || !total) return EH_EINVAL;
  Ctx* c = &ctx->c;
  Trie& t = const_cast<eh_trie*>(trie)->t;
  if (!t.host.symmetric || t.host.n_graphs != 1) {
    c->err = "the Lollipop count needs a symmetric single-graph trie";
    return EH_ESTATE;
  }
  eh_status st = hip_check(c, hipSetDevice(c->device), "hipSetDevice");
  if (st != EH_OK) return st;
  auto* acc = static_cast<unsigned long long*>(c->acc.p);
  if (c->tune.staging != EH_STAGE_SOURCE) {
    // each undirected edge {x, u} once, weighted by |N(x)| + |N(u)|
    Plan* p = nullptr;
    if ((st = get_plan(c, &t, EH_TRIANGLE, kStageHalf, &p)) != EH_OK) return st;
    if ((st = launch_fill_u64(c, c->stream, acc + 1, 1, 0)) != EH_OK) return st;
    if ((st = enqueue_count(c, t, p, 0, p->n_items, acc + 1, 0, nullptr, nullptr, true)) != EH_OK)
      return st;
    return read_back(c, acc + 1, total, 1);
  }
  // source staging: t(x) by first attribute over every arc, then the
  // degree-weighted sum
  DevBuf per;  // t(x) by original id
  if ((st = dev_alloc(c, per, sizeof(unsigned long long) * std::max<uint32_t>(t.host.n, 1))) !=
      EH_OK)
    return st;
  st = count_single(c, t, EH_TRIANGLE, acc, static_cast<unsigned long long*>(per.p));
  if (st == EH_OK) st = launch_fill_u64(c, c->stream, acc + 1, 1, 0);
  if (st == EH_OK)
    st = launch_degree_weighted_sum(c, c->stream, static_cast<const unsigned long long*>(per.p),
                                    static_cast<const uint32_t*>(t.vert.p),
                                    static_cast<const uint2*>(t.vdesc.p), t.host.n, acc + 1);
  if (st == EH_OK) st = read_back(c, acc + 1, total, 1);
  (void)hipStreamSynchronize(c->stream);
  dev_free(c, per);
  return st;
}

eh_status eh_count_async(eh_ctx* ctx, const eh_trie* trie, int pattern, uint64_t* d_total) {
  if (!ctx || !trie || !d_total) return EH_EINVAL;
  if (pattern != EH_TRIANGLE && pattern != EH_4CLIQUE) {
    ctx->c.err = "pattern must be EH_TRIANGLE or EH_4CLIQUE";
    return EH_EINVAL;
  }
  Trie& t = const_cast<eh_trie*>(trie)->t;
  return count_single(&ctx->c, t, pattern, reinterpret_cast<unsigned long long*>(d_total), nullptr);
}

eh_status eh_count_add_async(eh_ctx* ctx, const eh_trie* trie, int pattern, uint64_t* d_total) {
  if (!ctx || !trie || !d_total) return EH_EINVAL;
  if (pattern != EH_TRIANGLE && pattern != EH_4CLIQUE) {
    ctx->c.err = "pattern must be EH_TRIANGLE or EH_4CLIQUE";
    return EH_EINVAL;
  }
  Trie& t = const_cast<eh_trie*>(trie)->t;
  return count_single(&ctx->c, t, pattern, reinterpret_cast<unsigned long long*>(d_total), nullptr,
                      true);
}

eh_status eh_count_add_noalloc(eh_ctx* ctx, const eh_trie* trie, int pattern, uint64_t* d_total) {
  if (!ctx || !trie || !d_total) return EH_EINVAL;
  Ctx* c = &ctx->c;
  if (pattern != EH_TRIANGLE && pattern != EH_4CLIQUE) {
    c->err = "pattern must be EH_TRIANGLE or EH_4CLIQUE";
    return EH_EINVAL;
  }
  Trie& t = const_cast<eh_trie*>(trie)->t;
  if (t.host.n_graphs != 1) {
    c->err = "single-graph count called on a batch trie";
    return EH_ESTATE;
  }
  if (!c->noalloc_scratch) {
    c->err = "the context has no static scratch";
    return EH_ESTATE;
  }
  // the cursors the schedule uses must fit the scratch's cursor region
  const uint32_t parts = c->tune.xcds ? c->tune.xcds : 8u;
  if (size_t(parts) * kCursorWords * sizeof(uint32_t) > kNoAllocCursorBytes) {
    c->err = "the tuning's " + std::to_string(parts) + " item partitions need more cursors than "
             "the " + std::to_string(kNoAllocCursorBytes) + "-byte static scratch holds";
    return EH_EOVERFLOW;
  }
  const uint32_t staging = pattern == EH_TRIANGLE ? tri_staging(c, t, false, true) : EH_STAGE_SOURCE;
  Plan* p = find_plan(c, &t, pattern, staging);
  if (!p) {
    c->err = "no cached work-item plan for this pattern and tuning: count once with "
             "eh_count_async, eh_count_add_async or a blocking count first";
    return EH_ESTATE;
  }
  auto* base = static_cast<unsigned char*>(c->noalloc_scratch);
  auto* cursor = reinterpret_cast<uint32_t*>(base);
  auto* total = reinterpret_cast<unsigned long long*>(d_total);
  if (staging == kStageHalf) {
    // each undirected edge once: the ordered count is twice the launch's sum
    auto* half = reinterpret_cast<unsigned long long*>(base + kNoAllocCursorBytes);
    eh_status st = launch_fill_u64(c, c->stream, half, 1, 0);
    if (st != EH_OK) return st;
    if ((st = enqueue_count(c, t, p, 0, p->n_items, half, 0, nullptr, cursor)) != EH_OK) return st;
    return launch_add_scaled(c, c->stream, half, 2, total);
  }
  return enqueue_count(c, t, p, 0, p->n_items, total, 0, nullptr, cursor);
}

eh_status eh_count_rooted(eh_ctx* ctx, const eh_trie* trie, int pattern, const uint32_t* roots,
                          uint32_t n_roots, uint64_t* total) {
  if (!ctx || !trie || !roots || !total || n_roots == 0) return EH_EINVAL;
  Ctx* c = &ctx->c;
  if (pattern != EH_TRIANGLE && pattern != EH_4CLIQUE) {
    c->err = "pattern must be EH_TRIANGLE or EH_4CLIQUE";
    return EH_EINVAL;
  }
  Trie& t = const_cast<eh_trie*>(trie)->t;
  const HostTrie& h = t.host;
  if (h.n_graphs != 1) {
    c->err = "rooted count needs a single-graph trie";
    return EH_ESTATE;
  }
  std::vector<uint32_t> r;
  r.reserve(n_roots);
  for (uint32_t i = 0; i < n_roots; ++i) {
    if (roots[i] >= h.n) {
      c->err = "root id " + std::to_string(roots[i]) + " >= n";
      return EH_EINVAL;
    }
    r.push_back(h.rank[roots[i]]);
  }
  std::sort(r.begin(), r.end());
  r.erase(std::unique(r.begin(), r.end()), r.end());
  std::vector<Item> items;
  uint32_t item_dmax = 0;
  // 4-cliques: roots of out-degree <= 512 counted over their induced
  // out-neighbourhoods, whole roots after the S-list kernel's items
  const bool local = pattern == EH_4CLIQUE && c->tune.k4_local && !h.symmetric;
  std::vector<Item> lc[kK4LocalClasses];
  for (uint32_t u : r) {
    const uint32_t du = h.row[u + 1] - h.row[u];
    const int k = local ? k4_local_class(du) : -1;
    if (k >= 0) {
      lc[k].push_back(Item{u, h.row[u], du, 0});
      continue;
    }
    const size_t before = items.size();
    make_items_source(h, u, 0, c->tune.chunk_work, uint32_t(pattern), c->tune.use_bitsets != 0,
                      items);
    if (items.size() > before) item_dmax = std::max(item_dmax, du);
  }
  const size_t n_list = items.size();
  uint64_t loff[kK4LocalClasses + 1] = {n_list};
  for (uint32_t k = 0; k < kK4LocalClasses; ++k) {
    items.insert(items.end(), lc[k].begin(), lc[k].end());
    loff[k + 1] = items.size();
  }
  unsigned long long* acc = static_cast<unsigned long long*>(c->acc.p);
  eh_status st = launch_fill_u64(c, c->stream, acc, 1, 0);
  if (st != EH_OK) return st;
  DevBuf buf, lists;
  if (!items.empty()) {
    if ((st = dev_alloc(c, buf, sizeof(Item) * items.size())) != EH_OK) return st;
    if ((st = hip_check(c, hipMemcpyAsync(buf.p, items.data(), sizeof(Item) * items.size(),
                                          hipMemcpyHostToDevice, c->stream),
                        "upload request items")) != EH_OK) {
      dev_free(c, buf);
      return st;
    }
    Plan p;
    p.pattern = uint32_t(pattern);
    p.staging = EH_STAGE_SOURCE;
    p.items = buf;
    p.n_items = n_list;
    p.item_dmax = item_dmax;
    if (pattern == EH_4CLIQUE)
      st = prepare_k4_lists(c, h, items.data(), n_list, lists, p.k4s_waves, p.k4s_stride);
    p.k4s = lists;
    if (st == EH_OK && n_list) st = enqueue_count(c, t, &p, 0, n_list, acc, 0, nullptr);
    for (uint32_t k = 0; st == EH_OK && k < kK4LocalClasses; ++k) {
      LaunchArgs la = base_args(c, t);
      la.items = static_cast<const Item*>(buf.p) + loff[k];
      la.n_items = loff[k + 1] - loff[k];
      la.acc = acc;
      la.tag_base = 0;
      st = launch_4cliques_local_items(c, c->stream, la, int(k));
    }
  }
  if (st == EH_OK) st = read_back(c, acc, total, 1);
  (void)hipStreamSynchronize(c->stream);
  dev_free(c, buf);
  dev_free(c, lists);
  return st;
}

static eh_status batch_enqueue(Ctx* c, Trie& t, int pattern, uint32_t first, uint32_t count,
                               unsigned long long* d_out) {
  if (pattern != EH_TRIANGLE && pattern != EH_4CLIQUE) {
    c->err = "pattern must be EH_TRIANGLE or EH_4CLIQUE";
    return EH_EINVAL;
  }
  const HostTrie& h = t.host;
  if (count == 0 || uint64_t(first) + count > h.n_graphs) {
    c->err = "graph range out of bounds";
    return EH_EINVAL;
  }
  Plan* p = nullptr;
  // per-graph tags need source staging, which also keeps graphs contiguous
  const uint32_t staging =
      pattern == EH_TRIANGLE ? tri_staging(c, t, false) : uint32_t(EH_STAGE_SOURCE);
  eh_status st = get_plan(c, &t, uint32_t(pattern), staging, &p);
  if (st != EH_OK) return st;
  if ((st = launch_fill_u64(c, c->stream, d_out, count, 0)) != EH_OK) return st;
  const uint64_t i0 = p->g_item_off[first], i1 = p->g_item_off[first + count];
  if (h.n_graphs == 1) return enqueue_count(c, t, p, i0, i1, d_out, 0, nullptr);
  return enqueue_count(c, t, p, i0, i1, d_out, first, nullptr);
}

eh_status eh_count_batch(eh_ctx* ctx, const eh_trie* batch, int pattern, uint32_t first,
                         uint32_t count, uint64_t* out_counts) {
  if (!ctx || !batch || !out_counts) return EH_EINVAL;
  Ctx* c = &ctx->c;
  eh_status st = ensure_acc(c, count);
  if (st != EH_OK) return st;
  Trie& t = const_cast<eh_trie*>(batch)->t;
  unsigned long long* acc = static_cast<unsigned long long*>(c->acc.p);
  if ((st = batch_enqueue(c, t, pattern, first, count, acc)) != EH_OK) return st;
  return read_back(c, acc, out_counts, count);
}

eh_status eh_count_batch_async(eh_ctx* ctx, const eh_trie* batch, int pattern, uint32_t first,
                               uint32_t count, uint64_t* d_out) {
  if (!ctx || !batch || !d_out) return EH_EINVAL;
  Trie& t = const_cast<eh_trie*>(batch)->t;
  return batch_enqueue(&ctx->c, t, pattern, first, count,
                       reinterpret_cast<unsigned long long*>(d_out));
}

// ---- host-only trie ------------------------------------------------------------

eh_status eh_host_trie_build(const uint32_t* src, const uint32_t* dst, uint64_t n_edges,
                             uint32_t n_vertices, const eh_build_opts* opts, eh_host_trie** out) {
  if (!out || (n_edges && (!src || !dst))) return EH_EINVAL;
  *out = nullptr;
  if (opts && (opts->layout > EH_LAYOUT_BITSET_ALL || opts->order > EH_ORDER_STRONG_RUNS))
    return EH_EINVAL;
  eh_host_trie* x = new (std::nothrow) eh_host_trie();
  if (!x) return EH_ENOMEM;
  std::string err;
  eh_status st;
  try {
    st = host_build(src, dst, n_edges, n_vertices, resolve_opts(opts), x->h, err);
  } catch (const std::bad_alloc&) {
    st = EH_ENOMEM;
  }
  if (st != EH_OK) {
    g_err_no_ctx = err;
    delete x;
    return st;
  }
  *out = x;
  return EH_OK;
}

eh_status eh_host_trie_info(const eh_host_trie* h, eh_trie_info* out) {
  if (!h || !out) return EH_EINVAL;
  fill_info(h->h, out);
  return EH_OK;
}

eh_status eh_host_trie_arrays(const eh_host_trie* x, uint32_t* rank, uint32_t* row, uint32_t* col,
                              uint32_t* bs_off, uint32_t* bs_base, uint32_t* bs_nw,
                              uint32_t* bs_words) {
  if (!x) return EH_EINVAL;
  const HostTrie& h = x->h;
  auto cp = [](uint32_t* dst, const std::vector<uint32_t>& v) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(uint32_t));
  };
  cp(rank, h.rank);
  cp(row, h.row);
  cp(col, h.col);
  cp(bs_off, h.bs_off);
  cp(bs_base, h.bs_base);
  cp(bs_nw, h.bs_nw);
  cp(bs_words, h.bs_words);
  return EH_OK;
}

eh_status eh_host_trie_free(eh_host_trie* h) {
  if (!h) return EH_EINVAL;
  delete h;
  return EH_OK;
}

}  // extern "C"
