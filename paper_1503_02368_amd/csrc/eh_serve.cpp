// Serving: rooted triangle / 4-clique count requests against a resident trie.
//
// A request asks for the instances whose root (smallest-rank vertex) lies in
// a given vertex set -- an equality selection on the first attribute of the
// join, which the trie answers by starting Generic-Join's outer loop only at
// those vertices (appendix B.1 pushes such selections first).  Its work is
// the source-staged items of each root.
//
// Submission only validates and copies the roots.  Expansion workers then
// turn each request into work items (drop repeated roots, cut each root's
// out-list into items), in parallel with one another and with the device,
// and queue it for admission.  When a request could exceed the whole budget
// (known from the item count with every vertex a root), the submitting
// thread expands it itself, so that such a request is refused at submission.
//
// Continuous batching: a progress thread repeatedly (1) admits queued
// requests in arrival order while their work items fit the server's HBM
// arena (hbm_budget_bytes, first fit) and a counter slot is free, uploading
// each admitted request's items into its extent of the arena, (2) chooses up
// to step_items of the active requests' items, oldest request first (or, by
// option, those with the fewest items left first), which a gather kernel
// copies from the arena into the step's item list, (3) runs them as one
// device step (one launch per pattern, more for 4-cliques with roots of high
// out-degree) that adds into per-slot counters, and (4) retires every request
// whose items have all completed, freeing its extent.  Requests that
// arrive while a step runs join the next step; their work shares launches with
// requests admitted earlier.  The step after the one that finishes a request
// never waits for that request to be polled.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <ctime>
#include <iterator>
#include <map>

#include "eh_internal.h"

namespace eh {
namespace {

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return uint64_t(ts.tv_sec) * 1000000000ull + uint64_t(ts.tv_nsec);
}

struct Request {
  uint64_t ticket = 0;
  int pattern = 0;
  std::vector<uint32_t> roots;  // as submitted, until expanded
  std::vector<Item> items;  // tag filled at admission
  // 4-cliques: items[off[0] .. off[1]) go to the staged S-list kernel, and
  // items[off[1+k] .. off[2+k]) are whole roots of induced-neighbourhood class k
  uint64_t off[kK4LocalClasses + 2] = {};
  uint32_t item_dmax = 0;   // max out-degree of an item's root (S-list items)
  uint64_t footprint = 0;   // bytes its items take in the arena
  uint64_t arena_off = 0;   // item index of its extent in the arena
  uint64_t next_item = 0;   // next item to dispatch
  uint64_t done_items = 0;  // items whose step completed
  uint32_t slot = 0;
  bool zeroed = false;
  uint64_t count = 0;
  eh_req_stats stats{};
  bool finished = false;
};

}  // namespace

struct Server {
  Ctx* c = nullptr;
  Trie* t = nullptr;
  eh_server_opts o{};
  hipStream_t stream = nullptr;
  // the induced-neighbourhood classes of a step run beside its other launches
  // on streams of their own (default priority), forked from and joined back
  // into `stream` by events
  hipStream_t side[kK4LocalClasses] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kK4LocalClasses] = {};
  Tuning tune;             // the context's tuning when the server was created
  DevBuf cursor;           // work cursors of the server's own launches
  DevBuf items_d;          // step_items Items
  DevBuf acc_d;            // max_active uint64
  DevBuf arena;             // admitted requests' work items (hbm_budget_bytes)
  std::map<uint64_t, uint64_t> free_ext;  // free arena extents: first item -> items
  DevBuf pieces_d;         // per step: {first arena item, first step item, items, 0}
  uint4* pieces_h = nullptr;
  DevBuf k4s;              // 4-clique S lists in HBM, when some out-degree exceeds kK4ListMax
  uint32_t k4s_waves = 0, k4s_stride = 0;
  uint64_t* acc_h = nullptr;
  std::mutex mu;
  std::condition_variable cv_work;   // progress thread waits for work
  std::condition_variable cv_done;   // eh_wait waits for completions
  std::deque<std::shared_ptr<Request>> queue;
  std::vector<std::shared_ptr<Request>> active;  // by admission order
  std::unordered_map<uint64_t, std::shared_ptr<Request>> by_ticket;
  std::vector<uint32_t> free_slots;
  uint64_t footprint = 0;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::string fatal;  // first device error; every later request fails
  std::thread th;
  std::deque<std::shared_ptr<Request>> done;  // finished, in completion order
  // root de-duplication: a stamp per vertex, one table per expanding thread
  struct Dedup {
    std::vector<uint32_t> stamp;
    uint32_t epoch = 0;
  };
  std::mutex sync_mu;                          // guards sync_dedup
  Dedup sync_dedup;                            // expansion in eh_submit
  std::vector<Dedup> dedup;                    // one per worker
  std::deque<std::shared_ptr<Request>> incoming;  // submitted, not yet expanded
  std::condition_variable cv_incoming;
  std::vector<std::thread> workers;
  uint32_t chunk = 4096;                       // item size target, fixed at creation
  uint64_t arena_items = 0;                    // the arena's capacity in items
  bool async_ok[5] = {false, false, false, false, false};  // by pattern
  bool k4_local = false;   // 4-clique roots of out-degree <= 512 by induced neighbourhoods

  void run();
  bool step();
  bool arena_take(uint64_t n_items, uint64_t& off);
  void arena_give(uint64_t off, uint64_t n_items);
  void expand(Request& r, Dedup& d) const;
  void expand_loop(uint32_t w);
  void enqueue_expanded(const std::shared_ptr<Request>& r);  // caller holds mu
};

namespace {

// pattern: EH_TRIANGLE, EH_4CLIQUE (S-list kernel), or -1 - k for the
// induced-neighbourhood 4-clique kernel of class k (on ks when given)
eh_status server_launch(Server* s, uint64_t n_items, uint64_t off, int pattern,
                        uint32_t item_dmax, hipStream_t ks = nullptr) {
  if (n_items == 0) return EH_OK;
  Ctx* c = s->c;
  Trie& t = *s->t;
  LaunchArgs a;
  a.vdesc = static_cast<const uint2*>(t.vdesc.p);
  a.col = static_cast<const uint32_t*>(t.col.p);
  a.bsdesc = static_cast<const uint4*>(t.bsdesc.p);
  a.bsw = static_cast<const uint32_t*>(t.col.p);  // words live after col
  a.vert = static_cast<const uint32_t*>(t.vert.p);
  a.idx = static_cast<const uint32_t*>(t.col.p);
  a.items = static_cast<const Item*>(s->items_d.p) + off;
  a.n_items = n_items;
  a.acc = static_cast<unsigned long long*>(s->acc_d.p);
  a.tag_base = 0;
  const Tuning& tu = s->tune;
  a.use_bitsets = tu.use_bitsets && t.host.n_bs > 0;
  a.dynamic = tu.dynamic;
  a.grab = tu.grab;
  a.cursor = static_cast<uint32_t*>(s->cursor.p);
  a.k4s = static_cast<uint32_t*>(s->k4s.p);
  a.k4s_stride = s->k4s_stride;
  a.k4s_waves = s->k4s_waves;
  a.algo = tu.algo;
  a.gamma = tu.gamma;
  a.group_lanes = tu.group_lanes;
  a.dmax = t.host.dmax;
  a.item_dmax = item_dmax;
  a.stage_words = tu.stage_words;
  a.xcds = tu.xcds;
  a.unroll = tu.unroll;
  a.search_below = tu.search_below;
  a.symmetric = t.host.symmetric ? 1u : 0u;
  a.reverse = tu.reverse;
  if (pattern < 0) return launch_4cliques_local_items(c, ks ? ks : s->stream, a, -1 - pattern);
  if (pattern == EH_4CLIQUE) return launch_4cliques(c, s->stream, a, tu.kernel, tu.waves_per_cu);
  return launch_triangles(c, s->stream, a, tu.kernel, tu.waves_per_cu);
}

}  // namespace

// The server's streams and events, after their work has drained.
void destroy_streams(Server& s) {
  for (uint32_t q = 0; q < kK4LocalClasses; ++q) {
    if (s.side[q]) {
      (void)hipStreamSynchronize(s.side[q]);
      (void)hipStreamDestroy(s.side[q]);
    }
    if (s.join[q]) (void)hipEventDestroy(s.join[q]);
  }
  if (s.fork) (void)hipEventDestroy(s.fork);
  if (s.stream) (void)hipStreamDestroy(s.stream);
}

// First fit over the free extents of the arena (in items).
bool Server::arena_take(uint64_t n_items, uint64_t& off) {
  for (auto it = free_ext.begin(); it != free_ext.end(); ++it) {
    if (it->second < n_items) continue;
    off = it->first;
    const uint64_t rest = it->second - n_items;
    free_ext.erase(it);
    if (rest) free_ext.emplace(off + n_items, rest);
    return true;
  }
  return false;
}

// Returns an extent, merged with free neighbours.
void Server::arena_give(uint64_t off, uint64_t n_items) {
  auto next = free_ext.lower_bound(off);
  if (next != free_ext.end() && off + n_items == next->first) {
    n_items += next->second;
    next = free_ext.erase(next);
  }
  if (next != free_ext.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      prev->second += n_items;
      return;
    }
  }
  free_ext.emplace(off, n_items);
}

// One device step.  Returns false when there is nothing to do.
bool Server::step() {
  std::vector<std::shared_ptr<Request>> batch_reqs;
  std::vector<uint32_t> to_zero;
  std::vector<Request*> admitted;
  std::vector<uint4> tri, k4;  // pieces {first arena item, first step item, items, 0}
  std::vector<uint4> kl[kK4LocalClasses];  // the same for the induced-neighbourhood classes
  uint64_t n_tri = 0, n_k4 = 0, n_kl[kK4LocalClasses] = {};
  uint32_t dmax_tri = 0, dmax_k4 = 0;
  // requests stay alive in `active` until this thread retires them
  std::vector<std::pair<Request*, uint64_t>> dispatched;
  {
    std::unique_lock<std::mutex> lk(mu);
    // admission, arrival order: the request's items must fit the arena (a
    // request larger than the whole arena was refused at submission)
    while (!queue.empty() && !free_slots.empty() && !stop) {
      auto& r = queue.front();
      uint64_t off = 0;
      if (!arena_take(r->items.size(), off)) break;
      r->arena_off = off;
      r->slot = free_slots.back();
      free_slots.pop_back();
      for (auto& it : r->items) it.tag = r->slot;
      r->stats.t_admit_ns = now_ns();
      footprint += r->footprint;
      active.push_back(r);
      admitted.push_back(r.get());
      queue.pop_front();
    }
    if (active.empty()) return false;
    // gather items: oldest request first, or (EH_SERVE_SHORTEST) the
    // requests with the fewest items left first, ties by age
    std::vector<Request*> order;
    order.reserve(active.size());
    for (auto& r : active) order.push_back(r.get());
    if (o.policy == EH_SERVE_SHORTEST)
      std::stable_sort(order.begin(), order.end(), [](const Request* x, const Request* y) {
        return x->items.size() - x->next_item < y->items.size() - y->next_item;
      });
    uint64_t budget = o.step_items;
    for (Request* r : order) {
      if (!r->zeroed) {
        to_zero.push_back(r->slot);
        r->zeroed = true;
      }
      const uint64_t take = std::min<uint64_t>(budget, r->items.size() - r->next_item);
      if (take && r->pattern != EH_4CLIQUE) {
        dmax_tri = std::max(dmax_tri, r->item_dmax);
        tri.push_back(make_uint4(uint32_t(r->arena_off + r->next_item), uint32_t(n_tri),
                                 uint32_t(take), 0u));
        n_tri += take;
      } else if (take) {
        // the taken range, cut at the request's kernel regions
        const uint64_t a0 = r->next_item, a1 = a0 + take;
        for (uint32_t q = 0; q <= kK4LocalClasses; ++q) {
          const uint64_t lo = std::max(a0, r->off[q]), hi = std::min(a1, r->off[q + 1]);
          if (lo >= hi) continue;
          auto& dst = q == 0 ? k4 : kl[q - 1];
          uint64_t& filled = q == 0 ? n_k4 : n_kl[q - 1];
          if (q == 0) dmax_k4 = std::max(dmax_k4, r->item_dmax);
          dst.push_back(make_uint4(uint32_t(r->arena_off + lo), uint32_t(filled),
                                   uint32_t(hi - lo), 0u));
          filled += hi - lo;
        }
      }
      r->next_item += take;
      budget -= take;
      dispatched.emplace_back(r, take);
      if (budget == 0) break;
    }
  }
  // device step: upload the newly admitted requests' items into their
  // extents, zero new slots, gather the step's items from the arena, launch,
  // read counters.  The items of an active request stay in host memory
  // until it retires, so the uploads can be asynchronous.
  eh_status st = EH_OK;
  Item* arena_items = static_cast<Item*>(arena.p);
  for (Request* r : admitted)
    if (st == EH_OK)
      st = hip_check(c, hipMemcpyAsync(arena_items + r->arena_off, r->items.data(),
                                       r->items.size() * sizeof(Item), hipMemcpyHostToDevice,
                                       stream), "upload request items");
  for (uint32_t slot : to_zero)
    if (st == EH_OK)
      st = launch_fill_u64(c, stream, static_cast<unsigned long long*>(acc_d.p) + slot, 1, 0);
  // step items: the triangles', the S-list 4-cliques', then each class's
  uint64_t base[kK4LocalClasses + 2] = {0, n_tri};
  for (uint32_t q = 0; q < kK4LocalClasses; ++q) base[q + 2] = base[q + 1] + (q ? n_kl[q - 1] : n_k4);
  for (uint4& pc : k4) pc.y += uint32_t(base[1]);
  for (uint32_t q = 0; q < kK4LocalClasses; ++q)
    for (uint4& pc : kl[q]) pc.y += uint32_t(base[q + 2]);
  size_t n_pieces = tri.size() + k4.size();
  for (auto& v : kl) n_pieces += v.size();
  if (st == EH_OK && n_pieces) {
    uint4* ph = pieces_h;
    ph = std::copy(tri.begin(), tri.end(), ph);
    ph = std::copy(k4.begin(), k4.end(), ph);
    for (auto& v : kl) ph = std::copy(v.begin(), v.end(), ph);
    st = hip_check(c, hipMemcpyAsync(pieces_d.p, pieces_h, n_pieces * sizeof(uint4),
                                     hipMemcpyHostToDevice, stream), "upload step pieces");
    if (st == EH_OK)
      st = launch_gather_items(c, stream, arena_items, static_cast<const uint4*>(pieces_d.p),
                               uint32_t(n_pieces), static_cast<Item*>(items_d.p));
  }
  // the induced-neighbourhood classes start on their own streams once the
  // gather is done; the triangle and S-list launches (which share the work
  // cursors) follow one another on the server's stream
  bool forked = false;
  for (uint32_t q = 0; q < kK4LocalClasses && st == EH_OK; ++q) {
    if (!n_kl[q]) continue;
    if (!forked) {
      st = hip_check(c, hipEventRecord(fork, stream), "fork event");
      forked = st == EH_OK;
    }
    if (st == EH_OK) st = hip_check(c, hipStreamWaitEvent(side[q], fork, 0), "fork wait");
    if (st == EH_OK) st = server_launch(this, n_kl[q], base[q + 2], -1 - int(q), 0, side[q]);
    if (st == EH_OK) st = hip_check(c, hipEventRecord(join[q], side[q]), "join event");
  }
  if (st == EH_OK) st = server_launch(this, n_tri, 0, EH_TRIANGLE, dmax_tri);
  if (st == EH_OK) st = server_launch(this, n_k4, base[1], EH_4CLIQUE, dmax_k4);
  for (uint32_t q = 0; q < kK4LocalClasses && st == EH_OK; ++q)
    if (n_kl[q]) st = hip_check(c, hipStreamWaitEvent(stream, join[q], 0), "join wait");
  if (st == EH_OK)
    st = hip_check(c, hipMemcpyAsync(acc_h, acc_d.p, o.max_active * sizeof(uint64_t),
                                     hipMemcpyDeviceToHost, stream), "read counters");
  if (st == EH_OK) st = hip_check(c, hipStreamSynchronize(stream), "step sync");
  {
    std::unique_lock<std::mutex> lk(mu);
    if (st != EH_OK && fatal.empty()) fatal = c->err.empty() ? "device step failed" : c->err;
    for (auto& d : dispatched) d.first->done_items += d.second;
    const uint64_t t_done = now_ns();
    std::vector<std::shared_ptr<Request>> keep;
    for (auto& r : active) {
      if (r->done_items == r->items.size() || !fatal.empty()) {
        r->count = acc_h[r->slot];
        r->stats.t_done_ns = t_done;
        r->finished = true;
        footprint -= r->footprint;
        arena_give(r->arena_off, r->items.size());
        free_slots.push_back(r->slot);
        std::vector<Item>().swap(r->items);
        done.push_back(r);
      } else {
        keep.push_back(r);
      }
    }
    active.swap(keep);
  }
  cv_done.notify_all();
  return true;
}

void Server::run() {
  (void)hipSetDevice(c->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
      if (stop && active.empty()) {
        // cancel what was never admitted
        for (auto& r : queue) {
          r->finished = true;
          r->count = 0;
          r->stats.t_done_ns = now_ns();
          by_ticket.erase(r->ticket);
        }
        queue.clear();
        cv_done.notify_all();
        return;
      }
    }
    step();
  }
}

// Turns r.roots into work items: repeated roots are dropped with a stamp per
// vertex, and each root's out-list is cut into items whose size is estimated
// from its out-degree alone, so the cost is proportional to the roots.  The
// per-vertex tables are read at random: each pass prefetches a fixed distance
// ahead so that the cache misses of many roots overlap.
void Server::expand(Request& r, Dedup& d) const {
  const HostTrie& h = t->host;
  const uint32_t n_roots = uint32_t(r.roots.size());
  constexpr uint32_t kAhead = 24;
  std::vector<uint32_t> us(n_roots);
  const uint32_t* rank = h.rank.data();
  const uint32_t* roots = r.roots.data();
  for (uint32_t i = 0; i < n_roots; ++i) {
    if (i + kAhead < n_roots) __builtin_prefetch(rank + roots[i + kAhead]);
    us[i] = rank[roots[i]];
  }
  r.items.reserve(size_t(n_roots) + n_roots / 4);
  if (++d.epoch == 0) {
    std::fill(d.stamp.begin(), d.stamp.end(), 0u);
    d.epoch = 1;
  }
  uint32_t* stamp = d.stamp.data();
  const uint32_t* row = h.row.data();
  const bool local = k4_local && r.pattern == EH_4CLIQUE;
  std::vector<Item> lc[kK4LocalClasses];  // whole roots by induced-neighbourhood class
  for (uint32_t i = 0; i < n_roots; ++i) {
    if (i + kAhead < n_roots) {
      __builtin_prefetch(stamp + us[i + kAhead], 1);
      __builtin_prefetch(row + us[i + kAhead]);
    }
    const uint32_t u = us[i];
    if (stamp[u] == d.epoch) continue;
    stamp[u] = d.epoch;
    const int k = local ? k4_local_class(row[u + 1] - row[u]) : -1;
    if (k >= 0) {
      lc[k].push_back(Item{u, row[u], row[u + 1] - row[u], 0});
      continue;
    }
    const size_t before = r.items.size();
    make_items_estimated(h, u, 0, chunk, uint32_t(r.pattern), r.items);
    if (r.items.size() > before) r.item_dmax = std::max(r.item_dmax, row[u + 1] - row[u]);
  }
  r.off[0] = 0;
  r.off[1] = r.items.size();
  for (uint32_t k = 0; k < kK4LocalClasses; ++k) {
    r.items.insert(r.items.end(), lc[k].begin(), lc[k].end());
    r.off[k + 2] = r.items.size();
  }
  r.stats.items = r.items.size();
  r.footprint = sizeof(Item) * r.items.size();
  std::vector<uint32_t>().swap(r.roots);
}

void Server::enqueue_expanded(const std::shared_ptr<Request>& r) {
  if (r->items.empty()) {
    // no instance can be rooted here: done without device work
    r->finished = true;
    r->stats.t_admit_ns = r->stats.t_done_ns = now_ns();
    done.push_back(r);
  } else {
    queue.push_back(r);
  }
}

void Server::expand_loop(uint32_t w) {
  for (;;) {
    std::shared_ptr<Request> r;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_incoming.wait(lk, [&] { return stop || !incoming.empty(); });
      if (stop) return;  // eh_server_destroy cancels what is left
      r = incoming.front();
      incoming.pop_front();
    }
    expand(*r, dedup[w]);
    {
      std::unique_lock<std::mutex> lk(mu);
      if (stop) {
        r->finished = true;
        r->count = 0;
        r->stats.t_done_ns = now_ns();
        by_ticket.erase(r->ticket);
      } else {
        enqueue_expanded(r);
      }
    }
    cv_work.notify_one();
    cv_done.notify_all();
  }
}

}  // namespace eh

struct eh_server {
  eh::Server s;
};

using namespace eh;

extern "C" {

eh_status eh_server_create(eh_ctx* ctx, const eh_trie* resident, const eh_server_opts* opts,
                           eh_server** out) {
  if (!ctx || !resident || !out) return EH_EINVAL;
  *out = nullptr;
  Ctx* c = &ctx->c;
  Trie* t = &const_cast<eh_trie*>(resident)->t;
  if (t->host.n_graphs != 1) {
    c->err = "a server needs a single-graph trie";
    return EH_ESTATE;
  }
  eh_server* x = new (std::nothrow) eh_server();
  if (!x) return EH_ENOMEM;
  Server& s = x->s;
  s.c = c;
  s.t = t;
  s.tune = c->tune;
  s.k4_local = s.tune.k4_local && !t->host.symmetric;
  if (opts) s.o = *opts;
  if (!s.o.hbm_budget_bytes) s.o.hbm_budget_bytes = 2ull << 30;
  if (!s.o.max_active) s.o.max_active = 256;
  if (!s.o.max_queued) s.o.max_queued = 4096;
  if (!s.o.step_items) s.o.step_items = 1 << 18;
  eh_status st = hip_check(c, hipSetDevice(c->device), "hipSetDevice");
  if (st == EH_OK)
    st = hip_check(c, hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking), "server stream");
  for (uint32_t q = 0; q < kK4LocalClasses && st == EH_OK; ++q) {
    st = hip_check(c, hipStreamCreateWithFlags(&s.side[q], hipStreamNonBlocking), "server stream");
    if (st == EH_OK)
      st = hip_check(c, hipEventCreateWithFlags(&s.join[q], hipEventDisableTiming), "join event");
  }
  if (st == EH_OK)
    st = hip_check(c, hipEventCreateWithFlags(&s.fork, hipEventDisableTiming), "fork event");
  if (st == EH_OK) st = dev_alloc(c, s.items_d, sizeof(Item) * s.o.step_items);
  if (st == EH_OK) st = dev_alloc(c, s.acc_d, sizeof(uint64_t) * s.o.max_active);
  if (st == EH_OK) st = dev_alloc(c, s.cursor, sizeof(uint32_t) * kCursorWords * kMaxParts);
  if (st == EH_OK && t->host.dmax > kK4ListMax) {
    // 4-clique requests rooted at hubs keep S in HBM: lists for 4 waves per
    // compute unit, each as long as the largest out-degree
    s.k4s_waves = 4 * uint32_t(c->n_cu);
    s.k4s_stride = t->host.dmax;
    st = dev_alloc(c, s.k4s, sizeof(uint32_t) * size_t(s.k4s_stride) * s.k4s_waves);
  }
  s.arena_items = s.o.hbm_budget_bytes / sizeof(Item);
  if (st == EH_OK && s.arena_items > 0xFFFFFFFFull) {
    c->err = "hbm_budget_bytes above 64 GiB (2^32 work items)";
    st = EH_EINVAL;
  }
  if (st == EH_OK && s.arena_items == 0) {
    c->err = "hbm_budget_bytes holds no work item";
    st = EH_EINVAL;
  }
  if (st == EH_OK) st = dev_alloc(c, s.arena, s.arena_items * sizeof(Item));
  if (st == EH_OK) s.free_ext.emplace(0, s.arena_items);
  // a step takes one range of each active request, cut into at most one
  // piece per kernel region
  const size_t max_pieces = size_t(s.o.max_active) * (kK4LocalClasses + 1);
  if (st == EH_OK) st = dev_alloc(c, s.pieces_d, sizeof(uint4) * max_pieces);
  if (st == EH_OK)
    st = hip_check(c, hipHostMalloc((void**)&s.pieces_h, sizeof(uint4) * max_pieces,
                                    hipHostMallocDefault), "pinned pieces");
  if (st == EH_OK)
    st = hip_check(c, hipHostMalloc((void**)&s.acc_h, sizeof(uint64_t) * s.o.max_active,
                                    hipHostMallocDefault), "pinned counters");
  if (st != EH_OK) {
    dev_free(c, s.items_d);
    dev_free(c, s.acc_d);
    dev_free(c, s.cursor);
    dev_free(c, s.k4s);
    dev_free(c, s.arena);
    dev_free(c, s.pieces_d);
    if (s.pieces_h) (void)hipHostFree(s.pieces_h);
    if (s.acc_h) (void)hipHostFree(s.acc_h);
    destroy_streams(s);
    delete x;
    return st;
  }
  for (uint32_t i = s.o.max_active; i-- > 0;) s.free_slots.push_back(i);
  const HostTrie& h = t->host;
  s.chunk = std::max<uint32_t>(s.tune.chunk_work, 64);
  // the items with every vertex a root bound any request's footprint: when
  // that fits the budget, no request can be refused for its size, and
  // submission can leave the expansion to the workers
  for (uint32_t p : {uint32_t(EH_TRIANGLE), uint32_t(EH_4CLIQUE)}) {
    uint64_t all = 0;
    for (uint32_t u = 0; u < h.n; ++u) all += count_items_estimated(h, u, s.chunk, p);
    s.async_ok[p] = all <= s.arena_items;
  }
  const uint32_t hw = std::max(1u, std::thread::hardware_concurrency());
  const uint32_t n_workers = std::min(4u, std::max(1u, hw / 4));
  try {
    s.sync_dedup.stamp.assign(h.n, 0u);
    s.dedup.resize(n_workers);
    for (auto& d : s.dedup) d.stamp.assign(h.n, 0u);
  } catch (const std::bad_alloc&) {
    dev_free(c, s.items_d);
    dev_free(c, s.acc_d);
    dev_free(c, s.cursor);
    dev_free(c, s.k4s);
    dev_free(c, s.arena);
    dev_free(c, s.pieces_d);
    (void)hipHostFree(s.pieces_h);
    (void)hipHostFree(s.acc_h);
    destroy_streams(s);
    delete x;
    return EH_ENOMEM;
  }
  s.th = std::thread([&s] { s.run(); });
  for (uint32_t w = 0; w < n_workers; ++w) s.workers.emplace_back([&s, w] { s.expand_loop(w); });
  *out = x;
  return EH_OK;
}

eh_status eh_submit(eh_server* srv, int pattern, const uint32_t* roots, uint32_t n_roots,
                    uint64_t* ticket) {
  if (!srv || !roots || !ticket || n_roots == 0) return EH_EINVAL;
  if (pattern != EH_TRIANGLE && pattern != EH_4CLIQUE) return EH_EINVAL;
  Server& s = srv->s;
  const HostTrie& h = s.t->host;
  auto r = std::make_shared<Request>();
  r->pattern = pattern;
  r->stats.t_submit_ns = now_ns();
  for (uint32_t i = 0; i < n_roots; ++i)
    if (roots[i] >= h.n) return EH_EINVAL;
  r->roots.assign(roots, roots + n_roots);
  const bool async = s.async_ok[pattern];
  if (!async) {
    {
      std::lock_guard<std::mutex> lk(s.sync_mu);
      s.expand(*r, s.sync_dedup);
    }
    if (r->items.size() > s.arena_items) return EH_ENOMEM;
  }
  {
    std::unique_lock<std::mutex> lk(s.mu);
    if (s.stop) return EH_ESTATE;
    if (!s.fatal.empty()) return EH_EHIP;
    if (s.queue.size() + s.incoming.size() >= s.o.max_queued) return EH_EBUSY;
    r->ticket = s.next_ticket++;
    *ticket = r->ticket;
    s.by_ticket[r->ticket] = r;
    if (async)
      s.incoming.push_back(r);
    else
      s.enqueue_expanded(r);
  }
  if (async) {
    s.cv_incoming.notify_one();
  } else {
    s.cv_work.notify_one();
    s.cv_done.notify_all();
  }
  return EH_OK;
}

static eh_status take_result(Server& s, uint64_t ticket, uint64_t* count, eh_req_stats* stats) {
  auto itr = s.by_ticket.find(ticket);
  if (itr == s.by_ticket.end()) return EH_ENOTFOUND;
  auto& r = itr->second;
  if (!r->finished) return EH_PENDING;
  if (!s.fatal.empty()) {
    s.by_ticket.erase(itr);
    return EH_EHIP;
  }
  if (count) *count = r->count;
  if (stats) *stats = r->stats;
  s.by_ticket.erase(itr);
  return EH_OK;
}

eh_status eh_poll(eh_server* srv, uint64_t ticket, uint64_t* count, eh_req_stats* stats) {
  if (!srv) return EH_EINVAL;
  Server& s = srv->s;
  std::unique_lock<std::mutex> lk(s.mu);
  return take_result(s, ticket, count, stats);
}

eh_status eh_wait(eh_server* srv, uint64_t ticket, uint32_t timeout_ms, uint64_t* count,
                  eh_req_stats* stats) {
  if (!srv) return EH_EINVAL;
  Server& s = srv->s;
  std::unique_lock<std::mutex> lk(s.mu);
  const auto deadline = std::chrono::steady_clock::now() + std::chrono::milliseconds(timeout_ms);
  for (;;) {
    const eh_status st = take_result(s, ticket, count, stats);
    if (st != EH_PENDING) return st;
    if (s.cv_done.wait_until(lk, deadline) == std::cv_status::timeout) {
      return take_result(s, ticket, count, stats);
    }
  }
}

eh_status eh_server_drain(eh_server* srv, uint32_t cap, uint32_t timeout_ms, uint64_t* tickets,
                          uint64_t* counts, eh_req_stats* stats, uint32_t* n_out) {
  if (!srv || !tickets || !counts || !n_out || cap == 0) return EH_EINVAL;
  Server& s = srv->s;
  std::unique_lock<std::mutex> lk(s.mu);
  *n_out = 0;
  const auto deadline = std::chrono::steady_clock::now() + std::chrono::milliseconds(timeout_ms);
  for (;;) {
    uint32_t n = 0;
    while (n < cap && !s.done.empty()) {
      std::shared_ptr<Request> r = s.done.front();
      s.done.pop_front();
      auto itr = s.by_ticket.find(r->ticket);
      if (itr == s.by_ticket.end()) continue;  // already retired by eh_poll / eh_wait
      s.by_ticket.erase(itr);
      tickets[n] = r->ticket;
      counts[n] = r->count;
      if (stats) stats[n] = r->stats;
      ++n;
    }
    if (n > 0) {
      *n_out = n;
      return s.fatal.empty() ? EH_OK : EH_EHIP;
    }
    if (!s.fatal.empty()) return EH_EHIP;
    if (s.cv_done.wait_until(lk, deadline) == std::cv_status::timeout) return EH_OK;
  }
}

eh_status eh_server_destroy(eh_server* srv) {
  if (!srv) return EH_EINVAL;
  Server& s = srv->s;
  {
    std::unique_lock<std::mutex> lk(s.mu);
    s.stop = true;
  }
  s.cv_incoming.notify_all();
  s.cv_work.notify_all();
  for (auto& w : s.workers)
    if (w.joinable()) w.join();
  if (s.th.joinable()) s.th.join();
  {
    // cancel what was never expanded
    std::unique_lock<std::mutex> lk(s.mu);
    for (auto& r : s.incoming) {
      r->finished = true;
      r->count = 0;
      r->stats.t_done_ns = now_ns();
      s.by_ticket.erase(r->ticket);
    }
    s.incoming.clear();
  }
  s.cv_done.notify_all();
  (void)hipStreamSynchronize(s.stream);
  dev_free(s.c, s.items_d);
  dev_free(s.c, s.acc_d);
  dev_free(s.c, s.cursor);
  dev_free(s.c, s.k4s);
  dev_free(s.c, s.arena);
  dev_free(s.c, s.pieces_d);
  if (s.pieces_h) (void)hipHostFree(s.pieces_h);
  if (s.acc_h) (void)hipHostFree(s.acc_h);
  destroy_streams(s);
  delete srv;
  return EH_OK;
}

}  // extern "C"
