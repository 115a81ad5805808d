// Set stores: the uint, bitset and composite layouts of section 4.3 at the
// relation, set and block granularities, and the C ABI of pairwise
// intersection over them.
#include <algorithm>
#include <cstring>
#include <new>

#include "eh_internal.h"

namespace eh {
namespace {

struct SetRule {
  uint32_t layout = EH_SETS_COMPOSITE;
  uint32_t bl = 8;         // log2 of the block size in ids
  uint32_t block_min = 8;  // composite: members that make a block dense
  float tau = 32.0f;
  uint32_t s_min = 1;
};

eh_status resolve(const eh_set_opts* o, SetRule& r, std::string& err) {
  if (!o) return EH_OK;
  if (o->layout > EH_SETS_COMPOSITE) {
    err = "unknown set layout";
    return EH_EINVAL;
  }
  const uint32_t bl = o->block_log ? o->block_log : 8;
  if (bl < 5 || bl > 16) {
    err = "block_log must be 0 or in [5, 16]";
    return EH_EINVAL;
  }
  r.layout = o->layout;
  r.bl = bl;
  r.block_min = o->block_min ? o->block_min : (1u << bl) / 32u;
  r.tau = o->tau > 0.0f ? o->tau : 32.0f;
  r.s_min = o->s_min ? o->s_min : 1;
  return EH_OK;
}

// Writers of one segment.  Members m[k0 .. k1) lie in blocks b0 .. b1.
struct Encoder {
  HostSets& h;
  const uint32_t* m;
  uint32_t wpb;           // words per block
  bool overflow = false;  // a run would take the words past 2^31 - 1

  void put_uint(uint32_t b0, uint32_t b1, uint64_t k0, uint64_t k1) {
    h.seg.push_back(uint4{b0, b1, uint32_t(h.vals.size()), uint32_t(k1 - k0)});
    h.vals.insert(h.vals.end(), m + k0, m + k1);
  }
  void put_bits(uint32_t b0, uint32_t b1, uint64_t k0, uint64_t k1) {
    const size_t w0 = h.words.size();
    const uint64_t nw = (uint64_t(b1) - b0 + 1) * wpb;
    if (w0 + nw > kMaxIndex) {
      overflow = true;
      return;
    }
    h.words.resize(w0 + nw, 0u);
    const uint32_t first_word = b0 * wpb;  // = (b0 << block_log) / 32
    for (uint64_t k = k0; k < k1; ++k) {
      const uint32_t x = m[k];
      h.words[w0 + ((x >> 5) - first_word)] |= 1u << (x & 31);
    }
    h.seg.push_back(uint4{b0, b1, uint32_t(w0), uint32_t(k1 - k0) | kHiBit});
    h.n_bitset_segs++;
    h.bitset_blocks += uint64_t(b1) - b0 + 1;
  }
};

// Segments of one set m[0 .. len), strictly ascending.
void encode_set(Encoder& e, uint64_t len, const SetRule& r) {
  if (len == 0) return;
  const uint32_t* m = e.m;
  const uint32_t bl = r.bl;
  const uint32_t first = m[0], last = m[len - 1];
  if (r.layout == EH_SETS_UINT) {
    e.put_uint(first >> bl, last >> bl, 0, len);
    return;
  }
  if (r.layout == EH_SETS_SET) {
    const double range = double(last) - double(first) + 1.0;
    const bool dense = len >= r.s_min && range <= double(r.tau) * double(len);
    if (dense) e.put_bits(first >> bl, last >> bl, 0, len);
    else e.put_uint(first >> bl, last >> bl, 0, len);
    return;
  }
  // bitset / composite: classify each non-empty block, then emit maximal runs
  // (dense blocks only while consecutive; sparse blocks across any gap)
  bool open = false, run_bits = false;
  uint32_t run_b0 = 0, run_b1 = 0;
  uint64_t run_k0 = 0;
  uint64_t k = 0;
  while (k < len) {
    const uint32_t b = m[k] >> bl;
    uint64_t e_k = k + 1;
    while (e_k < len && (m[e_k] >> bl) == b) ++e_k;
    const bool dense = r.layout == EH_SETS_BITSET || e_k - k >= r.block_min;
    const bool extend = open && dense == run_bits && (!dense || b == run_b1 + 1);
    if (!extend) {
      if (open) {
        if (run_bits) e.put_bits(run_b0, run_b1, run_k0, k);
        else e.put_uint(run_b0, run_b1, run_k0, k);
      }
      open = true;
      run_bits = dense;
      run_b0 = b;
      run_k0 = k;
    }
    run_b1 = b;
    k = e_k;
  }
  if (run_bits) e.put_bits(run_b0, run_b1, run_k0, len);
  else e.put_uint(run_b0, run_b1, run_k0, len);
}

void fill_info(const HostSets& h, eh_sets_info* out) {
  std::memset(out, 0, sizeof(*out));
  out->n_sets = h.n_sets;
  out->block_log = h.block_log;
  out->n_members = h.n_members;
  out->n_segments = h.seg.size();
  out->n_bitset_segments = h.n_bitset_segs;
  out->uint_members = h.vals.size();
  out->bitset_blocks = h.bitset_blocks;
  out->bitset_words = h.words.size();
}

eh_status upload_buf(Ctx* c, DevBuf& b, const void* src, size_t bytes, const char* what) {
  eh_status st = dev_alloc(c, b, bytes);
  if (st != EH_OK || bytes == 0) return st;
  return hip_check(c, hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice), what);
}

void free_sets(Sets& s) {
  dev_free(s.ctx, s.seg_off);
  dev_free(s.ctx, s.seg);
  dev_free(s.ctx, s.vals);
  dev_free(s.ctx, s.words);
}

uint32_t auto_lanes(const eh_sets_info& i) {
  const uint64_t mean = i.n_sets ? i.n_members / i.n_sets : 0;
  return mean < 48 ? 4u : mean < 512 ? 16u : 64u;
}

eh_status check_pairs_args(Ctx* c, const eh_sets* sets, uint64_t n_pairs, const uint32_t* d_pairs,
                           uint32_t lanes) {
  if (!sets || (n_pairs && !d_pairs)) {
    c->err = "null set store or pair array";
    return EH_EINVAL;
  }
  if (sets->s.ctx != c) {
    c->err = "the set store belongs to another context";
    return EH_EINVAL;
  }
  if (n_pairs > 0xFFFFFFFFull) {
    c->err = "at most 2^32 - 1 pairs per call";
    return EH_EINVAL;
  }
  if (lanes != 0 && lanes != 4 && lanes != 16 && lanes != 64) {
    c->err = "lanes must be 0, 4, 16 or 64";
    return EH_EINVAL;
  }
  return EH_OK;
}

}  // namespace

eh_status host_sets_build(uint32_t n_sets, const uint64_t* off, const uint32_t* members,
                          const eh_set_opts* opts, HostSets& h, std::string& err) {
  SetRule r;
  eh_status st = resolve(opts, r, err);
  if (st != EH_OK) return st;
  if (!off) {
    err = "null offsets";
    return EH_EINVAL;
  }
  if (off[0] != 0) {
    err = "off[0] must be 0";
    return EH_EINVAL;
  }
  for (uint32_t i = 0; i < n_sets; ++i)
    if (off[i + 1] < off[i]) {
      err = "offsets decrease at set " + std::to_string(i);
      return EH_EINVAL;
    }
  const uint64_t total = off[n_sets];
  if (total && !members) {
    err = "null members";
    return EH_EINVAL;
  }
  if (total > kMaxIndex) {
    err = "members exceed 2^31-1";
    return EH_EOVERFLOW;
  }
  for (uint32_t i = 0; i < n_sets; ++i)
    for (uint64_t k = off[i] + 1; k < off[i + 1]; ++k)
      if (members[k] <= members[k - 1]) {
        err = "set " + std::to_string(i) + " is not strictly ascending";
        return EH_EINVAL;
      }
  h = HostSets{};
  h.n_sets = n_sets;
  h.block_log = r.bl;
  h.n_members = total;
  h.seg_off.resize(size_t(n_sets) + 1);
  h.vals.reserve(r.layout == EH_SETS_BITSET ? 0 : total);
  const uint32_t wpb = 1u << (r.bl - 5);
  for (uint32_t i = 0; i < n_sets; ++i) {
    h.seg_off[i] = uint32_t(h.seg.size());
    Encoder e{h, members + off[i], wpb};
    encode_set(e, off[i + 1] - off[i], r);
    if (e.overflow || h.seg.size() > kMaxIndex || h.words.size() > kMaxIndex) {
      err = "segments or bitset words exceed 2^31-1";
      return EH_EOVERFLOW;
    }
  }
  h.seg_off[n_sets] = uint32_t(h.seg.size());
  return EH_OK;
}

}  // namespace eh

using namespace eh;

extern "C" {

eh_status eh_host_sets_build(uint32_t n_sets, const uint64_t* off, const uint32_t* members,
                             const eh_set_opts* opts, eh_host_sets** out) {
  if (!out) return EH_EINVAL;
  *out = nullptr;
  eh_host_sets* x = new (std::nothrow) eh_host_sets();
  if (!x) return EH_ENOMEM;
  std::string err;
  eh_status st;
  try {
    st = host_sets_build(n_sets, off, members, opts, x->h, err);
  } catch (const std::bad_alloc&) {
    err = "host memory exhausted while encoding the sets";
    st = EH_ENOMEM;
  }
  if (st != EH_OK) {
    set_no_ctx_error(err);
    delete x;
    return st;
  }
  *out = x;
  return EH_OK;
}

eh_status eh_host_sets_info(const eh_host_sets* h, eh_sets_info* out) {
  if (!h || !out) return EH_EINVAL;
  fill_info(h->h, out);
  return EH_OK;
}

eh_status eh_host_sets_arrays(const eh_host_sets* x, uint32_t* seg_off, uint32_t* seg,
                              uint32_t* vals, uint32_t* words) {
  if (!x) return EH_EINVAL;
  const HostSets& h = x->h;
  if (seg_off) std::memcpy(seg_off, h.seg_off.data(), h.seg_off.size() * sizeof(uint32_t));
  if (seg && !h.seg.empty()) std::memcpy(seg, h.seg.data(), h.seg.size() * sizeof(uint4));
  if (vals && !h.vals.empty()) std::memcpy(vals, h.vals.data(), h.vals.size() * sizeof(uint32_t));
  if (words && !h.words.empty())
    std::memcpy(words, h.words.data(), h.words.size() * sizeof(uint32_t));
  return EH_OK;
}

eh_status eh_host_sets_free(eh_host_sets* h) {
  if (!h) return EH_EINVAL;
  delete h;
  return EH_OK;
}

eh_status eh_sets_build(eh_ctx* ctx, uint32_t n_sets, const uint64_t* off, const uint32_t* members,
                        const eh_set_opts* opts, eh_sets** out) {
  if (!ctx || !out) return EH_EINVAL;
  *out = nullptr;
  Ctx* c = &ctx->c;
  eh_status st = hip_check(c, hipSetDevice(c->device), "hipSetDevice");
  if (st != EH_OK) return st;
  eh_sets* x = new (std::nothrow) eh_sets();
  if (!x) return EH_ENOMEM;
  Sets& s = x->s;
  s.ctx = c;
  try {
    HostSets h;
    st = host_sets_build(n_sets, off, members, opts, h, c->err);
    if (st == EH_OK) {
      fill_info(h, &s.info);
      st = upload_buf(c, s.seg_off, h.seg_off.data(), h.seg_off.size() * sizeof(uint32_t),
                      "upload segment offsets");
      if (st == EH_OK)
        st = upload_buf(c, s.seg, h.seg.data(), h.seg.size() * sizeof(uint4), "upload segments");
      if (st == EH_OK)
        st = upload_buf(c, s.vals, h.vals.data(), h.vals.size() * sizeof(uint32_t),
                        "upload members");
      if (st == EH_OK)
        st = upload_buf(c, s.words, h.words.data(), h.words.size() * sizeof(uint32_t),
                        "upload bitset words");
    }
  } catch (const std::bad_alloc&) {
    c->err = "host memory exhausted while encoding the sets";
    st = EH_ENOMEM;
  }
  if (st != EH_OK) {
    free_sets(s);
    delete x;
    return st;
  }
  s.info.device_bytes = s.seg_off.bytes + s.seg.bytes + s.vals.bytes + s.words.bytes;
  *out = x;
  return EH_OK;
}

eh_status eh_sets_info_get(const eh_sets* sets, eh_sets_info* out) {
  if (!sets || !out) return EH_EINVAL;
  *out = sets->s.info;
  return EH_OK;
}

eh_status eh_sets_free(eh_sets* sets) {
  if (!sets) return EH_EINVAL;
  (void)hipStreamSynchronize(sets->s.ctx->stream);
  free_sets(sets->s);
  delete sets;
  return EH_OK;
}

eh_status eh_intersect_pairs(eh_ctx* ctx, const eh_sets* sets, uint64_t n_pairs,
                             const uint32_t* d_pairs, uint32_t* d_counts, uint32_t lanes,
                             uint64_t* total) {
  if (!ctx || !total) return EH_EINVAL;
  Ctx* c = &ctx->c;
  eh_status st = check_pairs_args(c, sets, n_pairs, d_pairs, lanes);
  if (st != EH_OK) return st;
  if ((st = hip_check(c, hipSetDevice(c->device), "hipSetDevice")) != EH_OK) return st;
  if ((st = ensure_acc(c, 2)) != EH_OK) return st;
  if ((st = ensure_pinned(c, 2)) != EH_OK) return st;
  auto* acc = static_cast<unsigned long long*>(c->acc.p);
  if ((st = launch_fill_u64(c, c->stream, acc, 2, 0)) != EH_OK) return st;
  const uint32_t g = lanes ? lanes : auto_lanes(sets->s.info);
  if ((st = launch_intersect_pairs(c, c->stream, sets->s, n_pairs, d_pairs, d_counts, g, acc,
                                   acc + 1)) != EH_OK)
    return st;
  if ((st = hip_check(c, hipMemcpyAsync(c->pinned, acc, 2 * sizeof(uint64_t),
                                        hipMemcpyDeviceToHost, c->stream),
                      "copy result")) != EH_OK)
    return st;
  if ((st = hip_check(c, hipStreamSynchronize(c->stream), "stream sync")) != EH_OK) return st;
  if (c->pinned[1]) {
    c->err = "a pair names a set index >= n_sets";
    return EH_EINVAL;
  }
  *total = c->pinned[0];
  return EH_OK;
}

eh_status eh_intersect_pairs_async(eh_ctx* ctx, const eh_sets* sets, uint64_t n_pairs,
                                   const uint32_t* d_pairs, uint32_t* d_counts, uint32_t lanes,
                                   uint64_t* d_total) {
  if (!ctx || !d_total) return EH_EINVAL;
  Ctx* c = &ctx->c;
  eh_status st = check_pairs_args(c, sets, n_pairs, d_pairs, lanes);
  if (st != EH_OK) return st;
  if ((st = hip_check(c, hipSetDevice(c->device), "hipSetDevice")) != EH_OK) return st;
  const uint32_t g = lanes ? lanes : auto_lanes(sets->s.info);
  return launch_intersect_pairs(c, c->stream, sets->s, n_pairs, d_pairs, d_counts, g,
                                reinterpret_cast<unsigned long long*>(d_total), nullptr);
}

}  // extern "C"
