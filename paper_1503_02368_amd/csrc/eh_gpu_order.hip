// Traversal node orderings on the GPU (appendix A, "node ordering"): the
// label sequence of BFS, of the hybrid (BFS, then a stable sort by degree
// descending) and of strong runs, computed from the deduplicated edges of a
// single graph without a sequential traversal.
//
// Vertices are visited in the order pos = (degree descending, id ascending).
//
// Strong runs: at its visit a vertex takes the next label if it has none,
// then its unlabelled neighbours take the next labels in ascending id.  So a
// vertex w is labelled at the first visit among w and its neighbours,
// event(w) = min(pos(w), min over neighbours x of pos(x)): by itself when
// that is pos(w), else as a neighbour.  Labels follow (event, by-itself
// first, id), one sort.
//
// BFS: each traversal starts at the unvisited vertex of smallest pos, and a
// dequeued vertex appends its unvisited neighbours in ascending id.  So the
// traversals are the connected components in the order of their smallest pos
// (found by propagating minima along edges), each component's labels form
// one contiguous block, and within a component the labels go level by level;
// a vertex of level L+1 is appended by its level-L neighbour of smallest
// label, so level L+1 is ordered by (that label, id).  All components advance
// one level per step; sorting a level by (parent label, id) also groups it by
// component, since the components' label blocks are ordered the same way.
#include <cstring>  // rocPRIM's headers use memset on the host
#include <hip/hip_runtime.h>
#include <rocprim/rocprim.hpp>

#include <algorithm>

#include "eh_internal.h"

namespace eh {
namespace {

constexpr uint32_t kB = 256;
constexpr uint32_t kNone = 0xFFFFFFFFu;

uint32_t grid_of(uint64_t n) {
  return uint32_t(std::max<uint64_t>(1, std::min<uint64_t>((n + kB - 1) / kB, 1u << 16)));
}
__device__ inline uint64_t gtid() { return uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; }
__device__ inline uint64_t gstride() { return uint64_t(gridDim.x) * blockDim.x; }

template <class T>
T* ptr(DevBuf& b) {
  return static_cast<T*>(b.p);
}

__global__ void __launch_bounds__(kB) k_pos_keys(const uint32_t* __restrict__ deg, uint32_t n,
                                                 uint32_t* __restrict__ key,
                                                 uint32_t* __restrict__ ids) {
  for (uint64_t v = gtid(); v < n; v += gstride()) {
    key[v] = ~deg[v];  // ascending sort of ~degree: degree descending
    ids[v] = uint32_t(v);
  }
}

// pos[seq[p]] = p
__global__ void __launch_bounds__(kB) k_invert(const uint32_t* __restrict__ seq, uint32_t n,
                                               uint32_t* __restrict__ pos) {
  for (uint64_t p = gtid(); p < n; p += gstride()) pos[seq[p]] = uint32_t(p);
}

__global__ void __launch_bounds__(kB) k_copy_u32(const uint32_t* __restrict__ a, uint64_t n,
                                                 uint32_t* __restrict__ b) {
  for (uint64_t i = gtid(); i < n; i += gstride()) b[i] = a[i];
}

__global__ void __launch_bounds__(kB) k_fill(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  for (uint64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}

// Strong runs: ev[w] = min(pos[w], min over neighbours of pos) (ev starts as pos).
__global__ void __launch_bounds__(kB) k_first_visit(const unsigned long long* __restrict__ key,
                                                    uint64_t m, uint32_t kb,
                                                    const uint32_t* __restrict__ pos,
                                                    uint32_t* __restrict__ ev) {
  const unsigned long long mask = (1ull << kb) - 1;
  for (uint64_t i = gtid(); i < m; i += gstride()) {
    const uint32_t a = uint32_t(key[i] >> kb), b = uint32_t(key[i] & mask);
    atomicMin(&ev[a], pos[b]);
    atomicMin(&ev[b], pos[a]);
  }
}

// Sort key (event, 0 if labelled by its own visit else 1, id).
__global__ void __launch_bounds__(kB) k_strong_keys(const uint32_t* __restrict__ ev,
                                                    const uint32_t* __restrict__ pos, uint32_t n,
                                                    uint32_t kb,
                                                    unsigned long long* __restrict__ out) {
  for (uint64_t v = gtid(); v < n; v += gstride()) {
    const unsigned long long by_nbr = ev[v] < pos[v] ? 1ull : 0ull;
    out[v] = (static_cast<unsigned long long>(ev[v]) << (kb + 1)) | (by_nbr << kb) | v;
  }
}

__global__ void __launch_bounds__(kB) k_low_bits(const unsigned long long* __restrict__ key,
                                                 uint64_t n, uint32_t kb, uint32_t* __restrict__ out) {
  const unsigned long long mask = (1ull << kb) - 1;
  for (uint64_t i = gtid(); i < n; i += gstride()) out[i] = uint32_t(key[i] & mask);
}

// Both arcs of every edge, as (from << kb | to).
__global__ void __launch_bounds__(kB) k_arcs(const unsigned long long* __restrict__ key, uint64_t m,
                                             uint32_t kb, unsigned long long* __restrict__ arcs) {
  const unsigned long long mask = (1ull << kb) - 1;
  for (uint64_t i = gtid(); i < m; i += gstride()) {
    const unsigned long long a = key[i] >> kb, b = key[i] & mask;
    arcs[i] = key[i];
    arcs[m + i] = (b << kb) | a;
  }
}

// row[v] = first arc of v in the sorted arcs (binary search).
__global__ void __launch_bounds__(kB) k_arc_rows(const unsigned long long* __restrict__ arcs,
                                                 uint64_t m2, uint32_t n, uint32_t kb,
                                                 uint32_t* __restrict__ row) {
  for (uint64_t v = gtid(); v <= n; v += gstride()) {
    const unsigned long long want = static_cast<unsigned long long>(v) << kb;
    uint64_t lo = 0, len = m2;
    while (len > 0) {
      const uint64_t half = len >> 1;
      if (arcs[lo + half] < want) {
        lo += half + 1;
        len -= half + 1;
      } else {
        len = half;
      }
    }
    row[v] = uint32_t(lo);
  }
}

// One round of minimum propagation along edges, then one pointer jump
// (cm[v] <- cm of the vertex at position cm[v]); *changed is set when any
// value fell.
__global__ void __launch_bounds__(kB) k_min_edges(const unsigned long long* __restrict__ key,
                                                  uint64_t m, uint32_t kb,
                                                  uint32_t* __restrict__ cm,
                                                  uint32_t* __restrict__ changed) {
  const unsigned long long mask = (1ull << kb) - 1;
  for (uint64_t i = gtid(); i < m; i += gstride()) {
    const uint32_t a = uint32_t(key[i] >> kb), b = uint32_t(key[i] & mask);
    const uint32_t ca = cm[a], cb = cm[b];
    if (ca < cb) {
      if (atomicMin(&cm[b], ca) > ca) *changed = 1;
    } else if (cb < ca) {
      if (atomicMin(&cm[a], cb) > cb) *changed = 1;
    }
  }
}

__global__ void __launch_bounds__(kB) k_jump(const uint32_t* __restrict__ seq, uint32_t n,
                                             uint32_t* __restrict__ cm) {
  for (uint64_t v = gtid(); v < n; v += gstride()) {
    const uint32_t c = cm[v];
    const uint32_t cc = cm[seq[c]];
    if (cc < c) atomicMin(&cm[v], cc);
  }
}

// Component sizes by the position of their first vertex.
__global__ void __launch_bounds__(kB) k_comp_sizes(const uint32_t* __restrict__ cm, uint32_t n,
                                                   uint32_t* __restrict__ size) {
  for (uint64_t v = gtid(); v < n; v += gstride()) atomicAdd(&size[cm[v]], 1u);
}

// Level 0: each component's first vertex takes its block's first label.
__global__ void __launch_bounds__(kB) k_roots(const uint32_t* __restrict__ seq, uint32_t n,
                                              const uint32_t* __restrict__ cm,
                                              const uint32_t* __restrict__ coff,
                                              uint32_t* __restrict__ lab,
                                              uint32_t* __restrict__ next_free,
                                              uint32_t* __restrict__ frontier,
                                              uint32_t* __restrict__ n_front) {
  for (uint64_t p = gtid(); p < n; p += gstride()) {
    const uint32_t v = seq[p];
    if (cm[v] != uint32_t(p)) continue;
    lab[v] = coff[p];
    next_free[p] = coff[p] + 1;
    frontier[atomicAdd(n_front, 1u)] = v;
  }
}

// Every unlabelled neighbour of a frontier vertex: the smallest label among
// its frontier neighbours, and one entry in the next level's list.
__global__ void __launch_bounds__(kB) k_expand(const uint32_t* __restrict__ frontier, uint32_t nf,
                                               const uint32_t* __restrict__ row,
                                               const uint32_t* __restrict__ adj,
                                               const uint32_t* __restrict__ lab,
                                               uint32_t* __restrict__ plab,
                                               uint32_t* __restrict__ seen,
                                               uint32_t* __restrict__ next,
                                               uint32_t* __restrict__ n_next) {
  for (uint64_t i = gtid(); i < nf; i += gstride()) {
    const uint32_t x = frontier[i];
    const uint32_t lx = lab[x];
    for (uint32_t e = row[x]; e < row[x + 1]; ++e) {
      const uint32_t w = adj[e];
      if (lab[w] != kNone) continue;
      atomicMin(&plab[w], lx);
      if (atomicExch(&seen[w], 1u) == 0u) next[atomicAdd(n_next, 1u)] = w;
    }
  }
}

__global__ void __launch_bounds__(kB) k_level_keys(const uint32_t* __restrict__ next, uint32_t nn,
                                                   const uint32_t* __restrict__ plab,
                                                   unsigned long long* __restrict__ key) {
  for (uint64_t i = gtid(); i < nn; i += gstride()) {
    const uint32_t w = next[i];
    key[i] = (static_cast<unsigned long long>(plab[w]) << 32) | w;
  }
}

// Sorted level: the first index of each component's run.
__global__ void __launch_bounds__(kB) k_run_starts(const unsigned long long* __restrict__ key,
                                                   uint32_t nn, const uint32_t* __restrict__ cm,
                                                   uint32_t* __restrict__ first) {
  for (uint64_t j = gtid(); j < nn; j += gstride()) {
    const uint32_t c = cm[uint32_t(key[j])];
    if (j == 0 || cm[uint32_t(key[j - 1])] != c) first[c] = uint32_t(j);
  }
}

// Labels of the level (the next frontier, in label order).
__global__ void __launch_bounds__(kB) k_level_labels(const unsigned long long* __restrict__ key,
                                                     uint32_t nn, const uint32_t* __restrict__ cm,
                                                     const uint32_t* __restrict__ first,
                                                     const uint32_t* __restrict__ next_free,
                                                     uint32_t* __restrict__ lab,
                                                     uint32_t* __restrict__ frontier) {
  for (uint64_t j = gtid(); j < nn; j += gstride()) {
    const uint32_t w = uint32_t(key[j]);
    const uint32_t c = cm[w];
    lab[w] = next_free[c] + uint32_t(j) - first[c];
    frontier[j] = w;
  }
}

// Each component with a run in the level moves its next label past the run
// (one run per component per level).
__global__ void __launch_bounds__(kB) k_level_advance(const unsigned long long* __restrict__ key,
                                                      uint32_t nn, const uint32_t* __restrict__ cm,
                                                      const uint32_t* __restrict__ first,
                                                      uint32_t* __restrict__ next_free) {
  for (uint64_t j = gtid(); j < nn; j += gstride()) {
    const uint32_t c = cm[uint32_t(key[j])];
    if (j + 1 == nn || cm[uint32_t(key[j + 1])] != c) next_free[c] += uint32_t(j) - first[c] + 1;
  }
}

// seq[lab[v]] = v
__global__ void __launch_bounds__(kB) k_by_label(const uint32_t* __restrict__ lab, uint32_t n,
                                                 uint32_t* __restrict__ seq) {
  for (uint64_t v = gtid(); v < n; v += gstride()) seq[lab[v]] = uint32_t(v);
}

// Hybrid: sort key (degree descending, BFS label).
__global__ void __launch_bounds__(kB) k_hybrid_keys(const uint32_t* __restrict__ deg,
                                                    const uint32_t* __restrict__ lab, uint32_t n,
                                                    unsigned long long* __restrict__ key) {
  for (uint64_t v = gtid(); v < n; v += gstride())
    key[v] = (static_cast<unsigned long long>(~deg[v]) << 32) | lab[v];
}

// label -> vertex for hybrid keys sorted by (~degree, BFS label): the label's
// vertex is found through the BFS sequence.
__global__ void __launch_bounds__(kB) k_hybrid_seq(const unsigned long long* __restrict__ key,
                                                   uint32_t n, const uint32_t* __restrict__ bfs_seq,
                                                   uint32_t* __restrict__ seq) {
  for (uint64_t p = gtid(); p < n; p += gstride())
    seq[p] = bfs_seq[uint32_t(key[p] & 0xFFFFFFFFull)];
}

}  // namespace

eh_status device_traversal_sequence(Ctx* c, const unsigned long long* edges, uint64_t m,
                                    uint32_t kb, uint32_t n, const uint32_t* deg, uint32_t order,
                                    uint32_t* seq_out) {
  if (n == 0) return EH_OK;
  if (n > 0x7FFFFFFFu) {
    c->err = "traversal orderings on the GPU need fewer than 2^31 vertices";
    return EH_EOVERFLOW;
  }
  hipStream_t s = c->stream;
  Scratch sc(c);
  DevBuf pkey, pkey2, ids, seq, pos, tmp, flag;
  eh_status st;
  auto chk = [&](hipError_t e, const char* what) { return hip_check(c, e, what); };
  if ((st = sc.get(pkey, 4ull * n)) != EH_OK || (st = sc.get(pkey2, 4ull * n)) != EH_OK ||
      (st = sc.get(ids, 4ull * n)) != EH_OK || (st = sc.get(seq, 4ull * n)) != EH_OK ||
      (st = sc.get(pos, 4ull * n)) != EH_OK || (st = sc.get(flag, 256)) != EH_OK)
    return st;
  // visiting order: (degree descending, id ascending); a stable sort keeps ids ascending
  hipLaunchKernelGGL(k_pos_keys, dim3(grid_of(n)), dim3(kB), 0, s, deg, n, ptr<uint32_t>(pkey),
                     ptr<uint32_t>(ids));
  size_t need = 0, b = 0;
  if ((st = chk(rocprim::radix_sort_pairs(nullptr, b, ptr<uint32_t>(pkey), ptr<uint32_t>(pkey2),
                                          ptr<uint32_t>(ids), ptr<uint32_t>(seq), size_t(n), 0, 32,
                                          s), "order sort size")) != EH_OK)
    return st;
  need = b;
  const uint64_t m2 = 2 * m;
  const uint64_t big = std::max<uint64_t>({m2, uint64_t(n), 1});
  DevBuf k64a, k64b;
  if ((st = sc.get(k64a, 8 * big)) != EH_OK || (st = sc.get(k64b, 8 * big)) != EH_OK) return st;
  rocprim::double_buffer<unsigned long long> db(ptr<unsigned long long>(k64a),
                                                ptr<unsigned long long>(k64b));
  if ((st = chk(rocprim::radix_sort_keys(nullptr, b, db, size_t(big), 0, 64, s),
                "order sort size")) != EH_OK)
    return st;
  need = std::max(need, b);
  if ((st = chk(rocprim::exclusive_scan(nullptr, b, ptr<uint32_t>(pkey), ptr<uint32_t>(pkey2), 0u,
                                        size_t(n), rocprim::plus<uint32_t>(), s),
                "order scan size")) != EH_OK)
    return st;
  need = std::max(need, b);
  if ((st = sc.get(tmp, need)) != EH_OK) return st;
  size_t tb = tmp.bytes;
  if ((st = chk(rocprim::radix_sort_pairs(tmp.p, tb, ptr<uint32_t>(pkey), ptr<uint32_t>(pkey2),
                                          ptr<uint32_t>(ids), ptr<uint32_t>(seq), size_t(n), 0, 32,
                                          s), "visiting order sort")) != EH_OK)
    return st;
  hipLaunchKernelGGL(k_invert, dim3(grid_of(n)), dim3(kB), 0, s, ptr<uint32_t>(seq), n,
                     ptr<uint32_t>(pos));

  if (order == EH_ORDER_STRONG_RUNS) {
    uint32_t* ev = ptr<uint32_t>(pkey);
    hipLaunchKernelGGL(k_copy_u32, dim3(grid_of(n)), dim3(kB), 0, s, ptr<uint32_t>(pos),
                       uint64_t(n), ev);
    if (m)
      hipLaunchKernelGGL(k_first_visit, dim3(grid_of(m)), dim3(kB), 0, s, edges, m, kb,
                         ptr<uint32_t>(pos), ev);
    hipLaunchKernelGGL(k_strong_keys, dim3(grid_of(n)), dim3(kB), 0, s, ev, ptr<uint32_t>(pos), n,
                       kb, ptr<unsigned long long>(k64a));
    rocprim::double_buffer<unsigned long long> sk(ptr<unsigned long long>(k64a),
                                                  ptr<unsigned long long>(k64b));
    tb = tmp.bytes;
    if ((st = chk(rocprim::radix_sort_keys(tmp.p, tb, sk, size_t(n), 0, 2 * kb + 1, s),
                  "strong-runs sort")) != EH_OK)
      return st;
    hipLaunchKernelGGL(k_low_bits, dim3(grid_of(n)), dim3(kB), 0, s, sk.current(), uint64_t(n), kb,
                       seq_out);
    return chk(hipGetLastError(), "strong-runs kernels");
  }

  // BFS (and the hybrid, which starts from it)
  DevBuf row, adj, cm, csize, coff, lab, plab, seen, next_free, first, front, nxt;
  if ((st = sc.get(row, 4ull * (n + 1))) != EH_OK || (st = sc.get(adj, 4 * std::max<uint64_t>(m2, 1))) != EH_OK ||
      (st = sc.get(cm, 4ull * n)) != EH_OK || (st = sc.get(csize, 4ull * n)) != EH_OK ||
      (st = sc.get(coff, 4ull * n)) != EH_OK || (st = sc.get(lab, 4ull * n)) != EH_OK ||
      (st = sc.get(plab, 4ull * n)) != EH_OK || (st = sc.get(seen, 4ull * n)) != EH_OK ||
      (st = sc.get(next_free, 4ull * n)) != EH_OK || (st = sc.get(first, 4ull * n)) != EH_OK ||
      (st = sc.get(front, 4ull * n)) != EH_OK || (st = sc.get(nxt, 4ull * n)) != EH_OK)
    return st;
  // adjacency in id space, both arcs of every edge, neighbours ascending
  unsigned long long* arcs = ptr<unsigned long long>(k64a);
  if (m) {
    hipLaunchKernelGGL(k_arcs, dim3(grid_of(m)), dim3(kB), 0, s, edges, m, kb, arcs);
    rocprim::double_buffer<unsigned long long> ab(ptr<unsigned long long>(k64a),
                                                  ptr<unsigned long long>(k64b));
    tb = tmp.bytes;
    if ((st = chk(rocprim::radix_sort_keys(tmp.p, tb, ab, size_t(m2), 0, 2 * kb, s),
                  "adjacency sort")) != EH_OK)
      return st;
    arcs = ab.current();
    hipLaunchKernelGGL(k_low_bits, dim3(grid_of(m2)), dim3(kB), 0, s, arcs, m2, kb,
                       ptr<uint32_t>(adj));
  }
  hipLaunchKernelGGL(k_arc_rows, dim3(grid_of(uint64_t(n) + 1)), dim3(kB), 0, s, arcs, m2, n, kb,
                     ptr<uint32_t>(row));
  // components: the smallest position in each, by propagation along edges
  uint32_t* cmp = ptr<uint32_t>(cm);
  hipLaunchKernelGGL(k_copy_u32, dim3(grid_of(n)), dim3(kB), 0, s, ptr<uint32_t>(pos), uint64_t(n),
                     cmp);
  uint32_t* h_flag = nullptr;
  if ((st = chk(hipHostMalloc((void**)&h_flag, 16, hipHostMallocDefault), "pinned flag")) != EH_OK)
    return st;
  auto free_flag = [&]() { (void)hipHostFree(h_flag); };
  for (uint32_t round = 0; m; ++round) {
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(kB), 0, s, ptr<uint32_t>(flag), uint64_t(4), 0u);
    hipLaunchKernelGGL(k_min_edges, dim3(grid_of(m)), dim3(kB), 0, s, edges, m, kb, cmp,
                       ptr<uint32_t>(flag));
    hipLaunchKernelGGL(k_jump, dim3(grid_of(n)), dim3(kB), 0, s, ptr<uint32_t>(seq), n, cmp);
    if ((st = chk(hipMemcpyAsync(h_flag, flag.p, 4, hipMemcpyDeviceToHost, s), "read flag")) !=
            EH_OK ||
        (st = chk(hipStreamSynchronize(s), "component sync")) != EH_OK) {
      free_flag();
      return st;
    }
    if (!h_flag[0]) break;
    if (round > n) {  // each round lowers some value; cannot happen
      free_flag();
      c->err = "component propagation did not converge";
      return EH_EHIP;
    }
  }
  // label blocks: exclusive scan of component sizes in position order
  hipLaunchKernelGGL(k_fill, dim3(grid_of(n)), dim3(kB), 0, s, ptr<uint32_t>(csize), uint64_t(n),
                     0u);
  hipLaunchKernelGGL(k_comp_sizes, dim3(grid_of(n)), dim3(kB), 0, s, cmp, n, ptr<uint32_t>(csize));
  tb = tmp.bytes;
  if ((st = chk(rocprim::exclusive_scan(tmp.p, tb, ptr<uint32_t>(csize), ptr<uint32_t>(coff), 0u,
                                        size_t(n), rocprim::plus<uint32_t>(), s),
                "component offsets")) != EH_OK) {
    free_flag();
    return st;
  }
  hipLaunchKernelGGL(k_fill, dim3(grid_of(n)), dim3(kB), 0, s, ptr<uint32_t>(lab), uint64_t(n),
                     kNone);
  hipLaunchKernelGGL(k_fill, dim3(grid_of(n)), dim3(kB), 0, s, ptr<uint32_t>(plab), uint64_t(n),
                     kNone);
  hipLaunchKernelGGL(k_fill, dim3(grid_of(n)), dim3(kB), 0, s, ptr<uint32_t>(seen), uint64_t(n),
                     0u);
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(kB), 0, s, ptr<uint32_t>(flag), uint64_t(4), 0u);
  hipLaunchKernelGGL(k_roots, dim3(grid_of(n)), dim3(kB), 0, s, ptr<uint32_t>(seq), n, cmp,
                     ptr<uint32_t>(coff), ptr<uint32_t>(lab), ptr<uint32_t>(next_free),
                     ptr<uint32_t>(front), ptr<uint32_t>(flag));
  if ((st = chk(hipMemcpyAsync(h_flag, flag.p, 4, hipMemcpyDeviceToHost, s), "read roots")) !=
          EH_OK ||
      (st = chk(hipStreamSynchronize(s), "root sync")) != EH_OK) {
    free_flag();
    return st;
  }
  uint32_t nf = h_flag[0];
  uint64_t labelled = nf;
  // roots are visited: no later level may take them
  // (their label is set, which k_expand checks)
  while (nf && m) {
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(kB), 0, s, ptr<uint32_t>(flag) + 1, uint64_t(1), 0u);
    hipLaunchKernelGGL(k_expand, dim3(grid_of(nf)), dim3(kB), 0, s, ptr<uint32_t>(front), nf,
                       ptr<uint32_t>(row), ptr<uint32_t>(adj), ptr<uint32_t>(lab),
                       ptr<uint32_t>(plab), ptr<uint32_t>(seen), ptr<uint32_t>(nxt),
                       ptr<uint32_t>(flag) + 1);
    if ((st = chk(hipMemcpyAsync(h_flag + 1, ptr<uint32_t>(flag) + 1, 4, hipMemcpyDeviceToHost, s),
                  "read level size")) != EH_OK ||
        (st = chk(hipStreamSynchronize(s), "level sync")) != EH_OK) {
      free_flag();
      return st;
    }
    const uint32_t nn = h_flag[1];
    if (!nn) break;
    labelled += nn;
    if (labelled > n) {  // each vertex enters one level; cannot happen
      free_flag();
      c->err = "BFS levels exceed the vertex count";
      return EH_EHIP;
    }
    hipLaunchKernelGGL(k_level_keys, dim3(grid_of(nn)), dim3(kB), 0, s, ptr<uint32_t>(nxt), nn,
                       ptr<uint32_t>(plab), ptr<unsigned long long>(k64a));
    rocprim::double_buffer<unsigned long long> lk(ptr<unsigned long long>(k64a),
                                                  ptr<unsigned long long>(k64b));
    tb = tmp.bytes;
    if ((st = chk(rocprim::radix_sort_keys(tmp.p, tb, lk, size_t(nn), 0, 64, s), "level sort")) !=
        EH_OK) {
      free_flag();
      return st;
    }
    hipLaunchKernelGGL(k_run_starts, dim3(grid_of(nn)), dim3(kB), 0, s, lk.current(), nn, cmp,
                       ptr<uint32_t>(first));
    hipLaunchKernelGGL(k_level_labels, dim3(grid_of(nn)), dim3(kB), 0, s, lk.current(), nn, cmp,
                       ptr<uint32_t>(first), ptr<uint32_t>(next_free), ptr<uint32_t>(lab),
                       ptr<uint32_t>(front));
    hipLaunchKernelGGL(k_level_advance, dim3(grid_of(nn)), dim3(kB), 0, s, lk.current(), nn, cmp,
                       ptr<uint32_t>(first), ptr<uint32_t>(next_free));
    nf = nn;
  }
  free_flag();
  if (order == EH_ORDER_HYBRID) {
    hipLaunchKernelGGL(k_by_label, dim3(grid_of(n)), dim3(kB), 0, s, ptr<uint32_t>(lab), n,
                       ptr<uint32_t>(seq));
    hipLaunchKernelGGL(k_hybrid_keys, dim3(grid_of(n)), dim3(kB), 0, s, deg, ptr<uint32_t>(lab), n,
                       ptr<unsigned long long>(k64a));
    rocprim::double_buffer<unsigned long long> hk(ptr<unsigned long long>(k64a),
                                                  ptr<unsigned long long>(k64b));
    tb = tmp.bytes;
    if ((st = chk(rocprim::radix_sort_keys(tmp.p, tb, hk, size_t(n), 0, 64, s), "hybrid sort")) !=
        EH_OK)
      return st;
    hipLaunchKernelGGL(k_hybrid_seq, dim3(grid_of(n)), dim3(kB), 0, s, hk.current(), n,
                       ptr<uint32_t>(seq), seq_out);
  } else {
    hipLaunchKernelGGL(k_by_label, dim3(grid_of(n)), dim3(kB), 0, s, ptr<uint32_t>(lab), n, seq_out);
  }
  if ((st = chk(hipGetLastError(), "BFS kernels")) != EH_OK) return st;
  return chk(hipStreamSynchronize(s), "order sync");
}

}  // namespace eh
