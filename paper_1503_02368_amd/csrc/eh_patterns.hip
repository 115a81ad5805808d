// Multi-attribute combinations of per-vertex counts (paper section 5.3).
//
// The Lollipop query L(x,y,z,w) :- R(x,y), S(y,z), T(x,z), U(x,w) on the
// unpruned relation is one Generic-Join whose innermost level over w is a
// single relation, not an intersection: its COUNT(*) is the sum over x of
// t(x) |N(x)|, where t(x) is the number of ordered triangles (x, y, z).  The
// staged kernel produces t by first attribute (the per-root vector of a
// symmetric trie); this kernel weights it by degree and sums it.
#include <hip/hip_runtime.h>

#include "eh_internal.h"

namespace eh {
namespace {

constexpr uint32_t kB = 256;

// out[0] += sum over ranks r of t_by_id[vert[r]] * |N(r)|
__global__ void __launch_bounds__(kB) k_degree_weighted_sum(const unsigned long long* __restrict__ t_by_id,
                                                            const uint32_t* __restrict__ vert,
                                                            const uint2* __restrict__ vdesc,
                                                            uint32_t n,
                                                            unsigned long long* __restrict__ out) {
  __shared__ unsigned long long part[kB / 64];
  unsigned long long sum = 0;
  for (uint64_t r = uint64_t(blockIdx.x) * kB + threadIdx.x; r < n; r += uint64_t(gridDim.x) * kB)
    sum += t_by_id[vert[r]] * static_cast<unsigned long long>(vdesc[r].y & kMaxIndex);
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x / 64] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t i = 1; i < kB / 64; ++i) sum += part[i];
    if (sum) atomicAdd(out, sum);
  }
}

// out[0] += f * in[0], one thread
__global__ void k_add_scaled(const unsigned long long* __restrict__ in, unsigned long long f,
                             unsigned long long* __restrict__ out) {
  if (threadIdx.x == 0) {
    const unsigned long long v = f * in[0];
    if (v) atomicAdd(out, v);
  }
}

}  // namespace

eh_status launch_add_scaled(Ctx* c, hipStream_t s, const unsigned long long* in,
                            unsigned long long f, unsigned long long* out) {
  hipLaunchKernelGGL(k_add_scaled, dim3(1), dim3(64), 0, s, in, f, out);
  return hip_check(c, hipGetLastError(), "scaled add launch");
}

eh_status launch_degree_weighted_sum(Ctx* c, hipStream_t s, const unsigned long long* t_by_id,
                                     const uint32_t* vert, const uint2* vdesc, uint32_t n,
                                     unsigned long long* out) {
  if (n == 0) return EH_OK;
  const uint32_t blocks = std::min<uint32_t>((n + kB - 1) / kB, 4096);
  hipLaunchKernelGGL(k_degree_weighted_sum, dim3(blocks), dim3(kB), 0, s, t_by_id, vert, vdesc, n,
                     out);
  return hip_check(c, hipGetLastError(), "degree-weighted sum launch");
}

}  // namespace eh
