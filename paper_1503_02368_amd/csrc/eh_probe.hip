// Streaming-read bandwidth probe: the ceiling a read-only kernel reaches on
// this GPU, measured beside the nominal HBM peak.  Every 16-byte word of the
// buffer is loaded once with 128-bit loads, four per lane in flight, over a
// grid-stride loop; the words are folded by XOR so the loads cannot be
// dropped, and each wave leaves one XOR in the sink.
#include <hip/hip_runtime.h>

#include "eh_internal.h"

namespace eh {
namespace {

constexpr int kProbeThreads = 256;

__global__ __launch_bounds__(kProbeThreads) void k_stream_read(const uint4* __restrict__ p,
                                                               uint64_t n16,
                                                               unsigned long long* sink) {
  const uint64_t stride = uint64_t(gridDim.x) * kProbeThreads;
  uint64_t i = uint64_t(blockIdx.x) * kProbeThreads + threadIdx.x;
  uint32_t x = 0;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const uint4 a = p[i], b = p[i + stride], c = p[i + 2 * stride], d = p[i + 3 * stride];
    x ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w;
    x ^= c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
  }
  for (; i < n16; i += stride) {
    const uint4 a = p[i];
    x ^= a.x ^ a.y ^ a.z ^ a.w;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x ^= uint32_t(__shfl_xor(int(x), o, 64));
  if ((threadIdx.x & 63) == 0 && x) atomicXor(sink, (unsigned long long)x);
}

}  // namespace
}  // namespace eh

using namespace eh;

extern "C" eh_status eh_stream_read(eh_ctx* ctx, const void* d_buf, uint64_t bytes,
                                    uint32_t blocks_per_cu, uint64_t* d_sink) {
  if (!ctx || !d_buf || !d_sink) return EH_EINVAL;
  Ctx* c = &ctx->c;
  if (bytes == 0 || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(d_buf) % 16 != 0) {
    c->err = "stream read needs a 16-byte aligned buffer of a positive multiple of 16 bytes";
    return EH_EINVAL;
  }
  if (blocks_per_cu == 0) blocks_per_cu = 8;
  if (blocks_per_cu > 64) {
    c->err = "blocks_per_cu must be at most 64";
    return EH_EINVAL;
  }
  const uint64_t n16 = bytes / 16;
  uint64_t blocks = uint64_t(c->n_cu) * blocks_per_cu;
  const uint64_t need = (n16 + kProbeThreads - 1) / kProbeThreads;
  if (blocks > need) blocks = need;
  hipLaunchKernelGGL(k_stream_read, dim3(uint32_t(blocks)), dim3(kProbeThreads), 0, c->stream,
                     static_cast<const uint4*>(d_buf), n16,
                     reinterpret_cast<unsigned long long*>(d_sink));
  return hip_check(c, hipGetLastError(), "stream read kernel launch");
}
