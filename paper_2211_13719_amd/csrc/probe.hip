// Read-bandwidth probe: a measurement helper for the rooflines of kernels
// bound by their L2 misses (the fine Wilson-clover kernel).  It tells which
// level of the memory system serves a working set of a given size, and at
// what rate: the L2s (4 MiB per XCD), the Infinity Cache (256 MiB), or HBM.
#include "internal.h"

namespace mrhs {
namespace {

// Every thread reads 16-byte words of the buffer in a grid-stride loop,
// `sweeps` times over, DEPTH independent words per trip (DEPTH loads in flight
// per thread before the first is used); the empty asm keeps the sum, and so
// the loads, alive without any store.
template <int DEPTH>
__global__ __launch_bounds__(256) void read_probe_kernel(const float4* __restrict__ p, size_t n4, int sweeps) {
  float acc = 0.f;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t first = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int s = 0; s < sweeps; ++s) {
    size_t i = first;
    for (; i + (DEPTH - 1) * stride < n4; i += DEPTH * stride) {
      float4 v[DEPTH];
#pragma unroll
      for (int k = 0; k < DEPTH; ++k) v[k] = p[i + k * stride];
#pragma unroll
      for (int k = 0; k < DEPTH; ++k) acc += v[k].x + v[k].y + v[k].z + v[k].w;
    }
    for (; i < n4; i += stride) {
      const float4 v = p[i];
      acc += v.x + v.y + v.z + v.w;
    }
  }
  asm volatile("" : : "v"(acc));
}

template <int DEPTH>
hipError_t launch_read_probe(const float4* p, size_t n4, int sweeps, int grid, hipStream_t s) {
  hipLaunchKernelGGL(read_probe_kernel<DEPTH>, dim3(grid), dim3(256), 0, s, p, n4, sweeps);
  return hipGetLastError();
}

hipError_t read_probe(int depth, const float4* p, size_t n4, int sweeps, int grid, hipStream_t s) {
  switch (depth) {
    case 1: return launch_read_probe<1>(p, n4, sweeps, grid, s);
    case 2: return launch_read_probe<2>(p, n4, sweeps, grid, s);
    case 4: return launch_read_probe<4>(p, n4, sweeps, grid, s);
    default: return launch_read_probe<8>(p, n4, sweeps, grid, s);
  }
}

}  // namespace
}  // namespace mrhs

using namespace mrhs;

extern "C" mrhs_status mrhs_read_probe(mrhs_ctx ctx, const void* buf, int64_t bytes, int32_t sweeps, int32_t grid,
                                       int32_t depth, float* ms) {
  if (!ctx) return MRHS_ERR_INVALID_ARG;
  if (!buf || !ms || !aligned16(buf)) return fail(ctx, MRHS_ERR_INVALID_ARG, "null or misaligned pointer");
  if (bytes < 16 || bytes % 16 || sweeps < 1 || sweeps > 100000 || grid < 1 || grid > (1 << 20))
    return fail(ctx, MRHS_ERR_INVALID_ARG, "bad probe size, sweeps or grid");
  if (depth != 1 && depth != 2 && depth != 4 && depth != 8)
    return fail(ctx, MRHS_ERR_INVALID_ARG, "probe depth %d not in {1, 2, 4, 8}", depth);
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (prev != ctx->device) MRHS_HIP(ctx, hipSetDevice(ctx->device));
  struct Restore {
    int p, d;
    ~Restore() {
      if (p >= 0 && p != d) (void)hipSetDevice(p);
    }
  } restore{prev, ctx->device};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  MRHS_HIP(ctx, hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  const size_t n4 = (size_t)bytes / 16;
  const auto* p = static_cast<const float4*>(buf);
  // one untimed sweep leaves the buffer in whatever cache holds it
  if (e == hipSuccess) e = read_probe(depth, p, n4, 1, grid, ctx->stream);
  if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
  if (e == hipSuccess) e = read_probe(depth, p, n4, sweeps, grid, ctx->stream);
  if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(ctx, e, "read probe");
  return MRHS_OK;
}
