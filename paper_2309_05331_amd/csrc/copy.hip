// A plain streaming copy: the bandwidth reference beside the stage kernels
// (what 16-byte-per-lane reads and writes reach on this device) and the known
// byte count that calibrates the HBM traffic counters.
#include <hip/hip_runtime.h>

#include "../../include/hode.h"

namespace {

__global__ __launch_bounds__(256) void copy16(const float4* __restrict__ s, float4* __restrict__ d, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) d[i] = s[i];
}

}  // namespace

extern "C" int hode_stream_copy(void* dst, const void* src, size_t bytes, int reps, double* avg_ms) {
  if (!dst || !src || bytes % 16 || reps < 1 || !avg_ms) return HODE_EINVAL;
  const int64_t n = (int64_t)(bytes / 16);
  int64_t grid = (n + 255) / 256;
  if (grid > 8192) grid = 8192;
  if (grid < 1) grid = 1;
  hipStream_t s;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return HODE_EHIP;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  copy16<<<(unsigned)grid, 256, 0, s>>>((const float4*)src, (float4*)dst, n);  // warm-up
  hipEventRecord(e0, s);
  for (int i = 0; i < reps; ++i) copy16<<<(unsigned)grid, 256, 0, s>>>((const float4*)src, (float4*)dst, n);
  hipEventRecord(e1, s);
  hipError_t e = hipEventSynchronize(e1);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipStreamDestroy(s);
  if (e != hipSuccess) return HODE_EHIP;
  *avg_ms = (double)ms / reps;
  return HODE_OK;
}
