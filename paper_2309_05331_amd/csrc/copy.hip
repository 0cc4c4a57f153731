// A plain streaming copy: the bandwidth reference beside the stage kernels
// (what 16-byte-per-lane reads and writes reach on this device) and the known
// byte count that calibrates the HBM traffic counters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "../../include/hode.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// Each workgroup moves 4 x 256 16-byte elements: all four loads are issued
// before the first store.  Loads are ordinary, stores non-temporal: the same
// access kinds as the stage kernels, so the counters it calibrates count the
// same way.
__global__ __launch_bounds__(256) void copy16(const f4* __restrict__ s, f4* __restrict__ d, int64_t n) {
  const int64_t base = (int64_t)blockIdx.x * (4 * 256) + threadIdx.x;
  f4 v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t i = base + u * 256;
    if (i < n) v[u] = s[i];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t i = base + u * 256;
    if (i < n) __builtin_nontemporal_store(v[u], &d[i]);
  }
}

}  // namespace

extern "C" int hode_stream_copy(void* dst, const void* src, size_t bytes, int reps, double* avg_ms) {
  if (!dst || !src || bytes % 16 || reps < 1 || !avg_ms) return HODE_EINVAL;
  if (((uintptr_t)dst | (uintptr_t)src) % 16) return HODE_EINVAL;  // 16-byte vector accesses
  const int64_t n = (int64_t)(bytes / 16);
  const int64_t grid = std::max<int64_t>(1, (n + 1023) / 1024);
  if (grid > INT32_MAX) return HODE_EINVAL;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float ms = 0;
  if (e == hipSuccess) {
    copy16<<<(unsigned)grid, 256, 0, s>>>((const f4*)src, (f4*)dst, n);  // warm-up
    e = hipEventRecord(e0, s);
    for (int i = 0; i < reps && e == hipSuccess; ++i) {
      copy16<<<(unsigned)grid, 256, 0, s>>>((const f4*)src, (f4*)dst, n);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) (void)hipStreamSynchronize(s);  // nothing left in flight on the buffers
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (e != hipSuccess) return HODE_EHIP;
  *avg_ms = (double)ms / reps;
  return HODE_OK;
}
