// Single-grid launches of the fused Runge-Kutta stage kernels: one tile
// (stage_tile, in stage.h) per workgroup over the whole grid.
//
// Block order is XCD-aware: workgroups are dealt round-robin to the 8 XCDs, so
// the linear block id is remapped to give each XCD a contiguous range of
// tiles, keeping y- and z-adjacent tiles (whose halo rows overlap) on one L2.
#include "stage.h"

namespace hode {

namespace {

// One stage over a whole grid: one tile per workgroup.  The linear block id
// is remapped XCD-aware: workgroups are dealt round-robin to the 8 XCDs, so
// each XCD gets a contiguous range of tiles and y/z-adjacent tiles (whose
// halo rows overlap) share an L2.  Consecutive stages sweep those ranges in
// opposite directions.
template <typename T, int KIND, int RY, int VW>
__global__ __launch_bounds__(256) void gs_stage(const GSLaunch a, DevCtrl* __restrict__ c) {
  __shared__ __align__(16) char smem[kTileSmem];
  if (c->done) return;
  const int N = a.N;
  const int nx = (N + 64 * VW - 1) / (64 * VW);
  const int ny = (N + 4 * RY - 1) / (4 * RY);
  const int nz = (N + a.zc - 1) / a.zc;
  const int per = (gridDim.x + 7) / 8;
  // Stages alternate their direction through each XCD's range, so a stage
  // starts on the tiles the previous stage wrote last, which are still in the
  // memory-side Infinity Cache.
  constexpr bool rev = KIND == K_R2 || KIND == K_R4 || KIND == K_D3 || KIND == K_D5 || KIND == K_D7 ||
                       KIND == K_D7F || KIND == K_C5;
  const int slot = rev ? per - 1 - (int)(blockIdx.x >> 3) : (int)(blockIdx.x >> 3);
  const int bb = (blockIdx.x & 7) * per + slot;
  if (bb >= nx * ny * nz) return;  // padding block of the remap (whole block)
  const int tz = bb / (nx * ny);
  stage_tile<T, KIND, RY, VW>(a, c, smem, bb % nx, (bb / nx) % ny, tz * a.zc, min(N, (tz + 1) * a.zc));
}

template <typename T, int RY, int VW>
hipError_t launch_t(int kind, const GSLaunch& a, DevCtrl* c, hipStream_t s) {
  constexpr int TX = 64 * VW;
  const int nx = (a.N + TX - 1) / TX;
  const int ny = (a.N + 4 * RY - 1) / (4 * RY);
  const int nz = (a.N + a.zc - 1) / a.zc;
  const int64_t nb = (int64_t)nx * ny * nz;
  const int64_t grid = (nb + 7) / 8 * 8;  // whole rounds of the XCD remap
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  switch (kind) {
#define HODE_CASE(K) \
  case K: gs_stage<T, K, RY, VW><<<dim3((unsigned)grid), dim3(256), 0, s>>>(a, c); break;
    HODE_CASE(K_D1) HODE_CASE(K_R2) HODE_CASE(K_R3) HODE_CASE(K_R4) HODE_CASE(K_D2) HODE_CASE(K_D3)
    HODE_CASE(K_D4) HODE_CASE(K_D5) HODE_CASE(K_D6) HODE_CASE(K_D7) HODE_CASE(K_D7F) HODE_CASE(K_C4)
    HODE_CASE(K_C5) HODE_CASE(K_C6) HODE_CASE(K_C6F) HODE_CASE(K_E1) HODE_CASE(K_COUNT)
#undef HODE_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int VW>
hipError_t launch_vw(int kind, int ry, const GSLaunch& a, DevCtrl* c, hipStream_t s) {
  if (ry == 1) return launch_t<T, 1, VW>(kind, a, c, s);
  if (ry == 2) return launch_t<T, 2, VW>(kind, a, c, s);
  if (ry == 4) return launch_t<T, 4, VW>(kind, a, c, s);
  return hipErrorInvalidValue;
}

}  // namespace

bool gs_ry_supported(int ry) { return ry == 1 || ry == 2 || ry == 4; }

// kind K_COUNT is the fixed-step stage 6 (new state only).  vw: cells per
// lane (0 = widest that divides N: 16-byte loads when possible).
hipError_t launch_gs(int kind, int dtype, int ry, int vw, const GSLaunch& a, DevCtrl* c, hipStream_t s) {
  if (a.N < 1 || a.zc < 1 || kind < 0 || kind > K_COUNT) return hipErrorInvalidValue;
  if (dtype == 1) {
    if (vw == 0) vw = a.N % 4 == 0 ? 4 : (a.N % 2 == 0 ? 2 : 1);
    if (a.N % vw) return hipErrorInvalidValue;
    if (vw == 4) return launch_vw<float, 4>(kind, ry, a, c, s);
    if (vw == 2) return launch_vw<float, 2>(kind, ry, a, c, s);
    if (vw == 1) return launch_vw<float, 1>(kind, ry, a, c, s);
    return hipErrorInvalidValue;
  }
  if (vw == 0) vw = a.N % 2 == 0 ? 2 : 1;
  if (a.N % vw) return hipErrorInvalidValue;
  if (vw == 2) return launch_vw<double, 2>(kind, ry, a, c, s);
  if (vw == 1) return launch_vw<double, 1>(kind, ry, a, c, s);
  return hipErrorInvalidValue;
}

}  // namespace hode
