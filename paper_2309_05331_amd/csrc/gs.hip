// Single-grid launches of the fused Runge-Kutta stage kernels of RK4, Dopri5,
// Cash-Karp 5(4) and Euler: one tile (stage_tile, in stage.h) per workgroup
// over the whole grid (gs_stage, in stage.h).  The Fehlberg 7(8) and
// Adams-Bashforth kinds are launched from gsx.hip.
#include "stage.h"

namespace hode {

namespace {

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
  if (kind > K_COUNT) return launch_gsx(kind, dtype, ry, vw, a, c, s);
  if (a.N < 1 || a.zc < 1 || kind < 0) return hipErrorInvalidValue;
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
