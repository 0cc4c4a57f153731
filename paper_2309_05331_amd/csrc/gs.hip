// Single-grid launches of the fused Runge-Kutta stage kernels of RK4, Dopri5,
// Cash-Karp 5(4) and Euler: one tile (stage_tile, in stage.h) per workgroup
// over the whole grid (gs_stage, in stage.h).  Tiles of four wavefronts for
// every row count and vector width; tiles of eight wavefronts (half the halo
// rows per tile row) for one- and two-row strips of 16-byte lanes.  The
// Fehlberg 7(8) and Adams-Bashforth kinds are launched from gsx.hip.
#include "stage.h"

namespace hode {

namespace {

template <typename T, int RY, int VW, int NW>
hipError_t launch_t(int kind, const GSLaunch& a, DevCtrl* c, hipStream_t s) {
  // (K_COUNT: the fixed-step stage 6, new state only)
  return launch_stage_t<T, RY, VW, NW, K_D1, K_R2, K_R3, K_R4, K_D2, K_D3, K_D4, K_D5, K_D6, K_D7, K_D7F, K_C4,
                        K_C5, K_C6, K_C6F, K_E1, K_COUNT>(kind, a, c, s);
}

template <typename T, int VW>
hipError_t launch_vw(int kind, int ry, int nw, const GSLaunch& a, DevCtrl* c, hipStream_t s) {
  constexpr bool wide = VW * sizeof(T) == 16;  // eight-wavefront tiles: 16-byte lanes only
  if (nw == 8) {
    if constexpr (wide) {
      if (ry == 1) return launch_t<T, 1, VW, 8>(kind, a, c, s);
      if (ry == 2) return launch_t<T, 2, VW, 8>(kind, a, c, s);
    }
    return hipErrorInvalidValue;
  }
  if (nw != 4) return hipErrorInvalidValue;
  if (ry == 1) return launch_t<T, 1, VW, 4>(kind, a, c, s);
  if (ry == 2) return launch_t<T, 2, VW, 4>(kind, a, c, s);
  if (ry == 4) return launch_t<T, 4, VW, 4>(kind, a, c, s);
  return hipErrorInvalidValue;
}

}  // namespace

bool gs_ry_supported(int ry) { return ry == 1 || ry == 2 || ry == 4; }

bool gs_tile_supported(int kind, int dtype, int ry, int vw, int nw, int N) {
  if (!gs_ry_supported(ry)) return false;
  if (nw == 4) return true;
  // eight wavefronts: the kinds of this file with one- and two-row strips,
  // the Fehlberg kinds (gsf.hip) with one-row strips; 16-byte lanes (vw 0
  // picks the widest lanes that divide N)
  const int wide = dtype == 1 ? 4 : 2;
  const int v = vw ? vw : (N % wide == 0 ? wide : 1);
  return nw == 8 && v == wide && ((kind <= K_COUNT && ry <= 2) || (gsf_kind(kind) && ry == 1));
}

// kind K_COUNT is the fixed-step stage 6 (new state only).  vw: cells per
// lane (0 = widest that divides N: 16-byte loads when possible).  nw:
// wavefronts per workgroup (4, or 8 for 16-byte lanes and ry <= 2; the
// Fehlberg kinds ry = 1).
hipError_t launch_gs(int kind, int dtype, int ry, int vw, int nw, const GSLaunch& a, DevCtrl* c, hipStream_t s) {
  if (kind > K_COUNT) {
    if (nw == 8) return launch_gsf8(kind, dtype, ry, vw, a, c, s);
    return nw == 4 ? launch_gsx(kind, dtype, ry, vw, a, c, s) : hipErrorInvalidValue;
  }
  if (a.N < 1 || a.zc < 1 || kind < 0) return hipErrorInvalidValue;
  if (dtype == 1) {
    if (vw == 0) vw = a.N % 4 == 0 ? 4 : (a.N % 2 == 0 ? 2 : 1);
    if (a.N % vw) return hipErrorInvalidValue;
    if (vw == 4) return launch_vw<float, 4>(kind, ry, nw, a, c, s);
    if (vw == 2) return launch_vw<float, 2>(kind, ry, nw, a, c, s);
    if (vw == 1) return launch_vw<float, 1>(kind, ry, nw, a, c, s);
    return hipErrorInvalidValue;
  }
  if (vw == 0) vw = a.N % 2 == 0 ? 2 : 1;
  if (a.N % vw) return hipErrorInvalidValue;
  if (vw == 2) return launch_vw<double, 2>(kind, ry, nw, a, c, s);
  if (vw == 1) return launch_vw<double, 1>(kind, ry, nw, a, c, s);
  return hipErrorInvalidValue;
}

}  // namespace hode
