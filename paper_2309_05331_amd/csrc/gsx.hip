// Single-grid launches of the Gray-Scott stage kernels of the higher-order
// and multi-step methods of the paper's Table 1: Runge-Kutta-Fehlberg 7(8)
// (13 stages; F13 forms the new state and, adaptive, the error norm at the
// own cell) and Adams-Bashforth with 1 to 8 steps (one right-hand side per
// step: f_n goes into the ring of past right-hand sides and the new state is
// formed from it and the s - 1 before); the Adams-Moulton correctors of
// Adams-Bashforth-Moulton (the Adams-Bashforth kinds write the prediction);
// the modified midpoint substeps (MM1 .. MM3); and the dense-output variant of
// Dopri5 stage 6 (D6K, which also stores k6).  Same tiles and block order as the
// other stage kernels (stage.h); a translation unit of its own so the two
// build in parallel.
#include "stage.h"

namespace hode {

namespace {

template <typename T, int RY, int VW>
hipError_t launch_t(int kind, const GSLaunch& a, DevCtrl* c, hipStream_t s) {
  return launch_stage_t<T, RY, VW, 4, K_F1, K_F2, K_F3, K_F4, K_F5, K_F6, K_F7, K_F8, K_F9, K_F10, K_F11, K_F12,
                        K_F13, K_F13F, K_AB1, K_AB2, K_AB3, K_AB4, K_AB5, K_AB6, K_AB7, K_AB8, K_D6K, K_ABC1,
                        K_ABC2, K_ABC3, K_ABC4, K_ABC5, K_ABC6, K_ABC7, K_ABC8, K_MM1, K_MM2, K_MM3>(kind, a, c, s);
}

template <typename T, int VW>
hipError_t launch_vw(int kind, int ry, const GSLaunch& a, DevCtrl* c, hipStream_t s) {
  if (ry == 1) return launch_t<T, 1, VW>(kind, a, c, s);
  if (ry == 2) return launch_t<T, 2, VW>(kind, a, c, s);
  if (ry == 4) return launch_t<T, 4, VW>(kind, a, c, s);
  return hipErrorInvalidValue;
}

}  // namespace

// Every kind here reads extra arrays through the table xk(a), which must hold them.
hipError_t launch_gsx(int kind, int dtype, int ry, int vw, const GSLaunch& a, DevCtrl* c, hipStream_t s) {
  if (a.N < 1 || a.zc < 1 || kind < K_F1 || kind >= K_ALL || xk(a) == nullptr) return hipErrorInvalidValue;
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
