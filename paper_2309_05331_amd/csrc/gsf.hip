// Single-grid launches of the Runge-Kutta-Fehlberg 7(8) stage kernels with
// tiles of eight wavefronts (one-row strips of 16-byte lanes).  The widest
// Fehlberg stages form their input from up to ten arrays; the halo rows above
// and below a tile are re-read from memory whenever a neighbouring tile's
// reads have already left L2, and an eight-row tile has half the halo rows per
// grid row of a four-row one.  Same tiles and block order as the other stage
// kernels (stage.h); a translation unit of its own so it builds in parallel.
#include "stage.h"

namespace hode {

namespace {

template <typename T, int VW>
hipError_t launch_t(int kind, const GSLaunch& a, DevCtrl* c, hipStream_t s) {
  return launch_stage_t<T, 1, VW, 8, K_F1, K_F2, K_F3, K_F4, K_F5, K_F6, K_F7, K_F8, K_F9, K_F10, K_F11, K_F12,
                        K_F13, K_F13F>(kind, a, c, s);
}

}  // namespace

bool gsf_kind(int kind) { return kind >= K_F1 && kind <= K_F13F; }

// Every kind here reads extra arrays through the table xk(a), which must hold them.
hipError_t launch_gsf8(int kind, int dtype, int ry, int vw, const GSLaunch& a, DevCtrl* c, hipStream_t s) {
  if (a.N < 1 || a.zc < 1 || !gsf_kind(kind) || ry != 1 || xk(a) == nullptr) return hipErrorInvalidValue;
  if (dtype == 1) {
    if (vw == 0) vw = a.N % 4 == 0 ? 4 : 1;
    return vw == 4 && a.N % 4 == 0 ? launch_t<float, 4>(kind, a, c, s) : hipErrorInvalidValue;
  }
  if (vw == 0) vw = a.N % 2 == 0 ? 2 : 1;
  return vw == 2 && a.N % 2 == 0 ? launch_t<double, 2>(kind, a, c, s) : hipErrorInvalidValue;
}

}  // namespace hode
