// Host-side declarations shared by the hode translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hode_dev.h"

namespace hode {

// Stage kernels of the Gray-Scott path.  D1 computes k1 = f(y) (also the
// first RK4 stage); R2..R4 are the remaining RK4 stages (R4 also forms the new
// state); D2..D5 are Dopri5 stages 2..5; D6 forms k6 and from it the new state
// and the partial error sum (D6F: new state only); D7 evaluates k7 = f(ynew)
// and completes the error norm (D7F: k7 only).  The control kernel follows the
// final stage of every attempt.
enum GSKind : int {
  K_D1 = 0, K_R2, K_R3, K_R4, K_D2, K_D3, K_D4, K_D5, K_D6, K_D7, K_D7F, K_COUNT,
  K_D6F = K_COUNT  // fixed-step stage 6: the new state only
};

struct GSLaunch {
  void* y[2];    // state, indexed by the device-side parity
  void* ks[2];   // first-same-as-last pair: k1 = ks[k1slot], k7 = ks[k1slot ^ 1]
  void* k[7];    // k[2] .. k[6]
  int64_t n3;    // N^3, the stride between the u and v fields
  int32_t N;
  int32_t zc;    // z-planes marched by one workgroup
  double Du_h2, Dv_h2, F, kk;
};

// ry: rows per wavefront strip (tile = 64*vw x 4*ry cells); vw: cells per
// lane (1, 2 or 4 for fp32, 1 or 2 for fp64, dividing N; 0 picks the widest).
hipError_t launch_gs(int kind, int dtype, int ry, int vw, const GSLaunch& a, DevCtrl* c, hipStream_t s);
bool gs_ry_supported(int ry);

// Element-wise families: the whole step runs in registers (one kernel per
// attempt).  mode: MODE_FIXED_RK4, MODE_FIXED_DP5 or MODE_ADAPTIVE.
hipError_t launch_ew(int dtype, int rhs, int mode, void* y0, void* y1, int64_t n, int grid, DevCtrl* c,
                     hipStream_t s);

// The step controller: one wavefront, run after the final stage kernel of
// every attempt or fixed step.
hipError_t launch_ctrl(DevCtrl* c, hipStream_t s);

// out = f(y) for the element-wise systems (no control block involved).
hipError_t launch_ew_rhs(int dtype, int rhs, const void* y, void* out, int64_t n, int grid, hipStream_t s);

// ---- batched ensemble -------------------------------------------------------
// One instance of the ensemble: its grid and arrays, its own control block
// (time, step, controller state, counters) and the barrier counter of the
// gang of workgroups that steps it.
struct EnsInst {
  GSLaunch a;
  DevCtrl ctrl;
  uint32_t bar;   // gang barrier arrivals (monotonic)
  int32_t gang;   // workgroups in the gang
  int32_t vw;     // cells per lane for this instance's tiles
  int32_t pad;
};

// One gang membership of a workgroup: instance, z-slab [z0, z1), rank.
struct EnsWork {
  int32_t inst, z0, z1, rank;
};

struct EnsSched {
  const EnsWork* items;  // memberships, grouped per workgroup
  const int32_t* offs;   // workgroup w owns items[offs[w] .. offs[w+1])
  uint32_t* error;       // set when a gang barrier waited past spin_limit
  int64_t spin_limit;
};

// The persistent ensemble kernel: grid = nwg co-resident workgroups.
hipError_t launch_ensemble(int dtype, EnsInst* inst, EnsSched s, int nwg, hipStream_t st);
// Workgroups of the persistent kernel that fit on one CU at once.
int ensemble_blocks_per_cu(int dtype);

}  // namespace hode
