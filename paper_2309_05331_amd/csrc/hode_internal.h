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
// Stage kernels: RK4 (D1 R2 R3 R4), Dopri5 (D1 D2 .. D7; D7F, D6F fixed
// step), Cash-Karp 5(4) (D1 D2 D3 share the Dopri5 stage shapes and
// coefficients; C4 C5, then C6 = stage 6 with new state and error norm, C6F
// its fixed-step form) and explicit Euler (E1: the new state y + h f(y)).
// Fehlberg 7(8): F1 .. F12 write k1 .. k12, F13 evaluates k13 and forms the
// new state and the error norm at the own cell (F13F: new state only).
// Adams-Bashforth with s steps: AB<s> writes f_n = f(y_n) into the ring of
// past right-hand sides and forms y_{n+1} from it and the s - 1 before.
enum GSKind : int {
  K_D1 = 0, K_R2, K_R3, K_R4, K_D2, K_D3, K_D4, K_D5, K_D6, K_D7, K_D7F, K_C4, K_C5, K_C6, K_C6F, K_E1, K_COUNT,
  K_D6F = K_COUNT,  // fixed-step stage 6: the new state only
  K_F1, K_F2, K_F3, K_F4, K_F5, K_F6, K_F7, K_F8, K_F9, K_F10, K_F11, K_F12, K_F13, K_F13F,
  K_AB1, K_AB2, K_AB3, K_AB4, K_AB5, K_AB6, K_AB7, K_AB8,
  K_D6K,  // Dopri5 stage 6 that also stores k6 (dense output)
  // Adams-Moulton correctors of Adams-Bashforth-Moulton with s steps: f(p)
  // of the prediction p (in the spare state buffer) and the corrected state,
  // written over y_n (each cell's y_n is read only by the thread that writes it)
  K_ABC1, K_ABC2, K_ABC3, K_ABC4, K_ABC5, K_ABC6, K_ABC7, K_ABC8,
  // modified midpoint (two substeps of h = H/2): MM1 z1 = y + h f(y), MM2
  // z2 = y + 2h f(z1), MM3 y_new = (z2 + z1 + h f(z2)) / 2
  K_MM1, K_MM2, K_MM3,
  K_ALL   // number of kinds
};

// Extra arrays of the Fehlberg and Adams-Bashforth kinds (device table
// xk(GSLaunch)): k1 .. k12 of Fehlberg 7(8) at 0 .. 11, the ring of the last
// s right-hand sides of Adams-Bashforth at kRingBase .. kRingBase + s - 1.
// k6 of Dopri5 for dense output at kXkK6; the modified midpoint's z1, z2
// at kXkZ1, kXkZ1 + 1.
constexpr int kXkF78 = 12, kXkK6 = 12, kXkZ1 = 13, kRingBase = 16, kXkCount = 24;

struct GSLaunch {
  void* y[2];    // state, indexed by the device-side parity
  void* ks[2];   // first-same-as-last pair: k1 = ks[k1slot], k7 = ks[k1slot ^ 1]
  void* k[7];    // k[2] .. k[6]; k[0]: device table of the extra arrays (void* [kXkCount], see xk())
  int64_t n3;    // N^3, the stride between the u and v fields
  int32_t N;
  int32_t zc;    // z-planes marched by one workgroup
  double Du_h2, Dv_h2, F, kk;
};

// ry: rows per wavefront strip (tile = 64*vw x nw*ry cells); vw: cells per
// lane (1, 2 or 4 for fp32, 1 or 2 for fp64, dividing N; 0 picks the widest).
// The device table of the extra arrays (null if none), kept in the unused
// stage slot k[0] so the layout of the launch arguments stays that of the
// other kinds.
__host__ __device__ inline void* const* xk(const GSLaunch& a) { return (void* const*)a.k[0]; }

// nw: wavefronts per workgroup (tile = 64*vw x nw*ry cells): 4, or 8 for the
// kinds of gs.hip with ry <= 2 and 16-byte lanes (gs_tile_supported).
hipError_t launch_gs(int kind, int dtype, int ry, int vw, int nw, const GSLaunch& a, DevCtrl* c, hipStream_t s);
// The Fehlberg and Adams-Bashforth kinds (K_F1 .. K_AB8), four wavefronts.
hipError_t launch_gsx(int kind, int dtype, int ry, int vw, const GSLaunch& a, DevCtrl* c, hipStream_t s);
// The Fehlberg kinds (K_F1 .. K_F13F) with eight wavefronts: one-row strips,
// 16-byte lanes.
hipError_t launch_gsf8(int kind, int dtype, int ry, int vw, const GSLaunch& a, DevCtrl* c, hipStream_t s);
bool gsf_kind(int kind);
bool gs_ry_supported(int ry);
bool gs_tile_supported(int kind, int dtype, int ry, int vw, int nw, int N);

// Element-wise families: the whole step runs in registers (one kernel per
// attempt).  mode: one of the Mode values (RK4, Dopri5 or Cash-Karp; fixed or adaptive).
hipError_t launch_ew(int dtype, int rhs, int mode, void* y0, void* y1, int64_t n, int grid, DevCtrl* c,
                     hipStream_t s);
// Fehlberg 7(8) and Adams-Bashforth steps of the element-wise families.
// xk: device table as for the Gray-Scott kinds (the ring of past right-hand
// sides); kout: if not null, the fixed Fehlberg step also stores k1 = f(y)
// there.
hipError_t launch_ewx(int dtype, int rhs, int mode, int ab_steps, void* y0, void* y1, void* const* xk, void* kout,
                      int64_t n, int grid, DevCtrl* c, hipStream_t s);

// Dense output of Dopri5 at theta in [0, 1] of the last accepted step of
// size h: out = y_n + h sum_j w_j(theta) k_j.  Gray-Scott: from the stored
// stages (k2 has weight 0); element-wise: the stages are evaluated again from
// y_n in registers, exactly as the step evaluated them.
hipError_t launch_dense_k(int dtype, void* out, const void* yn, const void* k1, const void* k3, const void* k4,
                          const void* k5, const void* k6, const void* k7, int64_t n, int grid, double h, double theta,
                          hipStream_t s);
hipError_t launch_dense_ew(int dtype, int rhs, void* out, const void* yn, int64_t n, int grid, double h,
                           double theta, hipStream_t s);

// The step controller: one wavefront, run after the final stage kernel of
// every attempt or fixed step.
hipError_t launch_ctrl(DevCtrl* c, hipStream_t s);

// out = f(y) for the element-wise systems (no control block involved).
hipError_t launch_ew_rhs(int dtype, int rhs, const void* y, void* out, int64_t n, int grid, hipStream_t s);

// ---- batched ensemble -------------------------------------------------------
// One instance of the ensemble: its grid and arrays, its own control block
// (time, step, controller state, counters).
struct EnsInst {
  GSLaunch a;
  DevCtrl ctrl;
  int64_t pause_at;   // the instance sits out the rest of a launch once ctrl.attempts reaches this
  int32_t vw;         // cells per lane for this instance's tiles
  int32_t k1_valid;   // k1 = f(y) is already in the first-same-as-last slot (resumed instance)
  int32_t seg;        // > 1: segmented rows (vw = 16 bytes / element, one row per 64/seg lanes, rounded down)
  int32_t ntiles;     // tiles of this instance in a stage phase
  uint32_t last_done; // last-stage tiles of the current round finished (zero at launch)
  int32_t rows;       // rows of one tile pass (the row chunk of this instance's tiles)
  int32_t zc_fix;     // planes per tile set for this instance (0: sized from the running cells)
  float weight;       // per-attempt work estimate (dealing to the per-XCD queues)
};

// One tile of a stage phase: rows [y0, y1) (y0 a multiple of the tile pass
// height of every stage kind) and planes [z0, z1) of one instance, all
// columns.
struct EnsTile {
  int32_t inst, y0, y1, z0, z1, pad;
};

// Launch parameters the kernel reads from device memory (so one captured
// graph serves every launch).
struct EnsParams {
  int32_t rounds;     // attempts per instance in this launch (at most)
  int32_t first_d1;   // run a stage-1 phase first (some instance has no k1 yet)
  int32_t n_inst;
  int32_t retile_at;  // re-tile once at most this many instances are running (0: never)
  int32_t tiles_cap;  // tiles the tile buffer holds
  int32_t pad[3];
};

// Wavefronts per workgroup of the persistent ensemble kernel: eight, so a
// tile pass covers twice the rows of a four-wavefront tile (half the halo
// rows per cell) at the same occupancy (two waves per SIMD either way).
constexpr int kEnsNW = 8;
// Instances up to which the persistent kernel re-tiles on the device (the
// re-tiling keeps its per-instance lists in the workgroup's tile LDS).
constexpr int kRetileMaxInst = 2048;
// Tiles per workgroup and phase that the plane ranges are sized for.
constexpr double kTilesPerWorkgroup = 0.5;

struct EnsSched {
  EnsTile* tiles;           // tiles, grouped in eight queues (one per XCD)
  int32_t* qoff;            // queue x holds tiles[qoff[x] .. qoff[x+1])
  const int32_t* order;     // every instance, largest work estimate first (dealing order)
  uint32_t* qctr;           // claim counters: two alternating sets of 8 (zero at launch)
  uint64_t* bar;            // grid barrier: XCDs whose workgroups have all arrived (zero at launch)
  uint64_t* xbar;           // grid barrier: arrivals per XCD, one 128-byte line each (zero at launch)
  uint32_t* live;           // instances still running after a round: two alternating (zero at launch)
  uint32_t* error;          // set when a barrier waited past spin_limit
  const EnsParams* params;
  int64_t spin_limit;
};

// The persistent ensemble kernel: grid = nwg co-resident workgroups.
hipError_t launch_ensemble(int dtype, EnsInst* inst, EnsSched s, int nwg, hipStream_t st);
// Workgroups of the persistent kernel that fit on one CU at once.
int ensemble_blocks_per_cu(int dtype);

}  // namespace hode
