// Fused Runge-Kutta stage kernels for the periodic 3D Gray-Scott system.
//
// System (the paper's Gray-Scott equation and its System functor listing):
//   du/dt = Du Lap(u) - u v^2 + F (1 - u)
//   dv/dt = Dv Lap(v) + u v^2 - (F + k) v
// with Lap the 7-point finite-difference Laplacian on an N^3 periodic grid of
// spacing L/N.  One kernel per Runge-Kutta stage fuses the Algebra (the stage
// input y + h sum_j a_sj k_j, formed on the fly, neighbour cells included),
// the System (stencil + reaction) and the stage's outputs.
//
// Layout: field-major SoA, u then v, each N^3 with x fastest.
//
// Work decomposition (2.5D blocking): a workgroup of NW wavefronts (4 or 8)
// owns a tile of 64*VW x NW*RY cells of an x-y plane and marches a chunk of zc
// planes in z.
// Each wavefront owns a strip of RY consecutive x-rows, VW cells per lane (one
// 16-byte load per lane per row).  Per plane, every row is loaded from memory
// once: the stage input is formed in registers, the z neighbours stay in
// registers (planes z-1, z, z+1), x neighbours come across lanes by shuffle,
// y neighbours inside a strip are the wave's own rows, and only the strips'
// first and last rows plus the tile halo (the rows above and below the tile,
// the two x-halo columns) pass through a small double-buffered LDS area: one
// barrier per plane.  Periodic wrap is folded into precomputed offsets; lanes
// and rows beyond a ragged edge load wrapped cells, which are exactly the
// neighbours the edge cells need, and write nothing.
//
// Dopri5 stages 6 and 7 are restructured so stage 7 reads 3 arrays instead of
// 6: stage 6 forms the new state y + h sum b_j k_j (= the stage-7 input, first
// same as last) and the partial error h sum_{j<=6} (b_j - bhat_j) k_j at the
// own cell and stores both instead of k6; stage 7 evaluates k7 = f(ynew) and
// completes the error with h (b_7 - bhat_7) k7.
#pragma once

#include "hode_internal.h"

namespace hode {

namespace {

// array ids: the state pair and the Runge-Kutta stages of RK4, Dopri5 and
// Cash-Karp; Fehlberg's k_j at A_X0 + j - 1; Adams-Bashforth's f_{n-j} (ring
// of past right-hand sides) at A_RG0 + j
enum : int { A_Y = 0, A_K1 = 1, A_K2, A_K3, A_K4, A_K5, A_E6 = 6, A_K7 = 7, A_YN = 8, A_X0 = 16, A_RG0 = 40 };

struct KindDesc {
  int ns;          // source arrays forming the stage input (first has coefficient 1)
  int src[10];
  double a[10];    // stage-input coefficients (times h); a[0] unused
  int nx;          // extra arrays needed at the own cell only
  int extra[8];
  int out;         // array receiving f(stage input), -1 none
  int fin;         // own-cell finish: 0 none, 1 RK4 new state, 2 Dopri5 new state (+ partial error),
                   // 3 Dopri5 error completion, 4 Cash-Karp new state (+ error norm),
                   // 5 Euler new state, 6 Fehlberg 7(8) new state (+ error norm),
                   // 7 Adams-Bashforth new state, 8 Adams-Moulton correction (in place),
                   // 9, 10, 11 modified midpoint z1, z2, new state
  bool err;        // error norm computed
  int ab;          // Adams-Bashforth steps (ring size), 0 otherwise
};

constexpr double B1 = 35.0 / 384.0, B3 = 500.0 / 1113.0, B4 = 125.0 / 192.0, B5 = -2187.0 / 6784.0,
                 B6 = 11.0 / 84.0;
constexpr double D1 = 35.0 / 384.0 - 5179.0 / 57600.0, D3 = 500.0 / 1113.0 - 7571.0 / 16695.0,
                 D4 = 125.0 / 192.0 - 393.0 / 640.0, D5 = -2187.0 / 6784.0 + 92097.0 / 339200.0,
                 D6 = 11.0 / 84.0 - 187.0 / 2100.0, D7 = -1.0 / 40.0;

// Cash-Karp 5(4) (Cash & Karp 1990): 5th-order weights CB (b2 = b5 = 0) and
// CE = b - bhat (the embedded estimate's weights; CE2 = 0).
constexpr double CB1 = 37.0 / 378.0, CB3 = 250.0 / 621.0, CB4 = 125.0 / 594.0, CB6 = 512.0 / 1771.0;
constexpr double CE1 = 37.0 / 378.0 - 2825.0 / 27648.0, CE3 = 250.0 / 621.0 - 18575.0 / 48384.0,
                 CE4 = 125.0 / 594.0 - 13525.0 / 55296.0, CE5 = -277.0 / 14336.0,
                 CE6 = 512.0 / 1771.0 - 1.0 / 4.0;

constexpr KindDesc kDesc[K_COUNT] = {
    /* D1  */ {1, {A_Y}, {0}, 0, {0, 0}, A_K1, 0, false},
    /* R2  */ {2, {A_Y, A_K1}, {0, 0.5}, 0, {0, 0}, A_K2, 0, false},
    /* R3  */ {2, {A_Y, A_K2}, {0, 0.5}, 0, {0, 0}, A_K3, 0, false},
    /* R4  */ {2, {A_Y, A_K3}, {0, 1.0}, 2, {A_K1, A_K2}, -1, 1, false},
    /* D2  */ {2, {A_Y, A_K1}, {0, 1.0 / 5.0}, 0, {0, 0}, A_K2, 0, false},
    /* D3  */ {3, {A_Y, A_K1, A_K2}, {0, 3.0 / 40.0, 9.0 / 40.0}, 0, {0, 0}, A_K3, 0, false},
    /* D4  */ {4, {A_Y, A_K1, A_K2, A_K3}, {0, 44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0}, 0, {0, 0}, A_K4, 0, false},
    /* D5  */ {5, {A_Y, A_K1, A_K2, A_K3, A_K4},
               {0, 19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0}, 0, {0, 0}, A_K5, 0,
               false},
    /* D6  */ {6, {A_Y, A_K1, A_K2, A_K3, A_K4, A_K5},
               {0, 9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0}, 0, {0, 0},
               -1, 2, true},
    /* D7  */ {1, {A_YN}, {0}, 2, {A_E6, A_Y}, A_K7, 3, true},
    /* D7F */ {1, {A_YN}, {0}, 0, {0, 0}, A_K7, 0, false},
    /* C4  */ {4, {A_Y, A_K1, A_K2, A_K3}, {0, 3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0}, 0, {0, 0}, A_K4, 0, false},
    /* C5  */ {5, {A_Y, A_K1, A_K2, A_K3, A_K4}, {0, -11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0}, 0, {0, 0},
               A_K5, 0, false},
    /* C6  */ {6, {A_Y, A_K1, A_K2, A_K3, A_K4, A_K5},
               {0, 1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0}, 0, {0, 0},
               -1, 4, true},
    /* C6F */ {6, {A_Y, A_K1, A_K2, A_K3, A_K4, A_K5},
               {0, 1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0}, 0, {0, 0},
               -1, 4, false},
    /* E1  */ {1, {A_Y}, {0}, 0, {0, 0}, -1, 5, false},
};
// D6 in fixed-step mode: the new state only (no partial error).
constexpr KindDesc kD6F = {6, {A_Y, A_K1, A_K2, A_K3, A_K4, A_K5},
                           {0, 9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0},
                           0, {0, 0}, -1, 2, false};

// Runge-Kutta-Fehlberg 7(8) (Fehlberg 1968): rows of the stage-input
// coefficients over the stages they use (zero columns skipped), the 8th-order
// weights FB (b1 = .. = b5 = b11 = 0) and the error weights: b - bhat is
// 41/840 times (-1, 0, .., 0, -1, 1, 1) over k1, k11, k12, k13.
constexpr int X1 = A_X0, X2 = A_X0 + 1, X3 = A_X0 + 2, X4 = A_X0 + 3, X5 = A_X0 + 4, X6 = A_X0 + 5,
              X7 = A_X0 + 6, X8 = A_X0 + 7, X9 = A_X0 + 8, X10 = A_X0 + 9, X11 = A_X0 + 10, X12 = A_X0 + 11;
constexpr double FB6 = 34.0 / 105.0, FB7 = 9.0 / 35.0, FB9 = 9.0 / 280.0, FB12 = 41.0 / 840.0, FE = 41.0 / 840.0;
#define HODE_F13_ROW                                                                                      \
  10, {A_Y, X1, X4, X5, X6, X7, X8, X9, X10, X12},                                                         \
      {0, -1777.0 / 4100.0, -341.0 / 164.0, 4496.0 / 1025.0, -289.0 / 82.0, 2193.0 / 4100.0, 51.0 / 82.0, \
       33.0 / 164.0, 12.0 / 41.0, 1.0}
constexpr KindDesc kDescX[K_ALL - K_F1] = {
    /* F1  */ {1, {A_Y}, {0}, 0, {0}, X1, 0, false, 0},
    /* F2  */ {2, {A_Y, X1}, {0, 2.0 / 27.0}, 0, {0}, X2, 0, false, 0},
    /* F3  */ {3, {A_Y, X1, X2}, {0, 1.0 / 36.0, 1.0 / 12.0}, 0, {0}, X3, 0, false, 0},
    /* F4  */ {3, {A_Y, X1, X3}, {0, 1.0 / 24.0, 1.0 / 8.0}, 0, {0}, X4, 0, false, 0},
    /* F5  */ {4, {A_Y, X1, X3, X4}, {0, 5.0 / 12.0, -25.0 / 16.0, 25.0 / 16.0}, 0, {0}, X5, 0, false, 0},
    /* F6  */ {4, {A_Y, X1, X4, X5}, {0, 1.0 / 20.0, 1.0 / 4.0, 1.0 / 5.0}, 0, {0}, X6, 0, false, 0},
    /* F7  */ {5, {A_Y, X1, X4, X5, X6}, {0, -25.0 / 108.0, 125.0 / 108.0, -65.0 / 27.0, 125.0 / 54.0}, 0, {0},
               X7, 0, false, 0},
    /* F8  */ {5, {A_Y, X1, X5, X6, X7}, {0, 31.0 / 300.0, 61.0 / 225.0, -2.0 / 9.0, 13.0 / 900.0}, 0, {0}, X8,
               0, false, 0},
    /* F9  */ {7, {A_Y, X1, X4, X5, X6, X7, X8},
               {0, 2.0, -53.0 / 6.0, 704.0 / 45.0, -107.0 / 9.0, 67.0 / 90.0, 3.0}, 0, {0}, X9, 0, false, 0},
    /* F10 */ {8, {A_Y, X1, X4, X5, X6, X7, X8, X9},
               {0, -91.0 / 108.0, 23.0 / 108.0, -976.0 / 135.0, 311.0 / 54.0, -19.0 / 60.0, 17.0 / 6.0,
                -1.0 / 12.0},
               0, {0}, X10, 0, false, 0},
    /* F11 */ {9, {A_Y, X1, X4, X5, X6, X7, X8, X9, X10},
               {0, 2383.0 / 4100.0, -341.0 / 164.0, 4496.0 / 1025.0, -301.0 / 82.0, 2133.0 / 4100.0,
                45.0 / 82.0, 45.0 / 164.0, 18.0 / 41.0},
               0, {0}, X11, 0, false, 0},
    /* F12 */ {7, {A_Y, X1, X6, X7, X8, X9, X10},
               {0, 3.0 / 205.0, -6.0 / 41.0, -3.0 / 205.0, -3.0 / 41.0, 3.0 / 41.0, 6.0 / 41.0}, 0, {0}, X12, 0,
               false, 0},
    /* F13 */ {HODE_F13_ROW, 1, {X11}, -1, 6, true, 0},
    /* F13F*/ {HODE_F13_ROW, 0, {0}, -1, 6, false, 0},
    /* AB1 */ {1, {A_Y}, {0}, 0, {0}, -1, 7, false, 1},
    /* AB2 */ {1, {A_Y}, {0}, 1, {A_RG0 + 1}, A_RG0, 7, false, 2},
    /* AB3 */ {1, {A_Y}, {0}, 2, {A_RG0 + 1, A_RG0 + 2}, A_RG0, 7, false, 3},
    /* AB4 */ {1, {A_Y}, {0}, 3, {A_RG0 + 1, A_RG0 + 2, A_RG0 + 3}, A_RG0, 7, false, 4},
    /* AB5 */ {1, {A_Y}, {0}, 4, {A_RG0 + 1, A_RG0 + 2, A_RG0 + 3, A_RG0 + 4}, A_RG0, 7, false, 5},
    /* AB6 */ {1, {A_Y}, {0}, 5, {A_RG0 + 1, A_RG0 + 2, A_RG0 + 3, A_RG0 + 4, A_RG0 + 5}, A_RG0, 7, false, 6},
    /* AB7 */ {1, {A_Y}, {0}, 6, {A_RG0 + 1, A_RG0 + 2, A_RG0 + 3, A_RG0 + 4, A_RG0 + 5, A_RG0 + 6}, A_RG0, 7,
               false, 7},
    /* AB8 */ {1, {A_Y}, {0}, 7, {A_RG0 + 1, A_RG0 + 2, A_RG0 + 3, A_RG0 + 4, A_RG0 + 5, A_RG0 + 6, A_RG0 + 7},
               A_RG0, 7, false, 8},
    /* D6K */ {6, {A_Y, A_K1, A_K2, A_K3, A_K4, A_K5},
               {0, 9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0}, 0, {0},
               A_X0 + kXkK6, 2, true, 0},
    // correctors: the stencil over the prediction (spare state buffer); at the
    // own cell y_n and f_n .. f_{n+2-s} from the ring
    /* ABC1 */ {1, {A_YN}, {0}, 1, {A_Y}, -1, 8, false, 1},
    /* ABC2 */ {1, {A_YN}, {0}, 2, {A_Y, A_RG0}, -1, 8, false, 2},
    /* ABC3 */ {1, {A_YN}, {0}, 3, {A_Y, A_RG0, A_RG0 + 1}, -1, 8, false, 3},
    /* ABC4 */ {1, {A_YN}, {0}, 4, {A_Y, A_RG0, A_RG0 + 1, A_RG0 + 2}, -1, 8, false, 4},
    /* ABC5 */ {1, {A_YN}, {0}, 5, {A_Y, A_RG0, A_RG0 + 1, A_RG0 + 2, A_RG0 + 3}, -1, 8, false, 5},
    /* ABC6 */ {1, {A_YN}, {0}, 6, {A_Y, A_RG0, A_RG0 + 1, A_RG0 + 2, A_RG0 + 3, A_RG0 + 4}, -1, 8, false, 6},
    /* ABC7 */ {1, {A_YN}, {0}, 7, {A_Y, A_RG0, A_RG0 + 1, A_RG0 + 2, A_RG0 + 3, A_RG0 + 4, A_RG0 + 5}, -1, 8,
                false, 7},
    /* ABC8 */ {1, {A_YN}, {0}, 8,
                {A_Y, A_RG0, A_RG0 + 1, A_RG0 + 2, A_RG0 + 3, A_RG0 + 4, A_RG0 + 5, A_RG0 + 6}, -1, 8, false, 8},
    /* MM1 */ {1, {A_Y}, {0}, 0, {0}, -1, 9, false, 0},
    /* MM2 */ {1, {A_X0 + kXkZ1}, {0}, 1, {A_Y}, -1, 10, false, 0},
    /* MM3 */ {1, {A_X0 + kXkZ1 + 1}, {0}, 1, {A_X0 + kXkZ1}, -1, 11, false, 0},
};
#undef HODE_F13_ROW

template <int KIND>
__host__ __device__ constexpr KindDesc desc() {
  return KIND < K_COUNT ? kDesc[KIND] : (KIND == K_COUNT ? kD6F : kDescX[KIND - K_F1]);
}

// rg: ring slot of f_n (Adams-Bashforth kinds), S: ring size
template <typename T>
__device__ inline T* array_ptr(const GSLaunch& a, int id, int p, int ks, int rg, int S) {
  if (id >= A_RG0) {
    const int j = id - A_RG0;
    return (T*)xk(a)[kRingBase + (rg + S - j) % S];
  }
  if (id >= A_X0) return (T*)xk(a)[id - A_X0];
  switch (id) {
    case A_Y: return (T*)a.y[p];
    case A_YN: return (T*)a.y[p ^ 1];
    case A_K1: return (T*)a.ks[ks];
    case A_K7: return (T*)a.ks[ks ^ 1];
    default: return (T*)a.k[id];
  }
}

template <typename T, int VW>
struct VecT;
template <>
struct VecT<float, 4> { using type = float4; };
template <>
struct VecT<float, 2> { using type = float2; };
template <>
struct VecT<float, 1> { using type = float; };
template <>
struct VecT<double, 2> { using type = double2; };
template <>
struct VecT<double, 1> { using type = double; };

template <typename T, int VW>
struct Pk {
  T v[VW];
};

template <typename T, int VW>
__device__ __forceinline__ Pk<T, VW> ldv(const T* __restrict__ p, int64_t g) {
  using V = typename VecT<T, VW>::type;
  const V x = *reinterpret_cast<const V*>(p + g);
  Pk<T, VW> r;
  __builtin_memcpy(&r, &x, sizeof(r));
  return r;
}

#ifndef HODE_NT_STORES
#define HODE_NT_STORES 1
#endif

// Stage outputs are streamed out with non-temporal stores: each array is
// written once and read by later stage kernels, far beyond what L2 holds.
template <typename T, int VW>
__device__ __forceinline__ void stv(T* __restrict__ p, int64_t g, const Pk<T, VW>& r) {
  if constexpr (HODE_NT_STORES) {
    if constexpr (VW == 1) {
      __builtin_nontemporal_store(r.v[0], p + g);
    } else {
      typedef T V __attribute__((ext_vector_type(VW)));
      V x;
#pragma unroll
      for (int e = 0; e < VW; ++e) x[e] = r.v[e];
      __builtin_nontemporal_store(x, reinterpret_cast<V*>(p + g));
    }
  } else {
    using V = typename VecT<T, VW>::type;
    V x;
    __builtin_memcpy(&x, &r, sizeof(r));
    *reinterpret_cast<V*>(p + g) = x;
  }
}

template <typename T>
__device__ __forceinline__ T shfl_up1(T v) {
  return __shfl_up(v, 1, 64);
}
template <typename T>
__device__ __forceinline__ T shfl_down1(T v) {
  return __shfl_down(v, 1, 64);
}

// LDS row slots of a tile, per buffer and field: the tile halo above (slot
// 0) and below (the last slot), and per wavefront the first and last row of
// its strip (one slot when the strip is one row).
template <int RY, int NW>
__host__ __device__ constexpr int row_slots() {
  return (RY == 1 ? NW : 2 * NW) + 2;
}
template <int RY>
__device__ constexpr int first_slot(int w) {
  return RY == 1 ? 1 + w : 1 + 2 * w;
}
template <int RY>
__device__ constexpr int last_slot(int w) {
  return RY == 1 ? 1 + w : 2 + 2 * w;
}

// Bytes of LDS one stage tile needs: the row slots of two buffers and two
// fields, and the x-halo cells (ordinary tiles only).
template <typename T, int VW, int RY, int NW, int SEG>
__host__ __device__ constexpr int tile_smem() {
  return 2 * 2 * row_slots<RY, NW>() * 64 * (int)sizeof(Pk<T, VW>) +
         2 * 2 * 2 * (SEG == 1 ? NW * RY : 1) * (int)sizeof(T);
}

// One stage over one tile: columns tx*64*VW .. (tx+1)*64*VW - 1, rows
// ty*TY .. (ty+1)*TY - 1 (TY = NW*RY*SEG), planes zbeg .. zend - 1 of the
// grid described by `a`, with step h, parity and first-same-as-last slot
// taken from the control block.  Called by all 64*NW threads of a workgroup;
// smem holds at least tile_smem<T, VW, RY, NW, SEG>() bytes of LDS.
//
// Segmented rows (SEG > 1, for grids whose rows are at most 64*VW/SEG cells):
// each wavefront is cut into SEG segments of 64/SEG lanes (rounded down: SEG
// need not divide 64, and the lanes left over load wrapped cells and write
// nothing) and every segment of a register row holds one whole x-row, so
// register row r of a wave holds rows r*SEG .. r*SEG + SEG - 1 of its strip
// of RY*SEG rows, and the tile is the full width of the grid (tx = 0).  x neighbours wrap inside the
// segment; the rows above and below come from the neighbouring segment, or
// the last/first segment of the neighbouring register row, by cross-lane
// permutes, and across strips from the LDS row slots as for the ordinary
// tiles; no x-halo is needed.  The arithmetic of every cell is the same
// expression in the same order, so the results are bitwise those of the
// ordinary tiles.
template <typename T, int KIND, int RY, int VW, int SEG = 1, int NW = 4>
__device__ void stage_tile(const GSLaunch& a, DevCtrl* __restrict__ c, char* smem, int tx, int ty, int zbeg,
                           int zend) {
  constexpr KindDesc D = desc<KIND>();
  static_assert(SEG >= 1 && 64 / SEG >= 4, "segments of at least four lanes");
  static_assert(NW >= 3, "three wavefronts carry the halo roles");
  constexpr int SL = 64 / SEG;  // lanes per segment (lanes SEG*SL .. 63 idle)
  constexpr int TX = 64 * VW;
  constexpr int TY = NW * RY * SEG;
  constexpr int TYX = SEG == 1 ? TY : 1;  // x-halo cells per column (ordinary tiles only)
  static_assert(SEG > 1 || 2 * TY <= 64, "the x-halo role holds both halo columns in one wavefront");
  constexpr int NS = row_slots<RY, NW>();
  using P = Pk<T, VW>;
  // LDS per buffer and field: the row slots (tile halo above, first and last
  // row of each wave's strip, tile halo below) and the x-halo cells; the
  // caller provides tile_smem<T, VW, RY, NW, SEG>() bytes
  P(*rows)[2][NS][64] = reinterpret_cast<P(*)[2][NS][64]>(smem);
  T(*xh)[2][2][TYX] = reinterpret_cast<T(*)[2][2][TYX]>(smem + 2 * 2 * NS * 64 * sizeof(P));
  __syncthreads();  // LDS may still be in use by the previous tile

  const double h = c->h;
  const int p = c->parity, ksl = c->k1slot;
  const int rg = D.ab > 1 ? c->ring : 0;
  const int N = a.N;
  const int64_t n3 = a.n3;
  const int64_t NN = (int64_t)N * N;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int seg = SEG == 1 ? 0 : lane / SL;  // segment of this lane
  const int jl = SEG == 1 ? lane : lane % SL;  // lane within the segment
  const int x0 = tx * TX, yt = ty * TY;
  const int y0 = yt + wv * RY * SEG + seg;  // first row of this lane's strip

  const T* src[10];
#pragma unroll
  for (int i = 0; i < D.ns; ++i) src[i] = array_ptr<T>(a, D.src[i], p, ksl, rg, D.ab);
  const T* ext[8];
#pragma unroll
  for (int i = 0; i < D.nx; ++i) ext[i] = array_ptr<T>(a, D.extra[i], p, ksl, rg, D.ab);
  T* out = D.out >= 0 ? array_ptr<T>(a, D.out, p, ksl, rg, D.ab) : nullptr;
  T* ynew = D.fin == 9    ? (T*)xk(a)[kXkZ1]
           : D.fin == 10 ? (T*)xk(a)[kXkZ1 + 1]
           : (D.fin == 1 || D.fin == 2 || D.fin >= 4) ? (T*)a.y[D.fin == 8 ? p : p ^ 1]
                                                       : nullptr;
  T* e6 = (D.fin == 2 && D.err) ? (T*)a.k[A_E6] : nullptr;

  T cf[10];
#pragma unroll
  for (int i = 1; i < D.ns; ++i) cf[i] = (T)(h * D.a[i]);
  const T Du = (T)a.Du_h2, Dv = (T)a.Dv_h2, F = (T)a.F, Fk = (T)(a.F + a.kk);
  const double atol = c->atol, rtol = c->rtol;
  (void)atol;
  (void)rtol;
  const T b16 = (T)(h * (1.0 / 6.0)), b13 = (T)(h * (1.0 / 3.0));
  const T q1 = (T)(h * B1), q3 = (T)(h * B3), q4 = (T)(h * B4), q5 = (T)(h * B5), q6 = (T)(h * B6);
  const double h1 = h * D1, h3 = h * D3, h4 = h * D4, h5 = h * D5, h6 = h * D6, h7 = h * D7;
  const T cq1 = (T)(h * CB1), cq3 = (T)(h * CB3), cq4 = (T)(h * CB4), cq6 = (T)(h * CB6);
  const T hT = (T)h;
  const T hm = (T)(0.5 * h), hm2 = (T)h;  // modified midpoint substep h/2 and 2 (h/2)
  const double ce1 = h * CE1, ce3 = h * CE3, ce4 = h * CE4, ce5 = h * CE5, ce6 = h * CE6;
  const T fb6 = (T)(h * FB6), fb7 = (T)(h * FB7), fb9 = (T)(h * FB9), fb12 = (T)(h * FB12);
  const double fe = h * FE;
  T abq[D.ab > 0 ? D.ab : 1];  // Adams-Bashforth (corrector: Adams-Moulton) weights times h
#pragma unroll
  for (int j = 0; j < D.ab; ++j) abq[j] = (T)(h * (D.fin == 8 ? AMW : ABW)[D.ab > 0 ? D.ab - 1 : 0][j]);

  // ---- offsets (periodic wrap folded in)
  const int xl = x0 + VW * jl;
  const int gx = xl % N;  // N % VW == 0, so gx .. gx+VW-1 are one aligned run
  const bool xval = xl < N;
  const int nl = N / VW;  // lanes holding a row (segmented rows)
  (void)nl;
  int rowoff[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) rowoff[r] = N * ((y0 + r * SEG) % N);
  // halo role of this wave: 0 the row above the tile, 1 the row below,
  // 2 the x-halo cells (lanes < TY left column, TY .. 2TY-1 right column)
  // (segmented rows: the row above is kept in the last segment's lanes and
  // the row below in the first segment's, where the strips' edge rows are)
  int hoff = 0;
  bool hact = false;
  if (wv == 0) { hoff = N * ((yt - 1 + N) % N) + gx; hact = SEG == 1 || seg == SEG - 1; }
  else if (wv == 1) { hoff = N * ((yt + TY) % N) + gx; hact = SEG == 1 || seg == 0; }
  else if (SEG == 1 && wv == 2 && lane < 2 * TY) {
    const int side = lane >= TY, rr = lane - side * TY;
    hoff = N * ((yt + rr) % N) + (side ? (x0 + TX) % N : (x0 - 1 + N) % N);
    hact = true;
  }

  // Partial own-cell finish of one row-field, formed at load time so the raw
  // sources need not stay live: RK4 y + h/6 k1 + h/3 k2 + h/3 k3; Dopri5
  // stage 6 y + h sum_{j<6} b_j k_j and (fp64) h sum_{j<6} (b_j - bhat_j) k_j;
  // stage 7 the stored partial error and y.
  struct Fin {
    T a[VW];
    double e[((D.fin == 2 || D.fin == 4 || D.fin == 6) && D.err) ? VW : 1];
    T b[(D.fin == 3 || ((D.fin == 4 || D.fin == 6) && D.err)) ? VW : 1];
  };

  auto stage_in = [&](int64_t g, Fin* fin) -> P {
    P s[10];
#pragma unroll
    for (int i = 0; i < D.ns; ++i) s[i] = ldv<T, VW>(src[i], g);
    P w = s[0];
#pragma unroll
    for (int i = 1; i < D.ns; ++i)
#pragma unroll
      for (int e = 0; e < VW; ++e) w.v[e] += cf[i] * s[i].v[e];
    if constexpr (D.fin != 0) {
      if (fin == nullptr) return w;  // halo cells need no finish
      P x[8];
#pragma unroll
      for (int i = 0; i < D.nx; ++i) x[i] = ldv<T, VW>(ext[i], g);
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        if constexpr (D.fin == 1) {
          // sources y, k3; extras k1, k2
          fin->a[e] = s[0].v[e] + b16 * x[0].v[e] + b13 * x[1].v[e] + b13 * s[1].v[e];
        } else if constexpr (D.fin == 2) {
          // sources y, k1 .. k5
          fin->a[e] = s[0].v[e] + q1 * s[1].v[e] + q3 * s[3].v[e] + q4 * s[4].v[e] + q5 * s[5].v[e];
          if constexpr (D.err)
            fin->e[e] = h1 * (double)s[1].v[e] + h3 * (double)s[3].v[e] + h4 * (double)s[4].v[e] +
                        h5 * (double)s[5].v[e];
        } else if constexpr (D.fin == 5) {
          // source y: Euler keeps the own cell's state for the new state
          fin->a[e] = s[0].v[e];
        } else if constexpr (D.fin == 6) {
          // sources y, k1, k4 .. k10, k12; extra k11: Fehlberg new state and
          // error without k13
          fin->a[e] = s[0].v[e] + fb6 * s[4].v[e] + fb7 * s[5].v[e] + fb7 * s[6].v[e] + fb9 * s[7].v[e] +
                      fb9 * s[8].v[e] + fb12 * s[9].v[e];
          if constexpr (D.err) {
            fin->e[e] = fe * ((double)s[9].v[e] - (double)s[1].v[e] - (double)x[0].v[e]);
            fin->b[e] = s[0].v[e];
          }
        } else if constexpr (D.fin == 7) {
          // source y; extras f_{n-1} .. f_{n-s+1}: Adams-Bashforth without f_n
          T acc = s[0].v[e];
#pragma unroll
          for (int j = 1; j < D.ab; ++j) acc += abq[j] * x[j - 1].v[e];
          fin->a[e] = acc;
        } else if constexpr (D.fin == 9) {
          // source y: z1 = y + (h/2) f(y)
          fin->a[e] = s[0].v[e];
        } else if constexpr (D.fin == 10) {
          // source z1; extra y: z2 = y + h f(z1)
          fin->a[e] = x[0].v[e];
        } else if constexpr (D.fin == 11) {
          // source z2; extra z1: (z2 + z1 + (h/2) f(z2)) / 2
          fin->a[e] = s[0].v[e] + x[0].v[e];
        } else if constexpr (D.fin == 8) {
          // source the prediction; extras y_n, f_n .. f_{n+2-s}: the
          // Adams-Moulton correction without f(p)
          T acc = x[0].v[e];
#pragma unroll
          for (int j = 1; j < D.ab; ++j) acc += abq[j] * x[j].v[e];
          fin->a[e] = acc;
        } else if constexpr (D.fin == 4) {
          // sources y, k1 .. k5: Cash-Karp new state and error without k6
          fin->a[e] = s[0].v[e] + cq1 * s[1].v[e] + cq3 * s[3].v[e] + cq4 * s[4].v[e];
          if constexpr (D.err) {
            fin->e[e] = ce1 * (double)s[1].v[e] + ce3 * (double)s[3].v[e] + ce4 * (double)s[4].v[e] +
                        ce5 * (double)s[5].v[e];
            fin->b[e] = s[0].v[e];
          }
        } else {
          // source ynew; extras partial error, y
          fin->a[e] = x[0].v[e];
          fin->b[e] = x[1].v[e];
        }
      }
    }
    return w;
  };
  auto stage_in1 = [&](int64_t g) -> T {
    T w = src[0][g];
#pragma unroll
    for (int i = 1; i < D.ns; ++i) w += cf[i] * src[i][g];
    return w;
  };

  P wp[2][RY], wc[2][RY], wn[2][RY];
  Fin fc[2][RY], fn[2][RY];
  P hv[2];  // halo data of this wave's role (scalar in .v[0] for the x-halo role)
  uint64_t emax = 0;

  auto load_plane = [&](int z, P (&w)[2][RY], Fin (&fin)[2][RY], bool halo) {
    const int64_t zb = (int64_t)z * NN;
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      const int64_t fb = f * n3 + zb;
#pragma unroll
      for (int r = 0; r < RY; ++r) w[f][r] = stage_in(fb + rowoff[r] + gx, &fin[f][r]);
      if (halo && hact) {
        if (wv < 2) hv[f] = stage_in(fb + hoff, nullptr);
        else hv[f].v[0] = stage_in1(fb + hoff);
      }
    }
  };
  // boundary rows of the strip and the halo role's data go to LDS buffer b
  auto publish = [&](int b, const P (&w)[2][RY]) {
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      rows[b][f][first_slot<RY>(wv)][lane] = w[f][0];
      if constexpr (RY > 1) rows[b][f][last_slot<RY>(wv)][lane] = w[f][RY - 1];
      if (hact) {
        if (wv == 0) rows[b][f][0][lane] = hv[f];
        else if (wv == 1) rows[b][f][NS - 1][lane] = hv[f];
        else if constexpr (SEG == 1) xh[b][f][lane >= TY][lane - (lane >= TY) * TY] = hv[f].v[0];
      }
    }
  };

  // prologue: own rows of plane zbeg-1 (z neighbours), plane zbeg in full
  {
    Fin tmpf[2][RY];
    load_plane((zbeg - 1 + N) % N, wp, tmpf, false);
  }
  load_plane(zbeg, wc, fc, true);
  publish(0, wc);

  for (int z = zbeg; z < zend; ++z) {
    const int b = (z - zbeg) & 1;
    load_plane(z + 1 == N ? 0 : z + 1, wn, fn, true);
    __syncthreads();
    const int64_t zb = (int64_t)z * NN;
    // neighbours across strip boundaries and the x-halo of the strip rows
    P above[2], below[2];
    T xlft[2][RY], xrgt[2][RY];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      if constexpr (SEG == 1) {
        above[f] = rows[b][f][wv == 0 ? 0 : last_slot<RY>(wv - 1)][lane];
        below[f] = rows[b][f][wv == NW - 1 ? NS - 1 : first_slot<RY>(wv + 1)][lane];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
          xlft[f][r] = xh[b][f][0][wv * RY + r];
          xrgt[f][r] = xh[b][f][1][wv * RY + r];
        }
      } else {
        // the strip above ends with its last segment, the strip below starts
        // with its first
        above[f] = rows[b][f][wv == 0 ? 0 : last_slot<RY>(wv - 1)][(SEG - 1) * SL + jl];
        below[f] = rows[b][f][wv == NW - 1 ? NS - 1 : first_slot<RY>(wv + 1)][jl];
      }
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      P fo[2];
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const P& cc = wc[f][r];
        P up, dn;
        T xm0, xpN;
        if constexpr (SEG == 1) {
          up = r == 0 ? above[f] : wc[f][r - 1];
          dn = r == RY - 1 ? below[f] : wc[f][r + 1];
          const T left = shfl_up1(cc.v[VW - 1]);
          const T right = shfl_down1(cc.v[0]);
          xm0 = lane == 0 ? xlft[f][r] : left;
          xpN = lane == 63 ? xrgt[f][r] : right;
        } else {
          // rows of the neighbouring segments (the first segment's upper
          // neighbour is the previous register row's last segment, the last
          // segment's lower one the next register row's first); x wraps
          // inside the segment
          const int lu = (lane - SL) & 63, ld = (lane + SL) & 63;
          const int lu2 = (lane + (SEG - 1) * SL) & 63, ld2 = (lane - (SEG - 1) * SL) & 63;
#pragma unroll
          for (int e = 0; e < VW; ++e) {
            const T vu = __shfl(cc.v[e], lu, 64), vd = __shfl(cc.v[e], ld, 64);
            const T vu2 = r == 0 ? above[f].v[e] : __shfl(wc[f][r > 0 ? r - 1 : 0].v[e], lu2, 64);
            const T vd2 = r == RY - 1 ? below[f].v[e] : __shfl(wc[f][r < RY - 1 ? r + 1 : 0].v[e], ld2, 64);
            up.v[e] = seg == 0 ? vu2 : vu;
            dn.v[e] = seg == SEG - 1 ? vd2 : vd;
          }
          const int base = lane - jl;
          xm0 = __shfl(cc.v[VW - 1], base + (jl == 0 ? nl - 1 : jl - 1), 64);
          xpN = __shfl(cc.v[0], base + (jl >= nl - 1 ? 0 : jl + 1), 64);
        }
#pragma unroll
        for (int e = 0; e < VW; ++e) {
          const T xm = e == 0 ? xm0 : cc.v[e - 1];
          const T xp = e == VW - 1 ? xpN : cc.v[e + 1];
          const T s = (xm + xp + up.v[e] + dn.v[e]);
          fo[f].v[e] = (s + wp[f][r].v[e] + wn[f][r].v[e]) - (T)6 * cc.v[e];
        }
      }
      // reaction terms
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        const T u = wc[0][r].v[e], v = wc[1][r].v[e];
        const T uvv = u * v * v;
        const T lu = fo[0].v[e], lv = fo[1].v[e];
        fo[0].v[e] = Du * lu - uvv + F * ((T)1 - u);
        fo[1].v[e] = Dv * lv + uvv - Fk * v;
      }
      const bool valid = xval && (64 % SEG == 0 || seg < SEG) && (y0 + r * SEG < N);
      if (valid) {
        const int64_t g = zb + rowoff[r] + gx;
        if (D.out >= 0) {
          stv<T, VW>(out, g, fo[0]);
          stv<T, VW>(out, n3 + g, fo[1]);
        }
        if constexpr (D.fin == 1) {
          // RK4 new state
#pragma unroll
          for (int f = 0; f < 2; ++f) {
            P yn;
#pragma unroll
            for (int e = 0; e < VW; ++e) yn.v[e] = fc[f][r].a[e] + b16 * fo[f].v[e];
            stv<T, VW>(ynew, f * n3 + g, yn);
          }
        } else if constexpr (D.fin == 2) {
          // Dopri5 new state (and partial error)
#pragma unroll
          for (int f = 0; f < 2; ++f) {
            P yn, ep;
#pragma unroll
            for (int e = 0; e < VW; ++e) {
              yn.v[e] = fc[f][r].a[e] + q6 * fo[f].v[e];
              if constexpr (D.err) ep.v[e] = (T)(fc[f][r].e[e] + h6 * (double)fo[f].v[e]);
            }
            stv<T, VW>(ynew, f * n3 + g, yn);
            if constexpr (D.err) stv<T, VW>(e6, f * n3 + g, ep);
          }
        } else if constexpr (D.fin == 5) {
          // Euler new state y + h f(y)
#pragma unroll
          for (int f = 0; f < 2; ++f) {
            P yn;
#pragma unroll
            for (int e = 0; e < VW; ++e) yn.v[e] = fc[f][r].a[e] + hT * fo[f].v[e];
            stv<T, VW>(ynew, f * n3 + g, yn);
          }
        } else if constexpr (D.fin == 9 || D.fin == 10 || D.fin == 11) {
          // modified midpoint substeps
#pragma unroll
          for (int f = 0; f < 2; ++f) {
            P yn;
#pragma unroll
            for (int e = 0; e < VW; ++e) {
              if constexpr (D.fin == 9) yn.v[e] = fc[f][r].a[e] + hm * fo[f].v[e];
              else if constexpr (D.fin == 10) yn.v[e] = fc[f][r].a[e] + hm2 * fo[f].v[e];
              else yn.v[e] = (T)0.5 * (fc[f][r].a[e] + hm * fo[f].v[e]);
            }
            stv<T, VW>(ynew, f * n3 + g, yn);
          }
        } else if constexpr (D.fin == 7 || D.fin == 8) {
          // Adams-Bashforth new state y + h sum_j beta_j f_{n-j}, or the
          // Adams-Moulton correction y_n + h (gamma_0 f(p) + sum_j gamma_j f_{n+1-j})
#pragma unroll
          for (int f = 0; f < 2; ++f) {
            P yn;
#pragma unroll
            for (int e = 0; e < VW; ++e) yn.v[e] = fc[f][r].a[e] + abq[0] * fo[f].v[e];
            stv<T, VW>(ynew, f * n3 + g, yn);
          }
        } else if constexpr (D.fin == 6) {
          // Fehlberg 7(8) new state y + h sum b_j k_j and, adaptive, the error
          // |h 41/840 (k12 + k13 - k1 - k11)| / (atol + rtol max(|y|, |ynew|))
#pragma unroll
          for (int f = 0; f < 2; ++f) {
            P yn;
#pragma unroll
            for (int e = 0; e < VW; ++e) yn.v[e] = fc[f][r].a[e] + fb12 * fo[f].v[e];
            stv<T, VW>(ynew, f * n3 + g, yn);
            if constexpr (D.err) {
#pragma unroll
              for (int e = 0; e < VW; ++e) {
                const double err = fc[f][r].e[e] + fe * (double)fo[f].v[e];
                const double sc = atol + rtol * fmax(fabs((double)fc[f][r].b[e]), fabs((double)yn.v[e]));
                const uint64_t bits = (uint64_t)__double_as_longlong(fabs(err) / sc);
                emax = bits > emax ? bits : emax;
              }
            }
          }
        } else if constexpr (D.fin == 4) {
          // Cash-Karp new state y + h sum b_j k_j and, adaptive, the error
          // |h sum (b_j - bhat_j) k_j| / (atol + rtol max(|y|, |ynew|))
#pragma unroll
          for (int f = 0; f < 2; ++f) {
            P yn;
#pragma unroll
            for (int e = 0; e < VW; ++e) yn.v[e] = fc[f][r].a[e] + cq6 * fo[f].v[e];
            stv<T, VW>(ynew, f * n3 + g, yn);
            if constexpr (D.err) {
#pragma unroll
              for (int e = 0; e < VW; ++e) {
                const double err = fc[f][r].e[e] + ce6 * (double)fo[f].v[e];
                const double sc = atol + rtol * fmax(fabs((double)fc[f][r].b[e]), fabs((double)yn.v[e]));
                const uint64_t bits = (uint64_t)__double_as_longlong(fabs(err) / sc);
                emax = bits > emax ? bits : emax;
              }
            }
          }
        } else if constexpr (D.fin == 3) {
          // Dopri5 error completion: |E6 + h d7 k7| / (atol + rtol max(|y|, |ynew|))
#pragma unroll
          for (int f = 0; f < 2; ++f) {
#pragma unroll
            for (int e = 0; e < VW; ++e) {
              const double err = (double)fc[f][r].a[e] + h7 * (double)fo[f].v[e];
              const double sc = atol + rtol * fmax(fabs((double)fc[f][r].b[e]), fabs((double)wc[f][r].v[e]));
              const uint64_t bits = (uint64_t)__double_as_longlong(fabs(err) / sc);
              emax = bits > emax ? bits : emax;
            }
          }
        }
      }
    }
    publish(b ^ 1, wn);
    // rotate planes
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        wp[f][r] = wc[f][r];
        wc[f][r] = wn[f][r];
        if constexpr (D.fin != 0) fc[f][r] = fn[f][r];
      }
    }
  }

  if constexpr (D.err && (D.fin == 3 || D.fin == 4 || D.fin == 6)) {
    emax = wave_max_u64(emax);
    if (lane == 0 && emax) atomicMax((unsigned long long*)&c->errmax_bits, (unsigned long long)emax);
  }
}

// One stage over a whole grid: one tile per workgroup.  The linear block id
// is remapped XCD-aware: workgroups are dealt round-robin to the 8 XCDs, so
// each XCD gets a contiguous range of tiles and y/z-adjacent tiles (whose
// halo rows overlap) share an L2.  Consecutive stages sweep those ranges in
// opposite directions.
template <typename T, int KIND, int RY, int VW, int NW = 4>
__global__ __launch_bounds__(64 * NW) void gs_stage(const GSLaunch a, DevCtrl* __restrict__ c) {
  __shared__ __align__(16) char smem[tile_smem<T, VW, RY, NW, 1>()];
  if (c->done) return;
  const int N = a.N;
  const int nx = (N + 64 * VW - 1) / (64 * VW);
  const int ny = (N + NW * RY - 1) / (NW * RY);
  const int nz = (N + a.zc - 1) / a.zc;
  const int per = (gridDim.x + 7) / 8;
  // Stages alternate their direction through each XCD's range, so a stage
  // starts on the tiles the previous stage wrote last, which are still in the
  // memory-side Infinity Cache.
  // (The Adams-Bashforth kinds alternate with the step; the Adams-Moulton
  // correctors, which keep the parity, sweep against their predictor.)
  constexpr bool rev_k = KIND == K_R2 || KIND == K_R4 || KIND == K_D3 || KIND == K_D5 || KIND == K_D7 ||
                         KIND == K_D7F || KIND == K_C5 || KIND == K_F2 || KIND == K_F4 || KIND == K_F6 ||
                         KIND == K_F8 || KIND == K_F10 || KIND == K_F12 || KIND == K_MM2;
  const bool rev = desc<KIND>().ab > 0 ? ((c->parity & 1) != 0) != (desc<KIND>().fin == 8) : rev_k;
  const int slot = rev ? per - 1 - (int)(blockIdx.x >> 3) : (int)(blockIdx.x >> 3);
  const int bb = (blockIdx.x & 7) * per + slot;
  if (bb >= nx * ny * nz) return;  // padding block of the remap (whole block)
  const int tz = bb / (nx * ny);
  stage_tile<T, KIND, RY, VW, 1, NW>(a, c, smem, bb % nx, (bb / nx) % ny, tz * a.zc, min(N, (tz + 1) * a.zc));
}

// Launches one stage kind over the whole grid with tiles of NW wavefronts x
// RY rows x 64*VW cells (KINDS: the kinds this launcher instantiates).
template <typename T, int RY, int VW, int NW, int... KINDS>
hipError_t launch_stage_t(int kind, const GSLaunch& a, DevCtrl* c, hipStream_t s) {
  constexpr int TX = 64 * VW;
  const int nx = (a.N + TX - 1) / TX;
  const int ny = (a.N + NW * RY - 1) / (NW * RY);
  const int nz = (a.N + a.zc - 1) / a.zc;
  const int64_t nb = (int64_t)nx * ny * nz;
  const int64_t grid = (nb + 7) / 8 * 8;  // whole rounds of the XCD remap
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  bool found = false;
  ((kind == KINDS ? (gs_stage<T, KINDS, RY, VW, NW><<<dim3((unsigned)grid), dim3(64 * NW), 0, s>>>(a, c),
                     found = true)
                  : false),
   ...);
  if (!found) return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

}  // namespace hode
