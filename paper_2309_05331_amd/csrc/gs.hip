// Fused Runge-Kutta stage kernels for the periodic 3D Gray-Scott system.
//
// System (the paper's Gray-Scott equation and its System functor listing):
//   du/dt = Du Lap(u) - u v^2 + F (1 - u)
//   dv/dt = Dv Lap(v) + u v^2 - (F + k) v
// with Lap the 7-point finite-difference Laplacian on an N^3 periodic grid of
// spacing L/N.  One kernel per Runge-Kutta stage fuses the Algebra (the stage
// input y + h sum_j a_sj k_j, formed on the fly, halo cells included), the
// System (stencil + reaction) and the stage's outputs.
//
// Layout: field-major SoA, u then v, each N^3 with x fastest.
// Tiling: a workgroup of 4 wavefronts owns a 64 x (4 ry) tile of an x-y plane
// and marches a chunk of zc planes in z.  Each wavefront covers one 64-cell x
// row per load (coalesced 256 B fp32 / 512 B fp64 rows).  The stage input of
// the current plane, with a one-cell x-y halo, sits in LDS (double buffered:
// one barrier per plane); the z neighbours stay in registers.  Periodic wrap
// is folded into per-thread in-plane offsets computed once, so ragged tiles
// (N not a multiple of the tile) read wrapped cells where the halo needs them.
#include "hode_internal.h"

namespace hode {

namespace {

// Array ids: 0 = y, 1..7 = k1..k7.
struct KindDesc {
  int ns;          // source arrays forming the stage input (first is y)
  int src[6];
  double a[6];     // stage-input coefficients (times h); a[0] unused (y)
  int nx;          // extra arrays needed at the own cell only
  int extra[2];
  int out;         // array id written with f(stage input); -1 none
  int final_kind;  // 0 no; 1 RK4 new state; 2 Dopri5 new state + k7 (+ error)
  bool err;
};

constexpr KindDesc kDesc[K_COUNT] = {
    /* D1 */ {1, {0}, {0}, 0, {0, 0}, 1, 0, false},
    /* R2 */ {2, {0, 1}, {0, 0.5}, 0, {0, 0}, 2, 0, false},
    /* R3 */ {2, {0, 2}, {0, 0.5}, 0, {0, 0}, 3, 0, false},
    /* R4 */ {2, {0, 3}, {0, 1.0}, 2, {1, 2}, -1, 1, false},
    /* D2 */ {2, {0, 1}, {0, 1.0 / 5.0}, 0, {0, 0}, 2, 0, false},
    /* D3 */ {3, {0, 1, 2}, {0, 3.0 / 40.0, 9.0 / 40.0}, 0, {0, 0}, 3, 0, false},
    /* D4 */ {4, {0, 1, 2, 3}, {0, 44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0}, 0, {0, 0}, 4, 0, false},
    /* D5 */ {5, {0, 1, 2, 3, 4},
              {0, 19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0}, 0, {0, 0}, 5, 0, false},
    /* D6 */ {6, {0, 1, 2, 3, 4, 5},
              {0, 9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0}, 0, {0, 0}, 6,
              0, false},
    /* D7 */ {6, {0, 1, 3, 4, 5, 6},
              {0, 35.0 / 384.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0}, 0, {0, 0}, 7, 2, true},
    /* D7F */ {6, {0, 1, 3, 4, 5, 6},
               {0, 35.0 / 384.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0}, 0, {0, 0}, 7, 2,
               false},
};

template <typename T>
struct Ptrs {
  const T* src[6];
  const T* extra[2];
  T* out;
  T* ynew;
};

template <typename T>
__device__ inline T* array_ptr(const GSLaunch& a, int id, int p, int ks) {
  if (id == 0) return (T*)a.y[p];
  if (id == 1) return (T*)a.ks[ks];
  if (id == 7) return (T*)a.ks[ks ^ 1];
  return (T*)a.k[id];
}

constexpr int TX = 64;

template <typename T, int KIND, int RY>
__global__ __launch_bounds__(256) void gs_stage(const GSLaunch a, DevCtrl* __restrict__ c) {
  constexpr KindDesc D = kDesc[KIND];
  constexpr int TY = 4 * RY;
  // raw own-cell values kept for the final combination / error
  constexpr int NR = D.final_kind == 1 ? (D.ns + D.nx) : (D.err ? D.ns : 0);
  __shared__ T lds[2][2][TY + 2][TX + 2];

  if (c->done) return;
  const double h = c->h;
  const int p = c->parity, ksl = c->k1slot;
  const int N = a.N;
  const int64_t n3 = a.n3;
  const int64_t NN = (int64_t)N * N;

  Ptrs<T> P;
#pragma unroll
  for (int i = 0; i < D.ns; ++i) P.src[i] = array_ptr<T>(a, D.src[i], p, ksl);
#pragma unroll
  for (int i = 0; i < D.nx; ++i) P.extra[i] = array_ptr<T>(a, D.extra[i], p, ksl);
  P.out = D.out >= 0 ? array_ptr<T>(a, D.out, p, ksl) : nullptr;
  P.ynew = D.final_kind ? (T*)a.y[p ^ 1] : nullptr;

  T cf[6];
#pragma unroll
  for (int i = 1; i < D.ns; ++i) cf[i] = (T)(h * D.a[i]);
  // RK4 final combination weights: y + h/6 k1 + h/3 k2 + h/3 k3 + h/6 k4
  const T b16 = (T)(h * (1.0 / 6.0)), b13 = (T)(h * (1.0 / 3.0));
  // Dopri5 error weights d_j = b_j - bhat_j (times h), in fp64
  constexpr double d1 = 35.0 / 384.0 - 5179.0 / 57600.0, d3 = 500.0 / 1113.0 - 7571.0 / 16695.0,
                   d4 = 125.0 / 192.0 - 393.0 / 640.0, d5 = -2187.0 / 6784.0 + 92097.0 / 339200.0,
                   d6 = 11.0 / 84.0 - 187.0 / 2100.0, d7 = -1.0 / 40.0;
  const double e1 = h * d1, e3 = h * d3, e4 = h * d4, e5 = h * d5, e6 = h * d6, e7 = h * d7;
  const double atol = c->atol, rtol = c->rtol;
  const T Du = (T)a.Du_h2, Dv = (T)a.Dv_h2, F = (T)a.F, Fk = (T)(a.F + a.kk);

  const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  const int zbeg = blockIdx.z * a.zc;
  const int zend = min(N, zbeg + a.zc);

  // per-thread in-plane offsets (periodic wrap folded in)
  const int gx = (x0 + lx) % N;
  int off[RY];
  bool valid[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int yy = y0 + ly + 4 * r;
    off[r] = gx + N * (yy % N);
    valid[r] = (x0 + lx < N) && (yy < N);
  }
  // halo cell of this thread: wave 0 row above, wave 1 row below, waves 2/3
  // the left/right columns (first TY lanes)
  int hoff = 0, hrow = 0, hcol = 0;
  bool hval = true;
  if (ly == 0) { hoff = gx + N * ((y0 - 1 + N) % N); hrow = 0; hcol = lx + 1; }
  else if (ly == 1) { hoff = gx + N * ((y0 + TY) % N); hrow = TY + 1; hcol = lx + 1; }
  else {
    hval = lx < TY;
    const int xx = (ly == 2) ? (x0 - 1 + N) % N : (x0 + TX) % N;
    hoff = xx + N * ((y0 + (hval ? lx : 0)) % N);
    hrow = (hval ? lx : 0) + 1;
    hcol = (ly == 2) ? 0 : TX + 1;
  }

  T wp[2][RY], wc[2][RY], wn[2][RY];
  T rawc[NR > 0 ? NR : 1][2][RY], rawn[NR > 0 ? NR : 1][2][RY];
  T hw[2];
  uint64_t emax = 0;

  auto stage_in = [&](int64_t g, T* raw, bool keep) -> T {
    T v0 = P.src[0][g];
    T w = v0;
    if (keep) raw[0] = v0;
#pragma unroll
    for (int i = 1; i < D.ns; ++i) {
      const T s = P.src[i][g];
      if (keep) raw[i] = s;
      w += cf[i] * s;
    }
    return w;
  };
  auto load_plane = [&](int z, T (&w)[2][RY], T (&raw)[NR > 0 ? NR : 1][2][RY], bool with_halo) {
    const int64_t zb = (int64_t)z * NN;
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        const int64_t g = f * n3 + zb + off[r];
        T tmp[6 + 2];
        w[f][r] = stage_in(g, tmp, NR > 0);
        if constexpr (NR > 0) {
#pragma unroll
          for (int i = 0; i < D.ns; ++i) raw[i][f][r] = tmp[i];
#pragma unroll
          for (int i = 0; i < D.nx; ++i) raw[D.ns + i][f][r] = P.extra[i][g];
        }
      }
      if (with_halo && hval) {
        T tmp[6 + 2];
        hw[f] = stage_in(f * n3 + zb + hoff, tmp, false);
      }
    }
  };
  auto store_lds = [&](int b, const T (&w)[2][RY]) {
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
      for (int r = 0; r < RY; ++r) lds[b][f][ly + 4 * r + 1][lx + 1] = w[f][r];
      if (hval) lds[b][f][hrow][hcol] = hw[f];
    }
  };

  if (zbeg < zend) {
    // prologue: centre of plane zbeg-1, plane zbeg with halo
    {
      T dummy[NR > 0 ? NR : 1][2][RY];
      load_plane((zbeg - 1 + N) % N, wp, dummy, false);
    }
    load_plane(zbeg, wc, rawc, true);
    store_lds(0, wc);

    for (int z = zbeg; z < zend; ++z) {
      const int b = (z - zbeg) & 1;
      load_plane(z + 1 == N ? 0 : z + 1, wn, rawn, true);
      __syncthreads();
      const int64_t zb = (int64_t)z * NN;
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        const int row = ly + 4 * r + 1;
        T lap[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
          const T s = lds[b][f][row][lx] + lds[b][f][row][lx + 2] + lds[b][f][row - 1][lx + 1] +
                      lds[b][f][row + 1][lx + 1];
          lap[f] = (s + wp[f][r] + wn[f][r]) - (T)6 * wc[f][r];
        }
        const T u = wc[0][r], v = wc[1][r];
        const T uvv = u * v * v;
        const T fu = Du * lap[0] - uvv + F * ((T)1 - u);
        const T fv = Dv * lap[1] + uvv - Fk * v;
        if (valid[r]) {
          const int64_t g = zb + off[r];
          if constexpr (D.final_kind == 0) {
            P.out[g] = fu;
            P.out[n3 + g] = fv;
          } else if constexpr (D.final_kind == 1) {
            // raw: [0]=y [1]=k3 [2]=k1 [3]=k2
#pragma unroll
            for (int f = 0; f < 2; ++f) {
              const T k4 = f ? fv : fu;
              const T yv = rawc[0][f][r], k3 = rawc[1][f][r], k1 = rawc[2][f][r], k2 = rawc[3][f][r];
              P.ynew[f * n3 + g] = yv + b16 * k1 + b13 * k2 + b13 * k3 + b16 * k4;
            }
          } else {
            P.ynew[g] = u;
            P.ynew[n3 + g] = v;
            P.out[g] = fu;
            P.out[n3 + g] = fv;
            if constexpr (D.err) {
              // raw: [0]=y [1]=k1 [2]=k3 [3]=k4 [4]=k5 [5]=k6
#pragma unroll
              for (int f = 0; f < 2; ++f) {
                const double k7 = (double)(f ? fv : fu);
                const double e = e1 * (double)rawc[1][f][r] + e3 * (double)rawc[2][f][r] +
                                 e4 * (double)rawc[3][f][r] + e5 * (double)rawc[4][f][r] +
                                 e6 * (double)rawc[5][f][r] + e7 * k7;
                const double yo = fabs((double)rawc[0][f][r]), yn = fabs((double)(f ? v : u));
                const double ratio = fabs(e) / (atol + rtol * fmax(yo, yn));
                const uint64_t bits = (uint64_t)__double_as_longlong(ratio);
                emax = bits > emax ? bits : emax;
              }
            }
          }
        }
      }
      store_lds(b ^ 1, wn);
#pragma unroll
      for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int r = 0; r < RY; ++r) {
          wp[f][r] = wc[f][r];
          wc[f][r] = wn[f][r];
        }
      if constexpr (NR > 0) {
#pragma unroll
        for (int i = 0; i < NR; ++i)
#pragma unroll
          for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int r = 0; r < RY; ++r) rawc[i][f][r] = rawn[i][f][r];
      }
    }
  }

  if constexpr (D.err) block_max_to<256>(emax, &c->errmax_bits);
}

template <typename T, int RY>
hipError_t launch_t(int kind, const GSLaunch& a, DevCtrl* c, hipStream_t s) {
  const int TY = 4 * RY;
  dim3 grid((a.N + TX - 1) / TX, (a.N + TY - 1) / TY, (a.N + a.zc - 1) / a.zc);
  dim3 block(256);
  switch (kind) {
#define HODE_CASE(K) \
  case K: gs_stage<T, K, RY><<<grid, block, 0, s>>>(a, c); break;
    HODE_CASE(K_D1) HODE_CASE(K_R2) HODE_CASE(K_R3) HODE_CASE(K_R4) HODE_CASE(K_D2) HODE_CASE(K_D3)
    HODE_CASE(K_D4) HODE_CASE(K_D5) HODE_CASE(K_D6) HODE_CASE(K_D7) HODE_CASE(K_D7F)
#undef HODE_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

bool gs_ry_supported(int ry) { return ry == 1 || ry == 2 || ry == 4; }

hipError_t launch_gs(int kind, int dtype, int ry, const GSLaunch& a, DevCtrl* c, hipStream_t s) {
  if (a.N < 1 || a.zc < 1) return hipErrorInvalidValue;
  if (dtype == 1) {
    if (ry == 1) return launch_t<float, 1>(kind, a, c, s);
    if (ry == 2) return launch_t<float, 2>(kind, a, c, s);
    if (ry == 4) return launch_t<float, 4>(kind, a, c, s);
  } else {
    if (ry == 1) return launch_t<double, 1>(kind, a, c, s);
    if (ry == 2) return launch_t<double, 2>(kind, a, c, s);
    if (ry == 4) return launch_t<double, 4>(kind, a, c, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace hode
