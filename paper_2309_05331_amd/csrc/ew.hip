// Whole-step kernel for the element-wise families of the accuracy benchmark:
// exponential dx/dt = x and sigmoidal (logistic) dx/dt = x (1 - x), one
// independent ODE per component.  With no spatial coupling every stage of a
// step needs only the component itself, so the entire Euler or RK4 step, Dopri5
// attempt (7 stages, first same as last), Cash-Karp 5(4) attempt (6 stages)
// or Fehlberg 7(8) attempt (13 stages) runs in registers: each component is
// read once and written once per attempt, and the embedded error's L-infinity
// norm is reduced on the fly (wavefront shuffle, LDS, one atomic per
// workgroup).  The one-wavefront control kernel then takes the decision.
// An Adams-Bashforth step reads the component's s - 1 past right-hand sides
// from the ring and writes the new one; an Adams-Bashforth-Moulton step
// does the same and corrects in registers, in place.
#include "hode_internal.h"

namespace hode {

namespace {

template <typename T, int RHS>
__device__ __forceinline__ T frhs(T x) {
  if constexpr (RHS == 1) return x;
  else return x * ((T)1 - x);
}

template <typename T>
struct DPCoef {
  T a21, a31, a32, a41, a42, a43, a51, a52, a53, a54, a61, a62, a63, a64, a65, b1, b3, b4, b5, b6;
  double e1, e3, e4, e5, e6, e7;
};

template <typename T>
__device__ inline DPCoef<T> dp_coef(double h) {
  DPCoef<T> q;
  q.a21 = (T)(h * (1.0 / 5.0));
  q.a31 = (T)(h * (3.0 / 40.0));
  q.a32 = (T)(h * (9.0 / 40.0));
  q.a41 = (T)(h * (44.0 / 45.0));
  q.a42 = (T)(h * (-56.0 / 15.0));
  q.a43 = (T)(h * (32.0 / 9.0));
  q.a51 = (T)(h * (19372.0 / 6561.0));
  q.a52 = (T)(h * (-25360.0 / 2187.0));
  q.a53 = (T)(h * (64448.0 / 6561.0));
  q.a54 = (T)(h * (-212.0 / 729.0));
  q.a61 = (T)(h * (9017.0 / 3168.0));
  q.a62 = (T)(h * (-355.0 / 33.0));
  q.a63 = (T)(h * (46732.0 / 5247.0));
  q.a64 = (T)(h * (49.0 / 176.0));
  q.a65 = (T)(h * (-5103.0 / 18656.0));
  q.b1 = (T)(h * (35.0 / 384.0));
  q.b3 = (T)(h * (500.0 / 1113.0));
  q.b4 = (T)(h * (125.0 / 192.0));
  q.b5 = (T)(h * (-2187.0 / 6784.0));
  q.b6 = (T)(h * (11.0 / 84.0));
  q.e1 = h * (35.0 / 384.0 - 5179.0 / 57600.0);
  q.e3 = h * (500.0 / 1113.0 - 7571.0 / 16695.0);
  q.e4 = h * (125.0 / 192.0 - 393.0 / 640.0);
  q.e5 = h * (-2187.0 / 6784.0 + 92097.0 / 339200.0);
  q.e6 = h * (11.0 / 84.0 - 187.0 / 2100.0);
  q.e7 = h * (-1.0 / 40.0);
  return q;
}

// Cash-Karp 5(4) (Cash & Karp 1990), times h: stage coefficients, the
// 5th-order weights (b2 = b5 = 0) and b - bhat of the embedded estimate.
template <typename T>
struct CKCoef {
  T a21, a31, a32, a41, a42, a43, a51, a52, a53, a54, a61, a62, a63, a64, a65, b1, b3, b4, b6;
  double e1, e3, e4, e5, e6;
};

template <typename T>
__device__ inline CKCoef<T> ck_coef(double h) {
  CKCoef<T> q;
  q.a21 = (T)(h * (1.0 / 5.0));
  q.a31 = (T)(h * (3.0 / 40.0));
  q.a32 = (T)(h * (9.0 / 40.0));
  q.a41 = (T)(h * (3.0 / 10.0));
  q.a42 = (T)(h * (-9.0 / 10.0));
  q.a43 = (T)(h * (6.0 / 5.0));
  q.a51 = (T)(h * (-11.0 / 54.0));
  q.a52 = (T)(h * (5.0 / 2.0));
  q.a53 = (T)(h * (-70.0 / 27.0));
  q.a54 = (T)(h * (35.0 / 27.0));
  q.a61 = (T)(h * (1631.0 / 55296.0));
  q.a62 = (T)(h * (175.0 / 512.0));
  q.a63 = (T)(h * (575.0 / 13824.0));
  q.a64 = (T)(h * (44275.0 / 110592.0));
  q.a65 = (T)(h * (253.0 / 4096.0));
  q.b1 = (T)(h * (37.0 / 378.0));
  q.b3 = (T)(h * (250.0 / 621.0));
  q.b4 = (T)(h * (125.0 / 594.0));
  q.b6 = (T)(h * (512.0 / 1771.0));
  q.e1 = h * (37.0 / 378.0 - 2825.0 / 27648.0);
  q.e3 = h * (250.0 / 621.0 - 18575.0 / 48384.0);
  q.e4 = h * (125.0 / 594.0 - 13525.0 / 55296.0);
  q.e5 = h * (-277.0 / 14336.0);
  q.e6 = h * (512.0 / 1771.0 - 1.0 / 4.0);
  return q;
}

// The seven Dopri5 stages of one component and the 5th-order solution
// (k7 = f(xn)); shared by the step and the dense output, which must see the
// same stage values.
template <typename T, int RHS>
__device__ __forceinline__ T dp_stages(T x, const DPCoef<T>& q, T (&k)[7]) {
  k[0] = frhs<T, RHS>(x);
  k[1] = frhs<T, RHS>(x + q.a21 * k[0]);
  k[2] = frhs<T, RHS>(x + q.a31 * k[0] + q.a32 * k[1]);
  k[3] = frhs<T, RHS>(x + q.a41 * k[0] + q.a42 * k[1] + q.a43 * k[2]);
  k[4] = frhs<T, RHS>(x + q.a51 * k[0] + q.a52 * k[1] + q.a53 * k[2] + q.a54 * k[3]);
  k[5] = frhs<T, RHS>(x + q.a61 * k[0] + q.a62 * k[1] + q.a63 * k[2] + q.a64 * k[3] + q.a65 * k[4]);
  const T xn = x + q.b1 * k[0] + q.b3 * k[2] + q.b4 * k[3] + q.b5 * k[4] + q.b6 * k[5];
  k[6] = frhs<T, RHS>(xn);
  return xn;
}

template <typename T, int RHS, int MODE>
__device__ __forceinline__ T step_one(T x, const DPCoef<T>& q, const CKCoef<T>& ck, T r2, T r1, T r16, T r13,
                                      double atol, double rtol, uint64_t& emax) {
  if constexpr (MODE == MODE_FIXED_EULER) {
    return x + r1 * frhs<T, RHS>(x);
  } else if constexpr (MODE == MODE_FIXED_MM) {
    // modified midpoint, two substeps of H/2 (r2 = H/2, r1 = H)
    const T z1 = x + r2 * frhs<T, RHS>(x);
    const T z2 = x + r1 * frhs<T, RHS>(z1);
    return (T)0.5 * (z2 + z1 + r2 * frhs<T, RHS>(z2));
  } else if constexpr (MODE == MODE_FIXED_CK || MODE == MODE_ADAPTIVE_CK) {
    const T k1 = frhs<T, RHS>(x);
    const T k2 = frhs<T, RHS>(x + ck.a21 * k1);
    const T k3 = frhs<T, RHS>(x + ck.a31 * k1 + ck.a32 * k2);
    const T k4 = frhs<T, RHS>(x + ck.a41 * k1 + ck.a42 * k2 + ck.a43 * k3);
    const T k5 = frhs<T, RHS>(x + ck.a51 * k1 + ck.a52 * k2 + ck.a53 * k3 + ck.a54 * k4);
    const T k6 = frhs<T, RHS>(x + ck.a61 * k1 + ck.a62 * k2 + ck.a63 * k3 + ck.a64 * k4 + ck.a65 * k5);
    const T xn = x + ck.b1 * k1 + ck.b3 * k3 + ck.b4 * k4 + ck.b6 * k6;
    if constexpr (MODE == MODE_ADAPTIVE_CK) {
      const double e = ck.e1 * (double)k1 + ck.e3 * (double)k3 + ck.e4 * (double)k4 + ck.e5 * (double)k5 +
                       ck.e6 * (double)k6;
      const double ratio = fabs(e) / (atol + rtol * fmax(fabs((double)x), fabs((double)xn)));
      const uint64_t bits = (uint64_t)__double_as_longlong(ratio);
      emax = bits > emax ? bits : emax;
    }
    return xn;
  } else if constexpr (MODE == MODE_FIXED_RK4) {
    const T k1 = frhs<T, RHS>(x);
    const T k2 = frhs<T, RHS>(x + r2 * k1);
    const T k3 = frhs<T, RHS>(x + r2 * k2);
    const T k4 = frhs<T, RHS>(x + r1 * k3);
    return x + r16 * k1 + r13 * k2 + r13 * k3 + r16 * k4;
  } else {
    T k[7];
    const T xn = dp_stages<T, RHS>(x, q, k);  // (k7 is dead code in fixed mode)
    if constexpr (MODE == MODE_ADAPTIVE) {
      const double e = q.e1 * (double)k[0] + q.e3 * (double)k[2] + q.e4 * (double)k[3] + q.e5 * (double)k[4] +
                       q.e6 * (double)k[5] + q.e7 * (double)k[6];
      const double ratio = fabs(e) / (atol + rtol * fmax(fabs((double)x), fabs((double)xn)));
      const uint64_t bits = (uint64_t)__double_as_longlong(ratio);
      emax = bits > emax ? bits : emax;
    }
    return xn;
  }
}

template <typename T>
struct Vec;
template <>
struct Vec<float> {
  using V = float4;
  static constexpr int W = 4;
};
template <>
struct Vec<double> {
  using V = double2;
  static constexpr int W = 2;
};

template <typename T, int RHS, int MODE>
__global__ __launch_bounds__(256) void ew_step(DevCtrl* __restrict__ c, T* __restrict__ b0, T* __restrict__ b1,
                                               int64_t n) {
  if (c->done) return;
  const double h = c->h;
  const T* __restrict__ y = c->parity ? b1 : b0;
  T* __restrict__ yn = c->parity ? b0 : b1;
  const double atol = c->atol, rtol = c->rtol;
  DPCoef<T> q = dp_coef<T>(h);
  CKCoef<T> ck = ck_coef<T>(h);
  const T r2 = (T)(h * 0.5), r1 = (T)h, r16 = (T)(h * (1.0 / 6.0)), r13 = (T)(h * (1.0 / 3.0));
  uint64_t emax = 0;

  using V = typename Vec<T>::V;
  constexpr int W = Vec<T>::W;
  const int64_t nv = n / W;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
    V v = reinterpret_cast<const V*>(y)[i];
    T* e = reinterpret_cast<T*>(&v);
#pragma unroll
    for (int j = 0; j < W; ++j) e[j] = step_one<T, RHS, MODE>(e[j], q, ck, r2, r1, r16, r13, atol, rtol, emax);
    reinterpret_cast<V*>(yn)[i] = v;
  }
  // ragged tail
  const int64_t tail = nv * W;
  if (blockIdx.x == gridDim.x - 1 && tail + threadIdx.x < n) {
    const int64_t i = tail + threadIdx.x;
    yn[i] = step_one<T, RHS, MODE>(y[i], q, ck, r2, r1, r16, r13, atol, rtol, emax);
  }
  if constexpr (mode_adaptive(MODE)) block_max_to<256>(emax, &c->errmax_bits);
}

// One Fehlberg 7(8) attempt of one component in registers (13 stages; zero
// tableau entries are skipped at compile time).  q = h F78A, qb = h F78B in
// the state's precision; the error h 41/840 (k12 + k13 - k1 - k11) in FP64.
template <typename T, int RHS, bool ADAPT>
__device__ __forceinline__ T f78_one(T x, const T (&q)[13][13], const T (&qb)[13], double qe, double atol,
                                     double rtol, uint64_t& emax, T& k1) {
  T k[13];
  k[0] = frhs<T, RHS>(x);
#pragma unroll
  for (int s = 1; s < 13; ++s) {
    T w = x;
#pragma unroll
    for (int j = 0; j < s; ++j)
      if (F78A[s][j] != 0.0) w += q[s][j] * k[j];
    k[s] = frhs<T, RHS>(w);
  }
  T xn = x;
#pragma unroll
  for (int j = 0; j < 13; ++j)
    if (F78B[j] != 0.0) xn += qb[j] * k[j];
  if constexpr (ADAPT) {
    const double e = qe * (((double)k[11] - (double)k[0] - (double)k[10]) + (double)k[12]);
    const double ratio = fabs(e) / (atol + rtol * fmax(fabs((double)x), fabs((double)xn)));
    const uint64_t bits = (uint64_t)__double_as_longlong(ratio);
    emax = bits > emax ? bits : emax;
  }
  k1 = k[0];
  return xn;
}

// Fehlberg 7(8) attempt (adaptive) or fixed step over all components; kout,
// if not null, receives k1 = f(y) (the right-hand side an Adams-Bashforth
// start-up step records).
template <typename T, int RHS, bool ADAPT>
__global__ __launch_bounds__(256) void ew_f78(DevCtrl* __restrict__ c, T* __restrict__ b0, T* __restrict__ b1,
                                              T* __restrict__ kout, int64_t n) {
  if (c->done) return;
  const double h = c->h;
  const T* __restrict__ y = c->parity ? b1 : b0;
  T* __restrict__ yn = c->parity ? b0 : b1;
  const double atol = c->atol, rtol = c->rtol;
  T q[13][13], qb[13];
#pragma unroll
  for (int s = 0; s < 13; ++s) {
#pragma unroll
    for (int j = 0; j < 13; ++j) q[s][j] = (T)(h * F78A[s][j]);
    qb[s] = (T)(h * F78B[s]);
  }
  const double qe = h * F78E;
  uint64_t emax = 0;
  using V = typename Vec<T>::V;
  constexpr int W = Vec<T>::W;
  const int64_t nv = n / W;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
    V v = reinterpret_cast<const V*>(y)[i];
    V kv;
    T* e = reinterpret_cast<T*>(&v);
    T* k1 = reinterpret_cast<T*>(&kv);
#pragma unroll
    for (int j = 0; j < W; ++j) e[j] = f78_one<T, RHS, ADAPT>(e[j], q, qb, qe, atol, rtol, emax, k1[j]);
    reinterpret_cast<V*>(yn)[i] = v;
    if (kout) reinterpret_cast<V*>(kout)[i] = kv;
  }
  const int64_t tail = nv * W;
  if (blockIdx.x == gridDim.x - 1 && tail + threadIdx.x < n) {
    const int64_t i = tail + threadIdx.x;
    T k1;
    yn[i] = f78_one<T, RHS, ADAPT>(y[i], q, qb, qe, atol, rtol, emax, k1);
    if (kout) kout[i] = k1;
  }
  if constexpr (ADAPT) block_max_to<256>(emax, &c->errmax_bits);
}

// One Adams-Bashforth step with S steps over all components: f_n = f(y_n)
// goes into ring slot c->ring (S > 1), and y_{n+1} = y_n + h sum_{j>=1}
// beta_j f_{n-j} + h beta_0 f_n with f_{n-j} from the ring (table xk).
template <typename T, int RHS, int S>
__global__ __launch_bounds__(256) void ew_ab(DevCtrl* __restrict__ c, T* __restrict__ b0, T* __restrict__ b1,
                                             void* const* __restrict__ xk, int64_t n) {
  if (c->done) return;
  const double h = c->h;
  const T* __restrict__ y = c->parity ? b1 : b0;
  T* __restrict__ yn = c->parity ? b0 : b1;
  const int rg = c->ring;
  T* __restrict__ fn = S > 1 ? (T*)xk[kRingBase + rg] : nullptr;
  const T* fp[S > 1 ? S : 1];
  T q[S];
#pragma unroll
  for (int j = 0; j < S; ++j) {
    q[j] = (T)(h * ABW[S - 1][j]);
    if (j > 0) fp[j] = (const T*)xk[kRingBase + (rg + S - j) % S];
  }
  using V = typename Vec<T>::V;
  constexpr int W = Vec<T>::W;
  const int64_t nv = n / W;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
    V v = reinterpret_cast<const V*>(y)[i];
    V past[S > 1 ? S : 1];
#pragma unroll
    for (int j = 1; j < S; ++j) past[j] = reinterpret_cast<const V*>(fp[j])[i];
    V fv;
    T* e = reinterpret_cast<T*>(&v);
    T* f = reinterpret_cast<T*>(&fv);
#pragma unroll
    for (int l = 0; l < W; ++l) {
      f[l] = frhs<T, RHS>(e[l]);
      T acc = e[l];
#pragma unroll
      for (int j = 1; j < S; ++j) acc += q[j] * reinterpret_cast<const T*>(&past[j])[l];
      e[l] = acc + q[0] * f[l];
    }
    reinterpret_cast<V*>(yn)[i] = v;
    if constexpr (S > 1) reinterpret_cast<V*>(fn)[i] = fv;
  }
  const int64_t tail = nv * W;
  if (blockIdx.x == gridDim.x - 1 && tail + threadIdx.x < n) {
    const int64_t i = tail + threadIdx.x;
    const T x = y[i];
    const T f = frhs<T, RHS>(x);
    T acc = x;
#pragma unroll
    for (int j = 1; j < S; ++j) acc += q[j] * fp[j][i];
    yn[i] = acc + q[0] * f;
    if constexpr (S > 1) fn[i] = f;
  }
}

// Weights h w_j(theta) of the Dopri5 continuous extension, in the state's
// precision (w_2 = 0).
template <typename T>
__device__ inline void dense_coef(double h, double th, T (&cw)[7]) {
  const double u = 1.0 - th;
  const double b[7] = {DPA[6][0], DPA[6][1], DPA[6][2], DPA[6][3], DPA[6][4], DPA[6][5], 0.0};
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    double w = b[j] * (3.0 * th * th - 2.0 * th * th * th) + DPC[j] * th * th * u * u;
    if (j == 0) w += th * u * u;
    if (j == 6) w -= th * th * u;
    cw[j] = (T)(h * w);
  }
}

// Dense output from stored stages (Gray-Scott): out = y_n + sum_j (h w_j) k_j.
template <typename T>
__global__ __launch_bounds__(256) void dense_k(T* __restrict__ out, const T* __restrict__ yn,
                                               const T* __restrict__ k1, const T* __restrict__ k3,
                                               const T* __restrict__ k4, const T* __restrict__ k5,
                                               const T* __restrict__ k6, const T* __restrict__ k7, int64_t n,
                                               double h, double th) {
  T cw[7];
  dense_coef<T>(h, th, cw);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = yn[i] + cw[0] * k1[i] + cw[2] * k3[i] + cw[3] * k4[i] + cw[4] * k5[i] + cw[5] * k6[i] + cw[6] * k7[i];
}

// Dense output of the element-wise families: the step's seven stages are
// evaluated again from y_n (same expressions, so the same values).
template <typename T, int RHS>
__global__ __launch_bounds__(256) void dense_ew(T* __restrict__ out, const T* __restrict__ yn, int64_t n, double h,
                                                double th) {
  const DPCoef<T> q = dp_coef<T>(h);
  T cw[7];
  dense_coef<T>(h, th, cw);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const T x = yn[i];
    T k[7];
    (void)dp_stages<T, RHS>(x, q, k);
    out[i] = x + cw[0] * k[0] + cw[2] * k[2] + cw[3] * k[3] + cw[4] * k[4] + cw[5] * k[5] + cw[6] * k[6];
  }
}

// One Adams-Bashforth-Moulton step with S steps over all components, in
// place: f_n = f(y_n) into ring slot c->ring (S > 1), the prediction
// p = y_n + h sum_j beta_j f_{n-j} (as ew_ab), and y_{n+1} = y_n + h (gamma_0
// f(p) + gamma_1 f_n + sum_{j>=2} gamma_j f_{n+1-j}) written over y_n.
template <typename T, int RHS, int S>
__global__ __launch_bounds__(256) void ew_abm(DevCtrl* __restrict__ c, T* __restrict__ b0, T* __restrict__ b1,
                                              void* const* __restrict__ xk, int64_t n) {
  if (c->done) return;
  const double h = c->h;
  T* __restrict__ y = c->parity ? b1 : b0;
  const int rg = c->ring;
  T* __restrict__ fn = S > 1 ? (T*)xk[kRingBase + rg] : nullptr;
  const T* fp[S > 1 ? S : 1];
  T q[S], g[S];
#pragma unroll
  for (int j = 0; j < S; ++j) {
    q[j] = (T)(h * ABW[S - 1][j]);
    g[j] = (T)(h * AMW[S - 1][j]);
    if (j > 0) fp[j] = (const T*)xk[kRingBase + (rg + S - j) % S];
  }
  auto one = [&](T x, const T* past, T& f) -> T {
    // past[j] = f_{n-j}, j = 1 .. S-1
    f = frhs<T, RHS>(x);
    T p = x;
#pragma unroll
    for (int j = 1; j < S; ++j) p += q[j] * past[j];
    p = p + q[0] * f;
    const T fpred = frhs<T, RHS>(p);
    T acc = x;
    if constexpr (S > 1) acc += g[1] * f;
#pragma unroll
    for (int j = 2; j < S; ++j) acc += g[j] * past[j - 1];
    return acc + g[0] * fpred;
  };
  using V = typename Vec<T>::V;
  constexpr int W = Vec<T>::W;
  const int64_t nv = n / W;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
    V v = reinterpret_cast<const V*>(y)[i];
    V pv[S > 1 ? S : 1];
#pragma unroll
    for (int j = 1; j < S; ++j) pv[j] = reinterpret_cast<const V*>(fp[j])[i];
    V fv;
    T* e = reinterpret_cast<T*>(&v);
    T* f = reinterpret_cast<T*>(&fv);
#pragma unroll
    for (int l = 0; l < W; ++l) {
      T past[S > 1 ? S : 1];
#pragma unroll
      for (int j = 1; j < S; ++j) past[j] = reinterpret_cast<const T*>(&pv[j])[l];
      e[l] = one(e[l], past, f[l]);
    }
    reinterpret_cast<V*>(y)[i] = v;
    if constexpr (S > 1) reinterpret_cast<V*>(fn)[i] = fv;
  }
  const int64_t tail = nv * W;
  if (blockIdx.x == gridDim.x - 1 && tail + threadIdx.x < n) {
    const int64_t i = tail + threadIdx.x;
    T past[S > 1 ? S : 1];
#pragma unroll
    for (int j = 1; j < S; ++j) past[j] = fp[j][i];
    T f;
    y[i] = one(y[i], past, f);
    if constexpr (S > 1) fn[i] = f;
  }
}

__global__ __launch_bounds__(64) void ctrl_kernel(DevCtrl* c) {
  if (c->done) return;
  ctrl_step(c);
}

template <typename T, int RHS>
__global__ __launch_bounds__(256) void ew_rhs(const T* __restrict__ y, T* __restrict__ out, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = frhs<T, RHS>(y[i]);
}

template <typename T, int RHS>
hipError_t launch_rhs(int mode, T* y0, T* y1, int64_t n, int grid, DevCtrl* c, hipStream_t s) {
  if (mode == MODE_FIXED_RK4) ew_step<T, RHS, MODE_FIXED_RK4><<<grid, 256, 0, s>>>(c, y0, y1, n);
  else if (mode == MODE_FIXED_DP5) ew_step<T, RHS, MODE_FIXED_DP5><<<grid, 256, 0, s>>>(c, y0, y1, n);
  else if (mode == MODE_FIXED_CK) ew_step<T, RHS, MODE_FIXED_CK><<<grid, 256, 0, s>>>(c, y0, y1, n);
  else if (mode == MODE_FIXED_EULER) ew_step<T, RHS, MODE_FIXED_EULER><<<grid, 256, 0, s>>>(c, y0, y1, n);
  else if (mode == MODE_FIXED_MM) ew_step<T, RHS, MODE_FIXED_MM><<<grid, 256, 0, s>>>(c, y0, y1, n);
  else if (mode == MODE_ADAPTIVE_CK) ew_step<T, RHS, MODE_ADAPTIVE_CK><<<grid, 256, 0, s>>>(c, y0, y1, n);
  else ew_step<T, RHS, MODE_ADAPTIVE><<<grid, 256, 0, s>>>(c, y0, y1, n);
  return hipGetLastError();
}

template <typename T, int RHS>
hipError_t launch_x(int mode, int ab_steps, T* y0, T* y1, void* const* xk, T* kout, int64_t n, int grid,
                    DevCtrl* c, hipStream_t s) {
  if (mode == MODE_FIXED_F78) ew_f78<T, RHS, false><<<grid, 256, 0, s>>>(c, y0, y1, kout, n);
  else if (mode == MODE_ADAPTIVE_F78) ew_f78<T, RHS, true><<<grid, 256, 0, s>>>(c, y0, y1, kout, n);
  else if (mode == MODE_FIXED_AB || mode == MODE_FIXED_ABM) {
    if (xk == nullptr && ab_steps > 1) return hipErrorInvalidValue;
    const bool abm = mode == MODE_FIXED_ABM;
    switch (ab_steps) {
#define HODE_AB(S)                                                                 \
  case S:                                                                          \
    if (abm) ew_abm<T, RHS, S><<<grid, 256, 0, s>>>(c, y0, y1, xk, n);             \
    else ew_ab<T, RHS, S><<<grid, 256, 0, s>>>(c, y0, y1, xk, n);                  \
    break;
      HODE_AB(1) HODE_AB(2) HODE_AB(3) HODE_AB(4) HODE_AB(5) HODE_AB(6) HODE_AB(7) HODE_AB(8)
#undef HODE_AB
      default: return hipErrorInvalidValue;
    }
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_ewx(int dtype, int rhs, int mode, int ab_steps, void* y0, void* y1, void* const* xk, void* kout,
                      int64_t n, int grid, DevCtrl* c, hipStream_t s) {
  if (grid < 1) return hipErrorInvalidValue;
  if (dtype == 1) {
    if (rhs == 1) return launch_x<float, 1>(mode, ab_steps, (float*)y0, (float*)y1, xk, (float*)kout, n, grid, c, s);
    return launch_x<float, 2>(mode, ab_steps, (float*)y0, (float*)y1, xk, (float*)kout, n, grid, c, s);
  }
  if (rhs == 1) return launch_x<double, 1>(mode, ab_steps, (double*)y0, (double*)y1, xk, (double*)kout, n, grid, c, s);
  return launch_x<double, 2>(mode, ab_steps, (double*)y0, (double*)y1, xk, (double*)kout, n, grid, c, s);
}

hipError_t launch_dense_k(int dtype, void* out, const void* yn, const void* k1, const void* k3, const void* k4,
                          const void* k5, const void* k6, const void* k7, int64_t n, int grid, double h, double theta,
                          hipStream_t s) {
  if (grid < 1) return hipErrorInvalidValue;
  if (dtype == 1)
    dense_k<float><<<grid, 256, 0, s>>>((float*)out, (const float*)yn, (const float*)k1, (const float*)k3,
                                        (const float*)k4, (const float*)k5, (const float*)k6, (const float*)k7, n, h,
                                        theta);
  else
    dense_k<double><<<grid, 256, 0, s>>>((double*)out, (const double*)yn, (const double*)k1, (const double*)k3,
                                         (const double*)k4, (const double*)k5, (const double*)k6, (const double*)k7,
                                         n, h, theta);
  return hipGetLastError();
}

hipError_t launch_dense_ew(int dtype, int rhs, void* out, const void* yn, int64_t n, int grid, double h,
                           double theta, hipStream_t s) {
  if (grid < 1) return hipErrorInvalidValue;
  if (dtype == 1) {
    if (rhs == 1) dense_ew<float, 1><<<grid, 256, 0, s>>>((float*)out, (const float*)yn, n, h, theta);
    else dense_ew<float, 2><<<grid, 256, 0, s>>>((float*)out, (const float*)yn, n, h, theta);
  } else {
    if (rhs == 1) dense_ew<double, 1><<<grid, 256, 0, s>>>((double*)out, (const double*)yn, n, h, theta);
    else dense_ew<double, 2><<<grid, 256, 0, s>>>((double*)out, (const double*)yn, n, h, theta);
  }
  return hipGetLastError();
}

hipError_t launch_ctrl(DevCtrl* c, hipStream_t s) {
  ctrl_kernel<<<1, 64, 0, s>>>(c);
  return hipGetLastError();
}

hipError_t launch_ew_rhs(int dtype, int rhs, const void* y, void* out, int64_t n, int grid, hipStream_t s) {
  if (grid < 1) return hipErrorInvalidValue;
  if (dtype == 1) {
    if (rhs == 1) ew_rhs<float, 1><<<grid, 256, 0, s>>>((const float*)y, (float*)out, n);
    else ew_rhs<float, 2><<<grid, 256, 0, s>>>((const float*)y, (float*)out, n);
  } else {
    if (rhs == 1) ew_rhs<double, 1><<<grid, 256, 0, s>>>((const double*)y, (double*)out, n);
    else ew_rhs<double, 2><<<grid, 256, 0, s>>>((const double*)y, (double*)out, n);
  }
  return hipGetLastError();
}

hipError_t launch_ew(int dtype, int rhs, int mode, void* y0, void* y1, int64_t n, int grid, DevCtrl* c,
                     hipStream_t s) {
  if (grid < 1) return hipErrorInvalidValue;
  if (dtype == 1) {
    if (rhs == 1) return launch_rhs<float, 1>(mode, (float*)y0, (float*)y1, n, grid, c, s);
    return launch_rhs<float, 2>(mode, (float*)y0, (float*)y1, n, grid, c, s);
  }
  if (rhs == 1) return launch_rhs<double, 1>(mode, (double*)y0, (double*)y1, n, grid, c, s);
  return launch_rhs<double, 2>(mode, (double*)y0, (double*)y1, n, grid, c, s);
}

}  // namespace hode
