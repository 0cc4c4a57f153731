// Device-side definitions shared by the hode kernels: the control block that
// keeps the whole time-stepping loop resident on the GPU, the Runge-Kutta
// tableaux, the L-infinity reduction and the step-size controller.
//
// Method (the paper's "Architecture and nomenclature of Boost Odeint"
// section): a state is advanced in place by a stepper that evaluates the
// System right-hand side once per stage and combines stages through an
// Algebra; error steppers report an embedded error estimate whose L-infinity
// norm drives an error-controlled adaptive step ("integrate_adaptive" with a
// tolerance, Reuse-potential section).  Here the Algebra is fused into the
// stage kernels and the control decision runs on the device in the last
// workgroup of each attempt, so a whole integration needs no host round-trip
// per step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hode {

enum Mode : int32_t {
  MODE_FIXED_RK4 = 1, MODE_FIXED_DP5 = 2, MODE_ADAPTIVE = 3,  // RK4, Dopri5 fixed, Dopri5 adaptive
  MODE_FIXED_CK = 4, MODE_ADAPTIVE_CK = 5,                    // Cash-Karp 5(4) fixed, adaptive
  MODE_FIXED_EULER = 6,                                       // explicit Euler
  MODE_FIXED_F78 = 7, MODE_ADAPTIVE_F78 = 8,                  // Fehlberg 7(8) fixed, adaptive
  MODE_FIXED_AB = 9,                                          // Adams-Bashforth (ab_steps steps)
  MODE_ADAPTIVE_DENSE = 10,  // Dopri5 adaptive, pausing after the accepted step that reaches stop_at
  MODE_FIXED_ABM = 11,       // Adams-Bashforth-Moulton (ab_steps steps; new state in place)
  MODE_FIXED_MM = 12         // modified midpoint (two substeps)
};

__host__ __device__ constexpr bool mode_adaptive(int m) {
  return m == MODE_ADAPTIVE || m == MODE_ADAPTIVE_CK || m == MODE_ADAPTIVE_F78 || m == MODE_ADAPTIVE_DENSE;
}
// Right-hand side evaluations of one attempt or fixed step (Dopri5: k1 of
// the first attempt comes on top; Adams-Bashforth steps after the start-up).
__host__ __device__ constexpr int mode_rhs_evals(int m) {
  return m == MODE_FIXED_RK4 ? 4
         : (m == MODE_FIXED_EULER || m == MODE_FIXED_AB) ? 1
         : m == MODE_FIXED_ABM                         ? 2
         : m == MODE_FIXED_MM                          ? 3
         : (m == MODE_FIXED_F78 || m == MODE_ADAPTIVE_F78) ? 13
                                                           : 6;
}
enum CtrlKind : int32_t { CTRL_PI = 1, CTRL_I = 2, CTRL_MLP = 3 };
enum Status : int32_t {
  ST_OK = 0,
  ST_EDT_UNDERFLOW = -5,
  ST_EMAXSTEPS = -6,
  ST_ENONFINITE = -7,
};

constexpr int TRACE_W = 24;  // doubles per trace record (8 scalars + 16 controller features)
constexpr int HIST = 4;     // attempts of history kept for the learned controller
constexpr int MLP_IN = 16, MLP_H = 64;
// packed bf16 weights: W1[64][16] b1[64] W2[64][64] b2[64] w3[64] b3[1]
constexpr int MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;

// Control block: one per integration, lives in device memory.  Written by the
// host before a run and by the last workgroup of every attempt; read by every
// kernel at entry.  FP64 for time, step and error; int64 counters.
struct DevCtrl {
  double t, t0, t1, dt, h;
  double atol, rtol;
  double err_prev, last_err;
  int64_t accepted, rejected, attempts, max_attempts, rhs_evals;
  int64_t nsteps;
  int32_t mode, ctrl_kind;
  int32_t parity, k1slot;
  int32_t done, status;
  int32_t last_rejected, last_flag;
  uint64_t errmax_bits;
  uint32_t pad_u32, hist_n;
  double hist_lerr[HIST], hist_lh[HIST], hist_acc[HIST];
  double* trace;
  int64_t trace_cap;
  const uint16_t* mlp_w;  // bf16 weights in device memory (CTRL_MLP)
  int64_t mlp_used, mlp_fallback;
  double stiff;  // spectral-radius scale of the System's Jacobian (feature of the learned controller)
  int32_t ab_steps;  // Adams-Bashforth: steps s (ring of s past right-hand sides)
  int32_t ring;      // Adams-Bashforth: ring slot receiving f_n of the next step
  double stop_at;    // dense output: the run pauses (done) after the accepted step that reaches it
  double h_acc;      // size of the last accepted step
};

// ---- tableaux (Dormand & Prince 1980; classical RK4) ------------------------
// Dormand-Prince 5(4): stage-input coefficients a[s][j] (s = 1..6 is stage
// s+1), 5th-order weights (= last row, first same as last) and the error
// weights d = b - bhat.
__device__ constexpr double DPA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0},
};
__device__ constexpr double DPD[7] = {
    35.0 / 384.0 - 5179.0 / 57600.0,         0.0,
    500.0 / 1113.0 - 7571.0 / 16695.0,       125.0 / 192.0 - 393.0 / 640.0,
    -2187.0 / 6784.0 + 92097.0 / 339200.0,   11.0 / 84.0 - 187.0 / 2100.0,
    -1.0 / 40.0,
};
__device__ constexpr double RKA[4] = {0.0, 0.5, 0.5, 1.0};  // stage s input: y + RKA[s] h k_{s}

// Runge-Kutta-Fehlberg 7(8) (Fehlberg 1968): stage-input coefficients
// F78A[s][j] (stage s+1 uses k_{j+1}), the 8th-order weights F78B; the error
// weights b - bhat are F78E times (-1, 0, .., 0, -1, 1, 1).
__device__ constexpr double F78A[13][13] = {
    {0},
    {2.0 / 27.0},
    {1.0 / 36.0, 1.0 / 12.0},
    {1.0 / 24.0, 0, 1.0 / 8.0},
    {5.0 / 12.0, 0, -25.0 / 16.0, 25.0 / 16.0},
    {1.0 / 20.0, 0, 0, 1.0 / 4.0, 1.0 / 5.0},
    {-25.0 / 108.0, 0, 0, 125.0 / 108.0, -65.0 / 27.0, 125.0 / 54.0},
    {31.0 / 300.0, 0, 0, 0, 61.0 / 225.0, -2.0 / 9.0, 13.0 / 900.0},
    {2.0, 0, 0, -53.0 / 6.0, 704.0 / 45.0, -107.0 / 9.0, 67.0 / 90.0, 3.0},
    {-91.0 / 108.0, 0, 0, 23.0 / 108.0, -976.0 / 135.0, 311.0 / 54.0, -19.0 / 60.0, 17.0 / 6.0, -1.0 / 12.0},
    {2383.0 / 4100.0, 0, 0, -341.0 / 164.0, 4496.0 / 1025.0, -301.0 / 82.0, 2133.0 / 4100.0, 45.0 / 82.0,
     45.0 / 164.0, 18.0 / 41.0},
    {3.0 / 205.0, 0, 0, 0, 0, -6.0 / 41.0, -3.0 / 205.0, -3.0 / 41.0, 3.0 / 41.0, 6.0 / 41.0, 0},
    {-1777.0 / 4100.0, 0, 0, -341.0 / 164.0, 4496.0 / 1025.0, -289.0 / 82.0, 2193.0 / 4100.0, 51.0 / 82.0,
     33.0 / 164.0, 12.0 / 41.0, 0, 1.0},
};
__device__ constexpr double F78B[13] = {0, 0, 0, 0, 0, 34.0 / 105.0, 9.0 / 35.0, 9.0 / 35.0, 9.0 / 280.0,
                                        9.0 / 280.0, 0, 41.0 / 840.0, 41.0 / 840.0};
__device__ constexpr double F78E = 41.0 / 840.0;

// Continuous extension of Dormand-Prince 5(4) (Dormand & Prince 1986;
// Hairer, Norsett & Wanner I, section II.6): y(t_n + theta h) = y_n + h
// sum_j w_j(theta) k_j with w_j = b_j (3 theta^2 - 2 theta^3) + DPC_j theta^2
// (1 - theta)^2 + [j = 1] theta (1 - theta)^2 - [j = 7] theta^2 (1 - theta):
// the quartic through y_n, y_{n+1} with end slopes k1, k7, made 4th-order
// accurate by the DPC term.
__device__ constexpr double DPC[7] = {-12715105075.0 / 11282082432.0, 0.0, 87487479700.0 / 32700410799.0,
                                      -10690763975.0 / 1880347072.0, 701980252875.0 / 199316789632.0,
                                      -1453857185.0 / 822651844.0, 69997945.0 / 29380423.0};

// Adams-Moulton weights for s values: y_{n+1} = y_n + h (AMW[s-1][0]
// f_{n+1} + sum_{j>=1} AMW[s-1][j] f_{n+1-j}) (the integral over one step of
// the polynomial through f_{n+1} .. f_{n+2-s}; Hairer, Norsett & Wanner I,
// section III.1), with f_{n+1} taken at the Adams-Bashforth prediction.
__device__ constexpr double AMW[8][8] = {
    {1.0},
    {1.0 / 2.0, 1.0 / 2.0},
    {5.0 / 12.0, 8.0 / 12.0, -1.0 / 12.0},
    {9.0 / 24.0, 19.0 / 24.0, -5.0 / 24.0, 1.0 / 24.0},
    {251.0 / 720.0, 646.0 / 720.0, -264.0 / 720.0, 106.0 / 720.0, -19.0 / 720.0},
    {475.0 / 1440.0, 1427.0 / 1440.0, -798.0 / 1440.0, 482.0 / 1440.0, -173.0 / 1440.0, 27.0 / 1440.0},
    {19087.0 / 60480.0, 65112.0 / 60480.0, -46461.0 / 60480.0, 37504.0 / 60480.0, -20211.0 / 60480.0,
     6312.0 / 60480.0, -863.0 / 60480.0},
    {36799.0 / 120960.0, 139849.0 / 120960.0, -121797.0 / 120960.0, 123133.0 / 120960.0, -88547.0 / 120960.0,
     41499.0 / 120960.0, -11351.0 / 120960.0, 1375.0 / 120960.0},
};

// Adams-Bashforth weights: with s steps, y_{n+1} = y_n + h sum_j ABW[s-1][j]
// f_{n-j} (the integral over one step of the polynomial through the last s
// right-hand sides; Hairer, Norsett & Wanner I, section III.1).
__device__ constexpr double ABW[8][8] = {
    {1.0},
    {3.0 / 2.0, -1.0 / 2.0},
    {23.0 / 12.0, -16.0 / 12.0, 5.0 / 12.0},
    {55.0 / 24.0, -59.0 / 24.0, 37.0 / 24.0, -9.0 / 24.0},
    {1901.0 / 720.0, -2774.0 / 720.0, 2616.0 / 720.0, -1274.0 / 720.0, 251.0 / 720.0},
    {4277.0 / 1440.0, -7923.0 / 1440.0, 9982.0 / 1440.0, -7298.0 / 1440.0, 2877.0 / 1440.0, -475.0 / 1440.0},
    {198721.0 / 60480.0, -447288.0 / 60480.0, 705549.0 / 60480.0, -688256.0 / 60480.0, 407139.0 / 60480.0,
     -134472.0 / 60480.0, 19087.0 / 60480.0},
    {434241.0 / 120960.0, -1152169.0 / 120960.0, 2183877.0 / 120960.0, -2664477.0 / 120960.0,
     2102243.0 / 120960.0, -1041723.0 / 120960.0, 295767.0 / 120960.0, -36799.0 / 120960.0},
};
__device__ constexpr double RKB[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};

// ---- reductions ---------------------------------------------------------------
// Error ratios are non-negative or NaN.  Their IEEE bit patterns order like the
// values as unsigned integers, and any NaN (after fabs) sits above +inf, so
// an integer max both reduces and propagates NaN, with a result independent
// of the reduction order.
__device__ inline uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(v, off, 64);
    v = v > o ? v : o;
  }
  return v;
}

template <int NT>
__device__ inline void block_max_to(uint64_t v, uint64_t* dst) {
  __shared__ uint64_t s_w[NT / 64];
  v = wave_max_u64(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) s_w[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t m = s_w[0];
#pragma unroll
    for (int i = 1; i < NT / 64; ++i) m = m > s_w[i] ? m : s_w[i];
    if (m) atomicMax((unsigned long long*)dst, (unsigned long long)m);
  }
}

// ---- learned step-size proposal -------------------------------------------------
__device__ inline float bf16_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// Features of the learned controller for an accepted attempt, after the
// attempt has been pushed into the history (newest first) and t advanced:
// for each of the last 4 attempts log(err) clamped to [-23, 23], log(h_i/h)
// and the accept flag (zeros where the history is shorter); the PI proposal's
// log-ratio; log(rtol); log(max(t1 - t, h)/h); log(h * stiff), where stiff
// scales the System's largest Jacobian eigenvalue (for the 7-point diffusion,
// 12 max(Du, Dv)/dx^2 + 1), so h*stiff measures the step against the
// explicit stability limit.
__device__ inline void mlp_features(const DevCtrl* c, double h, double pi_lr, float* x) {
  const double lh = log(h);
  for (int i = 0; i < HIST; ++i) {
    const bool have = (uint32_t)i < c->hist_n;
    x[3 * i + 0] = have ? (float)c->hist_lerr[i] : 0.f;
    x[3 * i + 1] = have ? (float)(c->hist_lh[i] - lh) : 0.f;
    x[3 * i + 2] = have ? (float)c->hist_acc[i] : 0.f;
  }
  x[12] = (float)pi_lr;
  x[13] = (float)log(c->rtol > 0 ? c->rtol : c->atol);
  x[14] = (float)log(fmax(c->t1 - c->t, h) / h);
  x[15] = (float)log(h * (c->stiff > 0 ? c->stiff : 1.0));
}

__device__ inline float bf16_round(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return f;
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return __uint_as_float(u & 0xffff0000u);
}

// Forward pass of the 16-64-64-1 tanh network by one wavefront (lane j owns
// hidden unit j), with the arithmetic of the training kernels: bf16 weights,
// inputs and first-layer activations, fp32 accumulation.  W is the packed
// layout W1[64][16] b1[64] W2[64][64] b2[64] w3[64] b3.  Returns the output in
// every lane.  s_h is 64 floats of LDS.
__device__ inline float mlp_forward_wave(const uint16_t* W, const float* x, float* s_h) {
  const int j = threadIdx.x & 63;
  const uint16_t* W1 = W;
  const uint16_t* b1 = W1 + MLP_H * MLP_IN;
  const uint16_t* W2 = b1 + MLP_H;
  const uint16_t* b2 = W2 + MLP_H * MLP_H;
  const uint16_t* w3 = b2 + MLP_H;
  const uint16_t* b3 = w3 + MLP_H;
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < MLP_IN; ++i) s += bf16_to_f32(W1[j * MLP_IN + i]) * bf16_round(x[i]);
  s_h[j] = bf16_round(tanhf(s + bf16_to_f32(b1[j])));
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  float s2 = 0.f;
  for (int i = 0; i < MLP_H; ++i) s2 += bf16_to_f32(W2[j * MLP_H + i]) * s_h[i];
  float o = bf16_to_f32(w3[j]) * tanhf(s2 + bf16_to_f32(b2[j]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) o += __shfl_xor(o, off, 64);
  return o + bf16_to_f32(b3[0]);
}

// ---- the control decision -----------------------------------------------------
// Runs after the error norm of the attempt is complete, in the last workgroup.
// Gustafsson PI controller (alpha = 0.7/k, beta = 0.4/k, safety 0.9, factor in
// [0.2, 5], no growth right after a reject, error floor 1e-10, reject factor
// 0.9 err^(-1/k)); the I variant uses alpha = 1/k, beta = 0.  k is 1 + the
// order of the embedded solution: 5 for the 5(4) pairs, 8 for Fehlberg 7(8).  With the learned controller the proposal for an
// accepted step comes from the network (log-ratio clamped to [log 0.2, log 5],
// never above 0 after a reject); a non-finite network output falls back to
// the PI proposal, and a rejected attempt always retries with the PI shrink.
// The embedded error estimate judges every attempt either way.
struct CtrlScratch {
  double err, fac, pi_lr;
  int ok, use_mlp;
  float x[MLP_IN];
  float h[MLP_H];
  float y;
};

__device__ inline void fixed_step_done(DevCtrl* c) {
  c->accepted += 1;
  c->attempts += 1;
  c->t = c->t0 + (double)c->accepted * c->h;
  // (Adams-Bashforth-Moulton corrects the state in place: no parity flip)
  if (c->mode != MODE_FIXED_ABM) c->parity ^= 1;
  c->k1slot ^= 1;
  c->rhs_evals += mode_rhs_evals(c->mode);
  if (c->mode == MODE_FIXED_AB || c->mode == MODE_FIXED_ABM) c->ring = c->ring + 1 == c->ab_steps ? 0 : c->ring + 1;
  if (c->accepted >= c->nsteps) c->done = 1;
}

// Phase A (one thread): decision and the PI proposal; history push.
__device__ inline void decide_a(DevCtrl* c, double err, CtrlScratch* s) {
  const double h = c->h;
  c->attempts += 1;
  c->rhs_evals += mode_rhs_evals(c->mode);
  c->last_err = err;
  const bool pi_kind = c->ctrl_kind != CTRL_I;
  const double k = c->mode == MODE_ADAPTIVE_F78 ? 8.0 : 5.0;
  const double alpha = pi_kind ? 0.7 / k : 1.0 / k;
  const double beta = pi_kind ? 0.4 / k : 0.0;
  const bool ok = err <= 1.0;
  for (int i = HIST - 1; i > 0; --i) {
    c->hist_lerr[i] = c->hist_lerr[i - 1];
    c->hist_lh[i] = c->hist_lh[i - 1];
    c->hist_acc[i] = c->hist_acc[i - 1];
  }
  c->hist_lerr[0] = isnan(err) ? 23.0 : fmin(23.0, fmax(-23.0, log(fmax(err, 1e-300))));
  c->hist_lh[0] = log(h);
  c->hist_acc[0] = ok ? 1.0 : 0.0;
  if (c->hist_n < HIST) c->hist_n += 1;
  double fac;
  if (ok) {
    const double e = fmax(err, 1e-10);
    double f = 0.9 * pow(e, -alpha) * pow(c->err_prev, beta);
    f = fmin(5.0, fmax(0.2, f));
    if (c->last_rejected) f = fmin(f, 1.0);
    fac = f;
    c->err_prev = e;
    c->t = c->last_flag ? c->t1 : c->t + h;
    c->h_acc = h;
    c->accepted += 1;
    c->parity ^= 1;
    c->k1slot ^= 1;
  } else {
    fac = isnan(err) ? 0.2 : fmax(0.2, 0.9 * pow(err, -1.0 / k));
    c->rejected += 1;
  }
  s->err = err;
  s->fac = fac;
  s->pi_lr = log(fac);
  s->ok = ok;
  s->use_mlp = ok && c->ctrl_kind == CTRL_MLP && c->mlp_w != nullptr && c->t < c->t1;
  if (ok) mlp_features(c, h, s->pi_lr, s->x);  // also recorded in the trace (training data)
}

// Phase C (one thread): apply the proposal, trace, prepare the next attempt.
__device__ inline void decide_c(DevCtrl* c, CtrlScratch* s) {
  const double h = c->h, err = s->err;
  double fac = s->fac;
  double mlp_lr = __longlong_as_double(0x7ff8000000000000LL);
  if (s->use_mlp) {
    if (isfinite(s->y)) {
      double lr = fmin(log(5.0), fmax(log(0.2), (double)s->y));
      if (c->last_rejected) lr = fmin(lr, 0.0);
      mlp_lr = lr;
      fac = exp(lr);
      c->mlp_used += 1;
    } else {
      c->mlp_fallback += 1;
    }
  }
  c->last_rejected = s->ok ? 0 : 1;
  c->dt = h * fac;
  if (c->trace && c->attempts <= c->trace_cap) {
    double* r = c->trace + TRACE_W * (c->attempts - 1);
    r[0] = h;
    r[1] = err;
    r[2] = s->ok ? 1.0 : 0.0;
    r[3] = c->t;
    r[4] = c->dt;
    r[5] = s->pi_lr;
    r[6] = mlp_lr;
    r[7] = c->last_flag ? 1.0 : 0.0;
    for (int i = 0; i < MLP_IN; ++i) r[8 + i] = s->ok ? (double)s->x[i] : __longlong_as_double(0x7ff8000000000000LL);
  }
  if (c->t >= c->t1) {
    c->done = 1;
    c->status = ST_OK;
    return;
  }
  if (c->attempts >= c->max_attempts) {
    c->done = 1;
    c->status = ST_EMAXSTEPS;
    return;
  }
  const bool last = c->dt >= c->t1 - c->t;
  const double hn = last ? c->t1 - c->t : c->dt;
  if (hn < 1e-12 * fmax(1.0, fabs(c->t))) {
    c->done = 1;
    c->status = isfinite(err) ? ST_EDT_UNDERFLOW : ST_ENONFINITE;
    return;
  }
  c->h = hn;
  c->last_flag = last ? 1 : 0;
  // dense output: hand back to the host, which interpolates inside this step
  if (c->mode == MODE_ADAPTIVE_DENSE && s->ok && c->t >= c->stop_at) c->done = 1;
}

// The whole control step: the body of the one-wavefront control kernel that
// follows the final stage kernel of every attempt (a kernel of its own so the
// transcendental control arithmetic does not raise the register budget of the
// streaming kernels).
__device__ inline void ctrl_step(DevCtrl* c) {
  __shared__ CtrlScratch s;
  __shared__ int s_adaptive;
  if (threadIdx.x == 0) {
    // read and clear with one atomic: the stage kernels' contributions are
    // atomics too, so this stays coherent with them when the controller
    // runs inside the same workgroup that produced them
    const uint64_t bits = atomicExch((unsigned long long*)&c->errmax_bits, 0ull);
    s_adaptive = mode_adaptive(c->mode);
    if (s_adaptive) decide_a(c, __longlong_as_double((long long)bits), &s);
    else if (c->mode != 0) fixed_step_done(c);  // mode 0: timing runs change nothing
  }
  __syncthreads();
  if (!s_adaptive) return;
  if (s.use_mlp && threadIdx.x < 64) {
    const float y = mlp_forward_wave(c->mlp_w, s.x, s.h);
    if (threadIdx.x == 0) s.y = y;
  }
  __syncthreads();
  if (threadIdx.x == 0) decide_c(c, &s);
}

}  // namespace hode
