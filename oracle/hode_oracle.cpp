// Plain FP64 CPU oracle for explicit Runge-Kutta time stepping.
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
// baseline leg of the benchmark may load this library.  It shares no source
// with the HIP path: tableaux, right-hand sides, the error norm and the step
// controller are written out here on their own.
//
// What it follows (Ahnert et al. 2011 / the paper's "Architecture and
// nomenclature of Boost Odeint" section): a *state* is advanced in place by a
// *stepper* that calls a *System* right-hand side once per stage; stages are
// combined by an *Algebra* (linear combinations of states); adaptive steppers
// bound the error with the L-infinity norm of the embedded error estimate.
//
//  * Steppers: explicit Euler, the modified midpoint method (Gragg, two
//    substeps), classical Runge-Kutta 4, Runge-Kutta-Dopri 5,
//    Runge-Kutta Cash-Karp 5(4) and Runge-Kutta-Fehlberg 7(8) (the paper's
//    Table 1, fixed and dynamic step size), and the multi-step
//    Adams-Bashforth methods of 1 to 8 steps (fixed step size).
//    Tableaux: Kutta 1901, Dormand & Prince 1980 (Hairer, Norsett & Wanner,
//    Solving ODEs I, Table II.5.2), Cash & Karp 1990 (ACM TOMS 16, 201) and
//    Fehlberg 1968 (NASA TR R-287).
//    Dopri 5 is first-same-as-last: k7 of an accepted step is k1 of the next;
//    Cash-Karp and Fehlberg evaluate their stages afresh every attempt.
//    Adams-Bashforth-Moulton with s steps (predict, evaluate, correct,
//    evaluate): the Adams-Bashforth prediction p, then the Adams-Moulton
//    correction y_{n+1} = y_n + h (gamma_0 f(p) + sum_{j>=1} gamma_j
//    f_{n+1-j}) over s right-hand sides (order s); f_{n+1} = f(y_{n+1}) is
//    the next step's first evaluation.
//    Adams-Bashforth with s steps: y_{n+1} = y_n + h sum_j beta_j f_{n-j},
//    beta_j the integral over one step of the Lagrange polynomial through
//    the last s right-hand sides; the first s-1 steps, before s right-hand
//    sides exist, are taken by the Fehlberg 7(8) fixed step, whose order 8
//    keeps the start-up error below that of every s <= 8.
//  * Systems: exponential dx/dt = x and sigmoidal (logistic) dx/dt = x(1-x),
//    the two families of the accuracy benchmark read as autonomous ODEs whose
//    solutions are x0 e^t and the logistic curve; and the 3D Gray-Scott
//    reaction-diffusion system of the scalability benchmark (equation of the
//    Gray-Scott model), with the Laplacian discretised by the periodic
//    7-point finite-difference stencil of spacing h = L/N.  The second
//    Gray-Scott equation is taken as +u v^2 - (F+k) v (the System listing).
//  * Error norm: max_i |e_i| / (atol + rtol max(|y_i|, |ynew_i|)).
//  * Controller (the paper gives none): Gustafsson's PI controller
//    (Hairer & Wanner, Solving ODEs II, section IV.2) with alpha = 0.7/k,
//    beta = 0.4/k, safety 0.9, factor clamp [0.2, 5], no growth right after a
//    reject (where the factor is max(0.2, 0.9 err^(-1/k))), error floor
//    1e-10, err_prev starting at 1; k = 1 + the order of the embedded
//    solution: 5 for the 5(4) pairs, 8 for Fehlberg 7(8).  The I variant sets
//    alpha = 1/k, beta = 0.
//
// Serial loops define the semantics.  The OpenMP pragmas only parallelise
// loops whose iterations are independent (and a max reduction, which is
// order-independent), so serial and threaded runs are bitwise identical.
// Build with -O2 -ffp-contract=off so no FMA contraction changes rounding.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>

extern "C" {

enum { ORC_EXP = 1, ORC_LOGISTIC = 2, ORC_GRAYSCOTT = 3 };
enum { ORC_RK4 = 1, ORC_DOPRI5 = 2, ORC_CASHKARP = 3, ORC_EULER = 4, ORC_FEHLBERG78 = 5, ORC_MIDPOINT = 6 };
// Adams-Bashforth with s steps (1 <= s <= 8) is method ORC_AB0 + s, the
// Adams-Bashforth-Moulton predictor-corrector with s steps ORC_ABM0 + s.
enum { ORC_AB0 = 10, ORC_ABM0 = 20 };
enum { ORC_CTRL_PI = 1, ORC_CTRL_I = 2 };
enum {
  ORC_OK = 0,
  ORC_EINVAL = -1,
  ORC_EDT_UNDERFLOW = -5,
  ORC_EMAXSTEPS = -6,
  ORC_ENONFINITE = -7,
};

struct orc_system {
  int32_t kind;
  int32_t pad;
  int64_t n;   // number of state elements (for Gray-Scott: 2 N^3)
  int64_t N;   // Gray-Scott grid edge
  double Du, Dv, F, k, L;
};

struct orc_stats {
  int64_t accepted, rejected, rhs_evals;
  double t, dt_next, last_err;
  int32_t status;
  int32_t pad;
};

}  // extern "C"

namespace {

// ---- Butcher tableaux -------------------------------------------------------

// Classical RK4.
const double RK4_C[4] = {0.0, 1.0 / 2.0, 1.0 / 2.0, 1.0};
const double RK4_A[4][4] = {
    {0, 0, 0, 0},
    {1.0 / 2.0, 0, 0, 0},
    {0, 1.0 / 2.0, 0, 0},
    {0, 0, 1.0, 0},
};
const double RK4_B[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};

// Dormand-Prince 5(4), 7 stages, FSAL.
const double DP_C[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};
const double DP_A[7][7] = {
    {0, 0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0, 0},
};
// 5th-order weights (equal to the last row of A) and 4th-order embedded weights.
const double DP_B[7] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0, 0.0};
const double DP_BHAT[7] = {5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0,
                           -92097.0 / 339200.0, 187.0 / 2100.0, 1.0 / 40.0};

// Continuous extension of Dormand-Prince 5(4) (Dormand & Prince 1986;
// Hairer, Norsett & Wanner I, section II.6): the quartic through y_n and
// y_{n+1} with slopes k1 and k7 at the ends, corrected by
// theta^2 (1-theta)^2 h sum_j DPD_j k_j, which makes it 4th-order accurate.
// Written as weights: y(t_n + theta h) = y_n + h sum_j w_j(theta) k_j.
const double DPD[7] = {-12715105075.0 / 11282082432.0, 0.0, 87487479700.0 / 32700410799.0,
                       -10690763975.0 / 1880347072.0, 701980252875.0 / 199316789632.0,
                       -1453857185.0 / 822651844.0, 69997945.0 / 29380423.0};

// w_j(theta) = b_j (3 theta^2 - 2 theta^3) + DPD_j theta^2 (1-theta)^2
//              + [j = 1] theta (1-theta)^2 - [j = 7] theta^2 (1-theta)
// (expanding y_n + theta D + theta (1-theta) (h k1 - D) + theta^2 (1-theta)
// (2 D - h k1 - h k7) + theta^2 (1-theta)^2 h sum_j DPD_j k_j, D = y_{n+1} - y_n).
void dopri5_dense_weights(double th, double* w) {
  const double u = 1.0 - th;
  for (int j = 0; j < 7; ++j) w[j] = DP_B[j] * (3.0 * th * th - 2.0 * th * th * th) + DPD[j] * th * th * u * u;
  w[0] += th * u * u;
  w[6] -= th * th * u;
}

// Cash-Karp 5(4), 6 stages: 5th-order weights b (the solution carried on) and
// 4th-order embedded weights bhat.
const double CK_C[6] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 3.0 / 5.0, 1.0, 7.0 / 8.0};
const double CK_A[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
    {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0, 0, 0},
    {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0, 0},
    {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0, 0},
};
const double CK_B[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0, 512.0 / 1771.0};
const double CK_BHAT[6] = {2825.0 / 27648.0, 0.0, 18575.0 / 48384.0, 13525.0 / 55296.0, 277.0 / 14336.0, 1.0 / 4.0};

// Runge-Kutta-Fehlberg 7(8), 13 stages: 8th-order weights b (the solution
// carried on) and 7th-order embedded weights bhat.
const double F78_C[13] = {0.0,       2.0 / 27.0, 1.0 / 9.0, 1.0 / 6.0, 5.0 / 12.0, 1.0 / 2.0, 5.0 / 6.0,
                          1.0 / 6.0, 2.0 / 3.0,  1.0 / 3.0, 1.0,       0.0,        1.0};
const double F78_A[13][13] = {
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
const double F78_B[13] = {0, 0, 0, 0, 0, 34.0 / 105.0, 9.0 / 35.0, 9.0 / 35.0, 9.0 / 280.0, 9.0 / 280.0, 0,
                          41.0 / 840.0, 41.0 / 840.0};
const double F78_BHAT[13] = {41.0 / 840.0, 0, 0, 0, 0, 34.0 / 105.0, 9.0 / 35.0, 9.0 / 35.0, 9.0 / 280.0,
                             9.0 / 280.0, 41.0 / 840.0, 0, 0};

// Adams-Bashforth weights for s steps, from their definition: with the
// right-hand sides f_{n-i} at the nodes u = -i (i = 0 .. s-1, in units of
// h), beta_j = integral over u in [0, 1] of the Lagrange basis polynomial
// prod_{i != j} (u + i) / (i - j).  The product is expanded into integer
// coefficients c_d; with L = lcm(1 .. s), the numerator sum_d c_d L/(d+1)
// and the denominator L prod_{i != j} (i - j) are exact integers, so the
// one division rounds beta_j correctly.
void ab_weights(int s, double* beta) {
  int64_t L = 1;
  for (int64_t d = 2; d <= s; ++d) {
    int64_t a = L, b = d;
    while (b) { const int64_t r = a % b; a = b; b = r; }
    L = L / a * d;
  }
  for (int j = 0; j < s; ++j) {
    int64_t poly[9] = {1};  // coefficients of u^0 .. u^8
    int deg = 0;
    int64_t denom = L;
    for (int i = 0; i < s; ++i) {
      if (i == j) continue;
      // multiply by (u + i)
      for (int d = deg + 1; d >= 1; --d) poly[d] = poly[d - 1] + (int64_t)i * poly[d];
      poly[0] *= i;
      ++deg;
      denom *= (i - j);
    }
    int64_t num = 0;
    for (int d = 0; d <= deg; ++d) num += poly[d] * (L / (d + 1));
    beta[j] = (double)num / (double)denom;
  }
}

// Adams-Moulton weights for s values, from their definition: with the
// right-hand sides at the nodes u = 1 - j (j = 0 .. s-1; u = 1 is the new
// point), gamma_j = integral over u in [0, 1] of prod_{i != j} (u - (1 - i))
// / ((1 - j) - (1 - i)) = prod_{i != j} (u - 1 + i) / (i - j); the same
// exact-integer evaluation as ab_weights.
void am_weights(int s, double* gamma) {
  int64_t L = 1;
  for (int64_t d = 2; d <= s; ++d) {
    int64_t a = L, b = d;
    while (b) { const int64_t r = a % b; a = b; b = r; }
    L = L / a * d;
  }
  for (int j = 0; j < s; ++j) {
    int64_t poly[9] = {1};  // coefficients of u^0 .. u^8
    int deg = 0;
    int64_t denom = L;
    for (int i = 0; i < s; ++i) {
      if (i == j) continue;
      // multiply by (u + (i - 1))
      for (int d = deg + 1; d >= 1; --d) poly[d] = poly[d - 1] + (int64_t)(i - 1) * poly[d];
      poly[0] *= (i - 1);
      ++deg;
      denom *= (i - j);
    }
    int64_t num = 0;
    for (int d = 0; d <= deg; ++d) num += poly[d] * (L / (d + 1));
    gamma[j] = (double)num / (double)denom;
  }
}

// ---- the System: right-hand sides -----------------------------------------

inline int64_t wrap(int64_t i, int64_t N) { return ((i % N) + N) % N; }

// Gray-Scott on an N^3 periodic grid, x fastest, u in [0, N^3), v in [N^3, 2N^3).
void gs_rhs(const orc_system& s, const double* y, double* f) {
  const int64_t N = s.N, n3 = N * N * N;
  const double h = s.L / (double)N;
  const double h2 = h * h;
  const double* u = y;
  const double* v = y + n3;
  double* du = f;
  double* dv = f + n3;
#pragma omp parallel for schedule(static)
  for (int64_t kz = 0; kz < N; ++kz) {
    for (int64_t jy = 0; jy < N; ++jy) {
      for (int64_t ix = 0; ix < N; ++ix) {
        const int64_t c = ix + N * (jy + N * kz);
        const int64_t xm = wrap(ix - 1, N) + N * (jy + N * kz);
        const int64_t xp = wrap(ix + 1, N) + N * (jy + N * kz);
        const int64_t ym = ix + N * (wrap(jy - 1, N) + N * kz);
        const int64_t yp = ix + N * (wrap(jy + 1, N) + N * kz);
        const int64_t zm = ix + N * (jy + N * wrap(kz - 1, N));
        const int64_t zp = ix + N * (jy + N * wrap(kz + 1, N));
        const double lap_u = (u[xm] + u[xp] + u[ym] + u[yp] + u[zm] + u[zp] - 6.0 * u[c]) / h2;
        const double lap_v = (v[xm] + v[xp] + v[ym] + v[yp] + v[zm] + v[zp] - 6.0 * v[c]) / h2;
        const double uvv = u[c] * v[c] * v[c];
        du[c] = s.Du * lap_u - uvv + s.F * (1.0 - u[c]);
        dv[c] = s.Dv * lap_v + uvv - (s.F + s.k) * v[c];
      }
    }
  }
}

void rhs(const orc_system& s, const double* y, double* f) {
  const int64_t n = s.n;
  switch (s.kind) {
    case ORC_EXP:
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i) f[i] = y[i];
      break;
    case ORC_LOGISTIC:
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i) f[i] = y[i] * (1.0 - y[i]);
      break;
    default:
      gs_rhs(s, y, f);
      break;
  }
}

bool valid(const orc_system* s) {
  if (!s) return false;
  if (s->kind == ORC_EXP || s->kind == ORC_LOGISTIC) return s->n >= 0;
  if (s->kind == ORC_GRAYSCOTT) return s->N >= 1 && s->n == 2 * s->N * s->N * s->N && s->L > 0;
  return false;
}

// ---- the Algebra: w = y + h * sum_j a_j k_j --------------------------------

void stage_input(int64_t n, const double* y, double h, int nk, const double* a, double* const* k, double* w) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < nk; ++j)
      if (a[j] != 0.0) s += a[j] * k[j][i];
    w[i] = y[i] + h * s;
  }
}

// ---- the L-infinity error norm ----------------------------------------------

double err_norm(int64_t n, const double* y, const double* ynew, const double* e, double atol, double rtol) {
  double m = 0.0;
  bool nan = false;
#pragma omp parallel for schedule(static) reduction(max : m) reduction(|| : nan)
  for (int64_t i = 0; i < n; ++i) {
    const double sc = atol + rtol * std::max(std::fabs(y[i]), std::fabs(ynew[i]));
    const double r = std::fabs(e[i]) / sc;
    if (std::isnan(r)) nan = true;
    else m = std::max(m, r);
  }
  return nan ? NAN : m;
}

// ---- steppers -----------------------------------------------------------------

struct Work {
  std::vector<std::vector<double>> k;
  std::vector<double> w;
  explicit Work(int64_t n, int nk) : k(nk, std::vector<double>(n)), w(n) {}
};

// One explicit Euler step in place: y += h f(y).
void euler_step(const orc_system& s, double* y, double h, Work& W) {
  const int64_t n = s.n;
  rhs(s, y, W.k[0].data());
  const double* k = W.k[0].data();
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) y[i] = y[i] + h * k[i];
}

// One modified midpoint step of size H in place, with m = 2 substeps of
// h = H/2 (Gragg; Hairer, Norsett & Wanner I, section II.9): z0 = y,
// z1 = z0 + h f(z0), z2 = z0 + 2h f(z1), y_new = (z2 + z1 + h f(z2)) / 2.
void midpoint_step(const orc_system& s, double* y, double H, Work& W) {
  const int64_t n = s.n;
  const double h = 0.5 * H;
  double* f = W.k[0].data();
  double* z1 = W.k[1].data();
  double* z2 = W.k[2].data();
  rhs(s, y, f);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) z1[i] = y[i] + h * f[i];
  rhs(s, z1, f);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) z2[i] = y[i] + 2.0 * h * f[i];
  rhs(s, z2, f);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) y[i] = 0.5 * (z2[i] + z1[i] + h * f[i]);
}

// One classical RK4 step in place.
void rk4_step(const orc_system& s, double* y, double h, Work& W) {
  const int64_t n = s.n;
  double* kp[4] = {W.k[0].data(), W.k[1].data(), W.k[2].data(), W.k[3].data()};
  rhs(s, y, kp[0]);
  for (int st = 1; st < 4; ++st) {
    stage_input(n, y, h, st, RK4_A[st], kp, W.w.data());
    rhs(s, W.w.data(), kp[st]);
  }
  stage_input(n, y, h, 4, RK4_B, kp, W.w.data());
  std::memcpy(y, W.w.data(), sizeof(double) * n);
}

// One Dopri5 attempt from (y, k1): writes ynew, k7 = f(ynew) and (if e != null)
// the embedded error e = h * sum_j (b_j - bhat_j) k_j.
void dopri5_attempt(const orc_system& s, const double* y, const double* k1, double h, double* ynew, double* k7,
                    double* e, Work& W) {
  const int64_t n = s.n;
  double* kp[7];
  for (int j = 0; j < 7; ++j) kp[j] = W.k[j].data();
  std::memcpy(kp[0], k1, sizeof(double) * n);
  for (int st = 1; st < 6; ++st) {
    stage_input(n, y, h, st, DP_A[st], kp, W.w.data());
    rhs(s, W.w.data(), kp[st]);
  }
  stage_input(n, y, h, 6, DP_A[6], kp, ynew);  // stage-7 input is the 5th-order solution
  rhs(s, ynew, kp[6]);
  std::memcpy(k7, kp[6], sizeof(double) * n);
  if (e) {
    double d[7];
    for (int j = 0; j < 7; ++j) d[j] = DP_B[j] - DP_BHAT[j];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int j = 0; j < 7; ++j)
        if (d[j] != 0.0) acc += d[j] * kp[j][i];
      e[i] = h * acc;
    }
  }
}

// One Cash-Karp attempt from y: k1 = f(y) and five more stages; writes ynew
// (5th order) and (if e != null) e = h * sum_j (b_j - bhat_j) k_j.
void cashkarp_attempt(const orc_system& s, const double* y, double h, double* ynew, double* e, Work& W) {
  const int64_t n = s.n;
  double* kp[6];
  for (int j = 0; j < 6; ++j) kp[j] = W.k[j].data();
  rhs(s, y, kp[0]);
  for (int st = 1; st < 6; ++st) {
    stage_input(n, y, h, st, CK_A[st], kp, W.w.data());
    rhs(s, W.w.data(), kp[st]);
  }
  stage_input(n, y, h, 6, CK_B, kp, ynew);
  if (e) {
    double d[6];
    for (int j = 0; j < 6; ++j) d[j] = CK_B[j] - CK_BHAT[j];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int j = 0; j < 6; ++j)
        if (d[j] != 0.0) acc += d[j] * kp[j][i];
      e[i] = h * acc;
    }
  }
}

// One Fehlberg 7(8) attempt from y with k1 = f(y) given: twelve more stages;
// writes ynew (8th order) and (if e != null) e = h * sum_j (b_j - bhat_j) k_j.
void fehlberg78_attempt(const orc_system& s, const double* y, const double* k1, double h, double* ynew, double* e,
                        Work& W) {
  const int64_t n = s.n;
  double* kp[13];
  for (int j = 0; j < 13; ++j) kp[j] = W.k[j].data();
  std::memcpy(kp[0], k1, sizeof(double) * n);
  for (int st = 1; st < 13; ++st) {
    stage_input(n, y, h, st, F78_A[st], kp, W.w.data());
    rhs(s, W.w.data(), kp[st]);
  }
  stage_input(n, y, h, 13, F78_B, kp, ynew);
  if (e) {
    double d[13];
    for (int j = 0; j < 13; ++j) d[j] = F78_B[j] - F78_BHAT[j];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int j = 0; j < 13; ++j)
        if (d[j] != 0.0) acc += d[j] * kp[j][i];
      e[i] = h * acc;
    }
  }
}

// Adams-Bashforth with s steps over nsteps fixed steps of size h from a fresh
// start (no stored right-hand sides): f_n = f(y_n) is kept for the last s
// steps; steps 0 .. s-2 are Fehlberg 7(8) steps (whose k1 is that f_n), later
// steps y_{n+1} = y_n + h sum_{j<s} beta_j f_{n-j}.  Returns the right-hand
// side evaluations made.
int64_t adams_bashforth(const orc_system& s, int steps, double* y, double h, int64_t nsteps) {
  const int64_t n = s.n;
  double beta[8];
  ab_weights(steps, beta);
  std::vector<std::vector<double>> f(steps, std::vector<double>(n));  // f[m % steps] = f_m
  Work W(n, 13);
  std::vector<double> ynew(n);
  int64_t evals = 0;
  for (int64_t m = 0; m < nsteps; ++m) {
    double* fm = f[m % steps].data();
    rhs(s, y, fm);
    evals += 1;
    if (m < steps - 1) {
      fehlberg78_attempt(s, y, fm, h, ynew.data(), nullptr, W);
      evals += 12;
      std::swap_ranges(ynew.begin(), ynew.end(), y);
      continue;
    }
    double* past[8];
    for (int j = 0; j < steps; ++j) past[j] = f[(m - j) % steps].data();
    stage_input(n, y, h, steps, beta, past, ynew.data());
    std::swap_ranges(ynew.begin(), ynew.end(), y);
  }
  return evals;
}

// Adams-Bashforth-Moulton (PECE) with s steps over nsteps fixed steps from a
// fresh start: the start-up as adams_bashforth, then per step f_n = f(y_n),
// the prediction p = y_n + h sum_j beta_j f_{n-j}, and the correction
// y_{n+1} = y_n + h (gamma_0 f(p) + sum_{j>=1} gamma_j f_{n+1-j}).  Returns
// the right-hand side evaluations made.
int64_t adams_bashforth_moulton(const orc_system& s, int steps, double* y, double h, int64_t nsteps) {
  const int64_t n = s.n;
  double beta[8], gamma[8];
  ab_weights(steps, beta);
  am_weights(steps, gamma);
  std::vector<std::vector<double>> f(steps, std::vector<double>(n));  // f[m % steps] = f_m
  Work W(n, 13);
  std::vector<double> p(n), fp(n), ynew(n);
  int64_t evals = 0;
  for (int64_t m = 0; m < nsteps; ++m) {
    double* fm = f[m % steps].data();
    rhs(s, y, fm);
    evals += 1;
    if (m < steps - 1) {
      fehlberg78_attempt(s, y, fm, h, ynew.data(), nullptr, W);
      evals += 12;
      std::swap_ranges(ynew.begin(), ynew.end(), y);
      continue;
    }
    double* past[8];
    for (int j = 0; j < steps; ++j) past[j] = f[(m - j) % steps].data();
    stage_input(n, y, h, steps, beta, past, p.data());
    rhs(s, p.data(), fp.data());
    evals += 1;
    // corrector values f(p), f_n, f_{n-1}, .., f_{n+2-s}
    double* cv[8];
    cv[0] = fp.data();
    for (int j = 1; j < steps; ++j) cv[j] = f[(m + 1 - j) % steps].data();
    stage_input(n, y, h, steps, gamma, cv, ynew.data());
    std::swap_ranges(ynew.begin(), ynew.end(), y);
  }
  return evals;
}

// ---- step-size controller -------------------------------------------------------

// k = 1 + the order of the embedded solution (5 for the 5(4) pairs, 8 for
// Fehlberg 7(8)).
struct Ctrl {
  double k, alpha, beta, safety = 0.9, fac_min = 0.2, fac_max = 5.0;
  double err_prev = 1.0;
  bool last_rejected = false;
  explicit Ctrl(int kind, double order_k = 5.0) : k(order_k) {
    if (kind == ORC_CTRL_I) { alpha = 1.0 / k; beta = 0.0; }
    else { alpha = 0.7 / k; beta = 0.4 / k; }
  }
  // Returns whether the attempt is accepted and the factor for the next step.
  bool decide(double err, double* fac) {
    if (err <= 1.0) {
      const double e = std::max(err, 1e-10);
      double f = safety * std::pow(e, -alpha) * std::pow(err_prev, beta);
      f = std::min(fac_max, std::max(fac_min, f));
      if (last_rejected) f = std::min(f, 1.0);
      err_prev = e;
      last_rejected = false;
      *fac = f;
      return true;
    }
    *fac = std::isnan(err) ? fac_min : std::max(fac_min, safety * std::pow(err, -1.0 / k));
    last_rejected = true;
    return false;
  }
};

}  // namespace

extern "C" {

int orc_rhs(const orc_system* s, const double* y, double* f) {
  if (!valid(s)) return ORC_EINVAL;
  rhs(*s, y, f);
  return ORC_OK;
}

void orc_tableau(int method, double* a, double* b, double* bhat, double* c) {
  if (method == ORC_RK4) {
    for (int i = 0; i < 4; ++i) {
      for (int j = 0; j < 4; ++j) a[i * 4 + j] = RK4_A[i][j];
      b[i] = RK4_B[i];
      c[i] = RK4_C[i];
      if (bhat) bhat[i] = 0.0;
    }
  } else if (method == ORC_FEHLBERG78) {
    for (int i = 0; i < 13; ++i) {
      for (int j = 0; j < 13; ++j) a[i * 13 + j] = F78_A[i][j];
      b[i] = F78_B[i];
      bhat[i] = F78_BHAT[i];
      c[i] = F78_C[i];
    }
  } else if (method == ORC_CASHKARP) {
    for (int i = 0; i < 6; ++i) {
      for (int j = 0; j < 6; ++j) a[i * 6 + j] = CK_A[i][j];
      b[i] = CK_B[i];
      bhat[i] = CK_BHAT[i];
      c[i] = CK_C[i];
    }
  } else {
    for (int i = 0; i < 7; ++i) {
      for (int j = 0; j < 7; ++j) a[i * 7 + j] = DP_A[i][j];
      b[i] = DP_B[i];
      bhat[i] = DP_BHAT[i];
      c[i] = DP_C[i];
    }
  }
}

double orc_err_norm(int64_t n, const double* y, const double* ynew, const double* e, double atol, double rtol) {
  return err_norm(n, y, ynew, e, atol, rtol);
}

// One controller decision: returns 1 if accepted; writes the step factor and the
// updated (err_prev, last_rejected).
void orc_ab_weights(int steps, double* beta) {
  if (steps >= 1 && steps <= 8) ab_weights(steps, beta);
}

void orc_am_weights(int steps, double* gamma) {
  if (steps >= 1 && steps <= 8) am_weights(steps, gamma);
}

int orc_ctrl_decide_k(int kind, double order_k, double err, double* err_prev, int* last_rejected, double* fac) {
  Ctrl c(kind, order_k);
  c.err_prev = *err_prev;
  c.last_rejected = *last_rejected != 0;
  const bool acc = c.decide(err, fac);
  *err_prev = c.err_prev;
  *last_rejected = c.last_rejected ? 1 : 0;
  return acc ? 1 : 0;
}

int orc_ctrl_decide(int kind, double err, double* err_prev, int* last_rejected, double* fac) {
  Ctrl c(kind);
  c.err_prev = *err_prev;
  c.last_rejected = *last_rejected != 0;
  const bool acc = c.decide(err, fac);
  *err_prev = c.err_prev;
  *last_rejected = c.last_rejected ? 1 : 0;
  return acc ? 1 : 0;
}

int orc_rk4_step(const orc_system* s, double* y, double h) {
  if (!valid(s)) return ORC_EINVAL;
  Work W(s->n, 4);
  rk4_step(*s, y, h, W);
  return ORC_OK;
}

// One Dopri5 attempt from y (k1 computed here).  ynew, k7 and e are outputs.
int orc_dopri5_attempt(const orc_system* s, const double* y, double h, double* ynew, double* k7, double* e) {
  if (!valid(s)) return ORC_EINVAL;
  Work W(s->n, 7);
  std::vector<double> k1(s->n);
  rhs(*s, y, k1.data());
  dopri5_attempt(*s, y, k1.data(), h, ynew, k7, e, W);
  return ORC_OK;
}

int orc_fehlberg78_attempt(const orc_system* s, const double* y, double h, double* ynew, double* e) {
  if (!valid(s)) return ORC_EINVAL;
  Work W(s->n, 13);
  std::vector<double> k1(s->n);
  rhs(*s, y, k1.data());
  fehlberg78_attempt(*s, y, k1.data(), h, ynew, e, W);
  return ORC_OK;
}

int orc_cashkarp_attempt(const orc_system* s, const double* y, double h, double* ynew, double* e) {
  if (!valid(s)) return ORC_EINVAL;
  Work W(s->n, 6);
  cashkarp_attempt(*s, y, h, ynew, e, W);
  return ORC_OK;
}

// Fixed steps: t_n = t0 + n dt (Odeint integrate_const / do_step).  An
// Adams-Bashforth run starts afresh (no stored right-hand sides).
int orc_integrate_n_steps_e(const orc_system* s, int method, double* y, double t0, double dt, int64_t nsteps,
                            double* t_end, int64_t* rhs_evals) {
  const bool ab = method > ORC_AB0 && method <= ORC_AB0 + 8;
  const bool abm = method > ORC_ABM0 && method <= ORC_ABM0 + 8;
  if (!valid(s) || nsteps < 0 ||
      !(method == ORC_RK4 || method == ORC_DOPRI5 || method == ORC_CASHKARP || method == ORC_EULER ||
        method == ORC_FEHLBERG78 || method == ORC_MIDPOINT || ab || abm))
    return ORC_EINVAL;
  const int64_t n = s->n;
  int64_t evals = 0;
  if (method == ORC_MIDPOINT) {
    Work W(n, 3);
    for (int64_t i = 0; i < nsteps; ++i) midpoint_step(*s, y, dt, W);
    evals = 3 * nsteps;
  } else if (ab) {
    evals = adams_bashforth(*s, method - ORC_AB0, y, dt, nsteps);
  } else if (abm) {
    evals = adams_bashforth_moulton(*s, method - ORC_ABM0, y, dt, nsteps);
  } else if (method == ORC_FEHLBERG78) {
    Work W(n, 13);
    std::vector<double> k1(n), ynew(n);
    for (int64_t i = 0; i < nsteps; ++i) {
      rhs(*s, y, k1.data());
      fehlberg78_attempt(*s, y, k1.data(), dt, ynew.data(), nullptr, W);
      std::swap_ranges(ynew.begin(), ynew.end(), y);
    }
    evals = 13 * nsteps;
  } else if (method == ORC_EULER) {
    Work W(n, 1);
    for (int64_t i = 0; i < nsteps; ++i) euler_step(*s, y, dt, W);
  } else if (method == ORC_RK4) {
    Work W(n, 4);
    for (int64_t i = 0; i < nsteps; ++i) rk4_step(*s, y, dt, W);
  } else if (method == ORC_CASHKARP) {
    Work W(n, 6);
    std::vector<double> ynew(n);
    for (int64_t i = 0; i < nsteps; ++i) {
      cashkarp_attempt(*s, y, dt, ynew.data(), nullptr, W);
      std::swap_ranges(ynew.begin(), ynew.end(), y);
    }
  } else {
    Work W(n, 7);
    std::vector<double> k1(n), k7(n), ynew(n);
    rhs(*s, y, k1.data());
    for (int64_t i = 0; i < nsteps; ++i) {
      dopri5_attempt(*s, y, k1.data(), dt, ynew.data(), k7.data(), nullptr, W);
      std::swap_ranges(ynew.begin(), ynew.end(), y);
      k1.swap(k7);
    }
  }
  if (!ab && !abm && method != ORC_FEHLBERG78 && method != ORC_MIDPOINT) {
    const int per = method == ORC_EULER ? 1 : (method == ORC_RK4 ? 4 : 6);
    evals = per * nsteps + (method == ORC_DOPRI5 && nsteps > 0 ? 1 : 0);
  }
  if (t_end) *t_end = t0 + (double)nsteps * dt;
  if (rhs_evals) *rhs_evals = evals;
  return ORC_OK;
}

int orc_integrate_n_steps(const orc_system* s, int method, double* y, double t0, double dt, int64_t nsteps,
                          double* t_end) {
  return orc_integrate_n_steps_e(s, method, y, t0, dt, nsteps, t_end, nullptr);
}

// Error-controlled integration from t0 to t1 with an embedded pair (Dopri5 or
// Cash-Karp; Odeint integrate_adaptive).  The trace, if given, receives 4
// doubles per attempt: h, err, accepted (0/1), t after.
// The state of an error-controlled integration that a run carries from one
// end time to the next: the embedded pair's k1 (first same as last), the
// proposed step, the controller and the counters.
struct Adaptive {
  const orc_system& s;
  int method;
  bool dp;
  double atol, rtol;
  Work W;
  std::vector<double> k1, k7, ynew, e;
  Ctrl c;
  double dt, last_err = 0.0;
  int64_t acc = 0, rej = 0, evals = 0, att = 0;
  Adaptive(const orc_system& sys, int method, const double* y, double dt0, double a, double r, int ctrl_kind)
      : s(sys), method(method), dp(method == ORC_DOPRI5), atol(a), rtol(r),
        W(sys.n, method == ORC_FEHLBERG78 ? 13 : 7), k1(sys.n), k7(sys.n),
        ynew(sys.n), e(sys.n), c(ctrl_kind, method == ORC_FEHLBERG78 ? 8.0 : 5.0), dt(dt0) {
    if (dp) {
      rhs(s, y, k1.data());
      evals = 1;
    }
  }
  // Advances y from *t to t1 (the last step clipped to land on t1); returns
  // the status.  max_steps bounds the attempts of the whole run.
  int advance(double* y, double* t, double t1, int64_t max_steps, double* trace, int64_t trace_cap) {
    const int64_t n = s.n;
    while (*t < t1) {
      if (att >= max_steps) return ORC_EMAXSTEPS;
      const bool last = dt >= t1 - *t;
      const double h = last ? t1 - *t : dt;
      if (h < 1e-12 * std::max(1.0, std::fabs(*t))) return std::isfinite(last_err) ? ORC_EDT_UNDERFLOW : ORC_ENONFINITE;
      if (dp) {
        dopri5_attempt(s, y, k1.data(), h, ynew.data(), k7.data(), e.data(), W);
        evals += 6;
      } else if (method == ORC_FEHLBERG78) {
        rhs(s, y, k1.data());
        fehlberg78_attempt(s, y, k1.data(), h, ynew.data(), e.data(), W);
        evals += 13;
      } else {
        cashkarp_attempt(s, y, h, ynew.data(), e.data(), W);
        evals += 6;
      }
      ++att;
      const double err = err_norm(n, y, ynew.data(), e.data(), atol, rtol);
      last_err = err;
      double fac;
      const bool ok = c.decide(err, &fac);
      if (ok) {
        std::swap_ranges(ynew.begin(), ynew.end(), y);
        if (dp) k1.swap(k7);
        *t = last ? t1 : *t + h;
        ++acc;
      } else {
        ++rej;
      }
      dt = h * fac;
      if (trace && att <= trace_cap) {
        double* r = trace + 4 * (att - 1);
        r[0] = h; r[1] = err; r[2] = ok ? 1.0 : 0.0; r[3] = *t;
      }
    }
    return ORC_OK;
  }
  void stats(orc_stats* st, double t, int status) const {
    if (!st) return;
    st->accepted = acc; st->rejected = rej; st->rhs_evals = evals;
    st->t = t; st->dt_next = dt; st->last_err = last_err; st->status = status;
  }
};

int orc_integrate_adaptive_m(const orc_system* s, int method, double* y, double t0, double t1, double dt0,
                             double atol, double rtol, int ctrl_kind, int64_t max_steps, orc_stats* st,
                             double* trace, int64_t trace_cap) {
  if (!valid(s) || !(t1 >= t0) || !(dt0 > 0) || !(atol >= 0) || !(rtol >= 0) || (atol == 0 && rtol == 0) ||
      !(method == ORC_DOPRI5 || method == ORC_CASHKARP || method == ORC_FEHLBERG78))
    return ORC_EINVAL;
  Adaptive A(*s, method, y, dt0, atol, rtol, ctrl_kind);
  double t = t0;
  const int status = A.advance(y, &t, t1, max_steps, trace, trace_cap);
  A.stats(st, t, status);
  return status;
}

// Odeint integrate_times: the state at times[0] is the current one; the run
// then advances to times[1], times[2], ... in turn, every step clipped to
// land on them, carrying the proposed step, the controller and (Dopri5) k1
// from one to the next, and out[i * n ..] receives the state at times[i].
// Stops at the first failing status (max_steps bounds the whole run).
int orc_integrate_times(const orc_system* s, int method, double* y, const double* times, int64_t nt, double dt0,
                        double atol, double rtol, int ctrl_kind, int64_t max_steps, double* out, orc_stats* st) {
  if (!valid(s) || nt < 1 || !(dt0 > 0) || !(atol >= 0) || !(rtol >= 0) || (atol == 0 && rtol == 0) ||
      !(method == ORC_DOPRI5 || method == ORC_CASHKARP || method == ORC_FEHLBERG78) || !out)
    return ORC_EINVAL;
  for (int64_t i = 1; i < nt; ++i)
    if (!(times[i] > times[i - 1])) return ORC_EINVAL;
  const int64_t n = s->n;
  Adaptive A(*s, method, y, dt0, atol, rtol, ctrl_kind);
  std::memcpy(out, y, sizeof(double) * n);
  double t = times[0];
  int status = ORC_OK;
  for (int64_t i = 1; i < nt && status == ORC_OK; ++i) {
    status = A.advance(y, &t, times[i], max_steps, nullptr, 0);
    if (status == ORC_OK) std::memcpy(out + i * n, y, sizeof(double) * n);
  }
  A.stats(st, t, status);
  return status;
}

// Dense output (Odeint's dense-output Dopri5 with integrate_times): the
// controlled steps run from times[0] to times[nt-1] exactly as
// integrate_adaptive does (only the last step clipped, to land on the end),
// and the state at every intermediate requested time comes from the
// continuous extension of the accepted step that covers it:
// t_prev < times[i] <= t_prev + h, theta = (times[i] - t_prev) / h with
// t_prev = t - h.  out[0] is the start state, out[nt-1] the end state.
int orc_integrate_dense_times(const orc_system* s, double* y, const double* times, int64_t nt, double dt0,
                              double atol, double rtol, int ctrl_kind, int64_t max_steps, double* out,
                              orc_stats* st) {
  if (!valid(s) || nt < 1 || !(dt0 > 0) || !(atol >= 0) || !(rtol >= 0) || (atol == 0 && rtol == 0) || !out)
    return ORC_EINVAL;
  for (int64_t i = 1; i < nt; ++i)
    if (!(times[i] > times[i - 1])) return ORC_EINVAL;
  const int64_t n = s->n;
  std::memcpy(out, y, sizeof(double) * n);
  const double t1 = times[nt - 1];
  Work W(n, 7);
  std::vector<double> k1(n), k7(n), ynew(n), e(n);
  rhs(*s, y, k1.data());
  Ctrl c(ctrl_kind);
  double t = times[0], dt = dt0, last_err = 0.0;
  int64_t acc = 0, rej = 0, evals = 1, att = 0, next = 1;
  int status = ORC_OK;
  while (t < t1) {
    if (att >= max_steps) { status = ORC_EMAXSTEPS; break; }
    const bool last = dt >= t1 - t;
    const double h = last ? t1 - t : dt;
    if (h < 1e-12 * std::max(1.0, std::fabs(t))) {
      status = std::isfinite(last_err) ? ORC_EDT_UNDERFLOW : ORC_ENONFINITE;
      break;
    }
    dopri5_attempt(*s, y, k1.data(), h, ynew.data(), k7.data(), e.data(), W);
    evals += 6;
    ++att;
    const double err = err_norm(n, y, ynew.data(), e.data(), atol, rtol);
    last_err = err;
    double fac;
    if (c.decide(err, &fac)) {
      const double tn = last ? t1 : t + h;
      // observations inside (t, tn], before y moves on (W.k holds k1 .. k7)
      for (; next < nt - 1 && times[next] <= tn; ++next) {
        const double th = (times[next] - (tn - h)) / h;
        double w[7];
        dopri5_dense_weights(th, w);
        double* o = out + next * n;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
          double sum = 0.0;
          for (int j = 0; j < 7; ++j)
            if (w[j] != 0.0) sum += w[j] * W.k[j][i];
          o[i] = y[i] + h * sum;
        }
      }
      std::swap_ranges(ynew.begin(), ynew.end(), y);
      k1.swap(k7);
      t = tn;
      ++acc;
    } else {
      ++rej;
    }
    dt = h * fac;
  }
  if (status == ORC_OK && nt > 1) std::memcpy(out + (nt - 1) * n, y, sizeof(double) * n);
  if (st) {
    st->accepted = acc; st->rejected = rej; st->rhs_evals = evals;
    st->t = t; st->dt_next = dt; st->last_err = last_err; st->status = status;
  }
  return status;
}

void orc_dopri5_dense_weights(double theta, double* w) { dopri5_dense_weights(theta, w); }

int orc_integrate_adaptive(const orc_system* s, double* y, double t0, double t1, double dt0, double atol,
                           double rtol, int ctrl_kind, int64_t max_steps, orc_stats* st, double* trace,
                           int64_t trace_cap) {
  return orc_integrate_adaptive_m(s, ORC_DOPRI5, y, t0, t1, dt0, atol, rtol, ctrl_kind, max_steps, st, trace,
                                  trace_cap);
}

// Replays a recorded step sequence: attempt i uses step h[i] and is accepted iff
// accepted[i] != 0 (the controller is bypassed).  errs (optional) receives the
// error norm of every attempt.
int orc_integrate_replay_m(const orc_system* s, int method, double* y, double t0, const double* hs,
                           const int32_t* accepted, int64_t n_att, double atol, double rtol, double* t_end,
                           double* errs) {
  if (!valid(s) || n_att < 0 || !(method == ORC_DOPRI5 || method == ORC_CASHKARP || method == ORC_FEHLBERG78))
    return ORC_EINVAL;
  const bool dp = method == ORC_DOPRI5;
  const int64_t n = s->n;
  Work W(n, method == ORC_FEHLBERG78 ? 13 : 7);
  std::vector<double> k1(n), k7(n), ynew(n), e(n);
  if (dp) rhs(*s, y, k1.data());
  double t = t0;
  for (int64_t i = 0; i < n_att; ++i) {
    if (dp) {
      dopri5_attempt(*s, y, k1.data(), hs[i], ynew.data(), k7.data(), e.data(), W);
    } else if (method == ORC_FEHLBERG78) {
      rhs(*s, y, k1.data());
      fehlberg78_attempt(*s, y, k1.data(), hs[i], ynew.data(), e.data(), W);
    } else {
      cashkarp_attempt(*s, y, hs[i], ynew.data(), e.data(), W);
    }
    if (errs) errs[i] = err_norm(n, y, ynew.data(), e.data(), atol, rtol);
    if (accepted[i]) {
      std::swap_ranges(ynew.begin(), ynew.end(), y);
      if (dp) k1.swap(k7);
      t += hs[i];
    }
  }
  if (t_end) *t_end = t;
  return ORC_OK;
}

int orc_integrate_replay(const orc_system* s, double* y, double t0, const double* hs, const int32_t* accepted,
                         int64_t n_att, double atol, double rtol, double* t_end, double* errs) {
  return orc_integrate_replay_m(s, ORC_DOPRI5, y, t0, hs, accepted, n_att, atol, rtol, t_end, errs);
}

int orc_num_threads(void);

}  // extern "C"

#ifdef _OPENMP
#include <omp.h>
extern "C" int orc_num_threads(void) { return omp_get_max_threads(); }
#else
extern "C" int orc_num_threads(void) { return 1; }
#endif
