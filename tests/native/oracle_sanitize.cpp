// Exercises every oracle entry point on small inputs; built with
// AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_oracle_sanitizers.py.  Any out-of-bounds access, leak or
// undefined operation aborts with a report.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" {
struct orc_system {
  int32_t kind, pad;
  int64_t n, N;
  double Du, Dv, F, k, L;
};
struct orc_stats {
  int64_t accepted, rejected, rhs_evals;
  double t, dt_next, last_err;
  int32_t status, pad;
};
int orc_integrate_n_steps_e(const orc_system*, int, double*, double, double, int64_t, double*, int64_t*);
int orc_integrate_adaptive_m(const orc_system*, int, double*, double, double, double, double, double, int, int64_t,
                             orc_stats*, double*, int64_t);
int orc_integrate_replay_m(const orc_system*, int, double*, double, const double*, const int32_t*, int64_t, double,
                           double, double*, double*);
int orc_integrate_times(const orc_system*, int, double*, const double*, int64_t, double, double, double, int, int64_t,
                        double*, orc_stats*);
int orc_integrate_dense_times(const orc_system*, double*, const double*, int64_t, double, double, double, int,
                              int64_t, double*, orc_stats*);
void orc_ab_weights(int, double*);
void orc_am_weights(int, double*);
}

int main() {
  int fails = 0;
  for (int N : {1, 2, 3, 5}) {
    orc_system s{3, 0, 2 * (int64_t)N * N * N, N, 2e-3, 1e-3, 0.053, 0.014, 2.5};
    std::vector<double> y0(s.n), y;
    for (int64_t i = 0; i < s.n; ++i) y0[i] = (i < s.n / 2 ? 1.0 : 0.0) + 0.01 * std::sin(0.37 * i);
    const int methods[] = {1, 2, 3, 4, 5, 6, 11, 14, 18, 21, 24, 28};
    for (int m : methods) {
      y = y0;
      double te;
      int64_t ev;
      fails += orc_integrate_n_steps_e(&s, m, y.data(), 0.0, 0.05, 9, &te, &ev) != 0;
    }
    for (int m : {2, 3, 5}) {
      y = y0;
      orc_stats st;
      std::vector<double> tr(4 * 64);
      fails += orc_integrate_adaptive_m(&s, m, y.data(), 0.0, 2.0, 0.1, 1e-7, 1e-7, 1, 64, &st, tr.data(), 64) != 0;
      const int64_t na = st.accepted + st.rejected;
      std::vector<double> hs(na), errs(na);
      std::vector<int32_t> acc(na);
      for (int64_t i = 0; i < na; ++i) { hs[i] = tr[4 * i]; acc[i] = tr[4 * i + 2] != 0.0; }
      y = y0;
      double te;
      fails += orc_integrate_replay_m(&s, m, y.data(), 0.0, hs.data(), acc.data(), na, 1e-7, 1e-7, &te,
                                      errs.data()) != 0;
      const double times[] = {0.0, 0.3, 1.1, 2.0};
      std::vector<double> out(4 * s.n);
      y = y0;
      fails += orc_integrate_times(&s, m, y.data(), times, 4, 0.1, 1e-7, 1e-7, 1, 1000, out.data(), &st) != 0;
    }
    const double times[] = {0.0, 0.01, 0.3, 1.1, 2.0};
    std::vector<double> out(5 * s.n);
    orc_stats st;
    y = y0;
    fails += orc_integrate_dense_times(&s, y.data(), times, 5, 0.1, 1e-7, 1e-7, 1, 1000, out.data(), &st) != 0;
  }
  double w[8];
  for (int k = 1; k <= 8; ++k) { orc_ab_weights(k, w); orc_am_weights(k, w); }
  std::printf("oracle sanitize run: %d failures\n", fails);
  return fails ? 1 : 0;
}
