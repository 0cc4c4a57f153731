// libhode host driver and C ABI.
//
// The integration loop is device-resident: the control block (time, step,
// counters, controller state) lives in device memory and is advanced by a
// one-wavefront control kernel after every attempt, so the host only launches
// hipGraph chunks
// of M attempts and reads the status word back once per chunk.  Kernels read
// the "done" flag at entry and exit at once after the run has finished, so a
// chunk that overshoots costs only empty launches.  Buffer rotation (the new
// state becoming the current one, k7 becoming k1 under first-same-as-last) is
// a parity flip in the control block, which keeps graph node arguments fixed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <map>
#include <new>
#include <queue>
#include <vector>
#include <string>
#include <utility>

#include "../../include/hode.h"
#include "hode_internal.h"

using hode::DevCtrl;

// ---- batched ensemble: host side -----------------------------------------------
struct Ensemble {
  int n = 0, dtype = 0;
  std::vector<int> N;
  std::vector<double> prm;  // n x {Du, Dv, F, k, L}
  std::vector<hode::EnsInst> inst;
  std::vector<int> parity, vw;
  std::vector<int> zc;         // planes per tile of each instance (0: sized from the launch's cell count)
  std::vector<double> weight;  // per-attempt work estimates (dealing instances to queues)
  std::vector<int64_t> attempts_last;
  hipEvent_t ev[2] = {nullptr, nullptr};
  double kernel_ms_last = 0;  // summed launch durations of the last integration
  int launches_last = 0;
  int epoch_first = 0, epoch_len = 0;  // attempts per instance per launch (0: the whole integration)
  int64_t barrier_polls = (int64_t)1 << 24;  // polls before a grid barrier gives up
  void* pool = nullptr;
  hode::EnsInst* d_inst = nullptr;
  hode::EnsTile* d_tiles = nullptr;
  size_t tiles_cap = 0;
  int32_t* d_order = nullptr;  // instances by work estimate, largest first (re-tiling order)
  // one device block: qoff[9] | params | bar | error | live[max_rounds] | qctr[8 (1 + 6 max_rounds)]
  void* d_sync = nullptr;
  int nwg = 0;
  double* d_trace = nullptr;
  int64_t trace_cap = 0;
  hipGraphExec_t graph = nullptr;
};

struct hode_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int rhs = 0;
  double prm[5] = {0, 0, 0, 0, 0};
  int dtype = 0;
  int64_t nelem = 0;  // elements per state array (EW n; GS 2 N^3)
  int N = 0;
  size_t esize = 0;
  void* y[2] = {nullptr, nullptr};
  void* ks[2] = {nullptr, nullptr};
  void* k[7] = {nullptr};
  DevCtrl* d_ctrl = nullptr;
  DevCtrl* d_ctrl_save = nullptr;
  DevCtrl* h_ctrl = nullptr;  // pinned mirror
  double* d_trace = nullptr;
  int64_t trace_cap = 0;
  uint16_t* d_mlp = nullptr;
  int ctrl_kind = hode::CTRL_PI;
  double atol = 1e-6, rtol = 1e-6;
  int ry = 0, zc = 0, ew_grid = 0, vw = 0;  // ry, zc: the tile of the widest stage kind
  int kry[hode::K_ALL] = {0}, kzc[hode::K_ALL] = {0};  // tile of every stage kind
  int knw[hode::K_ALL] = {0};  // wavefronts per workgroup of every stage kind (0: 4)
  int nw = 4;                  // requested wavefronts per workgroup (hode_set_tile_waves)
  // extra arrays (Fehlberg 7(8) stages k1 .. k12 on the Gray-Scott path, the
  // Adams-Bashforth ring of past right-hand sides), allocated on first use,
  // and their device table
  void* xk_arr[hode::kXkCount] = {nullptr};
  void** d_xk = nullptr;
  // Adams-Bashforth history (as an Odeint stepper object keeps it): steps s
  // (0: none), its step size, and the steps taken since it started
  int ab_steps = 0;
  bool ab_moulton = false;  // the history is that of Adams-Bashforth-Moulton
  double ab_dt = 0;
  int64_t ab_n = 0;
  void* d_obs = nullptr;  // staging for dense-output observations bound for host memory
  bool k1_valid = false;
  int parity = 0, k1slot = 0;
  bool use_graphs = true;      // replay captured chunks (else enqueue every kernel)
  int stepper = HODE_DOPRI5;   // embedded pair of the adaptive calls
  bool persist_valid = false;  // controller history carried between try_step calls
  DevCtrl persist;
  hode_stats last{};
  int64_t last_attempts = 0;
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  std::string err;
  Ensemble* ens = nullptr;
};

namespace {

int fail(hode_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                                      \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail(ctx, HODE_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
  } while (0)

bool is_gs(const hode_ctx* c) { return c->rhs == HODE_RHS_GRAYSCOTT3D; }

void clear_graphs(hode_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

void free_state(hode_ctx* c) {
  clear_graphs(c);
  for (void*& p : c->y) { if (p) (void)hipFree(p); p = nullptr; }
  for (void*& p : c->ks) { if (p) (void)hipFree(p); p = nullptr; }
  for (void*& p : c->k) { if (p) (void)hipFree(p); p = nullptr; }
  for (void*& p : c->xk_arr) { if (p) (void)hipFree(p); p = nullptr; }
  if (c->d_obs) (void)hipFree(c->d_obs);
  c->d_obs = nullptr;
  if (c->d_xk) (void)hipFree(c->d_xk);
  c->d_xk = nullptr;
  c->ab_steps = 0;
  c->nelem = 0;
  c->N = 0;
  c->dtype = 0;
  c->k1_valid = false;
  c->parity = c->k1slot = 0;
}

hode::GSLaunch gs_args(const hode_ctx* c) {
  hode::GSLaunch a{};
  for (int i = 0; i < 2; ++i) { a.y[i] = c->y[i]; a.ks[i] = c->ks[i]; }
  for (int i = 0; i < 7; ++i) a.k[i] = c->k[i];
  a.k[0] = (void*)c->d_xk;  // the extra arrays' table (see hode::xk)
  a.N = c->N;
  a.n3 = (int64_t)c->N * c->N * c->N;
  a.zc = c->zc;
  const double h = c->prm[4] / (double)c->N;
  a.Du_h2 = c->prm[0] / (h * h);
  a.Dv_h2 = c->prm[1] / (h * h);
  a.F = c->prm[2];
  a.kk = c->prm[3];
  return a;
}

// One stage kernel of `kind` with that kind's tile.
hipError_t launch_stage(const hode_ctx* c, int kind, hode::GSLaunch a) {
  a.zc = c->kzc[kind];
  return hode::launch_gs(kind, c->dtype, c->kry[kind], c->vw, c->knw[kind] ? c->knw[kind] : 4, a, c->d_ctrl,
                         c->stream);
}

// Sets one tile for every stage kind: ry rows per wavefront, zc planes, nw
// wavefronts per workgroup where the kind has such tiles (else 4).
void set_all_tiles(hode_ctx* c, int ry, int zc, int nw = 4) {
  c->ry = ry;
  c->zc = zc;
  for (int k = 0; k < hode::K_ALL; ++k) {
    c->kry[k] = ry;
    c->kzc[k] = zc;
    c->knw[k] = hode::gs_tile_supported(k, c->dtype, ry, c->vw, nw, c->N) ? nw : 4;
  }
}

int default_zc(int N, int ry) {
  const int nx = (N + 63) / 64, ny = (N + 4 * ry - 1) / (4 * ry);
  const int want = 2048;
  int nz = (want + nx * ny - 1) / (nx * ny);
  if (nz < 1) nz = 1;
  int zc = (N + nz - 1) / nz;
  if (zc < 8) zc = 8;
  return zc;
}

int default_ew_grid(int64_t n, int dtype) {
  const int64_t vec = dtype == HODE_F32 ? 4 : 2;
  int64_t g = (n / vec + 255) / 256;
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  return (int)g;
}

// Allocates the extra arrays a run needs (Gray-Scott Fehlberg stages; the
// first `ring` Adams-Bashforth ring slots; Gray-Scott k6 for dense output)
// and refreshes their device table.
int ensure_xk(hode_ctx* c, bool f78, int ring, bool k6 = false, bool mm = false) {
  bool changed = false;
  const size_t bytes = std::max<size_t>(256, (size_t)c->nelem * c->esize);
  auto need = [&](int i) -> bool {
    if (c->xk_arr[i]) return true;
    if (hipMalloc(&c->xk_arr[i], bytes) != hipSuccess) {
      c->xk_arr[i] = nullptr;
      return false;
    }
    changed = true;
    return true;
  };
  if (f78 && is_gs(c))
    for (int i = 0; i < hode::kXkF78; ++i)
      if (!need(i)) return fail(c, HODE_ENOMEM, "device allocation failed (Fehlberg stages)");
  for (int i = 0; i < ring; ++i)
    if (!need(hode::kRingBase + i)) return fail(c, HODE_ENOMEM, "device allocation failed (Adams-Bashforth ring)");
  if (k6 && is_gs(c) && !need(hode::kXkK6)) return fail(c, HODE_ENOMEM, "device allocation failed (k6)");
  if (mm && is_gs(c) && (!need(hode::kXkZ1) || !need(hode::kXkZ1 + 1)))
    return fail(c, HODE_ENOMEM, "device allocation failed (midpoint substeps)");
  if (!c->d_xk) {
    if (hipMalloc(&c->d_xk, sizeof(void*) * hode::kXkCount) != hipSuccess) {
      c->d_xk = nullptr;
      return fail(c, HODE_ENOMEM, "device allocation failed");
    }
    changed = true;
    clear_graphs(c);  // captured launches hold the table's address
  }
  if (changed) {
    HIPCHK(c, hipMemcpyAsync(c->d_xk, c->xk_arr, sizeof(void*) * hode::kXkCount, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return HODE_OK;
}

bool mode_f78(int mode) { return mode == hode::MODE_FIXED_F78 || mode == hode::MODE_ADAPTIVE_F78; }

bool mode_multistep(int mode) { return mode == hode::MODE_FIXED_AB || mode == hode::MODE_FIXED_ABM; }

// Enqueues the kernels of one attempt (or fixed step) in `mode`
// (Adams-Bashforth(-Moulton): with the context's current number of steps).
hipError_t enqueue_attempt(hode_ctx* c, int mode) {
  if (!is_gs(c)) {
    hipError_t e = mode_f78(mode) || mode_multistep(mode)
                       ? hode::launch_ewx(c->dtype, c->rhs, mode, c->ab_steps, c->y[0], c->y[1], c->d_xk, nullptr,
                                          c->nelem, c->ew_grid, c->d_ctrl, c->stream)
                       : hode::launch_ew(c->dtype, c->rhs, mode, c->y[0], c->y[1], c->nelem, c->ew_grid,
                                         c->d_ctrl, c->stream);
    return e != hipSuccess ? e : hode::launch_ctrl(c->d_ctrl, c->stream);
  }
  if (mode_f78(mode) || mode_multistep(mode)) {
    const hode::GSLaunch a = gs_args(c);
    if (mode_multistep(mode)) {
      if (c->ab_steps < 1 || c->ab_steps > 8) return hipErrorInvalidValue;
      // Adams-Bashforth (the prediction, for Adams-Bashforth-Moulton), then
      // the Adams-Moulton correction
      hipError_t e = launch_stage(c, hode::K_AB1 + c->ab_steps - 1, a);
      if (e == hipSuccess && mode == hode::MODE_FIXED_ABM) e = launch_stage(c, hode::K_ABC1 + c->ab_steps - 1, a);
      return e != hipSuccess ? e : hode::launch_ctrl(c->d_ctrl, c->stream);
    }
    for (int k = hode::K_F1; k <= hode::K_F12; ++k) {
      hipError_t e = launch_stage(c, k, a);
      if (e != hipSuccess) return e;
    }
    hipError_t e = launch_stage(c, mode == hode::MODE_ADAPTIVE_F78 ? hode::K_F13 : hode::K_F13F, a);
    return e != hipSuccess ? e : hode::launch_ctrl(c->d_ctrl, c->stream);
  }
  const hode::GSLaunch a = gs_args(c);
  static const int rk4[] = {hode::K_D1, hode::K_R2, hode::K_R3, hode::K_R4};
  static const int dp5f[] = {hode::K_D2, hode::K_D3, hode::K_D4, hode::K_D5, hode::K_D6F, hode::K_D7F};
  static const int dp5a[] = {hode::K_D2, hode::K_D3, hode::K_D4, hode::K_D5, hode::K_D6, hode::K_D7};
  static const int dp5d[] = {hode::K_D2, hode::K_D3, hode::K_D4, hode::K_D5, hode::K_D6K, hode::K_D7};
  // Cash-Karp: stages 1-3 have the Dopri5 shapes and coefficients
  static const int ckf[] = {hode::K_D1, hode::K_D2, hode::K_D3, hode::K_C4, hode::K_C5, hode::K_C6F};
  static const int cka[] = {hode::K_D1, hode::K_D2, hode::K_D3, hode::K_C4, hode::K_C5, hode::K_C6};
  static const int eul[] = {hode::K_E1};
  static const int mmd[] = {hode::K_MM1, hode::K_MM2, hode::K_MM3};
  const int* seq = mode == hode::MODE_FIXED_RK4   ? rk4
                   : mode == hode::MODE_FIXED_DP5 ? dp5f
                   : mode == hode::MODE_FIXED_CK  ? ckf
                   : mode == hode::MODE_ADAPTIVE_CK ? cka
                   : mode == hode::MODE_FIXED_EULER ? eul
                   : mode == hode::MODE_ADAPTIVE_DENSE ? dp5d
                   : mode == hode::MODE_FIXED_MM ? mmd
                                                    : dp5a;
  const int ns = mode == hode::MODE_FIXED_RK4 ? 4
                 : mode == hode::MODE_FIXED_EULER ? 1
                 : mode == hode::MODE_FIXED_MM ? 3
                                               : 6;
  for (int i = 0; i < ns; ++i) {
    hipError_t e = launch_stage(c, seq[i], a);
    if (e != hipSuccess) return e;
  }
  return hode::launch_ctrl(c->d_ctrl, c->stream);
}

int get_graph(hode_ctx* c, int mode, int M, hipGraphExec_t* out) {
  // Adams-Bashforth chunks differ by the number of steps
  auto key = std::make_pair(mode_multistep(mode) ? mode | (c->ab_steps << 8) : mode, M);
  auto it = c->graphs.find(key);
  if (it != c->graphs.end()) { *out = it->second; return HODE_OK; }
  hipGraph_t g = nullptr;
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  for (int i = 0; i < M && le == hipSuccess; ++i) le = enqueue_attempt(c, mode);
  hipError_t ee = hipStreamEndCapture(c->stream, &g);
  if (le != hipSuccess) { if (g) (void)hipGraphDestroy(g); return fail(c, HODE_EHIP, std::string("capture: ") + hipGetErrorString(le)); }
  if (ee != hipSuccess) return fail(c, HODE_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
  hipGraphExec_t ex = nullptr;
  hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) return fail(c, HODE_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
  c->graphs[key] = ex;
  *out = ex;
  return HODE_OK;
}

// Scale of the largest Jacobian eigenvalue of Gray-Scott on an N^3 grid: the
// 7-point Laplacian's spectral radius 12/dx^2 times the larger diffusivity,
// plus 1 for the reaction terms.
double gs_stiffness(const double* prm, int N) {
  const double dx = prm[4] / N;
  return 12.0 * std::max(std::fabs(prm[0]), std::fabs(prm[1])) / (dx * dx) + 1.0;
}

int adaptive_mode(const hode_ctx* c) {
  return c->stepper == HODE_CASHKARP54   ? hode::MODE_ADAPTIVE_CK
         : c->stepper == HODE_FEHLBERG78 ? hode::MODE_ADAPTIVE_F78
                                         : hode::MODE_ADAPTIVE;
}

// The learned controller was trained on the 5(4) pairs' error sequences.
int check_adaptive(hode_ctx* c) {
  if (c->ctrl_kind == hode::CTRL_MLP && c->stepper == HODE_FEHLBERG78)
    return fail(c, HODE_EINVAL, "the learned controller serves the 5(4) pairs; use PI or I with Fehlberg 7(8)");
  return HODE_OK;
}

DevCtrl base_ctrl(const hode_ctx* c, int mode) {
  DevCtrl d;
  std::memset(&d, 0, sizeof(d));
  d.mode = mode;
  d.ctrl_kind = c->ctrl_kind;
  d.parity = c->parity;
  d.k1slot = c->k1slot;
  d.atol = c->atol;
  d.rtol = c->rtol;
  d.err_prev = 1.0;
  d.trace = c->trace_cap > 0 ? c->d_trace : nullptr;
  d.trace_cap = c->trace_cap;
  d.mlp_w = c->d_mlp;
  d.max_attempts = INT64_MAX;
  d.stiff = 1.0;
  if (c->rhs == HODE_RHS_GRAYSCOTT3D && c->N > 0) d.stiff = gs_stiffness(c->prm, c->N);
  return d;
}

int launch_k1(hode_ctx* c) {
  if (!is_gs(c)) return HODE_OK;
  const hode::GSLaunch a = gs_args(c);
  HIPCHK(c, launch_stage(c, hode::K_D1, a));
  return HODE_OK;
}

int pow2_floor(int64_t x) {
  int m = 1;
  while ((int64_t)m * 2 <= x && m < 64) m *= 2;
  return m;
}

// Runs the device-resident loop from the control block `init` until done.
int run_loop(hode_ctx* c, const DevCtrl& init, bool need_k1) {
  if (mode_f78(init.mode) || mode_multistep(init.mode) || init.mode == hode::MODE_ADAPTIVE_DENSE ||
      init.mode == hode::MODE_FIXED_MM) {
    int rc = ensure_xk(c, mode_f78(init.mode), mode_multistep(init.mode) ? init.ab_steps : 0,
                       init.mode == hode::MODE_ADAPTIVE_DENSE, init.mode == hode::MODE_FIXED_MM);
    if (rc) return rc;
  }
  // every other stepping ends the Adams-Bashforth(-Moulton) history
  if (!mode_multistep(init.mode)) c->ab_steps = 0;
  *c->h_ctrl = init;
  HIPCHK(c, hipMemcpyAsync(c->d_ctrl, c->h_ctrl, sizeof(DevCtrl), hipMemcpyHostToDevice, c->stream));
  int64_t extra_evals = 0;
  if (need_k1 && !init.done) {
    int rc = launch_k1(c);
    if (rc) return rc;
    extra_evals = 1;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  DevCtrl cur = init;
  int64_t chunks = 0;
  while (!cur.done) {
    int M;
    if (hode::mode_adaptive(init.mode)) {
      const double est = std::ceil((cur.t1 - cur.t) / (cur.dt > 0 ? cur.dt : 1.0)) + 1.0;
      M = pow2_floor(est > 64 ? 64 : (int64_t)est);
    } else {
      M = pow2_floor(cur.nsteps - cur.accepted);
    }
    if (c->use_graphs) {
      hipGraphExec_t ex;
      int rc = get_graph(c, init.mode, M, &ex);
      if (rc) return rc;
      HIPCHK(c, hipGraphLaunch(ex, c->stream));
    } else {
      for (int i = 0; i < M; ++i) HIPCHK(c, enqueue_attempt(c, init.mode));
    }
    HIPCHK(c, hipMemcpyAsync(c->h_ctrl, c->d_ctrl, sizeof(DevCtrl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    cur = *c->h_ctrl;
    if (++chunks > (int64_t)1 << 40) return fail(c, HODE_EHIP, "control loop did not terminate");
  }
  c->parity = cur.parity;
  c->k1slot = cur.k1slot;
  // k1 = f(y) of the current state is in the first-same-as-last slot only
  // after the Dopri5 modes
  c->k1_valid = init.mode == hode::MODE_FIXED_DP5 || init.mode == hode::MODE_ADAPTIVE ||
                init.mode == hode::MODE_ADAPTIVE_DENSE;
  c->last.accepted = cur.accepted;
  c->last.rejected = cur.rejected;
  c->last.rhs_evals = cur.rhs_evals + extra_evals;
  c->last.t = cur.t;
  c->last.dt_next = hode::mode_adaptive(init.mode) ? cur.dt : cur.h;
  c->last.last_err = cur.last_err;
  c->last.status = cur.status;
  c->last_attempts = cur.attempts;
  c->persist = cur;
  return HODE_OK;
}

// One Adams-Bashforth start-up step: a Fehlberg 7(8) fixed step from the
// current state that also records f(y_n) (its k1) in ring slot `slot`.  d
// carries time and counters from step to step.
int ab_startup_step(hode_ctx* c, DevCtrl& d, int slot) {
  d.mode = hode::MODE_FIXED_F78;
  d.nsteps = d.accepted + 1;
  d.done = 0;
  d.parity = c->parity;
  d.k1slot = c->k1slot;
  *c->h_ctrl = d;
  HIPCHK(c, hipMemcpyAsync(c->d_ctrl, c->h_ctrl, sizeof(DevCtrl), hipMemcpyHostToDevice, c->stream));
  void* ring = c->xk_arr[hode::kRingBase + slot];
  if (is_gs(c)) {
    const hode::GSLaunch a = gs_args(c);
    for (int k = hode::K_F1; k <= hode::K_F12; ++k) HIPCHK(c, launch_stage(c, k, a));
    HIPCHK(c, launch_stage(c, hode::K_F13F, a));
    HIPCHK(c, hipMemcpyAsync(ring, c->xk_arr[0], (size_t)c->nelem * c->esize, hipMemcpyDeviceToDevice, c->stream));
  } else {
    HIPCHK(c, hode::launch_ewx(c->dtype, c->rhs, hode::MODE_FIXED_F78, 0, c->y[0], c->y[1], c->d_xk, ring,
                               c->nelem, c->ew_grid, c->d_ctrl, c->stream));
  }
  HIPCHK(c, hode::launch_ctrl(c->d_ctrl, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->h_ctrl, c->d_ctrl, sizeof(DevCtrl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  d = *c->h_ctrl;
  c->parity = d.parity;
  c->k1slot = d.k1slot;
  c->k1_valid = false;
  return HODE_OK;
}

// n fixed Adams-Bashforth (moulton: Adams-Bashforth-Moulton) steps with s
// steps.  The history (the last s right-hand sides) continues from the
// previous call when the method, s and dt are the same and no other stepping
// came in between; otherwise it starts afresh, and the first s - 1 steps are
// Fehlberg 7(8) steps that record f(y_n).
int ab_run(hode_ctx* c, int s, bool moulton, double t0, double dt, int64_t n) {
  if (!(c->ab_steps == s && c->ab_moulton == moulton && c->ab_dt == dt)) {
    c->ab_steps = s;
    c->ab_moulton = moulton;
    c->ab_dt = dt;
    c->ab_n = 0;
  }
  int rc = ensure_xk(c, c->ab_n < s - 1 && n > 0, s);
  if (rc) return rc;
  DevCtrl d = base_ctrl(c, moulton ? hode::MODE_FIXED_ABM : hode::MODE_FIXED_AB);
  d.t = d.t0 = t0;
  d.h = d.dt = dt;
  d.ab_steps = s;
  int64_t i = 0;
  for (; i < n && c->ab_n < s - 1; ++i) {
    rc = ab_startup_step(c, d, (int)(c->ab_n % s));
    if (rc) return rc;
    ++c->ab_n;
  }
  d.mode = moulton ? hode::MODE_FIXED_ABM : hode::MODE_FIXED_AB;
  d.nsteps = n;
  d.done = i >= n;
  d.ring = (int)(c->ab_n % s);
  d.parity = c->parity;
  d.k1slot = c->k1slot;
  rc = run_loop(c, d, false);
  if (rc) return rc;
  c->ab_n += n - i;
  return HODE_OK;
}

int check_ready(hode_ctx* c) {
  if (!c) return HODE_EINVAL;
  if (!c->rhs) return fail(c, HODE_ESTATE, "no RHS set");
  if (!c->dtype) return fail(c, HODE_ESTATE, "no state initialised");
  return HODE_OK;
}

void free_ensemble(hode_ctx* c) {
  Ensemble* e = c ? c->ens : nullptr;
  if (!e) return;
  if (e->graph) (void)hipGraphExecDestroy(e->graph);
  if (e->pool) (void)hipFree(e->pool);
  if (e->d_inst) (void)hipFree(e->d_inst);
  if (e->d_tiles) (void)hipFree(e->d_tiles);
  if (e->d_order) (void)hipFree(e->d_order);
  if (e->d_sync) (void)hipFree(e->d_sync);
  if (e->d_trace) (void)hipFree(e->d_trace);
  for (hipEvent_t& v : e->ev)
    if (v) (void)hipEventDestroy(v);
  delete e;
  c->ens = nullptr;
}

// Segments per wavefront of an ensemble instance's tiles: rows of at most
// 32 16-byte lanes are packed one per segment of 64/seg lanes (rounded down),
// as many segments as hold a row (seg 2, 3, 4, 5, 6, 8, 10 or 16; at least 4
// lanes a segment); 1 = ordinary tiles.
int ens_seg_for(int dtype, int N, int vw) {
  const int vf = dtype == HODE_F32 ? 4 : 2;
  if (vw != vf || N % vw) return 1;
  const int nl = N / vw;
  if (nl > 32) return 1;
  for (int seg : {16, 10, 8, 6, 5, 4, 3})
    if (64 / seg >= nl) return seg;
  return 2;
}

// Rows one pass of the ensemble's stage tiles covers for instance i (kEnsNW
// waves of 16 bytes of state per lane and field, or of two register rows of
// seg rows each; stage 6 excepted): a tile of exactly this many rows needs
// one pass, so no halo row of it is read twice.
int ens_tile_rows(const Ensemble& e, int i) {
  const int seg = ens_seg_for(e.dtype, e.N[i], e.vw[i]);
  if (seg > 1) return 2 * hode::kEnsNW * seg;
  const int per_lane = (e.dtype == HODE_F32 ? 4 : 2) / e.vw[i];
  return hode::kEnsNW * std::max(1, per_lane);
}


// The tiles of one launch: every active instance cut into row chunks of one
// tile pass (the last one ends at N) and plane chunks sized so a phase has
// about kTilesPerWorkgroup tiles per workgroup (at least 4096 cells, at least
// 4 planes), in plane-chunk-major, row-chunk-minor order (tiles that share
// halo rows are claimed close together).  Instances are dealt to eight
// queues, one per XCD, largest work first onto the least loaded queue.
void build_tiles(const Ensemble& e, int G, const std::vector<int>& active, std::vector<hode::EnsTile>& tiles,
                 std::vector<int32_t>& qoff) {
  double cells = 0;
  for (int i : active) cells += (double)e.N[i] * e.N[i] * e.N[i];
  const double target = std::max(4096.0, cells / (hode::kTilesPerWorkgroup * G));
  std::vector<int> order(active);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return e.weight[a] > e.weight[b]; });
  std::vector<std::vector<int>> q(8);
  std::vector<double> load(8, 0.0);
  for (int i : order) {
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    q[x].push_back(i);
    load[x] += e.weight[i];
  }
  tiles.clear();
  qoff.assign(9, 0);
  for (int x = 0; x < 8; ++x) {
    qoff[x] = (int32_t)tiles.size();
    for (int i : q[x]) {
      const int N = e.N[i];
      const int rows = ens_tile_rows(e, i);
      const int ny = (N + rows - 1) / rows;
      int zc = e.zc[i] > 0 ? e.zc[i] : (int)std::lround(target / ((double)N * rows));
      zc = std::max(e.zc[i] > 0 ? 1 : 4, std::min(N, zc));
      const int nz = (N + zc - 1) / zc;
      for (int kz = 0; kz < nz; ++kz) {
        const int z0 = (int)((int64_t)N * kz / nz), z1 = (int)((int64_t)N * (kz + 1) / nz);
        for (int ky = 0; ky < ny; ++ky)
          tiles.push_back({i, rows * ky, std::min(N, rows * (ky + 1)), z0, z1, 0});
      }
    }
  }
  qoff[8] = (int32_t)tiles.size();
}

}  // namespace

extern "C" {

int hode_create(hode_ctx** out, int device, void* stream) {
  if (!out) return HODE_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HODE_EINVAL;
  hode_ctx* c = new (std::nothrow) hode_ctx();
  if (!c) return HODE_ENOMEM;
  c->device = device;
  if (hipSetDevice(device) != hipSuccess) { delete c; return HODE_EHIP; }
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) { delete c; return HODE_EHIP; }
    c->own_stream = true;
  }
  if (hipMalloc(&c->d_ctrl, sizeof(DevCtrl)) != hipSuccess || hipMalloc(&c->d_ctrl_save, sizeof(DevCtrl)) != hipSuccess ||
      hipHostMalloc(&c->h_ctrl, sizeof(DevCtrl), hipHostMallocDefault) != hipSuccess) {
    hode_destroy(c);
    return HODE_ENOMEM;
  }
  std::memset(c->h_ctrl, 0, sizeof(DevCtrl));
  if (hipMemcpy(c->d_ctrl, c->h_ctrl, sizeof(DevCtrl), hipMemcpyHostToDevice) != hipSuccess) {
    hode_destroy(c);
    return HODE_EHIP;
  }
  *out = c;
  return HODE_OK;
}

void hode_destroy(hode_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  free_state(c);
  if (c->d_ctrl) (void)hipFree(c->d_ctrl);
  if (c->d_ctrl_save) (void)hipFree(c->d_ctrl_save);
  if (c->h_ctrl) (void)hipHostFree(c->h_ctrl);
  if (c->d_trace) (void)hipFree(c->d_trace);
  if (c->d_mlp) (void)hipFree(c->d_mlp);
  free_ensemble(c);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

int hode_set_rhs(hode_ctx* c, int rhs, const double* params, int nparams) {
  if (!c) return HODE_EINVAL;
  if (rhs == HODE_RHS_EXP || rhs == HODE_RHS_LOGISTIC) {
    if (nparams != 0) return fail(c, HODE_EINVAL, "element-wise systems take no parameters");
    if (c->dtype && c->N) return fail(c, HODE_ESTATE, "state is a Gray-Scott grid");
  } else if (rhs == HODE_RHS_GRAYSCOTT3D) {
    if (nparams != 5 || !params) return fail(c, HODE_EINVAL, "Gray-Scott takes {Du, Dv, F, k, L}");
    for (int i = 0; i < 5; ++i)
      if (!std::isfinite(params[i])) return fail(c, HODE_EINVAL, "non-finite parameter");
    if (!(params[4] > 0)) return fail(c, HODE_EINVAL, "L must be > 0");
    if (c->dtype && !c->N) return fail(c, HODE_ESTATE, "state is element-wise");
    for (int i = 0; i < 5; ++i) c->prm[i] = params[i];
  } else {
    return fail(c, HODE_EINVAL, "unknown rhs");
  }
  c->rhs = rhs;
  c->k1_valid = false;
  c->ab_steps = 0;
  clear_graphs(c);
  return HODE_OK;
}

int hode_init_state(hode_ctx* c, int dtype, int nfields, int ndim, const int64_t* shape, const void* src,
                    int src_on_device) {
  if (!c) return HODE_EINVAL;
  if (!c->rhs) return fail(c, HODE_ESTATE, "set the RHS before the state");
  if (dtype != HODE_F32 && dtype != HODE_F64) return fail(c, HODE_EINVAL, "dtype");
  if (!shape) return fail(c, HODE_EINVAL, "shape is NULL");
  int64_t nelem;
  int N = 0;
  if (is_gs(c)) {
    if (nfields != 2 || ndim != 3) return fail(c, HODE_EINVAL, "Gray-Scott needs nfields 2, ndim 3");
    if (shape[0] != shape[1] || shape[1] != shape[2]) return fail(c, HODE_EINVAL, "grid must be cubic");
    if (shape[0] < 1 || shape[0] > 2048) return fail(c, HODE_EINVAL, "grid edge out of [1, 2048]");
    N = (int)shape[0];
    nelem = 2 * (int64_t)N * N * N;
  } else {
    if (nfields != 1 || ndim != 1) return fail(c, HODE_EINVAL, "element-wise systems need nfields 1, ndim 1");
    if (shape[0] < 0 || shape[0] > ((int64_t)1 << 40)) return fail(c, HODE_EINVAL, "size out of range");
    nelem = shape[0];
  }
  if (nelem > 0 && !src) return fail(c, HODE_EINVAL, "src is NULL");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const size_t es = dtype == HODE_F32 ? 4 : 8;
  const size_t bytes = (size_t)nelem * es;
  const size_t alloc = bytes < 256 ? 256 : bytes;
  const int narr = is_gs(c) ? 2 + 2 + 5 : 2;
  // same shape and precision: keep the buffers (and the captured graphs)
  const bool reuse = c->dtype == dtype && c->nelem == nelem && c->N == N && c->y[0];
  if (!reuse) free_state(c);
  for (int i = 0; i < narr && !reuse; ++i) {
    void* p = nullptr;
    if (hipMalloc(&p, alloc) != hipSuccess) {
      free_state(c);
      return fail(c, HODE_ENOMEM, "device allocation failed");
    }
    if (i < 2) c->y[i] = p;
    else if (i < 4) c->ks[i - 2] = p;
    else c->k[i - 2] = p;  // k[2] .. k[6]
  }
  c->dtype = dtype;
  c->nelem = nelem;
  c->N = N;
  c->esize = es;
  if (bytes) {
    HIPCHK(c, hipMemcpyAsync(c->y[0], src, bytes, src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  c->parity = 0;
  c->k1slot = 0;
  c->k1_valid = false;
  c->persist_valid = false;
  c->ab_steps = 0;
  if (!reuse) {
    if (is_gs(c)) {
      const int ry = c->ry ? c->ry : (dtype == HODE_F32 ? 4 : 2);
      set_all_tiles(c, ry, default_zc(N, ry), c->nw);
      // the Fehlberg and Adams-Bashforth kinds hold up to 10 source rows per
      // register row: one row per wavefront keeps them out of scratch
      for (int k = hode::K_F1; k < hode::K_ALL; ++k) {
        c->kry[k] = 1;
        c->kzc[k] = default_zc(N, 1);
        c->knw[k] = 4;
      }
    } else {
      c->ew_grid = default_ew_grid(nelem, dtype);
    }
  }
  return HODE_OK;
}

size_t hode_state_bytes(const hode_ctx* c) { return c ? (size_t)c->nelem * c->esize : 0; }

// the device code's record width is the header's
static_assert(hode::TRACE_W == HODE_TRACE_W, "trace record width");

int hode_trace_width(void) { return HODE_TRACE_W; }

int hode_read_state(hode_ctx* c, void* dst, size_t dst_bytes, int dst_on_device) {
  int rc = check_ready(c);
  if (rc) return rc;
  const size_t bytes = (size_t)c->nelem * c->esize;
  if (dst_bytes < bytes) return fail(c, HODE_ESTATE, "destination too small");
  if (!bytes) return HODE_OK;
  if (!dst) return fail(c, HODE_EINVAL, "dst is NULL");
  HIPCHK(c, hipMemcpyAsync(dst, c->y[c->parity], bytes, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return HODE_OK;
}

int hode_set_tolerances(hode_ctx* c, double atol, double rtol) {
  if (!c) return HODE_EINVAL;
  if (!(atol >= 0) || !(rtol >= 0) || !std::isfinite(atol) || !std::isfinite(rtol) || (atol == 0 && rtol == 0))
    return fail(c, HODE_EINVAL, "tolerances must be finite, >= 0 and not both 0");
  c->atol = atol;
  c->rtol = rtol;
  return HODE_OK;
}

int hode_set_controller(hode_ctx* c, int kind, const void* weights, size_t nbytes) {
  if (!c) return HODE_EINVAL;
  if (kind == HODE_CTRL_PI || kind == HODE_CTRL_I) {
    c->ctrl_kind = kind;
    return HODE_OK;
  }
  if (kind != HODE_CTRL_MLP) return fail(c, HODE_EINVAL, "unknown controller");
  if (!weights || nbytes != 2 * (size_t)hode::MLP_NPARAM) return fail(c, HODE_EINVAL, "MLP weights must be 10626 bytes");
  if (!c->d_mlp) {
    if (hipMalloc(&c->d_mlp, nbytes) != hipSuccess) return fail(c, HODE_ENOMEM, "allocation failed");
  }
  HIPCHK(c, hipMemcpy(c->d_mlp, weights, nbytes, hipMemcpyHostToDevice));
  c->ctrl_kind = kind;
  return HODE_OK;
}

int hode_integrate_n_steps(hode_ctx* c, int method, double t0, double dt, int64_t n, double* t_end) {
  int rc = check_ready(c);
  if (rc) return rc;
  const bool ab = method >= HODE_AB1 && method <= HODE_AB8;
  const bool abm = method >= HODE_ABM1 && method <= HODE_ABM8;
  if (method != HODE_RK4 && method != HODE_DOPRI5 && method != HODE_CASHKARP54 && method != HODE_EULER &&
      method != HODE_FEHLBERG78 && method != HODE_MIDPOINT && !ab && !abm)
    return fail(c, HODE_EINVAL, "method");
  if (n < 0 || !std::isfinite(t0) || !std::isfinite(dt)) return fail(c, HODE_EINVAL, "bad step arguments");
  HIPCHK(c, hipSetDevice(c->device));
  if (ab || abm) {
    rc = ab_run(c, ab ? method - HODE_AB1 + 1 : method - HODE_ABM1 + 1, abm, t0, dt, n);
    if (rc) return rc;
    c->persist_valid = false;
    if (t_end) *t_end = t0 + (double)n * dt;
    return HODE_OK;
  }
  const int mode = method == HODE_RK4          ? hode::MODE_FIXED_RK4
                   : method == HODE_DOPRI5       ? hode::MODE_FIXED_DP5
                   : method == HODE_CASHKARP54   ? hode::MODE_FIXED_CK
                   : method == HODE_FEHLBERG78   ? hode::MODE_FIXED_F78
                   : method == HODE_MIDPOINT     ? hode::MODE_FIXED_MM
                                                 : hode::MODE_FIXED_EULER;
  DevCtrl d = base_ctrl(c, mode);
  d.t = d.t0 = t0;
  d.h = d.dt = dt;
  d.nsteps = n;
  d.done = n == 0;
  rc = run_loop(c, d, mode == hode::MODE_FIXED_DP5 && !c->k1_valid);
  if (rc) return rc;
  c->persist_valid = false;
  if (t_end) *t_end = t0 + (double)n * dt;
  return HODE_OK;
}

int hode_do_step(hode_ctx* c, int method, double t, double dt) {
  return hode_integrate_n_steps(c, method, t, dt, 1, nullptr);
}

int hode_integrate_adaptive(hode_ctx* c, double t0, double t1, double dt0, int64_t max_steps, hode_stats* out) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!std::isfinite(t0) || !std::isfinite(t1) || !(t1 >= t0) || !(dt0 > 0) || !std::isfinite(dt0) || max_steps < 0)
    return fail(c, HODE_EINVAL, "bad integration arguments");
  rc = check_adaptive(c);
  if (rc) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  DevCtrl d = base_ctrl(c, adaptive_mode(c));
  d.t = d.t0 = t0;
  d.t1 = t1;
  d.dt = dt0;
  d.max_attempts = max_steps;
  const bool last = dt0 >= t1 - t0;
  d.h = last ? t1 - t0 : dt0;
  d.last_flag = last;
  if (t0 >= t1) {
    d.done = 1;
  } else if (max_steps == 0) {
    d.done = 1;
    d.status = hode::ST_EMAXSTEPS;
  } else if (d.h < 1e-12 * std::fmax(1.0, std::fabs(t0))) {
    d.done = 1;
    d.status = hode::ST_EDT_UNDERFLOW;
  }
  rc = run_loop(c, d, c->stepper == HODE_DOPRI5 && !c->k1_valid);
  if (rc) return rc;
  c->persist_valid = false;
  if (out) *out = c->last;
  return c->last.status;
}

int hode_integrate_times(hode_ctx* c, const double* times, int64_t n_times, double dt0, int64_t max_steps,
                         void* dst, size_t dst_bytes, int dst_on_device, hode_stats* out) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!times || n_times < 1 || !(dt0 > 0) || !std::isfinite(dt0) || max_steps < 0)
    return fail(c, HODE_EINVAL, "bad integrate_times arguments");
  for (int64_t i = 0; i < n_times; ++i)
    if (!std::isfinite(times[i]) || (i > 0 && !(times[i] > times[i - 1])))
      return fail(c, HODE_EINVAL, "times must be finite and increasing");
  const size_t bytes = (size_t)c->nelem * c->esize;
  if (!dst || dst_bytes / (size_t)n_times < bytes) return fail(c, HODE_ESTATE, "destination too small");
  rc = check_adaptive(c);
  if (rc) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  // the observation at times[0]: the current state
  HIPCHK(c, hipMemcpyAsync(dst, c->y[c->parity], bytes, kind, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  hode_stats tot{};
  tot.t = times[0];
  tot.dt_next = dt0;
  double dt = dt0;
  int64_t left = max_steps;
  bool carry = false;
  DevCtrl prev{};
  for (int64_t i = 1; i < n_times; ++i) {
    // one segment times[i-1] -> times[i], landing on it; the proposed step,
    // the controller's memory and (Dopri5) k1 carry over from the last one
    DevCtrl d = base_ctrl(c, adaptive_mode(c));
    d.t = d.t0 = times[i - 1];
    d.t1 = times[i];
    d.dt = dt;
    d.max_attempts = left;
    const bool last = dt >= d.t1 - d.t0;
    d.h = last ? d.t1 - d.t0 : dt;
    d.last_flag = last;
    if (carry) {
      d.err_prev = prev.err_prev;
      d.last_rejected = prev.last_rejected;
      d.hist_n = prev.hist_n;
      for (int k = 0; k < hode::HIST; ++k) {
        d.hist_lerr[k] = prev.hist_lerr[k];
        d.hist_lh[k] = prev.hist_lh[k];
        d.hist_acc[k] = prev.hist_acc[k];
      }
    }
    if (left == 0) {
      d.done = 1;
      d.status = hode::ST_EMAXSTEPS;
    } else if (d.h < 1e-12 * std::fmax(1.0, std::fabs(d.t0))) {
      d.done = 1;
      d.status = hode::ST_EDT_UNDERFLOW;
    }
    rc = run_loop(c, d, c->stepper == HODE_DOPRI5 && !c->k1_valid);
    if (rc) return rc;
    const hode_stats& st = c->last;
    tot.accepted += st.accepted;
    tot.rejected += st.rejected;
    tot.rhs_evals += st.rhs_evals;
    tot.t = st.t;
    tot.dt_next = st.dt_next;
    tot.last_err = st.last_err;
    tot.status = st.status;
    left -= c->last_attempts;
    dt = st.dt_next;
    prev = c->persist;
    carry = true;
    if (st.status != HODE_OK) break;
    HIPCHK(c, hipMemcpyAsync((char*)dst + (size_t)i * bytes, c->y[c->parity], bytes, kind, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  c->persist_valid = false;
  c->last = tot;
  if (out) *out = tot;
  return tot.status;
}

int hode_integrate_times_dense(hode_ctx* c, const double* times, int64_t n_times, double dt0, int64_t max_steps,
                               void* dst, size_t dst_bytes, int dst_on_device, hode_stats* out) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!times || n_times < 1 || !(dt0 > 0) || !std::isfinite(dt0) || max_steps < 0)
    return fail(c, HODE_EINVAL, "bad integrate_times_dense arguments");
  for (int64_t i = 0; i < n_times; ++i)
    if (!std::isfinite(times[i]) || (i > 0 && !(times[i] > times[i - 1])))
      return fail(c, HODE_EINVAL, "times must be finite and increasing");
  if (c->stepper != HODE_DOPRI5) return fail(c, HODE_EINVAL, "dense output is Dopri5's continuous extension");
  const size_t bytes = (size_t)c->nelem * c->esize;
  if (!dst || dst_bytes / (size_t)n_times < bytes) return fail(c, HODE_ESTATE, "destination too small");
  rc = check_adaptive(c);
  if (rc) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (!dst_on_device && !c->d_obs && hipMalloc(&c->d_obs, std::max<size_t>(bytes, 256)) != hipSuccess) {
    c->d_obs = nullptr;
    return fail(c, HODE_ENOMEM, "device allocation failed (observation staging)");
  }
  rc = ensure_xk(c, false, 0, true);
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(dst, c->y[c->parity], bytes, kind, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double t0 = times[0], t1 = times[n_times - 1];
  DevCtrl d = base_ctrl(c, hode::MODE_ADAPTIVE_DENSE);
  d.t = d.t0 = t0;
  d.t1 = t1;
  d.dt = dt0;
  d.max_attempts = max_steps;
  const bool last = dt0 >= t1 - t0;
  d.h = last ? t1 - t0 : dt0;
  d.last_flag = last;
  if (t0 >= t1) {
    d.done = 1;
  } else if (max_steps == 0) {
    d.done = 1;
    d.status = hode::ST_EMAXSTEPS;
  } else if (d.h < 1e-12 * std::fmax(1.0, std::fabs(t0))) {
    d.done = 1;
    d.status = hode::ST_EDT_UNDERFLOW;
  }
  int64_t next = 1;  // next intermediate observation
  const bool need_k1 = !c->k1_valid && !d.done;
  bool first = true;
  for (;;) {
    d.stop_at = next < n_times - 1 ? times[next] : HUGE_VAL;
    rc = run_loop(c, d, first && need_k1);
    if (rc) return rc;
    first = false;
    const DevCtrl cur = c->persist;
    // every requested time the last accepted step reached lies inside it
    // (the run pauses at the first step that reaches one)
    const double tp = cur.t - cur.h_acc;
    for (; next < n_times - 1 && cur.accepted > 0 && times[next] <= cur.t; ++next) {
      const double th = (times[next] - tp) / cur.h_acc;
      void* o = dst_on_device ? (void*)((char*)dst + (size_t)next * bytes) : c->d_obs;
      const void* yn = c->y[cur.parity ^ 1];
      if (is_gs(c)) {
        HIPCHK(c, hode::launch_dense_k(c->dtype, o, yn, c->ks[cur.k1slot ^ 1], c->k[3], c->k[4], c->k[5],
                                       c->xk_arr[hode::kXkK6], c->ks[cur.k1slot], c->nelem,
                                       default_ew_grid(c->nelem, c->dtype), cur.h_acc, th, c->stream));
      } else {
        HIPCHK(c, hode::launch_dense_ew(c->dtype, c->rhs, o, yn, c->nelem, c->ew_grid, cur.h_acc, th, c->stream));
      }
      if (!dst_on_device)
        HIPCHK(c, hipMemcpyAsync((char*)dst + (size_t)next * bytes, c->d_obs, bytes, kind, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    if (cur.status != hode::ST_OK || cur.t >= t1 || !cur.done) break;
    d = cur;  // paused at an observation: resume where it stopped
    d.done = 0;
  }
  // the counters ran on across the pauses; the first k1 comes on top
  c->last.rhs_evals = c->persist.rhs_evals + (need_k1 ? 1 : 0);
  if (c->last.status == HODE_OK && n_times > 1) {
    HIPCHK(c, hipMemcpyAsync((char*)dst + (size_t)(n_times - 1) * bytes, c->y[c->parity], bytes, kind, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  c->persist_valid = false;
  if (out) *out = c->last;
  return c->last.status;
}

int hode_try_step(hode_ctx* c, double* t, double* dt, int* accepted) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!t || !dt || !accepted || !std::isfinite(*t) || !(*dt > 0) || !std::isfinite(*dt))
    return fail(c, HODE_EINVAL, "bad try_step arguments");
  rc = check_adaptive(c);
  if (rc) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  DevCtrl d = base_ctrl(c, adaptive_mode(c));
  if (c->persist_valid) {
    d.err_prev = c->persist.err_prev;
    d.last_rejected = c->persist.last_rejected;
    d.hist_n = c->persist.hist_n;
    for (int i = 0; i < hode::HIST; ++i) {
      d.hist_lerr[i] = c->persist.hist_lerr[i];
      d.hist_lh[i] = c->persist.hist_lh[i];
      d.hist_acc[i] = c->persist.hist_acc[i];
    }
  }
  d.t = d.t0 = *t;
  d.t1 = *t + *dt;
  d.h = *dt;
  d.dt = *dt;
  d.last_flag = 1;
  d.max_attempts = 1;
  rc = run_loop(c, d, c->stepper == HODE_DOPRI5 && !c->k1_valid);
  if (rc) return rc;
  c->persist_valid = true;
  *accepted = c->last.accepted > 0;
  if (*accepted) *t = d.t1;
  *dt = c->last.dt_next;
  return HODE_OK;
}

int hode_get_stats(hode_ctx* c, hode_stats* out) {
  if (!c || !out) return HODE_EINVAL;
  *out = c->last;
  return HODE_OK;
}

int hode_debug_poison(hode_ctx* c) {
  int rc = check_ready(c);
  if (rc) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  const size_t bytes = (size_t)c->nelem * c->esize;
  if (!bytes) return HODE_OK;
  // all-ones bytes are a NaN in FP32 and FP64
  auto poison = [&](void* p) -> hipError_t { return p ? hipMemsetAsync(p, 0xFF, bytes, c->stream) : hipSuccess; };
  HIPCHK(c, poison(c->y[c->parity ^ 1]));
  HIPCHK(c, poison(c->ks[c->k1slot ^ 1]));
  if (!c->k1_valid) HIPCHK(c, poison(c->ks[c->k1slot]));
  for (int i = 2; i < 7; ++i) HIPCHK(c, poison(c->k[i]));
  for (int i = 0; i < hode::kXkCount; ++i)
    if (i < hode::kRingBase || c->ab_steps == 0) HIPCHK(c, poison(c->xk_arr[i]));
  HIPCHK(c, poison(c->d_obs));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return HODE_OK;
}

int hode_get_ctrl(hode_ctx* c, void* blob, size_t* nbytes) {
  if (!c || !nbytes) return HODE_EINVAL;
  if (!blob) {
    *nbytes = sizeof(hode_checkpoint);
    return HODE_OK;
  }
  if (*nbytes < sizeof(hode_checkpoint)) return fail(c, HODE_ESTATE, "checkpoint buffer too small");
  if (c->persist.mode == 0) return fail(c, HODE_ESTATE, "no stepping call to checkpoint");
  const DevCtrl& d = c->persist;
  hode_checkpoint k;
  std::memset(&k, 0, sizeof(k));
  k.magic = HODE_CKPT_MAGIC;
  k.version = 1;
  k.t = d.t;
  k.dt_next = c->last.dt_next;
  k.err_prev = d.err_prev;
  k.last_rejected = d.last_rejected;
  k.hist_n = (int32_t)d.hist_n;
  for (int i = 0; i < hode::HIST; ++i) {
    k.hist_lerr[i] = d.hist_lerr[i];
    k.hist_lh[i] = d.hist_lh[i];
    k.hist_acc[i] = d.hist_acc[i];
  }
  k.accepted = c->last.accepted;
  k.rejected = c->last.rejected;
  k.rhs_evals = c->last.rhs_evals;
  std::memcpy(blob, &k, sizeof(k));
  *nbytes = sizeof(k);
  return HODE_OK;
}

int hode_set_ctrl(hode_ctx* c, const void* blob, size_t nbytes) {
  if (!c) return HODE_EINVAL;
  if (!blob || nbytes != sizeof(hode_checkpoint)) return fail(c, HODE_EINVAL, "checkpoint size");
  hode_checkpoint k;
  std::memcpy(&k, blob, sizeof(k));
  if (k.magic != HODE_CKPT_MAGIC || k.version != 1) return fail(c, HODE_EINVAL, "not a version-1 checkpoint");
  if (k.hist_n < 0 || k.hist_n > hode::HIST || !(k.err_prev > 0) || !std::isfinite(k.err_prev))
    return fail(c, HODE_EINVAL, "checkpoint out of range");
  DevCtrl& d = c->persist;
  d.err_prev = k.err_prev;
  d.last_rejected = k.last_rejected ? 1 : 0;
  d.hist_n = (uint32_t)k.hist_n;
  for (int i = 0; i < hode::HIST; ++i) {
    d.hist_lerr[i] = k.hist_lerr[i];
    d.hist_lh[i] = k.hist_lh[i];
    d.hist_acc[i] = k.hist_acc[i];
  }
  c->persist_valid = true;
  return HODE_OK;
}

int hode_set_trace(hode_ctx* c, int64_t capacity) {
  if (!c || capacity < 0) return HODE_EINVAL;
  if (c->d_trace) { (void)hipFree(c->d_trace); c->d_trace = nullptr; }
  c->trace_cap = 0;
  if (capacity > 0) {
    if (hipMalloc(&c->d_trace, sizeof(double) * hode::TRACE_W * (size_t)capacity) != hipSuccess)
      return fail(c, HODE_ENOMEM, "trace allocation failed");
    c->trace_cap = capacity;
  }
  return HODE_OK;
}

int hode_read_trace(hode_ctx* c, double* dst, int64_t cap, int64_t* n) {
  if (!c || cap < 0) return HODE_EINVAL;
  const int64_t avail = c->last_attempts < c->trace_cap ? c->last_attempts : c->trace_cap;
  const int64_t m = avail < cap ? avail : cap;
  if (n) *n = c->last_attempts;
  if (m > 0) {
    if (!dst) return fail(c, HODE_EINVAL, "dst is NULL");
    HIPCHK(c, hipMemcpy(dst, c->d_trace, sizeof(double) * hode::TRACE_W * (size_t)m, hipMemcpyDeviceToHost));
  }
  return HODE_OK;
}

int hode_eval_rhs(hode_ctx* c, void* dst, size_t dst_bytes, int dst_on_device) {
  int rc = check_ready(c);
  if (rc) return rc;
  const size_t bytes = (size_t)c->nelem * c->esize;
  if (dst_bytes < bytes) return fail(c, HODE_ESTATE, "destination too small");
  if (!bytes) return HODE_OK;
  HIPCHK(c, hipSetDevice(c->device));
  DevCtrl d = base_ctrl(c, 0);
  *c->h_ctrl = d;
  HIPCHK(c, hipMemcpyAsync(c->d_ctrl, c->h_ctrl, sizeof(DevCtrl), hipMemcpyHostToDevice, c->stream));
  void* src;
  if (is_gs(c)) {
    rc = launch_k1(c);
    if (rc) return rc;
    c->k1_valid = true;
    src = c->ks[c->k1slot];
  } else {
    HIPCHK(c, hode::launch_ew_rhs(c->dtype, c->rhs, c->y[c->parity], c->y[c->parity ^ 1], c->nelem, c->ew_grid,
                                  c->stream));
    src = c->y[c->parity ^ 1];
  }
  HIPCHK(c, hipMemcpyAsync(dst, src, bytes, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return HODE_OK;
}

int hode_set_tile(hode_ctx* c, int ry, int zc) {
  if (!c) return HODE_EINVAL;
  if (c->dtype && !is_gs(c)) {
    if (zc < 1) return fail(c, HODE_EINVAL, "workgroup cap must be >= 1");
    c->ew_grid = zc;
  } else {
    if (!hode::gs_ry_supported(ry) || zc < 1) return fail(c, HODE_EINVAL, "ry must be 1, 2 or 4 and zc >= 1");
    set_all_tiles(c, ry, zc, c->nw);
  }
  clear_graphs(c);
  return HODE_OK;
}

int hode_set_tile_waves(hode_ctx* c, int nw) {
  if (!c) return HODE_EINVAL;
  if (nw != 4 && nw != 8) return fail(c, HODE_EINVAL, "wavefronts per workgroup must be 4 or 8");
  c->nw = nw;
  if (c->dtype && is_gs(c)) {
    for (int k = 0; k < hode::K_ALL; ++k)
      c->knw[k] = hode::gs_tile_supported(k, c->dtype, c->kry[k], c->vw, nw, c->N) ? nw : 4;
    clear_graphs(c);
  }
  return HODE_OK;
}

int hode_set_vector_width(hode_ctx* c, int vw) {
  if (!c) return HODE_EINVAL;
  if (vw != 0 && vw != 1 && vw != 2 && vw != 4) return fail(c, HODE_EINVAL, "vector width 0, 1, 2 or 4");
  if (vw && c->dtype == HODE_F64 && vw > 2) return fail(c, HODE_EINVAL, "fp64 vector width at most 2");
  if (vw && c->N && c->N % vw) return fail(c, HODE_EINVAL, "vector width must divide N");
  c->vw = vw;
  // eight-wavefront tiles exist for 16-byte lanes only
  if (c->dtype && is_gs(c))
    for (int k = 0; k < hode::K_ALL; ++k)
      if (c->knw[k] == 8 && !hode::gs_tile_supported(k, c->dtype, c->kry[k], vw, 8, c->N)) c->knw[k] = 4;
  clear_graphs(c);
  return HODE_OK;
}

int hode_get_tile(const hode_ctx* c, int* ry, int* zc) {
  if (!c || !ry || !zc) return HODE_EINVAL;
  *ry = c->ry;
  *zc = is_gs(c) ? c->zc : c->ew_grid;
  return HODE_OK;
}

int hode_get_kind_tile(const hode_ctx* c, int kind, int* ry, int* zc, int* nw) {
  if (!c || !ry || !zc || !nw || kind < 0 || kind >= hode::K_ALL) return HODE_EINVAL;
  if (!c->dtype || !is_gs(c)) return HODE_ESTATE;
  *ry = c->kry[kind];
  *zc = c->kzc[kind];
  *nw = c->knw[kind] ? c->knw[kind] : 4;
  return HODE_OK;
}

int hode_time_kernel(hode_ctx* c, int kind, int reps, double* avg_ms) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (reps < 1 || !avg_ms) return fail(c, HODE_EINVAL, "reps >= 1 and avg_ms required");
  if (is_gs(c) && (kind < 0 || kind >= hode::K_ALL)) return fail(c, HODE_EINVAL, "kernel kind");
  if (!is_gs(c) && kind != HODE_RK4 && kind != HODE_DOPRI5) return fail(c, HODE_EINVAL, "kernel kind");
  HIPCHK(c, hipSetDevice(c->device));
  if (is_gs(c) && kind >= hode::K_F1) {
    // the Adams-Bashforth kinds write ring slot 0 (the correctors the state):
    // the history ends
    const int ring = kind >= hode::K_AB1 && kind <= hode::K_AB8     ? kind - hode::K_AB1 + 1
                     : kind >= hode::K_ABC1 && kind <= hode::K_ABC8 ? kind - hode::K_ABC1 + 1
                                                                    : 0;
    rc = ensure_xk(c, kind <= hode::K_F13F, ring, kind == hode::K_D6K, kind >= hode::K_MM1);
    if (rc) return rc;
    if (ring) c->ab_steps = 0;
  }
  // a control block in timing mode: kernels run with the last step size but
  // the epilogue changes nothing, so the current state and k1 stay intact
  DevCtrl d = base_ctrl(c, 0);
  d.h = c->last.dt_next > 0 ? c->last.dt_next : 0.01;
  *c->h_ctrl = d;
  HIPCHK(c, hipMemcpyAsync(c->d_ctrl, c->h_ctrl, sizeof(DevCtrl), hipMemcpyHostToDevice, c->stream));
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  const hode::GSLaunch a = is_gs(c) ? gs_args(c) : hode::GSLaunch{};
  auto launch = [&]() -> hipError_t {
    if (is_gs(c)) return launch_stage(c, kind, a);
    const int mode = kind == HODE_RK4 ? hode::MODE_FIXED_RK4 : hode::MODE_ADAPTIVE;
    return hode::launch_ew(c->dtype, c->rhs, mode, c->y[0], c->y[1], c->nelem, c->ew_grid, c->d_ctrl, c->stream);
  };
  hipError_t e = launch();  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
  for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(c, HODE_EHIP, std::string("timing: ") + hipGetErrorString(e));
  *avg_ms = (double)ms / reps;
  if (is_gs(c) && kind == hode::K_D1) c->k1_valid = true;
  return HODE_OK;
}

// Stage sequence of one attempt of `method` (adaptive for the embedded pairs;
// Adams-Bashforth: its one kernel).  seq holds up to 13 kinds.
static int stage_seq(int method, int* seq) {
  if (method >= HODE_AB1 && method <= HODE_AB8) {
    seq[0] = hode::K_AB1 + method - HODE_AB1;
    return 1;
  }
  if (method == HODE_FEHLBERG78) {
    for (int i = 0; i < 13; ++i) seq[i] = hode::K_F1 + i;
    return 13;
  }
  if (method == HODE_RK4) {
    const int s[] = {hode::K_D1, hode::K_R2, hode::K_R3, hode::K_R4};
    for (int i = 0; i < 4; ++i) seq[i] = s[i];
    return 4;
  }
  if (method == HODE_CASHKARP54) {
    const int s[] = {hode::K_D1, hode::K_D2, hode::K_D3, hode::K_C4, hode::K_C5, hode::K_C6};
    for (int i = 0; i < 6; ++i) seq[i] = s[i];
    return 6;
  }
  const int s[] = {hode::K_D2, hode::K_D3, hode::K_D4, hode::K_D5, hode::K_D6, hode::K_D7};
  for (int i = 0; i < 6; ++i) seq[i] = s[i];
  return 6;
}

int hode_profile_attempt(hode_ctx* c, int method, int reps, double* ms) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!is_gs(c)) return fail(c, HODE_EINVAL, "stage profiling is for the Gray-Scott path");
  const bool ab = method >= HODE_AB1 && method <= HODE_AB8;
  if (reps < 1 || !ms ||
      (method != HODE_RK4 && method != HODE_DOPRI5 && method != HODE_CASHKARP54 && method != HODE_FEHLBERG78 && !ab))
    return fail(c, HODE_EINVAL, "arguments");
  HIPCHK(c, hipSetDevice(c->device));
  if (method == HODE_FEHLBERG78 || ab) {
    rc = ensure_xk(c, !ab, ab ? method - HODE_AB1 + 1 : 0);
    if (rc) return rc;
    if (ab) c->ab_steps = 0;  // the timed steps overwrite ring slot 0
  }
  int seq[16];
  const int ns = stage_seq(method, seq);
  DevCtrl d = base_ctrl(c, 0);
  d.h = c->last.dt_next > 0 ? c->last.dt_next : 0.01;
  *c->h_ctrl = d;
  HIPCHK(c, hipMemcpyAsync(c->d_ctrl, c->h_ctrl, sizeof(DevCtrl), hipMemcpyHostToDevice, c->stream));
  const hode::GSLaunch a = gs_args(c);
  if (method == HODE_DOPRI5 && !c->k1_valid) {
    HIPCHK(c, launch_stage(c, hode::K_D1, a));
    c->k1_valid = true;
  }
  hipEvent_t ev[17];
  for (int i = 0; i <= ns; ++i) HIPCHK(c, hipEventCreate(&ev[i]));
  double acc[16] = {0};
  hipError_t e = hipSuccess;
  for (int r = 0; r <= reps && e == hipSuccess; ++r) {  // first round is warm-up
    for (int i = 0; i < ns && e == hipSuccess; ++i) {
      e = hipEventRecord(ev[i], c->stream);
      if (e == hipSuccess) e = launch_stage(c, seq[i], a);
    }
    if (e == hipSuccess) e = hipEventRecord(ev[ns], c->stream);
    if (e == hipSuccess) e = hode::launch_ctrl(c->d_ctrl, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev[ns]);
    for (int i = 0; i < ns && e == hipSuccess && r > 0; ++i) {
      float t = 0;
      e = hipEventElapsedTime(&t, ev[i], ev[i + 1]);
      acc[i] += t;
    }
  }
  for (int i = 0; i <= ns; ++i) (void)hipEventDestroy(ev[i]);
  HIPCHK(c, e);
  for (int i = 0; i < ns; ++i) ms[i] = acc[i] / reps;
  return HODE_OK;
}

int hode_autotune(hode_ctx* c, int method, int reps, int* best_ry, int* best_zc, double* best_ms) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!is_gs(c)) return fail(c, HODE_EINVAL, "autotuning is for the Gray-Scott path");
  if (method != HODE_RK4 && method != HODE_DOPRI5 && method != HODE_CASHKARP54 && method != HODE_FEHLBERG78 &&
      !(method >= HODE_AB1 && method <= HODE_AB8))
    return fail(c, HODE_EINVAL, "method");
  const int rys[] = {1, 2, 4};
  // plane chunks: powers of two, and the even splits of the grid into 1 .. 12
  // chunks (block counts that fill whole rounds of resident workgroups)
  std::vector<int> zcs;
  for (int zc = 8; zc <= 256; zc *= 2) zcs.push_back(zc);
  for (int nz = 1; nz <= 12; ++nz) zcs.push_back((c->N + nz - 1) / nz);
  std::sort(zcs.begin(), zcs.end());
  zcs.erase(std::unique(zcs.begin(), zcs.end()), zcs.end());
  // Adams-Bashforth starts a fresh history with Fehlberg 7(8) steps: its
  // stage kinds get their own tuned tiles first
  if (method >= HODE_AB1 && method <= HODE_AB8) {
    rc = hode_autotune(c, HODE_FEHLBERG78, reps, nullptr, nullptr, nullptr);
    if (rc) return rc;
  }
  int seq[16];
  const int ns = stage_seq(method, seq);
  // the tiles of the kinds this search does not time stay as they were (the
  // search sets every kind's tile while it times)
  int keep_ry[hode::K_ALL], keep_zc[hode::K_ALL], keep_nw[hode::K_ALL];
  for (int k = 0; k < hode::K_ALL; ++k) { keep_ry[k] = c->kry[k]; keep_zc[k] = c->kzc[k]; keep_nw[k] = c->knw[k]; }
  // every stage kind keeps its own fastest tile: rows per wavefront,
  // planes, and four or (16-byte lanes, one or two rows) eight wavefronts
  double best[16];
  int bry[16], bzc[16], bnw[16];
  for (int i = 0; i < ns; ++i) {
    best[i] = 1e300;
    bry[i] = c->kry[seq[i]];
    bzc[i] = c->kzc[seq[i]];
    bnw[i] = c->knw[seq[i]] ? c->knw[seq[i]] : 4;
  }
  for (int nw : {4, 8}) {
    for (int ry : rys) {
      bool any = false;
      for (int i = 0; i < ns; ++i) any = any || hode::gs_tile_supported(seq[i], c->dtype, ry, c->vw, nw, c->N);
      if (!any) continue;
      for (int zc : zcs) {
        if ((zc > c->N || zc < 8) && zc != 8) continue;
        set_all_tiles(c, ry, zc, nw);
        double ms[16];
        rc = hode_profile_attempt(c, method, reps, ms);
        if (rc) return rc;
        for (int i = 0; i < ns; ++i)
          if (ms[i] < best[i] && c->knw[seq[i]] == nw) { best[i] = ms[i]; bry[i] = ry; bzc[i] = zc; bnw[i] = nw; }
      }
    }
  }
  for (int k = 0; k < hode::K_ALL; ++k) { c->kry[k] = keep_ry[k]; c->kzc[k] = keep_zc[k]; c->knw[k] = keep_nw[k]; }
  double tot = 0;
  for (int i = 0; i < ns; ++i) {
    c->kry[seq[i]] = bry[i];
    c->kzc[seq[i]] = bzc[i];
    c->knw[seq[i]] = bnw[i];
    tot += best[i];
  }
  auto twin = [&](int dst, int src) {
    c->kry[dst] = c->kry[src];
    c->kzc[dst] = c->kzc[src];
    c->knw[dst] = c->knw[src];
  };
  if (method == HODE_DOPRI5) {
    // kinds of the same shape outside the timed attempt: the first k1, and
    // the fixed-step variants of stages 6 and 7
    twin(hode::K_D1, hode::K_D2);
    twin(hode::K_D6F, hode::K_D6);
    twin(hode::K_D7F, hode::K_D7);
  }
  if (method == HODE_CASHKARP54) twin(hode::K_C6F, hode::K_C6);
  if (method == HODE_FEHLBERG78) twin(hode::K_F13F, hode::K_F13);
  const int widest = method == HODE_RK4           ? hode::K_R4
                     : method == HODE_CASHKARP54  ? hode::K_C6
                     : method == HODE_FEHLBERG78  ? hode::K_F13
                     : method >= HODE_AB1         ? seq[0]
                                                  : hode::K_D6;
  c->ry = c->kry[widest];
  c->zc = c->kzc[widest];
  clear_graphs(c);
  if (best_ry) *best_ry = c->ry;
  if (best_zc) *best_zc = c->zc;
  if (best_ms) *best_ms = tot;
  return HODE_OK;
}

// Cache line: "hode-tune-v2 <arch> <dtype> <method> <N> <vw> <ry:zc:nw for every stage kind>".
static std::string tune_key(const hode_ctx* c, int method) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
    arch = prop.gcnArchName;
    for (char& ch : arch)
      if (ch == ' ') ch = '_';
  }
  char buf[256];
  std::snprintf(buf, sizeof(buf), "hode-tune-v2 %s %d %d %d %d", arch.c_str(), c->dtype, method, c->N, c->vw);
  return buf;
}

int hode_autotune_cached(hode_ctx* c, int method, int reps, const char* cache_path, int* from_cache) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!is_gs(c)) return fail(c, HODE_EINVAL, "autotuning is for the Gray-Scott path");
  if (from_cache) *from_cache = 0;
  const char* path = cache_path ? cache_path : std::getenv("HODE_TUNE_CACHE");
  const std::string key = tune_key(c, method);
  if (path && *path) {
    if (FILE* f = std::fopen(path, "r")) {
      // the last entry for this key wins
      std::vector<int> ry, zc, nw;
      char line[8192];
      while (std::fgets(line, sizeof(line), f)) {
        if (std::strncmp(line, key.c_str(), key.size()) != 0 || line[key.size()] != ' ') continue;
        std::vector<int> r, z, w;
        const char* q = line + key.size();
        int a, b, d, used;
        while (std::sscanf(q, " %d:%d:%d%n", &a, &b, &d, &used) == 3) {
          r.push_back(a);
          z.push_back(b);
          w.push_back(d);
          q += used;
        }
        if ((int)r.size() == hode::K_ALL) { ry = r; zc = z; nw = w; }
      }
      std::fclose(f);
      bool ok = !ry.empty();
      for (int k = 0; ok && k < hode::K_ALL; ++k)
        ok = hode::gs_tile_supported(k, c->dtype, ry[k], c->vw, nw[k], c->N) && zc[k] >= 1;
      if (ok) {
        for (int k = 0; k < hode::K_ALL; ++k) {
          c->kry[k] = ry[k];
          c->kzc[k] = zc[k];
          c->knw[k] = nw[k];
        }
        int seq[16];
        const int widest = stage_seq(method, seq) == 1 ? seq[0] : (method == HODE_RK4 ? hode::K_R4
                                                                    : method == HODE_CASHKARP54 ? hode::K_C6
                                                                    : method == HODE_FEHLBERG78 ? hode::K_F13
                                                                                                : hode::K_D6);
        c->ry = c->kry[widest];
        c->zc = c->kzc[widest];
        clear_graphs(c);
        if (from_cache) *from_cache = 1;
        return HODE_OK;
      }
    }
  }
  rc = hode_autotune(c, method, reps, nullptr, nullptr, nullptr);
  if (rc) return rc;
  if (path && *path) {
    FILE* f = std::fopen(path, "a");
    if (!f) return fail(c, HODE_EINVAL, std::string("cannot append to the tuning cache ") + path);
    std::string line = key;
    char buf[32];
    for (int k = 0; k < hode::K_ALL; ++k) {
      std::snprintf(buf, sizeof(buf), " %d:%d:%d", c->kry[k], c->kzc[k], c->knw[k] ? c->knw[k] : 4);
      line += buf;
    }
    line += "\n";
    const bool w = std::fputs(line.c_str(), f) >= 0;
    const bool cl = std::fclose(f) == 0;
    if (!w || !cl) return fail(c, HODE_EINVAL, std::string("cannot write the tuning cache ") + path);
  }
  return HODE_OK;
}

int hode_set_stepper(hode_ctx* c, int method) {
  if (!c) return HODE_EINVAL;
  if (method != HODE_DOPRI5 && method != HODE_CASHKARP54 && method != HODE_FEHLBERG78)
    return fail(c, HODE_EINVAL, "adaptive stepper: Dopri5, Cash-Karp or Fehlberg 7(8)");
  if (c->ens) return fail(c, HODE_EINVAL, "the ensemble steps with Dopri5");
  c->stepper = method;
  c->persist_valid = false;
  return HODE_OK;
}

int hode_set_graphs(hode_ctx* c, int enable) {
  if (!c) return HODE_EINVAL;
  c->use_graphs = enable != 0;
  return HODE_OK;
}

int hode_ensemble_create(hode_ctx** out, int device, void* stream, int n, const int64_t* edges,
                         const double* params, int dtype) {
  if (!out || n < 1 || !edges || !params || (dtype != HODE_F32 && dtype != HODE_F64)) return HODE_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (edges[i] < 1 || edges[i] > 1024) return HODE_EINVAL;
    for (int j = 0; j < 5; ++j)
      if (!std::isfinite(params[5 * i + j])) return HODE_EINVAL;
    if (!(params[5 * i + 4] > 0)) return HODE_EINVAL;
  }
  int rc = hode_create(out, device, stream);
  if (rc) return rc;
  hode_ctx* c = *out;
  Ensemble* e = new (std::nothrow) Ensemble();
  if (!e) { hode_destroy(c); *out = nullptr; return HODE_ENOMEM; }
  c->ens = e;
  c->rhs = HODE_RHS_GRAYSCOTT3D;
  c->dtype = dtype;
  c->esize = dtype == HODE_F32 ? 4 : 8;
  e->n = n;
  e->dtype = dtype;
  e->N.assign(edges, edges + n);
  e->prm.assign(params, params + 5 * n);
  e->parity.assign(n, 0);
  e->vw.assign(n, 0);
  e->zc.assign(n, 0);
  e->attempts_last.assign(n, 0);
  e->weight.resize(n);
  e->inst.resize(n);
  // default per-attempt work estimates: the cells the instance's tiles cover
  // (rows padded to the 64-lane tile width)
  for (int i = 0; i < n; ++i) {
    const double Nd = (double)e->N[i];
    e->weight[i] = std::ceil(Nd / 64.0) * 64.0 * Nd * Nd;
  }
  // one pool: 9 arrays of 2 N^3 elements per instance, 256-byte aligned
  std::vector<size_t> off(n);
  size_t tot = 0;
  for (int i = 0; i < n; ++i) {
    off[i] = tot;
    const size_t ab = ((size_t)2 * e->N[i] * e->N[i] * e->N[i] * c->esize + 255) / 256 * 256;
    tot += 9 * ab;
  }
  if (hipMalloc(&e->pool, tot) != hipSuccess) { hode_destroy(c); *out = nullptr; return HODE_ENOMEM; }
  for (int i = 0; i < n; ++i) {
    const int Ni = e->N[i];
    const size_t ab = ((size_t)2 * Ni * Ni * Ni * c->esize + 255) / 256 * 256;
    char* b = (char*)e->pool + off[i];
    hode::EnsInst& I = e->inst[i];
    std::memset(&I, 0, sizeof(I));
    I.a.y[0] = b;
    I.a.y[1] = b + ab;
    I.a.ks[0] = b + 2 * ab;
    I.a.ks[1] = b + 3 * ab;
    for (int k = 2; k <= 6; ++k) I.a.k[k] = b + (2 + k) * ab;
    I.a.N = Ni;
    I.a.n3 = (int64_t)Ni * Ni * Ni;
    I.a.zc = Ni;
    const double hh = params[5 * i + 4] / Ni;
    I.a.Du_h2 = params[5 * i + 0] / (hh * hh);
    I.a.Dv_h2 = params[5 * i + 1] / (hh * hh);
    I.a.F = params[5 * i + 2];
    I.a.kk = params[5 * i + 3];
    const int maxvw = dtype == HODE_F32 ? 4 : 2;
    int v = 1;
    while (v * 2 <= maxvw && Ni % (v * 2) == 0 && 64 * v < Ni) v *= 2;  // narrowest that still fills a row
    if (ens_seg_for(dtype, Ni, maxvw) > 1) v = maxvw;                   // short rows: segmented 16-byte lanes
    e->vw[i] = v;
  }
  if (hipMalloc(&e->d_inst, sizeof(hode::EnsInst) * n) != hipSuccess) {
    hode_destroy(c);
    *out = nullptr;
    return HODE_ENOMEM;
  }
  // the persistent grid: every workgroup resident at once (grid barriers)
  const int bpc = hode::ensemble_blocks_per_cu(dtype);
  int cus = 0;
  if (bpc < 1 || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) {
    hode_destroy(c);
    *out = nullptr;
    return HODE_EHIP;
  }
  e->nwg = bpc * cus;
  if (hipEventCreate(&e->ev[0]) != hipSuccess || hipEventCreate(&e->ev[1]) != hipSuccess) {
    hode_destroy(c);
    *out = nullptr;
    return HODE_EHIP;
  }
  return HODE_OK;
}

static int ens_check(hode_ctx* c, int i) {
  if (!c) return HODE_EINVAL;
  if (!c->ens) return fail(c, HODE_ESTATE, "not an ensemble context");
  if (i < 0 || i >= c->ens->n) return fail(c, HODE_EINVAL, "instance index out of range");
  return HODE_OK;
}

int hode_ensemble_size(const hode_ctx* c) { return c && c->ens ? c->ens->n : 0; }

int hode_ensemble_init_state(hode_ctx* c, int i, const void* src, int src_on_device) {
  int rc = ens_check(c, i);
  if (rc) return rc;
  Ensemble* e = c->ens;
  if (!src) return fail(c, HODE_EINVAL, "src is NULL");
  const size_t bytes = (size_t)2 * e->N[i] * e->N[i] * e->N[i] * c->esize;
  e->parity[i] = 0;
  HIPCHK(c, hipMemcpy(e->inst[i].a.y[0], src, bytes, src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
  return HODE_OK;
}

int hode_ensemble_read_state(hode_ctx* c, int i, void* dst, size_t dst_bytes, int dst_on_device) {
  int rc = ens_check(c, i);
  if (rc) return rc;
  Ensemble* e = c->ens;
  const size_t bytes = (size_t)2 * e->N[i] * e->N[i] * e->N[i] * c->esize;
  if (dst_bytes < bytes) return fail(c, HODE_ESTATE, "destination too small");
  if (!dst) return fail(c, HODE_EINVAL, "dst is NULL");
  HIPCHK(c, hipMemcpy(dst, e->inst[i].a.y[e->parity[i]], bytes,
                      dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
  return HODE_OK;
}

int hode_ensemble_set_weights(hode_ctx* c, const double* w) {
  int rc = ens_check(c, 0);
  if (rc) return rc;
  if (!w) return fail(c, HODE_EINVAL, "weights are NULL");
  for (int i = 0; i < c->ens->n; ++i)
    if (!(w[i] > 0) || !std::isfinite(w[i])) return fail(c, HODE_EINVAL, "weights must be positive");
  c->ens->weight.assign(w, w + c->ens->n);
  return HODE_OK;
}

int hode_ensemble_set_vector_width(hode_ctx* c, int i, int vw) {
  int rc = ens_check(c, i);
  if (rc) return rc;
  const int maxvw = c->dtype == HODE_F32 ? 4 : 2;
  if (vw != 1 && vw != 2 && vw != 4) return fail(c, HODE_EINVAL, "vector width 1, 2 or 4");
  if (vw > maxvw || c->ens->N[i] % vw) return fail(c, HODE_EINVAL, "vector width must divide N (fp64: at most 2)");
  c->ens->vw[i] = vw;
  return HODE_OK;
}

int hode_ensemble_set_plane_chunk(hode_ctx* c, int i, int zc) {
  int rc = ens_check(c, i);
  if (rc) return rc;
  if (zc < 0) return fail(c, HODE_EINVAL, "plane chunk must be >= 0");
  c->ens->zc[i] = zc;
  return HODE_OK;
}

int hode_ensemble_get_tile(const hode_ctx* c, int i, int* vw, int* zc) {
  if (!c || !c->ens || i < 0 || i >= c->ens->n || !vw || !zc) return HODE_EINVAL;
  *vw = c->ens->vw[i];
  *zc = c->ens->zc[i];
  return HODE_OK;
}

int hode_ensemble_set_trace(hode_ctx* c, int64_t capacity) {
  int rc = ens_check(c, 0);
  if (rc) return rc;
  if (capacity < 0) return fail(c, HODE_EINVAL, "capacity");
  Ensemble* e = c->ens;
  if (e->d_trace) { (void)hipFree(e->d_trace); e->d_trace = nullptr; }
  e->trace_cap = 0;
  if (capacity > 0) {
    if (hipMalloc(&e->d_trace, sizeof(double) * hode::TRACE_W * (size_t)capacity * e->n) != hipSuccess)
      return fail(c, HODE_ENOMEM, "trace allocation failed");
    e->trace_cap = capacity;
  }
  return HODE_OK;
}

int hode_ensemble_read_trace(hode_ctx* c, int i, double* dst, int64_t cap, int64_t* n) {
  int rc = ens_check(c, i);
  if (rc) return rc;
  Ensemble* e = c->ens;
  const int64_t att = e->attempts_last[i];
  const int64_t m = std::min(std::min(att, e->trace_cap), std::max<int64_t>(cap, 0));
  if (n) *n = att;
  if (m > 0) {
    if (!dst) return fail(c, HODE_EINVAL, "dst is NULL");
    HIPCHK(c, hipMemcpy(dst, e->d_trace + (size_t)hode::TRACE_W * e->trace_cap * i,
                        sizeof(double) * hode::TRACE_W * (size_t)m, hipMemcpyDeviceToHost));
  }
  return HODE_OK;
}

int hode_ensemble_set_epoch(hode_ctx* c, int first, int rest) {
  int rc = ens_check(c, 0);
  if (rc) return rc;
  const bool whole = first == 0 && rest == 0;
  if (!whole && (first < 1 || rest < 1 || first > 4096 || rest > 4096))
    return fail(c, HODE_EINVAL, "attempts per launch must be in 1 .. 4096 (or both 0)");
  c->ens->epoch_first = first;
  c->ens->epoch_len = rest;
  return HODE_OK;
}

int hode_ensemble_set_barrier_limit(hode_ctx* c, int64_t polls) {
  int rc = ens_check(c, 0);
  if (rc) return rc;
  if (polls < 1) return fail(c, HODE_EINVAL, "barrier poll limit must be >= 1");
  Ensemble* e = c->ens;
  if (polls != e->barrier_polls && e->graph) {
    // the limit is a kernel argument of the captured launch: capture again
    (void)hipGraphExecDestroy(e->graph);
    e->graph = nullptr;
  }
  e->barrier_polls = polls;
  return HODE_OK;
}

int hode_ensemble_timing(hode_ctx* c, double* kernel_ms, int* launches) {
  int rc = ens_check(c, 0);
  if (rc) return rc;
  if (kernel_ms) *kernel_ms = c->ens->kernel_ms_last;
  if (launches) *launches = c->ens->launches_last;
  return HODE_OK;
}

// Device block of the launch bookkeeping, sized for `rounds` rounds.
// The ensemble's bookkeeping block: queue offsets, launch parameters, then
// (cleared before every launch) the barrier's global counter, its eight
// per-XCD counters (one 128-byte line each), the error flag, the two
// running-instance counts and the two sets of claim counters.
struct SyncLayout {
  size_t qoff = 0, params = 64, bar = 128, xbar = 256, error = 256 + 8 * 128, live = error + 4, qctr = live + 8,
         bytes = qctr + 4 * 16;
};

int hode_ensemble_integrate_adaptive(hode_ctx* c, double t0, double t1, double dt0, int64_t max_steps,
                                     hode_stats* per_instance) {
  int rc = ens_check(c, 0);
  if (rc) return rc;
  if (!std::isfinite(t0) || !std::isfinite(t1) || !(t1 > t0) || !(dt0 > 0) || max_steps < 1)
    return fail(c, HODE_EINVAL, "bad integration arguments");
  Ensemble* e = c->ens;
  HIPCHK(c, hipSetDevice(c->device));
  // per-instance control blocks
  for (int i = 0; i < e->n; ++i) {
    hode::EnsInst& I = e->inst[i];
    DevCtrl d = base_ctrl(c, hode::MODE_ADAPTIVE);
    d.parity = e->parity[i];
    d.k1slot = 0;
    d.t = d.t0 = t0;
    d.t1 = t1;
    d.dt = dt0;
    const bool last = dt0 >= t1 - t0;
    d.h = last ? t1 - t0 : dt0;
    d.last_flag = last;
    d.max_attempts = max_steps;
    d.trace = e->trace_cap > 0 ? e->d_trace + (size_t)hode::TRACE_W * e->trace_cap * i : nullptr;
    d.trace_cap = e->trace_cap;
    d.stiff = gs_stiffness(&e->prm[5 * i], e->N[i]);
    I.ctrl = d;
    I.vw = e->vw[i];
    I.seg = ens_seg_for(e->dtype, e->N[i], e->vw[i]);
    I.k1_valid = 0;
  }
  // bookkeeping block and tile buffer (the captured graph holds their addresses)
  const SyncLayout L;
  static_assert(sizeof(hode::EnsParams) <= 64, "launch parameters fit their slot");
  if (!e->d_sync) {
    if (hipMalloc(&e->d_sync, L.bytes) != hipSuccess)
      return fail(c, HODE_ENOMEM, "ensemble bookkeeping allocation failed");
  }
  char* sb = (char*)e->d_sync;
  e->kernel_ms_last = 0;
  e->launches_last = 0;
  std::vector<int> active;
  std::vector<hode::EnsTile> tiles;
  std::vector<int32_t> qoff;
  for (int launch = 0;; ++launch) {
    active.clear();
    for (int i = 0; i < e->n; ++i)
      if (!e->inst[i].ctrl.done) active.push_back(i);
    if (active.empty()) break;
    // one launch for the whole integration (every instance is done after at
    // most max_steps rounds), unless epochs were set
    const int64_t ep = launch == 0 ? e->epoch_first : e->epoch_len;
    const int rounds = (int)std::min<int64_t>(ep > 0 ? ep : max_steps, 0x7fffffff);
    build_tiles(*e, e->nwg, active, tiles, qoff);
    // the tile buffer holds the finest cut the kernel's re-tiling can make
    // (every plane chunk at its smallest), and the kernel reads the dealing
    // order of the instances from the device
    size_t cap = tiles.size();
    if (e->n <= hode::kRetileMaxInst) {
      size_t finest = 0;
      for (int i : active) {
        const int N = e->N[i], rows = ens_tile_rows(*e, i), zmin = e->zc[i] > 0 ? std::min(N, e->zc[i]) : std::min(N, 4);
        finest += (size_t)((N + rows - 1) / rows) * ((N + zmin - 1) / zmin);
      }
      cap = std::max(cap, finest);
    }
    if (cap > e->tiles_cap || !e->d_order) {
      if (e->graph) { (void)hipGraphExecDestroy(e->graph); e->graph = nullptr; }
      if (cap > e->tiles_cap) {
        if (e->d_tiles) (void)hipFree(e->d_tiles);
        e->d_tiles = nullptr;
        e->tiles_cap = std::max(cap, (size_t)1024);
        if (hipMalloc(&e->d_tiles, sizeof(hode::EnsTile) * e->tiles_cap) != hipSuccess)
          return fail(c, HODE_ENOMEM, "tile allocation failed");
      }
      if (!e->d_order && hipMalloc(&e->d_order, sizeof(int32_t) * e->n) != hipSuccess)
        return fail(c, HODE_ENOMEM, "ensemble order allocation failed");
    }
    {
      std::vector<int32_t> order(e->n);
      for (int i = 0; i < e->n; ++i) order[i] = i;
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return e->weight[a] > e->weight[b]; });
      HIPCHK(c, hipMemcpy(e->d_order, order.data(), sizeof(int32_t) * e->n, hipMemcpyHostToDevice));
    }
    bool need_d1 = false;
    for (int i = 0; i < e->n; ++i) {
      hode::EnsInst& I = e->inst[i];
      I.ntiles = 0;
      I.last_done = 0;
      I.rows = ens_tile_rows(*e, i);
      I.zc_fix = e->zc[i];
      I.weight = (float)e->weight[i];
    }
    for (int i : active) {
      hode::EnsInst& I = e->inst[i];
      I.pause_at = I.ctrl.attempts + rounds;
      need_d1 = need_d1 || !I.k1_valid;
    }
    for (const hode::EnsTile& tl : tiles) ++e->inst[tl.inst].ntiles;
    // re-tile on the device each time the running instances have halved
    const int retile_at = e->n <= hode::kRetileMaxInst && active.size() >= 2 ? (int)active.size() / 2 : 0;
    const hode::EnsParams prm{rounds, need_d1 ? 1 : 0, e->n, retile_at, (int32_t)e->tiles_cap, {0, 0, 0}};
    HIPCHK(c, hipMemcpy(e->d_tiles, tiles.data(), sizeof(hode::EnsTile) * tiles.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemsetAsync(sb + L.bar, 0, L.bytes - L.bar, c->stream));
    HIPCHK(c, hipMemcpyAsync(sb + L.qoff, qoff.data(), sizeof(int32_t) * 9, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(sb + L.params, &prm, sizeof(prm), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(e->d_inst, e->inst.data(), sizeof(hode::EnsInst) * e->n, hipMemcpyHostToDevice,
                             c->stream));
    // the persistent kernel, captured once into a graph: its arguments are
    // the fixed buffers above, refilled before every launch
    if (!e->graph) {
      hode::EnsSched sch{e->d_tiles,
                         (int32_t*)(sb + L.qoff),
                         e->d_order,
                         (uint32_t*)(sb + L.qctr),
                         (uint64_t*)(sb + L.bar),
                         (uint64_t*)(sb + L.xbar),
                         (uint32_t*)(sb + L.live),
                         (uint32_t*)(sb + L.error),
                         (const hode::EnsParams*)(sb + L.params),
                         e->barrier_polls};
      HIPCHK(c, hipStreamSynchronize(c->stream));
      hipGraph_t g = nullptr;
      HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      hipError_t le = hode::launch_ensemble(e->dtype, e->d_inst, sch, e->nwg, c->stream);
      hipError_t ee = hipStreamEndCapture(c->stream, &g);
      if (le != hipSuccess || ee != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(c, HODE_EHIP, std::string("ensemble capture: ") + hipGetErrorString(le != hipSuccess ? le : ee));
      }
      hipError_t ie = hipGraphInstantiate(&e->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIPCHK(c, ie);
    }
    HIPCHK(c, hipEventRecord(e->ev[0], c->stream));
    HIPCHK(c, hipGraphLaunch(e->graph, c->stream));
    HIPCHK(c, hipEventRecord(e->ev[1], c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    float kms = 0;
    HIPCHK(c, hipEventElapsedTime(&kms, e->ev[0], e->ev[1]));
    e->kernel_ms_last += kms;
    ++e->launches_last;
    uint32_t err = 0;
    HIPCHK(c, hipMemcpy(&err, sb + L.error, sizeof(err), hipMemcpyDeviceToHost));
    if (err == 3) return fail(c, HODE_EHIP, "ensemble re-tiling exceeded the tile buffer");
    if (err) return fail(c, HODE_EHIP, "ensemble grid barrier timed out (workgroups not co-resident?)");
    std::vector<int64_t> before(e->n);
    for (int i = 0; i < e->n; ++i) before[i] = e->inst[i].ctrl.attempts;
    HIPCHK(c, hipMemcpy(e->inst.data(), e->d_inst, sizeof(hode::EnsInst) * e->n, hipMemcpyDeviceToHost));
    for (int i : active) {
      hode::EnsInst& I = e->inst[i];
      if (I.ctrl.attempts == before[i] && !I.ctrl.done) return fail(c, HODE_EHIP, "ensemble launch made no progress");
      I.k1_valid = 1;
    }
  }
  int worst = HODE_OK;
  for (int i = 0; i < e->n; ++i) {
    const DevCtrl& d = e->inst[i].ctrl;
    e->parity[i] = d.parity;
    e->attempts_last[i] = d.attempts;
    if (per_instance) {
      hode_stats& st = per_instance[i];
      st.accepted = d.accepted;
      st.rejected = d.rejected;
      st.rhs_evals = d.rhs_evals + 1;
      st.t = d.t;
      st.dt_next = d.dt;
      st.last_err = d.last_err;
      st.status = d.status;
      st.pad = 0;
    }
    if (d.status != HODE_OK && worst == HODE_OK) worst = d.status;
  }
  return worst;
}

// Ensemble tile autotuner: the persistent kernel is timed on a twin of the
// whole ensemble (same edges and parameters, started from this ensemble's
// current states, so this ensemble is left unchanged) for `reps` attempts
// per candidate.  Edge by edge, largest total cells first, every
// cells-per-lane width dividing the edge is tried for that edge's instances
// (16-byte lanes give segmented rows where rows are at most 32 lanes,
// narrower widths 64-lane rows) with the other edges at their current
// choice; the width with the shortest total kernel time is kept.  Timing the
// whole ensemble measures a shape by the throughput it gives next to every
// other instance: a sub-ensemble of one edge does not fill the GPU, so its
// time follows the latency of a single tile and favours narrow, many-tiled
// shapes.  Plane ranges are not tuned: they are sized from the running cells
// at every launch and re-cut as instances finish, which measured faster over
// the whole integration than any fixed per-edge choice.  With a cache file
// (HODE_TUNE_CACHE) the choices of earlier runs for the same architecture,
// precision, workgroup count and edge list are read instead of timed, and
// new ones appended.
static std::string ens_tune_key(const hode_ctx* c) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
    arch = prop.gcnArchName;
    for (char& ch : arch)
      if (ch == ' ') ch = '_';
  }
  // the edge multiset identifies the workload shape (FNV-1a over the edges)
  uint64_t hsh = 1469598103934665603ull;
  for (int N : c->ens->N) {
    hsh ^= (uint64_t)N;
    hsh *= 1099511628211ull;
  }
  char buf[256];
  std::snprintf(buf, sizeof(buf), "hode-ens-tune-v2 %s %d %d %d %016llx", arch.c_str(), c->dtype, c->ens->n,
                c->ens->nwg, (unsigned long long)hsh);
  return buf;
}

int hode_ensemble_autotune(hode_ctx* c, int reps, int* vw_out, double* ms_out) {
  int rc = ens_check(c, 0);
  if (rc) return rc;
  if (reps < 1) return fail(c, HODE_EINVAL, "reps >= 1");
  Ensemble* e = c->ens;
  const char* path = std::getenv("HODE_TUNE_CACHE");
  std::map<int, std::vector<int>> members;  // edge -> instances with it
  for (int i = 0; i < e->n; ++i) members[e->N[i]].push_back(i);
  std::map<int, int> best;  // edge -> width
  double best_ms = 0;
  const std::string key = ens_tune_key(c);
  if (path && *path) {
    if (FILE* f = std::fopen(path, "r")) {
      char line[512];
      while (std::fgets(line, sizeof(line), f)) {
        if (std::strncmp(line, key.c_str(), key.size()) != 0 || line[key.size()] != ' ') continue;
        int N = 0, v = 0;
        double ms = 0;
        if (std::sscanf(line + key.size(), " %d %d %lf", &N, &v, &ms) == 3 && members.count(N) && v >= 1 &&
            N % v == 0) {
          best[N] = v;
          best_ms = ms;
        }
      }
      std::fclose(f);
    }
  }
  const int maxvw = c->dtype == HODE_F32 ? 4 : 2;
  if (best.size() < members.size()) {
    std::vector<int64_t> edges(e->N.begin(), e->N.end());
    hode_ctx* t = nullptr;
    rc = hode_ensemble_create(&t, c->device, nullptr, e->n, edges.data(), e->prm.data(), c->dtype);
    if (rc) return fail(c, rc, "ensemble autotune: context");
    rc = hode_set_tolerances(t, c->atol, c->rtol);
    std::vector<hode_stats> st(e->n);
    std::vector<int> cur(e->vw);
    // one timed run of the twin with widths `vw` (kernel time in ms)
    auto run = [&](const std::vector<int>& vw, double* ms) -> int {
      for (int i = 0; i < e->n; ++i) {
        int r = hode_ensemble_init_state(t, i, e->inst[i].a.y[e->parity[i]], 1);
        if (!r) r = hode_ensemble_set_vector_width(t, i, vw[i]);
        if (r) return r;
      }
      const int r2 = hode_ensemble_integrate_adaptive(t, 0.0, 1e300, 0.1, reps, st.data());
      if (r2 != HODE_OK && r2 != HODE_EMAXSTEPS) return r2;
      *ms = t->ens->kernel_ms_last;
      return HODE_OK;
    };
    std::vector<std::pair<double, int>> by_cells;
    for (auto& kv : members) by_cells.push_back({-(double)kv.second.size() * kv.first * kv.first * kv.first, kv.first});
    std::sort(by_cells.begin(), by_cells.end());
    double ms = 0;
    if (!rc) rc = run(cur, &ms);  // warm-up (graph capture, first touch)
    for (auto& bc : by_cells) {
      const int N = bc.second;
      if (rc) break;
      if (best.count(N)) {
        for (int i : members[N]) cur[i] = best[N];
        continue;
      }
      int bv = cur[members[N][0]];
      double bms = 1e300;
      for (int v = 1; v <= maxvw && !rc; v *= 2) {
        if (N % v) continue;
        for (int i : members[N]) cur[i] = v;
        rc = run(cur, &ms);
        if (!rc && ms < bms) {
          bms = ms;
          bv = v;
        }
      }
      for (int i : members[N]) cur[i] = bv;
      best[N] = bv;
      best_ms = bms;
      if (!rc && path && *path) {
        FILE* f = std::fopen(path, "a");
        const bool w = f && std::fprintf(f, "%s %d %d %.6g\n", key.c_str(), N, bv, bms) > 0;
        const bool cl = f && std::fclose(f) == 0;
        if (!w || !cl) {
          hode_destroy(t);
          return fail(c, HODE_EINVAL, std::string("cannot write the tuning cache ") + path);
        }
      }
    }
    const std::string msg = rc ? hode_last_error(t) : "";
    hode_destroy(t);
    if (rc) return fail(c, rc, "ensemble autotune: " + msg);
  }
  for (int i = 0; i < e->n; ++i) {
    e->vw[i] = best[e->N[i]];
    e->zc[i] = 0;
    if (vw_out) vw_out[i] = e->vw[i];
    if (ms_out) ms_out[i] = best_ms;
  }
  return HODE_OK;
}

const char* hode_last_error(const hode_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
