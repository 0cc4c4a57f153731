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
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <utility>

#include "../../include/hode.h"
#include "hode_internal.h"

using hode::DevCtrl;

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
  int ry = 0, zc = 0, ew_grid = 0;
  bool k1_valid = false;
  int parity = 0, k1slot = 0;
  bool persist_valid = false;  // controller history carried between try_step calls
  DevCtrl persist;
  hode_stats last{};
  int64_t last_attempts = 0;
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  std::string err;
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
  for (auto& kv : c->graphs) hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

void free_state(hode_ctx* c) {
  clear_graphs(c);
  for (void*& p : c->y) { if (p) hipFree(p); p = nullptr; }
  for (void*& p : c->ks) { if (p) hipFree(p); p = nullptr; }
  for (void*& p : c->k) { if (p) hipFree(p); p = nullptr; }
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

// Enqueues the kernels of one attempt (or fixed step) in `mode`.
hipError_t enqueue_attempt(hode_ctx* c, int mode) {
  if (!is_gs(c)) {
    hipError_t e = hode::launch_ew(c->dtype, c->rhs, mode, c->y[0], c->y[1], c->nelem, c->ew_grid, c->d_ctrl,
                                   c->stream);
    return e != hipSuccess ? e : hode::launch_ctrl(c->d_ctrl, c->stream);
  }
  const hode::GSLaunch a = gs_args(c);
  static const int rk4[] = {hode::K_D1, hode::K_R2, hode::K_R3, hode::K_R4};
  static const int dp5f[] = {hode::K_D2, hode::K_D3, hode::K_D4, hode::K_D5, hode::K_D6F, hode::K_D7F};
  static const int dp5a[] = {hode::K_D2, hode::K_D3, hode::K_D4, hode::K_D5, hode::K_D6, hode::K_D7};
  const int* seq = mode == hode::MODE_FIXED_RK4 ? rk4 : (mode == hode::MODE_FIXED_DP5 ? dp5f : dp5a);
  const int ns = mode == hode::MODE_FIXED_RK4 ? 4 : 6;
  for (int i = 0; i < ns; ++i) {
    hipError_t e = hode::launch_gs(seq[i], c->dtype, c->ry, a, c->d_ctrl, c->stream);
    if (e != hipSuccess) return e;
  }
  return hode::launch_ctrl(c->d_ctrl, c->stream);
}

int get_graph(hode_ctx* c, int mode, int M, hipGraphExec_t* out) {
  auto key = std::make_pair(mode, M);
  auto it = c->graphs.find(key);
  if (it != c->graphs.end()) { *out = it->second; return HODE_OK; }
  hipGraph_t g = nullptr;
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  for (int i = 0; i < M && le == hipSuccess; ++i) le = enqueue_attempt(c, mode);
  hipError_t ee = hipStreamEndCapture(c->stream, &g);
  if (le != hipSuccess) { if (g) hipGraphDestroy(g); return fail(c, HODE_EHIP, std::string("capture: ") + hipGetErrorString(le)); }
  if (ee != hipSuccess) return fail(c, HODE_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
  hipGraphExec_t ex = nullptr;
  hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (ie != hipSuccess) return fail(c, HODE_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
  c->graphs[key] = ex;
  *out = ex;
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
  return d;
}

int launch_k1(hode_ctx* c) {
  if (!is_gs(c)) return HODE_OK;
  const hode::GSLaunch a = gs_args(c);
  HIPCHK(c, hode::launch_gs(hode::K_D1, c->dtype, c->ry, a, c->d_ctrl, c->stream));
  return HODE_OK;
}

int pow2_floor(int64_t x) {
  int m = 1;
  while ((int64_t)m * 2 <= x && m < 64) m *= 2;
  return m;
}

// Runs the device-resident loop from the control block `init` until done.
int run_loop(hode_ctx* c, const DevCtrl& init, bool need_k1) {
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
    if (init.mode == hode::MODE_ADAPTIVE) {
      const double est = std::ceil((cur.t1 - cur.t) / (cur.dt > 0 ? cur.dt : 1.0)) + 1.0;
      M = pow2_floor(est > 64 ? 64 : (int64_t)est);
    } else {
      M = pow2_floor(cur.nsteps - cur.accepted);
    }
    hipGraphExec_t ex;
    int rc = get_graph(c, init.mode, M, &ex);
    if (rc) return rc;
    HIPCHK(c, hipGraphLaunch(ex, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->h_ctrl, c->d_ctrl, sizeof(DevCtrl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    cur = *c->h_ctrl;
    if (++chunks > (int64_t)1 << 40) return fail(c, HODE_EHIP, "control loop did not terminate");
  }
  c->parity = cur.parity;
  c->k1slot = cur.k1slot;
  if (init.mode != hode::MODE_FIXED_RK4) c->k1_valid = true;
  c->last.accepted = cur.accepted;
  c->last.rejected = cur.rejected;
  c->last.rhs_evals = cur.rhs_evals + extra_evals;
  c->last.t = cur.t;
  c->last.dt_next = init.mode == hode::MODE_ADAPTIVE ? cur.dt : cur.h;
  c->last.last_err = cur.last_err;
  c->last.status = cur.status;
  c->last_attempts = cur.attempts;
  c->persist = cur;
  return HODE_OK;
}

int check_ready(hode_ctx* c) {
  if (!c) return HODE_EINVAL;
  if (!c->rhs) return fail(c, HODE_ESTATE, "no RHS set");
  if (!c->dtype) return fail(c, HODE_ESTATE, "no state initialised");
  return HODE_OK;
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
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  free_state(c);
  if (c->d_ctrl) hipFree(c->d_ctrl);
  if (c->d_ctrl_save) hipFree(c->d_ctrl_save);
  if (c->h_ctrl) hipHostFree(c->h_ctrl);
  if (c->d_trace) hipFree(c->d_trace);
  if (c->d_mlp) hipFree(c->d_mlp);
  if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
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
  if (!reuse) {
    if (is_gs(c)) {
      if (!c->ry) c->ry = dtype == HODE_F32 ? 4 : 2;
      c->zc = default_zc(N, c->ry);
    } else {
      c->ew_grid = default_ew_grid(nelem, dtype);
    }
  }
  return HODE_OK;
}

size_t hode_state_bytes(const hode_ctx* c) { return c ? (size_t)c->nelem * c->esize : 0; }

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
  if (!weights || nbytes != 2 * (size_t)hode::MLP_NPARAM) return fail(c, HODE_EINVAL, "MLP weights must be 10498 bytes");
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
  if (method != HODE_RK4 && method != HODE_DOPRI5) return fail(c, HODE_EINVAL, "method");
  if (n < 0 || !std::isfinite(t0) || !std::isfinite(dt)) return fail(c, HODE_EINVAL, "bad step arguments");
  HIPCHK(c, hipSetDevice(c->device));
  const int mode = method == HODE_RK4 ? hode::MODE_FIXED_RK4 : hode::MODE_FIXED_DP5;
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
  HIPCHK(c, hipSetDevice(c->device));
  DevCtrl d = base_ctrl(c, hode::MODE_ADAPTIVE);
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
  rc = run_loop(c, d, !c->k1_valid);
  if (rc) return rc;
  c->persist_valid = false;
  if (out) *out = c->last;
  return c->last.status;
}

int hode_try_step(hode_ctx* c, double* t, double* dt, int* accepted) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!t || !dt || !accepted || !std::isfinite(*t) || !(*dt > 0) || !std::isfinite(*dt))
    return fail(c, HODE_EINVAL, "bad try_step arguments");
  HIPCHK(c, hipSetDevice(c->device));
  DevCtrl d = base_ctrl(c, hode::MODE_ADAPTIVE);
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
  rc = run_loop(c, d, !c->k1_valid);
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

int hode_set_trace(hode_ctx* c, int64_t capacity) {
  if (!c || capacity < 0) return HODE_EINVAL;
  if (c->d_trace) { hipFree(c->d_trace); c->d_trace = nullptr; }
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
    c->ry = ry;
    c->zc = zc;
  }
  clear_graphs(c);
  return HODE_OK;
}

int hode_get_tile(const hode_ctx* c, int* ry, int* zc) {
  if (!c || !ry || !zc) return HODE_EINVAL;
  *ry = c->ry;
  *zc = is_gs(c) ? c->zc : c->ew_grid;
  return HODE_OK;
}

int hode_time_kernel(hode_ctx* c, int kind, int reps, double* avg_ms) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (reps < 1 || !avg_ms) return fail(c, HODE_EINVAL, "reps >= 1 and avg_ms required");
  if (is_gs(c) && (kind < 0 || kind > hode::K_D6F)) return fail(c, HODE_EINVAL, "kernel kind");
  if (!is_gs(c) && kind != HODE_RK4 && kind != HODE_DOPRI5) return fail(c, HODE_EINVAL, "kernel kind");
  HIPCHK(c, hipSetDevice(c->device));
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
    if (is_gs(c)) return hode::launch_gs(kind, c->dtype, c->ry, a, c->d_ctrl, c->stream);
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
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (e != hipSuccess) return fail(c, HODE_EHIP, std::string("timing: ") + hipGetErrorString(e));
  *avg_ms = (double)ms / reps;
  if (is_gs(c) && kind == hode::K_D1) c->k1_valid = true;
  return HODE_OK;
}

// Stage sequence of one attempt of `method` (adaptive Dopri5 for HODE_DOPRI5).
static int stage_seq(int method, int* seq) {
  if (method == HODE_RK4) {
    const int s[] = {hode::K_D1, hode::K_R2, hode::K_R3, hode::K_R4};
    for (int i = 0; i < 4; ++i) seq[i] = s[i];
    return 4;
  }
  const int s[] = {hode::K_D2, hode::K_D3, hode::K_D4, hode::K_D5, hode::K_D6, hode::K_D7};
  for (int i = 0; i < 6; ++i) seq[i] = s[i];
  return 6;
}

int hode_profile_attempt(hode_ctx* c, int method, int reps, double* ms) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!is_gs(c)) return fail(c, HODE_EINVAL, "stage profiling is for the Gray-Scott path");
  if (reps < 1 || !ms || (method != HODE_RK4 && method != HODE_DOPRI5)) return fail(c, HODE_EINVAL, "arguments");
  HIPCHK(c, hipSetDevice(c->device));
  int seq[8];
  const int ns = stage_seq(method, seq);
  DevCtrl d = base_ctrl(c, 0);
  d.h = c->last.dt_next > 0 ? c->last.dt_next : 0.01;
  *c->h_ctrl = d;
  HIPCHK(c, hipMemcpyAsync(c->d_ctrl, c->h_ctrl, sizeof(DevCtrl), hipMemcpyHostToDevice, c->stream));
  const hode::GSLaunch a = gs_args(c);
  if (method == HODE_DOPRI5 && !c->k1_valid) {
    HIPCHK(c, hode::launch_gs(hode::K_D1, c->dtype, c->ry, a, c->d_ctrl, c->stream));
    c->k1_valid = true;
  }
  hipEvent_t ev[9];
  for (int i = 0; i <= ns; ++i) HIPCHK(c, hipEventCreate(&ev[i]));
  double acc[8] = {0};
  hipError_t e = hipSuccess;
  for (int r = 0; r <= reps && e == hipSuccess; ++r) {  // first round is warm-up
    for (int i = 0; i < ns && e == hipSuccess; ++i) {
      e = hipEventRecord(ev[i], c->stream);
      if (e == hipSuccess) e = hode::launch_gs(seq[i], c->dtype, c->ry, a, c->d_ctrl, c->stream);
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
  for (int i = 0; i <= ns; ++i) hipEventDestroy(ev[i]);
  HIPCHK(c, e);
  for (int i = 0; i < ns; ++i) ms[i] = acc[i] / reps;
  return HODE_OK;
}

int hode_autotune(hode_ctx* c, int method, int reps, int* best_ry, int* best_zc, double* best_ms) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!is_gs(c)) return fail(c, HODE_EINVAL, "autotuning is for the Gray-Scott path");
  const int rys[] = {1, 2, 4};
  const int zcs[] = {8, 16, 32, 64, 128, 256};
  double best = 1e300;
  int bry = c->ry, bzc = c->zc;
  for (int ry : rys) {
    for (int zc : zcs) {
      if (zc > c->N && zc != zcs[0]) continue;
      c->ry = ry;
      c->zc = zc;
      double ms[8];
      rc = hode_profile_attempt(c, method, reps, ms);
      if (rc) return rc;
      const int ns = method == HODE_RK4 ? 4 : 6;
      double tot = 0;
      for (int i = 0; i < ns; ++i) tot += ms[i];
      if (tot < best) { best = tot; bry = ry; bzc = zc; }
    }
  }
  c->ry = bry;
  c->zc = bzc;
  clear_graphs(c);
  if (best_ry) *best_ry = bry;
  if (best_zc) *best_zc = bzc;
  if (best_ms) *best_ms = best;
  return HODE_OK;
}

const char* hode_last_error(const hode_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
