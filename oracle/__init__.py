"""FP64 CPU oracle for the explicit Runge-Kutta hot path (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP path.  The C++ source
(``hode_oracle.cpp``) is compiled with ``g++ -O2 -ffp-contract=off -fopenmp``
into ``liboracle.so`` next to it, on first use or by :func:`build`.

Every function here is a thin ctypes wrapper; the arithmetic lives in the C++
file, which cites what each part follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hode_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

EXP, LOGISTIC, GRAYSCOTT = 1, 2, 3
RK4, DOPRI5, CASHKARP, EULER, FEHLBERG78, MIDPOINT = 1, 2, 3, 4, 5, 6


def AB(steps: int) -> int:
    """Method code of Adams-Bashforth with `steps` steps (1 .. 8)."""
    assert 1 <= steps <= 8
    return 10 + steps


def ABM(steps: int) -> int:
    """Method code of the Adams-Bashforth-Moulton predictor-corrector (1 .. 8 steps)."""
    assert 1 <= steps <= 8
    return 20 + steps


CTRL_PI, CTRL_I = 1, 2
OK, EINVAL, EDT_UNDERFLOW, EMAXSTEPS, ENONFINITE = 0, -1, -5, -6, -7


class System(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad", C.c_int32), ("n", C.c_int64), ("N", C.c_int64),
                ("Du", C.c_double), ("Dv", C.c_double), ("F", C.c_double), ("k", C.c_double),
                ("L", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("accepted", C.c_int64), ("rejected", C.c_int64), ("rhs_evals", C.c_int64),
                ("t", C.c_double), ("dt_next", C.c_double), ("last_err", C.c_double),
                ("status", C.c_int32), ("pad", C.c_int32)]


def build(force: bool = False) -> str:
    """Compiles ``liboracle.so`` (always when ``force``; else only if stale)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                               "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.orc_rhs.argtypes = [C.POINTER(System), P, P]
        L.orc_tableau.argtypes = [C.c_int, P, P, P, P]
        L.orc_tableau.restype = None
        L.orc_err_norm.argtypes = [C.c_int64, P, P, P, C.c_double, C.c_double]
        L.orc_err_norm.restype = C.c_double
        L.orc_ctrl_decide.argtypes = [C.c_int, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_int),
                                      C.POINTER(C.c_double)]
        L.orc_rk4_step.argtypes = [C.POINTER(System), P, C.c_double]
        L.orc_dopri5_attempt.argtypes = [C.POINTER(System), P, C.c_double, P, P, P]
        L.orc_integrate_n_steps.argtypes = [C.POINTER(System), C.c_int, P, C.c_double, C.c_double,
                                            C.c_int64, C.POINTER(C.c_double)]
        L.orc_integrate_adaptive.argtypes = [C.POINTER(System), P, C.c_double, C.c_double, C.c_double,
                                             C.c_double, C.c_double, C.c_int, C.c_int64,
                                             C.POINTER(Stats), P, C.c_int64]
        L.orc_integrate_replay.argtypes = [C.POINTER(System), P, C.c_double, P, P, C.c_int64,
                                           C.c_double, C.c_double, C.POINTER(C.c_double), P]
        L.orc_cashkarp_attempt.argtypes = [C.POINTER(System), P, C.c_double, P, P]
        L.orc_fehlberg78_attempt.argtypes = [C.POINTER(System), P, C.c_double, P, P]
        L.orc_integrate_dense_times.argtypes = [C.POINTER(System), P, P, C.c_int64, C.c_double, C.c_double,
                                                C.c_double, C.c_int, C.c_int64, P, C.POINTER(Stats)]
        L.orc_dopri5_dense_weights.argtypes = [C.c_double, P]
        L.orc_dopri5_dense_weights.restype = None
        L.orc_ab_weights.argtypes = [C.c_int, P]
        L.orc_ab_weights.restype = None
        L.orc_am_weights.argtypes = [C.c_int, P]
        L.orc_am_weights.restype = None
        L.orc_ctrl_decide_k.argtypes = [C.c_int, C.c_double, C.c_double, C.POINTER(C.c_double),
                                        C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.orc_integrate_n_steps_e.argtypes = [C.POINTER(System), C.c_int, P, C.c_double, C.c_double,
                                              C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.orc_integrate_times.argtypes = [C.POINTER(System), C.c_int, P, P, C.c_int64, C.c_double, C.c_double,
                                          C.c_double, C.c_int, C.c_int64, P, C.POINTER(Stats)]
        L.orc_integrate_adaptive_m.argtypes = [C.POINTER(System), C.c_int, P, C.c_double, C.c_double, C.c_double,
                                               C.c_double, C.c_double, C.c_int, C.c_int64,
                                               C.POINTER(Stats), P, C.c_int64]
        L.orc_integrate_replay_m.argtypes = [C.POINTER(System), C.c_int, P, C.c_double, P, P, C.c_int64,
                                             C.c_double, C.c_double, C.POINTER(C.c_double), P]
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def ew_system(kind: int, n: int) -> System:
    return System(kind=kind, n=n, N=0)


def gs_system(N: int, Du=2e-5, Dv=1e-5, F=0.053, k=0.014, L=2.5) -> System:
    return System(kind=GRAYSCOTT, n=2 * N ** 3, N=N, Du=Du, Dv=Dv, F=F, k=k, L=L)


def rhs(sysd: System, y) -> np.ndarray:
    y = _f64(y).ravel()
    f = np.empty_like(y)
    rc = lib().orc_rhs(C.byref(sysd), _ptr(y), _ptr(f))
    assert rc == OK, rc
    return f


def tableau(method: int):
    s = {RK4: 4, DOPRI5: 7, CASHKARP: 6, FEHLBERG78: 13}[method]
    a = np.zeros(s * s)
    b = np.zeros(s)
    bh = np.zeros(s)
    c = np.zeros(s)
    lib().orc_tableau(method, _ptr(a), _ptr(b), _ptr(bh), _ptr(c))
    return a.reshape(s, s), b, bh, c


def err_norm(y, ynew, e, atol, rtol) -> float:
    y, ynew, e = _f64(y).ravel(), _f64(ynew).ravel(), _f64(e).ravel()
    return lib().orc_err_norm(y.size, _ptr(y), _ptr(ynew), _ptr(e), atol, rtol)


def ctrl_decide(kind: int, err: float, err_prev: float, last_rejected: bool, order_k=None):
    """One controller decision; order_k = 1 + the embedded order (default 5)."""
    ep = C.c_double(err_prev)
    lr = C.c_int(1 if last_rejected else 0)
    fac = C.c_double(0)
    if order_k is None:
        acc = lib().orc_ctrl_decide(kind, err, C.byref(ep), C.byref(lr), C.byref(fac))
    else:
        acc = lib().orc_ctrl_decide_k(kind, order_k, err, C.byref(ep), C.byref(lr), C.byref(fac))
    return bool(acc), fac.value, ep.value, bool(lr.value)


def am_weights(steps: int) -> np.ndarray:
    """Adams-Moulton weights gamma_0 .. gamma_{steps-1} (gamma_j multiplies f_{n+1-j})."""
    g = np.zeros(8)
    lib().orc_am_weights(steps, _ptr(g))
    return g[:steps]


def ab_weights(steps: int) -> np.ndarray:
    """Adams-Bashforth weights beta_0 .. beta_{steps-1} (beta_j multiplies f_{n-j})."""
    b = np.zeros(8)
    lib().orc_ab_weights(steps, _ptr(b))
    return b[:steps]


def rk4_step(sysd: System, y, h: float) -> np.ndarray:
    y = _f64(y).ravel().copy()
    assert lib().orc_rk4_step(C.byref(sysd), _ptr(y), h) == OK
    return y


def dopri5_attempt(sysd: System, y, h: float):
    """One Dopri5 attempt from y: returns (ynew, k7, e)."""
    y = _f64(y).ravel()
    yn, k7, e = np.empty_like(y), np.empty_like(y), np.empty_like(y)
    assert lib().orc_dopri5_attempt(C.byref(sysd), _ptr(y), h, _ptr(yn), _ptr(k7), _ptr(e)) == OK
    return yn, k7, e


def cashkarp_attempt(sysd: System, y, h: float):
    """One Cash-Karp 5(4) attempt from y: returns (ynew, e)."""
    y = _f64(y).ravel()
    yn, e = np.empty_like(y), np.empty_like(y)
    assert lib().orc_cashkarp_attempt(C.byref(sysd), _ptr(y), h, _ptr(yn), _ptr(e)) == OK
    return yn, e


def fehlberg78_attempt(sysd: System, y, h: float):
    """One Fehlberg 7(8) attempt from y: returns (ynew, e)."""
    y = _f64(y).ravel()
    yn, e = np.empty_like(y), np.empty_like(y)
    assert lib().orc_fehlberg78_attempt(C.byref(sysd), _ptr(y), h, _ptr(yn), _ptr(e)) == OK
    return yn, e


def integrate_n_steps(sysd: System, method: int, y, t0: float, dt: float, n: int, evals: bool = False):
    """n fixed steps (an Adams-Bashforth method, AB(s), starts afresh);
    returns (y, t_end) or, with evals, (y, t_end, right-hand side evaluations)."""
    y = _f64(y).ravel().copy()
    te = C.c_double(0)
    ne = C.c_int64(0)
    rc = lib().orc_integrate_n_steps_e(C.byref(sysd), method, _ptr(y), t0, dt, n, C.byref(te), C.byref(ne))
    assert rc == OK, rc
    return (y, te.value, ne.value) if evals else (y, te.value)


def integrate_adaptive(sysd: System, y, t0, t1, dt0, atol, rtol, ctrl=CTRL_PI, max_steps=10 ** 7,
                       trace_cap=0, method=None):
    """Returns (y, stats dict, trace array of shape (attempts, 4) or None).
    method: DOPRI5 (default), CASHKARP or FEHLBERG78."""
    y = _f64(y).ravel().copy()
    st = Stats()
    tr = np.zeros((max(trace_cap, 1), 4))
    lib().orc_integrate_adaptive_m(C.byref(sysd), DOPRI5 if method is None else method, _ptr(y), t0, t1, dt0,
                                   atol, rtol, ctrl, max_steps, C.byref(st), _ptr(tr) if trace_cap else None,
                                   trace_cap)
    stats = {f: getattr(st, f) for f, _ in Stats._fields_ if f != "pad"}
    n_att = stats["accepted"] + stats["rejected"]
    return y, stats, (tr[:min(n_att, trace_cap)] if trace_cap else None)


def integrate_times(sysd: System, y, times, dt0, atol, rtol, ctrl=CTRL_PI, max_steps=10 ** 7, method=None):
    """States at times[0], times[1], ... (rows of the returned array; rows
    after a failing status stay zero) and the stats dict."""
    y = _f64(y).ravel().copy()
    times = _f64(times).ravel()
    out = np.zeros((times.size, y.size))
    st = Stats()
    rc = lib().orc_integrate_times(C.byref(sysd), DOPRI5 if method is None else method, _ptr(y), _ptr(times),
                                   times.size, dt0, atol, rtol, ctrl, max_steps, _ptr(out), C.byref(st))
    if rc == EINVAL:
        raise ValueError("integrate_times: invalid arguments (times must increase)")
    return out, {f: getattr(st, f) for f, _ in Stats._fields_ if f != "pad"}


def integrate_dense_times(sysd: System, y, times, dt0, atol, rtol, ctrl=CTRL_PI, max_steps=10 ** 7):
    """Dopri5 dense output: free controlled steps from times[0] to
    times[-1], intermediate states from the continuous extension.  Returns
    (rows of states, stats dict)."""
    y = _f64(y).ravel().copy()
    times = _f64(times).ravel()
    out = np.zeros((times.size, y.size))
    st = Stats()
    rc = lib().orc_integrate_dense_times(C.byref(sysd), _ptr(y), _ptr(times), times.size, dt0, atol, rtol, ctrl,
                                         max_steps, _ptr(out), C.byref(st))
    if rc == EINVAL:
        raise ValueError("integrate_dense_times: invalid arguments (times must increase)")
    return out, {f: getattr(st, f) for f, _ in Stats._fields_ if f != "pad"}


def dopri5_dense_weights(theta: float) -> np.ndarray:
    """w_j(theta) of the continuous extension: y(t_n + theta h) = y_n + h sum_j w_j k_j."""
    w = np.zeros(7)
    lib().orc_dopri5_dense_weights(theta, _ptr(w))
    return w


def integrate_replay(sysd: System, y, t0, hs, accepted, atol=1e-6, rtol=1e-6, method=None):
    """Replays (h, accepted) pairs; returns (y, t_end, per-attempt error norms).
    method: DOPRI5 (default), CASHKARP or FEHLBERG78."""
    y = _f64(y).ravel().copy()
    hs = _f64(hs).ravel()
    acc = np.ascontiguousarray(np.asarray(accepted, dtype=np.int32).ravel())
    errs = np.zeros(max(hs.size, 1))
    te = C.c_double(0)
    rc = lib().orc_integrate_replay_m(C.byref(sysd), DOPRI5 if method is None else method, _ptr(y), t0, _ptr(hs),
                                      _ptr(acc), hs.size, atol, rtol, C.byref(te), _ptr(errs))
    assert rc == OK, rc
    return y, te.value, errs[:hs.size]


def num_threads() -> int:
    return lib().orc_num_threads()
