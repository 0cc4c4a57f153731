"""ctypes binding of libhode.so (argument marshalling only).

Functions carry the C names of ``include/hode.h``.  Device work runs in the
library's HIP kernels; this module only converts Python/numpy/torch arguments
to plain pointers and sizes and raises on error codes.  If the library has not
been built the import of :func:`lib` fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libhode.so")

F32, F64 = 1, 2
RHS_EXP, RHS_LOGISTIC, RHS_GRAYSCOTT3D = 1, 2, 3
RK4, DOPRI5, CASHKARP54, EULER, FEHLBERG78, MIDPOINT = 1, 2, 3, 4, 5, 6


def ABM(steps):
    """Method code of Adams-Bashforth-Moulton with `steps` steps (1 .. 8)."""
    if not 1 <= steps <= 8:
        raise ValueError("Adams-Bashforth-Moulton steps must be 1 .. 8")
    return 20 + steps


def AB(steps):
    """Method code of Adams-Bashforth with `steps` steps (1 .. 8)."""
    if not 1 <= steps <= 8:
        raise ValueError("Adams-Bashforth steps must be 1 .. 8")
    return 10 + steps


CTRL_PI, CTRL_I, CTRL_MLP = 1, 2, 3
OK, EINVAL, ESTATE, EHIP, ENOMEM, EDT_UNDERFLOW, EMAXSTEPS, ENONFINITE = 0, -1, -2, -3, -4, -5, -6, -7
# doubles per trace record (h, err, accepted, t after, dt next, PI log-ratio,
# learned log-ratio, landed, 16 features): HODE_TRACE_W, read from the library
# by lib()
TRACE_W = None
MLP_NPARAM = 64 * 16 + 64 + 64 * 64 + 64 + 64 + 1

# Gray-Scott stage kernels, as numbered by hode_time_kernel
K_D1, K_R2, K_R3, K_R4, K_D2, K_D3, K_D4, K_D5, K_D6, K_D7, K_D7F, K_C4, K_C5, K_C6, K_C6F, K_E1, K_D6F = range(17)
K_F = list(range(17, 30))  # Fehlberg 7(8) stages F1 .. F13
K_F13F = 30
K_AB = list(range(31, 39))  # Adams-Bashforth with 1 .. 8 steps
K_D6K = 39  # Dopri5 stage 6 storing k6 (dense output)
K_ABC = list(range(40, 48))  # Adams-Moulton correctors with 1 .. 8 steps
K_MM = [48, 49, 50]  # modified midpoint substeps


class hode_stats(C.Structure):
    _fields_ = [("accepted", C.c_int64), ("rejected", C.c_int64), ("rhs_evals", C.c_int64), ("t", C.c_double),
                ("dt_next", C.c_double), ("last_err", C.c_double), ("status", C.c_int32), ("pad", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


class HodeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("hode error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    """Loads libhode.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError("libhode.so is not built: run python -m paper_2309_05331_amd.build")
        # torch bundles its own HIP runtime under the same soname; load it
        # first so the process holds one runtime that both torch (device
        # memory, streams) and this library use
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIBPATH)
        P, I, I64, D, S = C.c_void_p, C.c_int, C.c_int64, C.c_double, C.c_size_t
        sig = {
            "hode_create": ([C.POINTER(P), I, P], I),
            "hode_destroy": ([P], None),
            "hode_set_rhs": ([P, I, C.POINTER(D), I], I),
            "hode_init_state": ([P, I, I, I, C.POINTER(I64), P, I], I),
            "hode_read_state": ([P, P, S, I], I),
            "hode_state_bytes": ([P], S),
            "hode_set_tolerances": ([P, D, D], I),
            "hode_set_controller": ([P, I, P, S], I),
            "hode_do_step": ([P, I, D, D], I),
            "hode_integrate_n_steps": ([P, I, D, D, I64, C.POINTER(D)], I),
            "hode_integrate_times": ([P, C.POINTER(D), I64, D, I64, P, S, I, C.POINTER(hode_stats)], I),
            "hode_integrate_times_dense": ([P, C.POINTER(D), I64, D, I64, P, S, I, C.POINTER(hode_stats)], I),
            "hode_get_ctrl": ([P, P, C.POINTER(S)], I),
            "hode_autotune_cached": ([P, I, I, C.c_char_p, C.POINTER(I)], I),
            "hode_debug_poison": ([P], I),
            "hode_set_ctrl": ([P, P, S], I),
            "hode_try_step": ([P, C.POINTER(D), C.POINTER(D), C.POINTER(I)], I),
            "hode_integrate_adaptive": ([P, D, D, D, I64, C.POINTER(hode_stats)], I),
            "hode_get_stats": ([P, C.POINTER(hode_stats)], I),
            "hode_set_trace": ([P, I64], I),
            "hode_read_trace": ([P, P, I64, C.POINTER(I64)], I),
            "hode_eval_rhs": ([P, P, S, I], I),
            "hode_set_stepper": ([P, I], I),
            "hode_set_graphs": ([P, I], I),
            "hode_set_tile": ([P, I, I], I),
            "hode_get_tile": ([P, C.POINTER(I), C.POINTER(I)], I),
            "hode_set_tile_waves": ([P, I], I),
            "hode_get_kind_tile": ([P, I, C.POINTER(I), C.POINTER(I), C.POINTER(I)], I),
            "hode_time_kernel": ([P, I, I, C.POINTER(D)], I),
            "hode_profile_attempt": ([P, I, I, C.POINTER(D)], I),
            "hode_autotune": ([P, I, I, C.POINTER(I), C.POINTER(I), C.POINTER(D)], I),
            "hode_stream_copy": ([P, P, S, I, C.POINTER(D)], I),
            "hode_set_vector_width": ([P, I], I),
            "hode_ensemble_create": ([C.POINTER(P), I, P, I, C.POINTER(I64), C.POINTER(D), I], I),
            "hode_ensemble_size": ([P], I),
            "hode_ensemble_init_state": ([P, I, P, I], I),
            "hode_ensemble_read_state": ([P, I, P, S, I], I),
            "hode_ensemble_set_weights": ([P, C.POINTER(D)], I),
            "hode_ensemble_set_epoch": ([P, I, I], I),
            "hode_ensemble_set_barrier_limit": ([P, I64], I),
            "hode_ensemble_timing": ([P, C.POINTER(D), C.POINTER(I)], I),
            "hode_ensemble_set_vector_width": ([P, I, I], I),
            "hode_ensemble_set_plane_chunk": ([P, I, I], I),
            "hode_ensemble_get_tile": ([P, I, C.POINTER(I), C.POINTER(I)], I),
            "hode_ensemble_set_trace": ([P, I64], I),
            "hode_ensemble_read_trace": ([P, I, P, I64, C.POINTER(I64)], I),
            "hode_ensemble_integrate_adaptive": ([P, D, D, D, I64, C.POINTER(hode_stats)], I),
            "hode_ensemble_autotune": ([P, I, C.POINTER(I), C.POINTER(D)], I),
            "hode_mlp_forward": ([P, P, P, I64, P], I),
            "hode_mlp_quantize": ([P, P, P], I),
            "hode_mlp_loss_grad": ([P, P, P, P, P, I64, P, P, C.POINTER(D), P], I),
            "hode_mlp_train_step": ([P, P, P, P, I64, P, P, P, P, P, P, I64, C.c_float, C.POINTER(D), P], I),
            "hode_mlp_train_step_noalloc": ([P, P, P, P, I64, P, P, P, P, I64, C.c_float, C.POINTER(D), P], I),
            "hode_last_error": ([P], C.c_char_p),
            "hode_trace_width": ([], I),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        global TRACE_W
        TRACE_W = L.hode_trace_width()
        _lib = L
    return _lib


def stream_copy(dst, src, reps=20):
    """Times the reference copy kernel between two equal-size device tensors;
    returns (ms per copy, GB/s counting read + write)."""
    ms = C.c_double()
    nb = src.numel() * src.element_size()
    rc = lib().hode_stream_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nb, reps, C.byref(ms))
    if rc != OK:
        raise HodeError(rc, "stream copy")
    return ms.value, 2 * nb / (ms.value * 1e-3) / 1e9


def exported_symbols():
    """Names declared in include/hode.h (for the export check)."""
    import re
    hdr = os.path.join(os.path.dirname(HERE), "include", "hode.h")
    return sorted(set(re.findall(r"\b(hode_[a-z_0-9]+)\s*\(", open(hdr).read())))


def _ptr_of(buf):
    """(pointer, nbytes, on_device) for a numpy array or a torch tensor."""
    if isinstance(buf, np.ndarray):
        assert buf.flags["C_CONTIGUOUS"]
        return buf.ctypes.data_as(C.c_void_p), buf.nbytes, 0
    # torch tensor
    assert buf.is_contiguous()
    on_dev = 1 if buf.is_cuda else 0
    return C.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(), on_dev


class Context:
    """A hode_ctx* with the C functions as methods (same names minus the prefix)."""

    def __init__(self, device: int = 0, stream: int | None = None):
        self.L = lib()
        self.h = C.c_void_p()
        self._check(self.L.hode_create(C.byref(self.h), device, C.c_void_p(stream) if stream else None))

    def close(self):
        if self.h:
            self.L.hode_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=()):
        if rc != OK and rc not in allow:
            msg = self.L.hode_last_error(self.h).decode() if self.h else ""
            raise HodeError(rc, msg)
        return rc

    def set_rhs(self, rhs, params=None):
        if params is None:
            return self._check(self.L.hode_set_rhs(self.h, rhs, None, 0))
        arr = (C.c_double * len(params))(*params)
        return self._check(self.L.hode_set_rhs(self.h, rhs, arr, len(params)))

    def init_state(self, src, dtype=None, grid=None):
        """src: numpy array or torch tensor (float32/float64), flat or (2,N,N,N)."""
        is_f32 = str(src.dtype) in ("float32", "torch.float32")
        dt = dtype or (F32 if is_f32 else F64)
        if grid is not None:
            shape = (C.c_int64 * 3)(grid, grid, grid)
            nf, nd = 2, 3
        else:
            n = src.size if isinstance(src, np.ndarray) else src.numel()
            shape = (C.c_int64 * 1)(n)
            nf, nd = 1, 1
        p, _, on_dev = _ptr_of(src)
        return self._check(self.L.hode_init_state(self.h, dt, nf, nd, shape, p, on_dev))

    def state_bytes(self):
        return self.L.hode_state_bytes(self.h)

    def read_state(self, dst):
        p, nb, on_dev = _ptr_of(dst)
        return self._check(self.L.hode_read_state(self.h, p, nb, on_dev))

    def set_tolerances(self, atol, rtol):
        return self._check(self.L.hode_set_tolerances(self.h, atol, rtol))

    def set_controller(self, kind, weights_bf16=None):
        if weights_bf16 is None:
            return self._check(self.L.hode_set_controller(self.h, kind, None, 0))
        w = np.ascontiguousarray(weights_bf16, dtype=np.uint16)
        return self._check(self.L.hode_set_controller(self.h, kind, w.ctypes.data_as(C.c_void_p), w.nbytes))

    def do_step(self, method, t, dt):
        return self._check(self.L.hode_do_step(self.h, method, t, dt))

    def integrate_n_steps(self, method, t0, dt, n):
        te = C.c_double()
        self._check(self.L.hode_integrate_n_steps(self.h, method, t0, dt, n, C.byref(te)))
        return te.value

    def try_step(self, t, dt):
        tt, dd, acc = C.c_double(t), C.c_double(dt), C.c_int()
        self._check(self.L.hode_try_step(self.h, C.byref(tt), C.byref(dd), C.byref(acc)))
        return tt.value, dd.value, bool(acc.value)

    def integrate_adaptive(self, t0, t1, dt0, max_steps=10 ** 9, allow=(EMAXSTEPS, EDT_UNDERFLOW, ENONFINITE)):
        st = hode_stats()
        self._check(self.L.hode_integrate_adaptive(self.h, t0, t1, dt0, max_steps, C.byref(st)), allow)
        return st.as_dict()

    def integrate_times(self, times, dt0, dst, max_steps=10 ** 9, allow=(EMAXSTEPS, EDT_UNDERFLOW, ENONFINITE)):
        """States at the given times into dst (numpy array or device tensor of
        len(times) * state elements); returns the summed stats."""
        arr = (C.c_double * len(times))(*[float(t) for t in times])
        p, nb, on_dev = _ptr_of(dst)
        st = hode_stats()
        self._check(self.L.hode_integrate_times(self.h, arr, len(times), dt0, max_steps, p, nb, on_dev, C.byref(st)),
                    allow)
        return st.as_dict()

    def integrate_dense_times(self, times, dt0, dst, max_steps=10 ** 9,
                              allow=(EMAXSTEPS, EDT_UNDERFLOW, ENONFINITE)):
        """Dopri5 dense output: the states at the given times into dst (as
        integrate_times), intermediate ones interpolated inside the free
        steps; returns the stats."""
        arr = (C.c_double * len(times))(*[float(t) for t in times])
        p, nb, on_dev = _ptr_of(dst)
        st = hode_stats()
        self._check(self.L.hode_integrate_times_dense(self.h, arr, len(times), dt0, max_steps, p, nb, on_dev,
                                                      C.byref(st)), allow)
        return st.as_dict()

    def get_ctrl(self):
        """Checkpoint of the step control (bytes of a hode_checkpoint)."""
        n = C.c_size_t(0)
        self._check(self.L.hode_get_ctrl(self.h, None, C.byref(n)))
        buf = (C.c_char * n.value)()
        self._check(self.L.hode_get_ctrl(self.h, buf, C.byref(n)))
        return bytes(buf)[: n.value]

    def set_ctrl(self, blob):
        buf = C.create_string_buffer(bytes(blob), len(blob))
        return self._check(self.L.hode_set_ctrl(self.h, buf, len(blob)))

    def get_stats(self):
        st = hode_stats()
        self._check(self.L.hode_get_stats(self.h, C.byref(st)))
        return st.as_dict()

    def set_trace(self, capacity):
        return self._check(self.L.hode_set_trace(self.h, capacity))

    def read_trace(self, cap=None):
        n = C.c_int64()
        self._check(self.L.hode_read_trace(self.h, None, 0, C.byref(n)))
        m = n.value if cap is None else min(cap, n.value)
        out = np.zeros((max(m, 1), TRACE_W))
        self._check(self.L.hode_read_trace(self.h, out.ctypes.data_as(C.c_void_p), m, C.byref(n)))
        return out[:m]

    def eval_rhs(self, dst):
        p, nb, on_dev = _ptr_of(dst)
        return self._check(self.L.hode_eval_rhs(self.h, p, nb, on_dev))

    def set_stepper(self, method):
        return self._check(self.L.hode_set_stepper(self.h, method))

    def set_graphs(self, enable):
        return self._check(self.L.hode_set_graphs(self.h, 1 if enable else 0))

    def set_tile(self, ry, zc):
        return self._check(self.L.hode_set_tile(self.h, ry, zc))

    def get_tile(self):
        a, b = C.c_int(), C.c_int()
        self._check(self.L.hode_get_tile(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def profile_attempt(self, method, reps):
        ms = (C.c_double * 16)()
        self._check(self.L.hode_profile_attempt(self.h, method, reps, ms))
        ns = 4 if method == RK4 else (13 if method == FEHLBERG78 else (1 if method > 10 else 6))
        return list(ms)[:ns]

    def autotune(self, method, reps=3):
        ry, zc, ms = C.c_int(), C.c_int(), C.c_double()
        self._check(self.L.hode_autotune(self.h, method, reps, C.byref(ry), C.byref(zc), C.byref(ms)))
        return ry.value, zc.value, ms.value

    def autotune_cached(self, method, reps=3, cache_path=None):
        """hode_autotune through a persistent cache file (cache_path, else
        $HODE_TUNE_CACHE); returns True when the tiles came from the file."""
        hit = C.c_int(0)
        p = None if cache_path is None else os.fsencode(str(cache_path))
        self._check(self.L.hode_autotune_cached(self.h, method, reps, p, C.byref(hit)))
        return bool(hit.value)

    def debug_poison(self):
        """Fills the library's scratch buffers with NaN (testing aid)."""
        return self._check(self.L.hode_debug_poison(self.h))

    def set_tile_waves(self, nw):
        """Wavefronts per workgroup of the Gray-Scott tiles (4 or 8)."""
        return self._check(self.L.hode_set_tile_waves(self.h, nw))

    def kind_tile(self, kind):
        """(ry, zc, nw) of one stage kind."""
        ry, zc, nw = C.c_int(), C.c_int(), C.c_int()
        self._check(self.L.hode_get_kind_tile(self.h, kind, C.byref(ry), C.byref(zc), C.byref(nw)))
        return ry.value, zc.value, nw.value

    def set_vector_width(self, vw):
        return self._check(self.L.hode_set_vector_width(self.h, vw))

    def time_kernel(self, kind, reps):
        ms = C.c_double()
        self._check(self.L.hode_time_kernel(self.h, kind, reps, C.byref(ms)))
        return ms.value


class Ensemble(Context):
    """An ensemble context (hode_ensemble_*): n Gray-Scott instances stepped by
    one persistent kernel."""

    def __init__(self, edges, params, dtype=F32, device=0, stream=None):
        self.L = lib()
        self.h = C.c_void_p()
        self.edges = [int(e) for e in edges]
        n = len(self.edges)
        e = (C.c_int64 * n)(*self.edges)
        flat = [float(v) for row in params for v in row]
        assert len(flat) == 5 * n
        p = (C.c_double * (5 * n))(*flat)
        self.dtype = dtype
        self._check(self.L.hode_ensemble_create(C.byref(self.h), device, C.c_void_p(stream) if stream else None,
                                                n, e, p, dtype))

    def __len__(self):
        return self.L.hode_ensemble_size(self.h)

    def init_instance(self, i, src):
        p, _, on_dev = _ptr_of(src)
        return self._check(self.L.hode_ensemble_init_state(self.h, i, p, on_dev))

    def read_instance(self, i, dst):
        p, nb, on_dev = _ptr_of(dst)
        return self._check(self.L.hode_ensemble_read_state(self.h, i, p, nb, on_dev))

    def set_weights(self, w):
        arr = (C.c_double * len(w))(*[float(v) for v in w])
        return self._check(self.L.hode_ensemble_set_weights(self.h, arr))

    def set_epoch(self, first, rest):
        return self._check(self.L.hode_ensemble_set_epoch(self.h, first, rest))

    def set_barrier_limit(self, polls):
        return self._check(self.L.hode_ensemble_set_barrier_limit(self.h, polls))

    def timing(self):
        """(summed kernel ms, launches) of the last integration."""
        ms, n = C.c_double(), C.c_int()
        self._check(self.L.hode_ensemble_timing(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def set_instance_vector_width(self, i, vw):
        return self._check(self.L.hode_ensemble_set_vector_width(self.h, i, vw))

    def set_trace(self, capacity):
        return self._check(self.L.hode_ensemble_set_trace(self.h, capacity))

    def set_plane_chunk(self, i, zc):
        return self._check(self.L.hode_ensemble_set_plane_chunk(self.h, i, zc))

    def instance_tile(self, i):
        """(vector width, planes per tile) of instance i."""
        vw, zc = C.c_int(), C.c_int()
        self._check(self.L.hode_ensemble_get_tile(self.h, i, C.byref(vw), C.byref(zc)))
        return vw.value, zc.value

    def read_instance_trace(self, i, cap=None):
        n = C.c_int64()
        self._check(self.L.hode_ensemble_read_trace(self.h, i, None, 0, C.byref(n)))
        m = n.value if cap is None else min(cap, n.value)
        out = np.zeros((max(m, 1), TRACE_W))
        self._check(self.L.hode_ensemble_read_trace(self.h, i, out.ctypes.data_as(C.c_void_p), m, C.byref(n)))
        return out[:m]

    def autotune(self, reps=3):
        n = len(self)
        vw = (C.c_int * n)()
        ms = (C.c_double * n)()
        self._check(self.L.hode_ensemble_autotune(self.h, reps, vw, ms))
        return list(vw), list(ms)

    def integrate_adaptive(self, t0, t1, dt0, max_steps=10 ** 9, allow=(EMAXSTEPS, EDT_UNDERFLOW, ENONFINITE)):
        n = len(self)
        st = (hode_stats * n)()
        self._check(self.L.hode_ensemble_integrate_adaptive(self.h, t0, t1, dt0, max_steps, st), allow)
        return [s.as_dict() for s in st]
