"""GPU: the allocation-free training step (hode_mlp_train_step_noalloc),
called through the C ABI, against hode_mlp_train_step with caller-owned
gradient and scratch buffers: two calls in a row from the same start, the
second with a smaller minibatch (a ragged tail of the 64-sample tiles and a
different index set), so a gradient or loss sum left over from the first
call in the shared scratch would show.

Both paths run the same kernels; the gradient is summed across workgroups
with fp32 atomics whose order varies from run to run, so the comparison
allows that rounding: the loss to 1e-9 relative, Adam's moments to 1e-4
relative (norm), the master weights to 1e-3 of one learning-rate step
(max-abs), and the bf16 copy to one bf16 ulp where the master weight sits
within that tolerance of a rounding boundary."""
import ctypes as C

import numpy as np
import pytest

from paper_2309_05331_amd import controller, hode

pytestmark = pytest.mark.gpu


def _dev(t, a, dtype):
    return t.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def _p(x):
    return C.c_void_p(x.data_ptr())


def test_noalloc_train_step_matches_workspace_entry_point():
    import torch as t
    L = hode.lib()
    rng = np.random.default_rng(7)
    nrows = 6000
    X = _dev(t, rng.normal(size=(nrows, 16)).astype(np.float32), t.float32)
    T = _dev(t, rng.normal(scale=0.5, size=nrows).astype(np.float32), t.float32)
    W = _dev(t, rng.uniform(0.5, 2.0, size=nrows).astype(np.float32), t.float32)
    p0 = controller.init_params(seed=3)
    lr = 2e-3
    # warm Adam's moments with one ordinary step so the update direction is a
    # smooth function of the gradient (at step 1 it is sign(g))
    Wm = _dev(t, p0, t.float32)
    Wb = t.zeros(hode.MLP_NPARAM, dtype=t.int16, device="cuda:0")
    m, v, g = t.zeros_like(Wm), t.zeros_like(Wm), t.zeros_like(Wm)
    acc = t.zeros(2, dtype=t.float64, device="cuda:0")
    assert L.hode_mlp_quantize(_p(Wm), _p(Wb), None) == 0
    loss = C.c_double()
    assert L.hode_mlp_train_step(_p(X), _p(T), _p(W), None, nrows, _p(Wm), _p(Wb), _p(m), _p(v), _p(g), _p(acc),
                                 1, C.c_float(lr), C.byref(loss), None) == 0
    for call, B in enumerate((4096, 1000)):
        idx = _dev(t, rng.permutation(nrows)[:B].astype(np.int64), t.int64)
        ref = [x.clone() for x in (Wm, Wb, m, v)]
        new = [x.clone() for x in (Wm, Wb, m, v)]
        lr_ref, lr_new = C.c_double(), C.c_double()
        assert L.hode_mlp_train_step(_p(X), _p(T), _p(W), _p(idx), B, _p(ref[0]), _p(ref[1]), _p(ref[2]),
                                     _p(ref[3]), _p(g), _p(acc), 2, C.c_float(lr), C.byref(lr_ref), None) == 0
        assert L.hode_mlp_train_step_noalloc(_p(X), _p(T), _p(W), _p(idx), B, _p(new[0]), _p(new[1]), _p(new[2]),
                                             _p(new[3]), 2, C.c_float(lr), C.byref(lr_new), None) == 0
        t.cuda.synchronize()
        a = [x.cpu().numpy() for x in ref]
        b = [x.cpu().numpy() for x in new]
        dl = abs(lr_new.value - lr_ref.value) / abs(lr_ref.value)
        dm = np.linalg.norm(b[2] - a[2]) / np.linalg.norm(a[2])
        dv = np.linalg.norm(b[3] - a[3]) / np.linalg.norm(a[3])
        dw = float(np.max(np.abs(b[0] - a[0])))
        print("call %d (B=%d): loss %.9g vs %.9g (rel %.2e); m rel %.2e, v rel %.2e, Wm max-abs %.2e"
              % (call, B, lr_new.value, lr_ref.value, dl, dm, dv, dw), flush=True)
        assert np.isfinite(lr_new.value) and dl <= 1e-9
        assert dm <= 1e-4 and dv <= 1e-4
        assert dw <= 1e-3 * lr
        # the bf16 copy is the rounding of the master weights
        qb = b[1].view(np.uint16).astype(np.int64)
        qa = a[1].view(np.uint16).astype(np.int64)
        assert np.all(np.abs(qb - qa) <= 1)
    # argument checks: sizes outside 1 .. HODE_MLP_NOALLOC_MAX_B are refused
    for bad in (0, -1, 2 ** 31):
        assert L.hode_mlp_train_step_noalloc(_p(X), _p(T), _p(W), None, bad, _p(Wm), _p(Wb), _p(m), _p(v), 2,
                                             C.c_float(lr), C.byref(loss), None) == hode.EINVAL
