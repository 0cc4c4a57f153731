"""GPU: checkpoint and resume of the step control through the C ABI
(hode_get_ctrl / hode_set_ctrl).  A sequence of controlled attempts split by
a checkpoint, restored into a fresh context with the saved state, equals the
unsplit sequence bitwise (PI and the learned controller, whose history the
checkpoint carries); malformed blobs are refused."""
import os

import numpy as np
import pytest

from paper_2309_05331_amd import hode, inputs
from gpu_util import gs_ctx, read

pytestmark = pytest.mark.gpu

PRM_D = dict(Du=2e-3, Dv=1e-3, F=0.053, k=0.014, L=2.5)
WEIGHTS = os.path.join(os.path.dirname(hode.__file__), "controller_weights.npy")


def _attempts(ctx, t, dt, n):
    for _ in range(n):
        t, dt, _ = ctx.try_step(t, dt)
    return t, dt


@pytest.mark.parametrize("ctrl", ["pi", "learned"])
def test_try_step_sequence_resumes_bitwise(ctrl):
    N = 20
    y0 = inputs.gray_scott_ic(N, seed=95)

    def make(y):
        ctx = gs_ctx(y, N, PRM_D)
        ctx.set_tolerances(1e-7, 1e-7)
        if ctrl == "learned":
            ctx.set_controller(hode.CTRL_MLP, np.load(WEIGHTS))
        return ctx

    a = make(y0)
    ta, dta = _attempts(a, 0.0, 0.1, 30)
    ya = read(a, np.float64, 2 * N ** 3)
    a.close()
    b = make(y0)
    tb, dtb = _attempts(b, 0.0, 0.1, 12)
    blob = b.get_ctrl()
    yb = read(b, np.float64, 2 * N ** 3)
    b.close()
    import struct
    magic, version, t_ck, dt_ck = struct.unpack_from("<IIdd", blob)
    assert magic == 0x48434B50 and version == 1 and (t_ck, dt_ck) == (tb, dtb)
    c = make(yb)
    c.set_ctrl(blob)
    tc, dtc = _attempts(c, t_ck, dt_ck, 18)
    yc = read(c, np.float64, 2 * N ** 3)
    assert np.array_equal(yc, ya) and (tc, dtc) == (ta, dta)
    c.close()


def test_checkpoint_checks():
    N = 8
    ctx = gs_ctx(inputs.gray_scott_ic(N, seed=96), N, PRM_D)
    with pytest.raises(hode.HodeError):
        ctx.get_ctrl()  # nothing to checkpoint yet
    ctx.try_step(0.0, 0.1)
    blob = ctx.get_ctrl()
    with pytest.raises(hode.HodeError):
        ctx.set_ctrl(blob[:-8])
    bad = bytearray(blob)
    bad[0] ^= 0xFF
    with pytest.raises(hode.HodeError):
        ctx.set_ctrl(bytes(bad))
    ctx.set_ctrl(blob)
    ctx.close()
