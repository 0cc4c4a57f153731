"""GPU: the streaming-copy reference (the bandwidth ceiling and counter
calibration beside the benchmark) copies exactly and checks its arguments on
the host; the state size query."""
import numpy as np
import pytest

from paper_2309_05331_amd import hode, inputs
from gpu_util import ew_ctx, gs_ctx

pytestmark = pytest.mark.gpu


def test_stream_copy_is_exact_and_checks_arguments():
    import ctypes as C
    import torch

    n = (1 << 22) + 12  # 16-byte elements: a ragged last block of the 1024-element grid
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (4 * n,), dtype=torch.int32, device="cuda:0")
    dst = torch.zeros_like(src)
    torch.cuda.synchronize()
    ms, gbs = hode.stream_copy(dst, src, reps=3)
    assert ms > 0 and gbs > 0
    assert torch.equal(dst, src)
    L, out = hode.lib(), C.c_double()
    p, q = C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr())
    assert L.hode_stream_copy(p, q, 8, 1, C.byref(out)) == hode.EINVAL          # not a multiple of 16
    assert L.hode_stream_copy(p, q, 64, 0, C.byref(out)) == hode.EINVAL         # reps < 1
    assert L.hode_stream_copy(None, q, 64, 1, C.byref(out)) == hode.EINVAL      # null pointer
    assert L.hode_stream_copy(C.c_void_p(dst.data_ptr() + 4), q, 64, 1, C.byref(out)) == hode.EINVAL  # misaligned
    assert L.hode_stream_copy(p, q, 64, 1, None) == hode.EINVAL


def test_state_bytes():
    ctx = hode.Context(0)
    assert ctx.state_bytes() == 0
    ctx.close()
    N = 12
    ctx = gs_ctx(inputs.gray_scott_ic(N, seed=3, dtype=np.float32), N)
    assert ctx.state_bytes() == 2 * N ** 3 * 4
    ctx.close()
    ctx = ew_ctx(hode.RHS_EXP, inputs.exp_family_x0(1001, seed=3))
    assert ctx.state_bytes() == 1001 * 8
    ctx.close()
