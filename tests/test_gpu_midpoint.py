"""GPU parity of the modified midpoint method (the paper's Table 1, Gragg's
two-substep form) through the C ABI against the FP64 oracle: element-wise
and 3D Gray-Scott, FP64 and FP32, tile independence of its three stencil
kernels."""
import numpy as np
import pytest

from paper_2309_05331_amd import hode, inputs
from gpu_util import ew_ctx, gs_ctx, read, rel_err, rel_err_fields

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
PRM = dict(Du=2e-5, Dv=1e-5, F=0.053, k=0.014, L=2.5)
PRM_D = dict(Du=2e-3, Dv=1e-3, F=0.053, k=0.014, L=2.5)


@pytest.mark.parametrize("kind", [hode.RHS_EXP, hode.RHS_LOGISTIC])
@pytest.mark.parametrize("n", [1, 1000, 100003])
def test_midpoint_fp64_elementwise(orc, kind, n):
    x0 = inputs.exp_family_x0(n, seed=91)
    ctx = ew_ctx(kind, x0)
    ctx.integrate_n_steps(hode.MIDPOINT, 0.0, 0.05, 100)
    g = read(ctx, np.float64, n)
    o, _, ev = orc.integrate_n_steps(orc.ew_system(kind, n), orc.MIDPOINT, x0, 0.0, 0.05, 100, evals=True)
    assert rel_err(g, o) <= TOL64, rel_err(g, o)
    st = ctx.get_stats()
    assert st["accepted"] == 100 and st["rhs_evals"] == ev == 300
    ctx.close()


@pytest.mark.parametrize("N", [5, 24, 33])
def test_midpoint_fp64_grayscott(orc, N):
    y0 = inputs.gray_scott_ic(N, seed=92)
    ctx = gs_ctx(y0, N, PRM_D)
    ctx.integrate_n_steps(hode.MIDPOINT, 0.0, 0.1, 20)
    g = read(ctx, np.float64, 2 * N ** 3)
    o, _ = orc.integrate_n_steps(orc.gs_system(N, **PRM_D), orc.MIDPOINT, y0.ravel(), 0.0, 0.1, 20)
    assert rel_err_fields(g, o, 2) <= TOL64
    ctx.close()


def test_midpoint_tiles_and_fp32(orc):
    N = 40
    y0 = inputs.gray_scott_ic(N, seed=93)
    ref = None
    for tile in (None, (1, 8), (2, 16), (4, 40)):
        ctx = gs_ctx(y0, N, PRM_D, tile=tile)
        ctx.integrate_n_steps(hode.MIDPOINT, 0.0, 0.05, 10)
        g = read(ctx, np.float64, 2 * N ** 3)
        ctx.close()
        if ref is None:
            ref = g
        assert np.array_equal(g, ref), tile
    N = 32
    y32 = inputs.gray_scott_ic(N, seed=1, dtype=np.float32)
    ctx = gs_ctx(y32, N, PRM)
    ctx.integrate_n_steps(hode.MIDPOINT, 0.0, 0.1, 100)
    g = read(ctx, np.float32, 2 * N ** 3)
    o, _ = orc.integrate_n_steps(orc.gs_system(N, **PRM), orc.MIDPOINT, y32.astype(np.float64).ravel(), 0.0, 0.1, 100)
    err = np.max(np.abs(g.astype(np.float64) - o))
    print("32^3 FP32 modified midpoint x100 max-abs vs FP64 oracle: %.3e" % err)
    assert err <= 1e-4
    for k in hode.K_MM:
        assert ctx.time_kernel(k, 2) > 0
    ctx.close()
