"""GPU parity of explicit Euler (the first stepper of the paper's Table 1)
through the C ABI against the FP64 oracle: fixed steps on the element-wise
families and on 3D Gray-Scott, FP64 within 1e-12 relative, FP32 within the
max-abs bound."""
import numpy as np
import pytest

from paper_2309_05331_amd import hode, inputs
from gpu_util import ew_ctx, gs_ctx, read, rel_err, rel_err_fields

pytestmark = pytest.mark.gpu

PRM_D = dict(Du=2e-3, Dv=1e-3, F=0.053, k=0.014, L=2.5)


@pytest.mark.parametrize("kind", [hode.RHS_EXP, hode.RHS_LOGISTIC])
@pytest.mark.parametrize("n", [1, 1000, 100003])
def test_euler_elementwise_fp64(orc, kind, n):
    x0 = inputs.exp_family_x0(n, seed=51)
    ctx = ew_ctx(kind, x0)
    ctx.integrate_n_steps(hode.EULER, 0.0, 0.01, 500)
    g = read(ctx, np.float64, n)
    o, _ = orc.integrate_n_steps(orc.ew_system(kind, n), orc.EULER, x0, 0.0, 0.01, 500)
    assert rel_err(g, o) <= 1e-12
    st = ctx.get_stats()
    assert st["accepted"] == 500 and st["rhs_evals"] == 500
    ctx.close()


@pytest.mark.parametrize("N", [5, 24])
def test_euler_grayscott_fp64_and_fp32(orc, N):
    y0 = inputs.gray_scott_ic(N, seed=52)
    ctx = gs_ctx(y0, N, PRM_D)
    ctx.integrate_n_steps(hode.EULER, 0.0, 0.05, 40)
    g = read(ctx, np.float64, 2 * N ** 3)
    sysd = orc.gs_system(N, **PRM_D)
    o, _ = orc.integrate_n_steps(sysd, orc.EULER, y0.ravel(), 0.0, 0.05, 40)
    assert rel_err_fields(g, o, 2) <= 1e-12
    ctx.close()
    y32 = y0.astype(np.float32)
    ctx = gs_ctx(y32, N, PRM_D)
    ctx.integrate_n_steps(hode.EULER, 0.0, 0.05, 40)
    g = read(ctx, np.float32, 2 * N ** 3)
    o, _ = orc.integrate_n_steps(sysd, orc.EULER, y32.astype(np.float64).ravel(), 0.0, 0.05, 40)
    assert np.max(np.abs(g - o)) <= 1e-4
    ctx.close()
