"""GPU parity of the Cash-Karp 5(4) stepper (the paper's Table 1 error
stepper, the second embedded pair next to Dopri5) through the C ABI against
the FP64 oracle: fixed steps and adaptive runs (free-running counts and the
oracle replaying the GPU's step sequence) on the element-wise families and
on 3D Gray-Scott; FP32 state against the oracle replay (max-abs 1e-4); and
switching steppers on one context keeps every result consistent."""
import numpy as np
import pytest

from paper_2309_05331_amd import hode, inputs
from gpu_util import ew_ctx, gs_ctx, read, rel_err, rel_err_fields

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
FREE64 = 1e-10
TOL32_ABS = 1e-4
PRM = dict(Du=2e-5, Dv=1e-5, F=0.053, k=0.014, L=2.5)
PRM_D = dict(Du=2e-3, Dv=1e-3, F=0.053, k=0.014, L=2.5)


@pytest.mark.parametrize("kind", [hode.RHS_EXP, hode.RHS_LOGISTIC])
@pytest.mark.parametrize("n", [1, 1000, 100003])
def test_fixed_steps_fp64_elementwise(orc, kind, n):
    x0 = inputs.exp_family_x0(n, seed=41)
    ctx = ew_ctx(kind, x0)
    ctx.integrate_n_steps(hode.CASHKARP54, 0.0, 0.05, 100)
    g = read(ctx, np.float64, n)
    o, _ = orc.integrate_n_steps(orc.ew_system(kind, n), orc.CASHKARP, x0, 0.0, 0.05, 100)
    assert rel_err(g, o) <= TOL64, rel_err(g, o)
    st = ctx.get_stats()
    assert st["accepted"] == 100 and st["rhs_evals"] == 600
    ctx.close()


@pytest.mark.parametrize("kind", [hode.RHS_EXP, hode.RHS_LOGISTIC])
def test_adaptive_fp64_elementwise_free_and_replay(orc, kind):
    n = 100003
    x0 = inputs.exp_family_x0(n, seed=2)
    ctx = ew_ctx(kind, x0)
    ctx.set_stepper(hode.CASHKARP54)
    ctx.set_tolerances(1e-6, 1e-6)
    ctx.set_trace(10000)
    st = ctx.integrate_adaptive(0.0, 5.0, 0.01, max_steps=200000)
    g = read(ctx, np.float64, n)
    tr = ctx.read_trace()
    sysd = orc.ew_system(kind, n)
    o, ost, otr = orc.integrate_adaptive(sysd, x0, 0.0, 5.0, 0.01, 1e-6, 1e-6, trace_cap=10000,
                                         method=orc.CASHKARP)
    assert (st["accepted"], st["rejected"]) == (ost["accepted"], ost["rejected"])
    assert st["t"] == 5.0 and st["status"] == 0
    assert st["rhs_evals"] == 6 * (st["accepted"] + st["rejected"])  # no first-same-as-last
    assert rel_err(g, o) <= FREE64
    r, te, errs = orc.integrate_replay(sysd, x0, 0.0, tr[:, 0], tr[:, 2].astype(np.int32), 1e-6, 1e-6,
                                       method=orc.CASHKARP)
    assert rel_err(g, r) <= TOL64
    np.testing.assert_allclose(tr[:, 1], errs, rtol=1e-6, atol=1e-9)
    ctx.close()


@pytest.mark.parametrize("N", [5, 24, 33])
def test_fixed_steps_fp64_grayscott(orc, N):
    y0 = inputs.gray_scott_ic(N, seed=42)
    ctx = gs_ctx(y0, N, PRM_D)
    ctx.integrate_n_steps(hode.CASHKARP54, 0.0, 0.2, 15)
    g = read(ctx, np.float64, 2 * N ** 3)
    o, _ = orc.integrate_n_steps(orc.gs_system(N, **PRM_D), orc.CASHKARP, y0.ravel(), 0.0, 0.2, 15)
    assert rel_err_fields(g, o, 2) <= TOL64
    ctx.close()


@pytest.mark.parametrize("N", [16, 37])
def test_adaptive_fp64_grayscott_free_and_replay(orc, N):
    y0 = inputs.gray_scott_ic(N, seed=43)
    ctx = gs_ctx(y0, N, PRM_D)
    ctx.set_stepper(hode.CASHKARP54)
    ctx.set_tolerances(1e-7, 1e-7)
    ctx.set_trace(100000)
    st = ctx.integrate_adaptive(0.0, 20.0, 0.1, max_steps=100000)
    assert st["status"] == 0 and st["t"] == 20.0
    g = read(ctx, np.float64, 2 * N ** 3)
    tr = ctx.read_trace()
    sysd = orc.gs_system(N, **PRM_D)
    r, te, errs = orc.integrate_replay(sysd, y0.ravel(), 0.0, tr[:, 0], tr[:, 2].astype(np.int32), 1e-7, 1e-7,
                                       method=orc.CASHKARP)
    assert abs(te - 20.0) < 1e-9
    assert rel_err_fields(g, r, 2) <= TOL64
    o, ost, _ = orc.integrate_adaptive(sysd, y0.ravel(), 0.0, 20.0, 0.1, 1e-7, 1e-7, method=orc.CASHKARP)
    assert (st["accepted"], st["rejected"]) == (ost["accepted"], ost["rejected"])
    assert rel_err_fields(g, o, 2) <= FREE64
    ctx.close()


def test_adaptive_fp32_grayscott_replay(orc):
    N = 32
    y32 = inputs.gray_scott_ic(N, seed=1, dtype=np.float32)
    ctx = gs_ctx(y32, N, PRM)
    ctx.set_stepper(hode.CASHKARP54)
    ctx.set_trace(100000)
    st = ctx.integrate_adaptive(0.0, 30.0, 0.1, max_steps=100000)
    assert st["status"] == 0 and st["t"] == 30.0
    g = read(ctx, np.float32, 2 * N ** 3)
    tr = ctx.read_trace()
    r, _, _ = orc.integrate_replay(orc.gs_system(N, **PRM), y32.astype(np.float64).ravel(), 0.0, tr[:, 0],
                                   tr[:, 2].astype(np.int32), method=orc.CASHKARP)
    err = np.max(np.abs(g.astype(np.float64) - r))
    print("32^3 FP32 Cash-Karp adaptive max-abs vs FP64 oracle (replay): %.3e" % err)
    assert err <= TOL32_ABS
    ctx.close()


def test_stepper_switches_stay_consistent(orc):
    # Dopri5 adaptive, RK4 fixed, Cash-Karp adaptive, Dopri5 again on one
    # context: the first-same-as-last k1 must be recomputed whenever another
    # stepper moved the state
    N = 20
    y0 = inputs.gray_scott_ic(N, seed=44)
    sysd = orc.gs_system(N, **PRM_D)
    ctx = gs_ctx(y0, N, PRM_D)
    ctx.set_tolerances(1e-8, 1e-8)
    y = y0.ravel().copy()
    st = ctx.integrate_adaptive(0.0, 2.0, 0.1, max_steps=100000)
    y, ost, _ = orc.integrate_adaptive(sysd, y, 0.0, 2.0, 0.1, 1e-8, 1e-8)
    assert (st["accepted"], st["rejected"]) == (ost["accepted"], ost["rejected"])
    ctx.integrate_n_steps(hode.RK4, 2.0, 0.1, 5)
    y, _ = orc.integrate_n_steps(sysd, orc.RK4, y, 2.0, 0.1, 5)
    ctx.set_stepper(hode.CASHKARP54)
    st = ctx.integrate_adaptive(2.5, 4.0, 0.1, max_steps=100000)
    y, ost, _ = orc.integrate_adaptive(sysd, y, 2.5, 4.0, 0.1, 1e-8, 1e-8, method=orc.CASHKARP)
    assert (st["accepted"], st["rejected"]) == (ost["accepted"], ost["rejected"])
    ctx.set_stepper(hode.DOPRI5)
    st = ctx.integrate_adaptive(4.0, 6.0, 0.1, max_steps=100000)
    y, ost, _ = orc.integrate_adaptive(sysd, y, 4.0, 6.0, 0.1, 1e-8, 1e-8)
    assert (st["accepted"], st["rejected"]) == (ost["accepted"], ost["rejected"])
    g = read(ctx, np.float64, 2 * N ** 3)
    assert rel_err_fields(g, y, 2) <= FREE64
    with pytest.raises(hode.HodeError):
        ctx.set_stepper(hode.RK4)
    ctx.close()
