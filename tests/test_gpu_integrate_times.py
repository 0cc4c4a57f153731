"""GPU: integrate_times (Odeint's observer at requested times) through the C
ABI against the FP64 oracle's integrate_times: the recorded states, the
summed counts, host and device destinations, both embedded pairs, and the
argument checks."""
import numpy as np
import pytest
import torch

from paper_2309_05331_amd import hode, inputs
from gpu_util import ew_ctx, gs_ctx, rel_err, rel_err_fields

pytestmark = pytest.mark.gpu

FREE64 = 1e-10
PRM_D = dict(Du=2e-3, Dv=1e-3, F=0.053, k=0.014, L=2.5)
TIMES = [0.0, 0.37, 1.0, 2.5, 2.51, 5.0]


@pytest.mark.parametrize("stepper,om", [(hode.DOPRI5, 2), (hode.CASHKARP54, 3)])
@pytest.mark.parametrize("kind", [hode.RHS_EXP, hode.RHS_LOGISTIC])
def test_elementwise_times_match_oracle(orc, stepper, om, kind):
    n = 20011
    x0 = inputs.exp_family_x0(n, seed=61)
    ctx = ew_ctx(kind, x0)
    ctx.set_stepper(stepper)
    ctx.set_tolerances(1e-8, 1e-8)
    dst = np.zeros((len(TIMES), n))
    st = ctx.integrate_times(TIMES, 0.01, dst)
    out, ost = orc.integrate_times(orc.ew_system(kind, n), x0, TIMES, 0.01, 1e-8, 1e-8, method=om)
    assert st["status"] == 0 and st["t"] == 5.0
    assert (st["accepted"], st["rejected"], st["rhs_evals"]) == (ost["accepted"], ost["rejected"], ost["rhs_evals"])
    assert np.array_equal(dst[0], x0)
    for i in range(len(TIMES)):
        assert rel_err(dst[i], out[i]) <= FREE64, i
    ctx.close()


def test_grayscott_times_device_destination(orc):
    N = 12
    y0 = inputs.gray_scott_ic(N, seed=62)
    ctx = gs_ctx(y0, N, PRM_D)
    ctx.set_tolerances(1e-8, 1e-8)
    dst = torch.zeros(len(TIMES) * 2 * N ** 3, dtype=torch.float64, device="cuda:0")
    st = ctx.integrate_times(TIMES, 0.1, dst)
    got = dst.cpu().numpy().reshape(len(TIMES), -1)
    out, ost = orc.integrate_times(orc.gs_system(N, **PRM_D), y0.ravel(), TIMES, 0.1, 1e-8, 1e-8)
    assert (st["accepted"], st["rejected"]) == (ost["accepted"], ost["rejected"])
    for i in range(len(TIMES)):
        assert rel_err_fields(got[i], out[i], 2) <= FREE64, i
    # the context continues from the last observation
    final = np.empty(2 * N ** 3)
    ctx.read_state(final)
    assert np.array_equal(final, got[-1])
    ctx.close()


def test_times_argument_checks():
    x0 = inputs.exp_family_x0(64, seed=63)
    ctx = ew_ctx(hode.RHS_EXP, x0)
    with pytest.raises(hode.HodeError):
        ctx.integrate_times([0.0, 1.0, 1.0], 0.01, np.zeros((3, 64)))
    with pytest.raises(hode.HodeError):
        ctx.integrate_times([0.0, 1.0, 2.0], 0.01, np.zeros((2, 64)))
    st = ctx.integrate_times([0.0, 1.0, 2.0], 0.01, np.zeros((3, 64)), max_steps=3)
    assert st["status"] == hode.EMAXSTEPS and st["accepted"] + st["rejected"] == 3
    ctx.close()
