"""GPU parity of Runge-Kutta-Fehlberg 7(8) and the Adams-Bashforth methods of
1 to 8 steps (the paper's Table 1; its multi-step accuracy test) through the C
ABI against the FP64 oracle: fixed steps, adaptive Fehlberg runs (free-running
counts and the oracle replaying the GPU's steps), element-wise and 3D
Gray-Scott, FP64 and FP32; the Adams-Bashforth history across calls; tile
independence of the new stencil kernels; and the argument checks."""
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


# Adams-Bashforth parity runs keep h * lambda_max <= 0.01, inside every
# method's real stability interval (AB8: 0.0244, the narrowest): outside it
# the parasitic roots amplify the rounding-order differences of any two
# implementations step after step.
def _dt_ab(N, prm):
    lam = 12.0 * max(prm["Du"], prm["Dv"]) / (prm["L"] / N) ** 2 + 1.0
    return 0.01 / lam


def _ab_evals(s, n):
    m = min(n, s - 1)
    return 13 * m + (n - m)


@pytest.mark.parametrize("kind", [hode.RHS_EXP, hode.RHS_LOGISTIC])
@pytest.mark.parametrize("n", [1, 1000, 100003])
def test_fehlberg_fixed_fp64_elementwise(orc, kind, n):
    x0 = inputs.exp_family_x0(n, seed=71)
    ctx = ew_ctx(kind, x0)
    ctx.integrate_n_steps(hode.FEHLBERG78, 0.0, 0.1, 50)
    g = read(ctx, np.float64, n)
    o, _ = orc.integrate_n_steps(orc.ew_system(kind, n), orc.FEHLBERG78, x0, 0.0, 0.1, 50)
    assert rel_err(g, o) <= TOL64, rel_err(g, o)
    st = ctx.get_stats()
    assert st["accepted"] == 50 and st["rhs_evals"] == 13 * 50
    ctx.close()


@pytest.mark.parametrize("kind", [hode.RHS_EXP, hode.RHS_LOGISTIC])
@pytest.mark.parametrize("steps", range(1, 9))
def test_adams_bashforth_fp64_elementwise(orc, kind, steps):
    n = 40009
    x0 = inputs.exp_family_x0(n, seed=72)
    ctx = ew_ctx(kind, x0)
    ctx.integrate_n_steps(hode.AB(steps), 0.0, 0.01, 100)  # |f'| <= 1
    g = read(ctx, np.float64, n)
    o, _, ev = orc.integrate_n_steps(orc.ew_system(kind, n), orc.AB(steps), x0, 0.0, 0.01, 100, evals=True)
    assert rel_err(g, o) <= TOL64, rel_err(g, o)
    st = ctx.get_stats()
    assert st["accepted"] == 100 and st["rhs_evals"] == ev == _ab_evals(steps, 100)
    ctx.close()


@pytest.mark.parametrize("kind", [hode.RHS_EXP, hode.RHS_LOGISTIC])
def test_fehlberg_adaptive_fp64_elementwise_free_and_replay(orc, kind):
    n = 100003
    x0 = inputs.exp_family_x0(n, seed=2)
    ctx = ew_ctx(kind, x0)
    ctx.set_stepper(hode.FEHLBERG78)
    ctx.set_tolerances(1e-10, 1e-10)
    ctx.set_trace(10000)
    st = ctx.integrate_adaptive(0.0, 5.0, 0.01, max_steps=200000)
    g = read(ctx, np.float64, n)
    tr = ctx.read_trace()
    sysd = orc.ew_system(kind, n)
    o, ost, _ = orc.integrate_adaptive(sysd, x0, 0.0, 5.0, 0.01, 1e-10, 1e-10, method=orc.FEHLBERG78)
    assert (st["accepted"], st["rejected"]) == (ost["accepted"], ost["rejected"])
    assert st["t"] == 5.0 and st["status"] == 0 and st["accepted"] > 5
    assert st["rhs_evals"] == 13 * (st["accepted"] + st["rejected"])
    assert rel_err(g, o) <= FREE64
    r, te, errs = orc.integrate_replay(sysd, x0, 0.0, tr[:, 0], tr[:, 2].astype(np.int32), 1e-10, 1e-10,
                                       method=orc.FEHLBERG78)
    assert rel_err(g, r) <= TOL64
    # the estimate h 41/840 (k12 + k13 - k1 - k11) cancels four nearly equal
    # stage values: its rounding, 4 eps h 41/840 |k| / (rtol |x|), is ~1e-7
    # in units of the tolerance at rtol = 1e-10, whatever the summation order
    np.testing.assert_allclose(tr[:, 1], errs, rtol=1e-6, atol=1e-6)
    ctx.close()


@pytest.mark.parametrize("N", [5, 24, 33, 97])
def test_fehlberg_fixed_fp64_grayscott(orc, N):
    y0 = inputs.gray_scott_ic(N, seed=73)
    ctx = gs_ctx(y0, N, PRM_D)
    steps = 3 if N == 97 else 8
    dt = min(0.2, 200 * _dt_ab(N, PRM_D))  # h * lambda_max <= 2, inside the stability region
    ctx.integrate_n_steps(hode.FEHLBERG78, 0.0, dt, steps)
    g = read(ctx, np.float64, 2 * N ** 3)
    o, _ = orc.integrate_n_steps(orc.gs_system(N, **PRM_D), orc.FEHLBERG78, y0.ravel(), 0.0, dt, steps)
    assert np.all(np.isfinite(o))
    assert rel_err_fields(g, o, 2) <= TOL64
    ctx.close()


@pytest.mark.parametrize("N", [12, 33, 97])
@pytest.mark.parametrize("steps", [1, 2, 5, 8])
def test_adams_bashforth_fp64_grayscott(orc, N, steps):
    y0 = inputs.gray_scott_ic(N, seed=74)
    ctx = gs_ctx(y0, N, PRM_D)
    n = 12 if N == 97 else 30
    dt = _dt_ab(N, PRM_D)
    ctx.integrate_n_steps(hode.AB(steps), 0.0, dt, n)
    g = read(ctx, np.float64, 2 * N ** 3)
    o, _, ev = orc.integrate_n_steps(orc.gs_system(N, **PRM_D), orc.AB(steps), y0.ravel(), 0.0, dt, n,
                                     evals=True)
    assert rel_err_fields(g, o, 2) <= TOL64
    assert ctx.get_stats()["rhs_evals"] == ev
    ctx.close()


@pytest.mark.parametrize("N", [16, 37])
def test_fehlberg_adaptive_fp64_grayscott_free_and_replay(orc, N):
    y0 = inputs.gray_scott_ic(N, seed=75)
    ctx = gs_ctx(y0, N, PRM_D)
    ctx.set_stepper(hode.FEHLBERG78)
    ctx.set_tolerances(1e-9, 1e-9)
    ctx.set_trace(100000)
    st = ctx.integrate_adaptive(0.0, 10.0, 0.1, max_steps=100000)
    assert st["status"] == 0 and st["t"] == 10.0
    g = read(ctx, np.float64, 2 * N ** 3)
    tr = ctx.read_trace()
    sysd = orc.gs_system(N, **PRM_D)
    r, te, _ = orc.integrate_replay(sysd, y0.ravel(), 0.0, tr[:, 0], tr[:, 2].astype(np.int32), 1e-9, 1e-9,
                                    method=orc.FEHLBERG78)
    assert abs(te - 10.0) < 1e-9
    assert rel_err_fields(g, r, 2) <= TOL64
    o, ost, _ = orc.integrate_adaptive(sysd, y0.ravel(), 0.0, 10.0, 0.1, 1e-9, 1e-9, method=orc.FEHLBERG78)
    assert (st["accepted"], st["rejected"]) == (ost["accepted"], ost["rejected"])
    assert rel_err_fields(g, o, 2) <= FREE64
    ctx.close()


def test_fp32_grayscott_fehlberg_replay_and_ab8(orc):
    N = 32
    y32 = inputs.gray_scott_ic(N, seed=1, dtype=np.float32)
    y64 = y32.astype(np.float64).ravel()
    sysd = orc.gs_system(N, **PRM)
    ctx = gs_ctx(y32, N, PRM)
    ctx.set_stepper(hode.FEHLBERG78)
    ctx.set_trace(100000)
    st = ctx.integrate_adaptive(0.0, 30.0, 0.1, max_steps=100000)
    assert st["status"] == 0 and st["t"] == 30.0
    g = read(ctx, np.float32, 2 * N ** 3)
    tr = ctx.read_trace()
    r, _, _ = orc.integrate_replay(sysd, y64, 0.0, tr[:, 0], tr[:, 2].astype(np.int32), method=orc.FEHLBERG78)
    err = np.max(np.abs(g.astype(np.float64) - r))
    print("32^3 FP32 Fehlberg 7(8) adaptive max-abs vs FP64 oracle (replay): %.3e" % err)
    assert err <= TOL32_ABS
    ctx.close()
    ctx = gs_ctx(y32, N, PRM)
    dt = _dt_ab(N, PRM)
    ctx.integrate_n_steps(hode.AB(8), 0.0, dt, 200)
    g = read(ctx, np.float32, 2 * N ** 3)
    o, _ = orc.integrate_n_steps(sysd, orc.AB(8), y64, 0.0, dt, 200)
    err = np.max(np.abs(g.astype(np.float64) - o))
    print("32^3 FP32 Adams-Bashforth 8 x200 max-abs vs FP64 oracle: %.3e" % err)
    assert err <= TOL32_ABS
    ctx.close()


@pytest.mark.parametrize("gs", [False, True])
def test_adams_bashforth_history_across_calls(orc, gs):
    # n steps in several calls equal n in one (bitwise), the start-up may span
    # calls; a new dt or another stepper starts a fresh history
    if gs:
        N = 20
        y0 = inputs.gray_scott_ic(N, seed=76).ravel()
        sysd = orc.gs_system(N, **PRM_D)
        make = lambda: gs_ctx(y0, N, PRM_D)
        h1 = _dt_ab(N, PRM_D) / 2
    else:
        y0 = inputs.exp_family_x0(5003, seed=76)
        sysd = orc.ew_system(orc.LOGISTIC, y0.size)
        make = lambda: ew_ctx(hode.RHS_LOGISTIC, y0)
        h1 = 0.005
    h2 = 2 * h1
    for s in (4, 8):
        one = make()
        one.integrate_n_steps(hode.AB(s), 0.0, h1, 20)
        want = read(one, np.float64, y0.size)
        one.close()
        split = make()
        t = 0.0
        for m in (3, 1, 9, 7):
            split.integrate_n_steps(hode.AB(s), t, h1, m)
            t += m * h1
        got = read(split, np.float64, y0.size)
        assert np.array_equal(got, want), s
        assert split.get_stats()["rhs_evals"] == 7  # the last call: AB steps only
        # a new step size restarts from the current state
        split.integrate_n_steps(hode.AB(s), t, h2, 10)
        o, _ = orc.integrate_n_steps(sysd, orc.AB(s), want, t, h2, 10)
        assert rel_err(read(split, np.float64, y0.size), o) <= TOL64
        # so does another stepper in between
        cur = read(split, np.float64, y0.size)
        split.integrate_n_steps(hode.RK4, t, h1, 1)
        cur, _ = orc.integrate_n_steps(sysd, orc.RK4, cur, t, h1, 1)
        split.integrate_n_steps(hode.AB(s), t, h2, 10)
        o, _ = orc.integrate_n_steps(sysd, orc.AB(s), cur, t, h2, 10)
        assert rel_err(read(split, np.float64, y0.size), o) <= TOL64
        split.close()


@pytest.mark.parametrize("method", ["F78", "AB8", "AB3"])
def test_new_stencil_kernels_tile_independent(orc, method):
    # every tile shape, eight-wavefront Fehlberg tiles included (N = 44: a
    # ragged last row of eight-row tiles), gives bitwise the same steps
    N = 44
    y0 = inputs.gray_scott_ic(N, seed=77)
    ref = None
    m = hode.FEHLBERG78 if method == "F78" else hode.AB(int(method[2]))
    for tile in (None, (1, 8), (2, 16), (4, 44), (1, 13), (1, 16, 8), (1, 44, 8)):
        ctx = gs_ctx(y0, N, PRM_D, tile=tile[:2] if tile else None)
        if tile and len(tile) == 3:
            ctx.set_tile_waves(tile[2])
            ctx.set_tile(tile[0], tile[1])
            if method == "F78":
                assert ctx.kind_tile(hode.K_F[12])[2] == 8
        ctx.integrate_n_steps(m, 0.0, 0.01, 12)
        g = read(ctx, np.float64, 2 * N ** 3)
        ctx.close()
        if ref is None:
            ref = g
        assert np.array_equal(g, ref), tile


def test_fehlberg_integrate_times_and_checks(orc):
    # Fehlberg's estimate h 41/840 (k12 + k13 - k1 - k11) of the first, tiny
    # steps lies below the FP64 resolution of the stage values (error norms
    # ~1e-9 of the tolerance), so the controller grows the step from rounding
    # noise and two correct implementations follow step sequences that differ
    # at ~1e-3 relative (the replay test above pins the stepper itself to
    # 1e-12).  Checked here: the closed forms at every requested time, the
    # single-interval call equal to integrate_adaptive bitwise, and the step
    # count within one step per interval of the oracle's.
    x0 = inputs.exp_family_x0(4097, seed=78)
    times = [0.0, 0.37, 1.0, 2.5, 5.0]
    ctx = ew_ctx(hode.RHS_EXP, x0)
    ctx.set_stepper(hode.FEHLBERG78)
    ctx.set_tolerances(1e-9, 1e-9)
    dst = np.zeros((len(times), x0.size))
    st = ctx.integrate_times(times, 0.01, dst)
    assert st["status"] == 0 and st["t"] == 5.0
    _, ost = orc.integrate_times(orc.ew_system(orc.EXP, x0.size), x0, times, 0.01, 1e-9, 1e-9,
                                 method=orc.FEHLBERG78)
    assert abs(st["accepted"] - ost["accepted"]) <= len(times) - 1 and st["rejected"] == ost["rejected"] == 0
    for i, t in enumerate(times):
        exact = x0 * np.exp(t)
        assert np.max(np.abs(dst[i] - exact) / (1 + np.abs(exact))) < 30e-9, t
    one = np.zeros((2, x0.size))
    ctx.init_state(x0)
    st1 = ctx.integrate_times([0.0, 5.0], 0.01, one)
    ctx.init_state(x0)
    st2 = ctx.integrate_adaptive(0.0, 5.0, 0.01)
    assert np.array_equal(one[1], read(ctx, np.float64, x0.size)) and st1["accepted"] == st2["accepted"]
    # the learned controller serves the 5(4) pairs only
    w = np.zeros(hode.MLP_NPARAM, dtype=np.uint16)
    ctx.set_controller(hode.CTRL_MLP, w)
    with pytest.raises(hode.HodeError):
        ctx.integrate_adaptive(0.0, 1.0, 0.01)
    ctx.set_controller(hode.CTRL_PI)
    with pytest.raises(ValueError):
        hode.AB(9)
    with pytest.raises(hode.HodeError):
        ctx.integrate_n_steps(19, 0.0, 0.1, 1)
    ctx.close()


def test_time_and_profile_new_kinds():
    N = 64
    y0 = inputs.gray_scott_ic(N, seed=79, dtype=np.float32)
    ctx = gs_ctx(y0, N, PRM)
    for k in hode.K_F + [hode.K_F13F] + hode.K_AB:
        assert ctx.time_kernel(k, 2) > 0
    ms = ctx.profile_attempt(hode.FEHLBERG78, 2)
    assert len(ms) == 13 and min(ms) > 0
    ry, zc, tot = ctx.autotune(hode.AB(8), 1)
    assert ry in (1, 2, 4) and tot > 0
    ctx.close()


# ------------------------------------------- Adams-Bashforth-Moulton (PECE)

@pytest.mark.parametrize("kind", [hode.RHS_EXP, hode.RHS_LOGISTIC])
@pytest.mark.parametrize("steps", range(1, 9))
def test_abm_fp64_elementwise(orc, kind, steps):
    n = 40009
    x0 = inputs.exp_family_x0(n, seed=85)
    ctx = ew_ctx(kind, x0)
    ctx.integrate_n_steps(hode.ABM(steps), 0.0, 0.01, 100)
    g = read(ctx, np.float64, n)
    o, _, ev = orc.integrate_n_steps(orc.ew_system(kind, n), orc.ABM(steps), x0, 0.0, 0.01, 100, evals=True)
    assert rel_err(g, o) <= TOL64, rel_err(g, o)
    st = ctx.get_stats()
    assert st["accepted"] == 100 and st["rhs_evals"] == ev
    ctx.close()


@pytest.mark.parametrize("N", [12, 33])
@pytest.mark.parametrize("steps", [1, 2, 5, 8])
def test_abm_fp64_grayscott(orc, N, steps):
    y0 = inputs.gray_scott_ic(N, seed=86)
    ctx = gs_ctx(y0, N, PRM_D)
    dt = _dt_ab(N, PRM_D)
    ctx.integrate_n_steps(hode.ABM(steps), 0.0, dt, 30)
    g = read(ctx, np.float64, 2 * N ** 3)
    o, _, ev = orc.integrate_n_steps(orc.gs_system(N, **PRM_D), orc.ABM(steps), y0.ravel(), 0.0, dt, 30,
                                     evals=True)
    assert rel_err_fields(g, o, 2) <= TOL64
    assert ctx.get_stats()["rhs_evals"] == ev
    ctx.close()


@pytest.mark.parametrize("gs", [False, True])
def test_abm_history_and_switches(orc, gs):
    if gs:
        N = 20
        y0 = inputs.gray_scott_ic(N, seed=87).ravel()
        sysd = orc.gs_system(N, **PRM_D)
        make = lambda: gs_ctx(y0, N, PRM_D)
        h = _dt_ab(N, PRM_D)
    else:
        y0 = inputs.exp_family_x0(5003, seed=87)
        sysd = orc.ew_system(orc.LOGISTIC, y0.size)
        make = lambda: ew_ctx(hode.RHS_LOGISTIC, y0)
        h = 0.01
    for s in (3, 8):
        one = make()
        one.integrate_n_steps(hode.ABM(s), 0.0, h, 20)
        want = read(one, np.float64, y0.size)
        one.close()
        split = make()
        t = 0.0
        for m in (2, 6, 5, 7):
            split.integrate_n_steps(hode.ABM(s), t, h, m)
            t += m * h
        assert np.array_equal(read(split, np.float64, y0.size), want), s
        # Adams-Bashforth with the same s and dt is another method: a fresh history
        split.integrate_n_steps(hode.AB(s), t, h, 10)
        o, _ = orc.integrate_n_steps(sysd, orc.AB(s), want, t, h, 10)
        assert rel_err(read(split, np.float64, y0.size), o) <= TOL64
        split.close()


def test_abm_tile_independent_and_fp32(orc):
    N = 40
    y0 = inputs.gray_scott_ic(N, seed=88)
    ref = None
    for tile in (None, (1, 8), (2, 16), (4, 40)):
        ctx = gs_ctx(y0, N, PRM_D, tile=tile)
        ctx.integrate_n_steps(hode.ABM(8), 0.0, 0.001, 12)
        g = read(ctx, np.float64, 2 * N ** 3)
        ctx.close()
        if ref is None:
            ref = g
        assert np.array_equal(g, ref), tile
    N = 32
    y32 = inputs.gray_scott_ic(N, seed=1, dtype=np.float32)
    ctx = gs_ctx(y32, N, PRM)
    dt = _dt_ab(N, PRM)
    ctx.integrate_n_steps(hode.ABM(8), 0.0, dt, 200)
    g = read(ctx, np.float32, 2 * N ** 3)
    o, _ = orc.integrate_n_steps(orc.gs_system(N, **PRM), orc.ABM(8), y32.astype(np.float64).ravel(), 0.0, dt, 200)
    err = np.max(np.abs(g.astype(np.float64) - o))
    print("32^3 FP32 Adams-Bashforth-Moulton 8 x200 max-abs vs FP64 oracle: %.3e" % err)
    assert err <= TOL32_ABS
    ctx.close()
