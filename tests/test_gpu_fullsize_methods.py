"""GPU parity at full size for the further steppers' benchmark workloads:
512^3 FP32 Gray-Scott with adaptive Cash-Karp 5(4), adaptive Fehlberg 7(8)
and fixed-step Adams-Bashforth 4, each in the benchmark's launch
configuration (the project autotuner's tiles for that method), on sampled
cells.

The windowing argument of the other full-size tests: a cell's value after E
right-hand-side evaluations depends only on cells within E grid steps, so
the FP64 oracle integrates the periodic window of edge 2R + 1 around each
sampled cell (R above the evaluations on the path to the result), replaying
the GPU's recorded (h, accepted) sequence for the adaptive pairs.  The
initial condition is drawn on the device by the torch form of the shared
generator and on the host only at the windows' cells."""
import numpy as np
import pytest

from paper_2309_05331_amd import hode, inputs

pytestmark = pytest.mark.gpu

TOL32_ABS = 1e-4
PRM = [2e-5, 1e-5, 0.053, 0.014, 2.5]
N, SEED = 512, 5


def _samples():
    a, b, m = 3 * N // 8, 5 * N // 8 - 1, N // 2
    pts = [(a, a, a), (b, b, b), (m, m, m), (a, m, b), (0, 0, 0), (N - 1, N - 1, N - 1), (0, N - 1, m),
           (a - 1, a, b + 1)]
    rng = np.random.default_rng(21)
    return pts + [tuple(int(v) for v in rng.integers(0, N, size=3)) for _ in range(2)]


def _window(R, c):
    ax = [np.arange(ci - R, ci + R + 1) % N for ci in c]
    z, y, x = np.meshgrid(*ax, indexing="ij")
    return np.stack([inputs.gray_scott_ic_at(N, SEED, f, z, y, x).astype(np.float32) for f in (0, 1)]
                    ).astype(np.float64).ravel()


def _gpu(method, adaptive, t1=None, dt=None, nsteps=None):
    import torch

    pts = _samples()
    flat = np.array([[f * N ** 3 + x + N * (y + N * z) for (z, y, x) in pts] for f in (0, 1)], dtype=np.int64)
    ti = torch.from_numpy(flat.ravel()).to("cuda:0")
    ic = inputs.gray_scott_ic_torch(N, SEED, dtype=torch.float32, device="cuda:0")
    torch.cuda.synchronize()
    ctx = hode.Context(0)
    try:
        ctx.set_rhs(hode.RHS_GRAYSCOTT3D, PRM)
        ctx.init_state(ic, grid=N)
        ctx.set_tolerances(1e-6, 1e-6)
        if adaptive:
            ctx.set_stepper(method)
        tile = ctx.autotune(method, 3)
        print("%s: autotuned tile (ry, zc) = (%d, %d)" % (method, tile[0], tile[1]), flush=True)
        trace = None
        if adaptive:
            ctx.set_trace(256)
            st = ctx.integrate_adaptive(0.0, t1, dt, max_steps=256)
            assert st["status"] == 0 and st["t"] == t1
            trace = ctx.read_trace()
        else:
            ctx.integrate_n_steps(method, 0.0, dt, nsteps)
        ctx.read_state(ic)
        g = ic[ti].cpu().numpy().reshape(2, -1).astype(np.float64)
    finally:
        ctx.close()
        del ic
        torch.cuda.empty_cache()
    return pts, g, trace


def _check_adaptive(orc, method, attempt, stages, t1):
    pts, g, tr = _gpu(method, True, t1=t1, dt=0.1)
    hs, errs, acc = tr[:, 0], tr[:, 1], tr[:, 2].astype(bool)
    assert np.all(acc == (errs <= 1.0))
    R = stages * int(acc.sum()) + stages + 1
    W = 2 * R + 1
    sysd = orc.gs_system(W, *PRM[:4], L=PRM[4] * W / N)
    ctr = np.array([0, 1]) * W ** 3 + (R * W + R) * W + R
    worst, sampled = 0.0, np.zeros(len(hs))
    for j, c in enumerate(pts):
        yw = _window(R, c)
        for a, h in enumerate(hs):
            yn, e = attempt(sysd, yw, h)
            sampled[a] = max(sampled[a], orc.err_norm(yw[ctr], yn[ctr], e[ctr], 1e-6, 1e-6))
            if acc[a]:
                yw = yn
        worst = max(worst, float(np.max(np.abs(g[:, j] - yw[ctr]))))
    print("512^3 %s adaptive (%d attempts): sampled max-abs vs FP64 oracle %.3e" % (method, len(hs), worst))
    assert worst <= TOL32_ABS
    return errs, sampled


def test_full_size_512_fp32_cashkarp_adaptive_sampled(orc):
    errs, sampled = _check_adaptive(orc, hode.CASHKARP54, orc.cashkarp_attempt, 6, 1.0)
    # the global norm bounds every sampled cell's ratio (FP32 stages perturb
    # a ratio by ~1e-3 at this tolerance)
    assert np.all(errs >= sampled - 1e-2)


def test_full_size_512_fp32_fehlberg78_adaptive_sampled(orc):
    # the Fehlberg estimate cancels four nearly equal stage values, so the
    # FP32 stages leave it too noisy to compare with a sampled bound; the
    # states are compared
    _check_adaptive(orc, hode.FEHLBERG78, orc.fehlberg78_attempt, 13, 0.2)


def test_full_size_512_fp32_adams_bashforth4_sampled(orc):
    steps, dt = 8, 0.025  # the benchmark's step; 3 Fehlberg start-up steps, then 5 Adams-Bashforth steps
    pts, g, _ = _gpu(hode.AB(4), False, dt=dt, nsteps=steps)
    R = 13 * 3 + (steps - 3) + 1
    W = 2 * R + 1
    sysd = orc.gs_system(W, *PRM[:4], L=PRM[4] * W / N)
    ctr = np.array([0, 1]) * W ** 3 + (R * W + R) * W + R
    worst = 0.0
    for j, c in enumerate(pts):
        yw, _ = orc.integrate_n_steps(sysd, orc.AB(4), _window(R, c), 0.0, dt, steps)
        worst = max(worst, float(np.max(np.abs(g[:, j] - yw[ctr]))))
    print("512^3 AB4 x%d sampled max-abs vs FP64 oracle %.3e" % (steps, worst))
    assert worst <= TOL32_ABS
