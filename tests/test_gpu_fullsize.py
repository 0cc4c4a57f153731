"""GPU parity at the benchmark's full sizes and launch configuration (the
tile the project autotuner picks), on sampled cells.

A 7-point stencil moves information one cell per right-hand-side
evaluation, so a cell's value after E evaluations depends only on the cells
within E grid steps of it.  For each sampled cell the FP64 oracle integrates
the periodic window of edge 2R + 1 centred on it (R at least the number of
evaluations), with the domain length scaled so the grid spacing is that of
the full grid: the window's wrapped faces are wrong, but the error moves
inward one cell per evaluation and never reaches the centre.  The oracle
replays the GPU's recorded (h, accepted) sequence; the GPU's state at the
sampled cells must match the window centres, every sampled cell's error
ratio is a lower bound of the GPU's global error norm, and each accept
decision follows from that norm."""
import numpy as np
import pytest

from paper_2309_05331_amd import hode, inputs

pytestmark = pytest.mark.gpu

PRM = [2e-5, 1e-5, 0.053, 0.014, 2.5]
TOL32_ABS = 1e-4


def _samples(N, extra, seed=0):
    """Cube corners and faces, the domain's corners (wrap-around), the centre
    and a few seeded random cells, as (z, y, x)."""
    a, b, m = 3 * N // 8, 5 * N // 8 - 1, N // 2
    pts = [(a, a, a), (b, b, b), (a, b, a), (b, a, b), (a, m, m), (m, m, b), (m, a, m), (m, m, m),
           (0, 0, 0), (N - 1, N - 1, N - 1), (0, N - 1, m), (m, 0, N - 1), (a - 1, a, b + 1)]
    rng = np.random.default_rng(seed)
    pts += [tuple(int(v) for v in rng.integers(0, N, size=3)) for _ in range(extra)]
    return pts


def _window(y, N, R, c):
    """The (2, W, W, W) periodic window of edge W = 2R + 1 centred on cell c."""
    idx = [np.arange(ci - R, ci + R + 1) % N for ci in c]
    return y[:, idx[0]][:, :, idx[1]][:, :, :, idx[2]]


def _run(N, seed, method, t1=None, dt=None, nsteps=None):
    y32 = inputs.gray_scott_ic(N, seed=seed, dtype=np.float32)
    ctx = hode.Context(0)
    ctx.set_rhs(hode.RHS_GRAYSCOTT3D, PRM)
    ctx.init_state(y32.ravel(), grid=N)
    ctx.set_tolerances(1e-6, 1e-6)
    tile = ctx.autotune(method, 3)
    print("N=%d autotuned tile (ry, zc) = (%d, %d)" % (N, tile[0], tile[1]), flush=True)
    trace = None
    if method == hode.DOPRI5:
        ctx.set_trace(256)
        st = ctx.integrate_adaptive(0.0, t1, dt, max_steps=256)
        assert st["status"] == 0 and st["t"] == t1
        trace = ctx.read_trace()
    else:
        ctx.integrate_n_steps(hode.RK4, 0.0, dt, nsteps)
    out = np.empty(2 * N ** 3, dtype=np.float32)
    ctx.read_state(out)
    ctx.close()
    return y32, out.reshape(2, N, N, N), trace


def test_full_size_512_fp32_dopri5_adaptive_sampled(orc):
    N = 512
    y32, g, trace = _run(N, 5, hode.DOPRI5, t1=1.0, dt=0.1)
    hs, errs, acc = trace[:, 0], trace[:, 1], trace[:, 2].astype(bool)
    print("attempts %d accepted %d" % (len(hs), acc.sum()), flush=True)
    assert np.all(acc == (errs <= 1.0))
    # k1 = f(y), then 6 evaluations per attempt; the last attempt's error needs k7
    R = 6 * int(acc.sum()) + 8
    W = 2 * R + 1
    sysd = orc.gs_system(W, *PRM[:4], L=PRM[4] * W / N)
    ctr = np.array([0, 1]) * W ** 3 + (R * W + R) * W + R
    worst = 0.0
    sampled_err = np.zeros(len(hs))
    for c in _samples(N, 8):
        yw = _window(y32, N, R, c).astype(np.float64).ravel()
        for j, h in enumerate(hs):
            yn, _, e = orc.dopri5_attempt(sysd, yw, h)
            sampled_err[j] = max(sampled_err[j], orc.err_norm(yw[ctr], yn[ctr], e[ctr], 1e-6, 1e-6))
            if acc[j]:
                yw = yn
        d = np.max(np.abs(g[:, c[0], c[1], c[2]] - yw[ctr]))
        worst = max(worst, d)
    print("512^3 sampled max-abs vs FP64 oracle %.3e; GPU err norms %s; sampled lower bounds %s"
          % (worst, np.array2string(errs, precision=4), np.array2string(sampled_err, precision=4)))
    assert worst <= TOL32_ABS
    # the global L-inf norm bounds every sampled cell's ratio (FP32 stages
    # perturb a ratio by ~1e-3 at these tolerances)
    assert np.all(errs >= sampled_err - 1e-2)


def test_full_size_256_fp32_rk4_sampled(orc):
    N, steps = 256, 10
    y32, g, _ = _run(N, 3, hode.RK4, dt=0.1, nsteps=steps)
    R = 4 * steps + 1
    W = 2 * R + 1
    sysd = orc.gs_system(W, *PRM[:4], L=PRM[4] * W / N)
    ctr = np.array([0, 1]) * W ** 3 + (R * W + R) * W + R
    worst = 0.0
    for c in _samples(N, 8, seed=1):
        yw = _window(y32, N, R, c).astype(np.float64).ravel()
        yw, _ = orc.integrate_n_steps(sysd, orc.RK4, yw, 0.0, 0.1, steps)
        worst = max(worst, np.max(np.abs(g[:, c[0], c[1], c[2]] - yw[ctr])))
    print("256^3 RK4 x%d sampled max-abs vs FP64 oracle %.3e" % (steps, worst))
    assert worst <= TOL32_ABS
