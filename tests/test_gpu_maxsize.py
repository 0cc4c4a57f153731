"""GPU parity at maximum sizes: states past 2**31 elements, where any 32-bit
index, offset or launch-size computation on the path would wrap.

* Element-wise FP64, n = 2**31 + 4099 components (17 GB per array; a ragged
  tail for every vector width): fixed RK4 steps, then free-running adaptive
  Dopri5 replayed by the oracle, on sampled components (the components are
  independent, so the oracle integrates only the sampled ones).
* Gray-Scott FP32 on a 1300^3 grid: each field alone holds more than 2**31
  cells and the state 4.4e9 elements (17.6 GB per array, nine arrays for
  Dopri5); rows end in a ragged tile.  Fixed RK4 steps and adaptive Dopri5
  are checked on periodic windows around sampled cells (the windowing
  argument of the full-size tests), including cells on both sides of flat
  index 2**31 in field 0.

The inputs are drawn on the device by the torch version of the shared
counter-based generator (bitwise the host one, checked by the CPU tests and
here again at the sampled positions); the oracle's windows are drawn on the
host at the window cells only."""
import numpy as np
import pytest

from paper_2309_05331_amd import hode, inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32_ABS = 1e-4
PRM = [2e-5, 1e-5, 0.053, 0.014, 2.5]


@pytest.fixture
def torch_dev():
    import torch

    yield torch, torch.device("cuda:0")
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_max_size_elementwise_fp64_past_int32(orc, torch_dev):
    torch, dev = torch_dev
    n = (1 << 31) + 4099
    B = 1 << 31
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([
        np.arange(0, 6), np.arange(B - 4, B + 4), np.arange(n - 4105, n - 4095), np.arange(n - 6, n),
        rng.integers(0, n, size=16)]))
    x0 = inputs.exp_family_x0_torch(n, seed=21, device=dev)
    torch.cuda.synchronize()
    want0 = 0.01 + 0.49 * inputs.uniform_at(21, 0, idx)
    ti = torch.from_numpy(idx).to(dev)
    assert np.array_equal(x0[ti].cpu().numpy(), want0)
    out = torch.empty_like(x0)
    sysd = orc.ew_system(orc.LOGISTIC, idx.size)
    ctx = hode.Context(0)
    try:
        ctx.set_rhs(hode.RHS_LOGISTIC)
        ctx.init_state(x0)
        te = ctx.integrate_n_steps(hode.RK4, 0.0, 0.1, 3)
        assert te == pytest.approx(0.3)
        ctx.read_state(out)
        got = out[ti].cpu().numpy()
        want, _ = orc.integrate_n_steps(sysd, orc.RK4, want0, 0.0, 0.1, 3)
        rk4_err = float(np.max(np.abs(got - want) / np.abs(want)))
        print("n = %d RK4 x3: sampled relative error %.3e" % (n, rk4_err), flush=True)
        assert rk4_err <= TOL64

        ctx.init_state(x0)
        ctx.set_tolerances(1e-6, 1e-6)
        ctx.set_trace(256)
        st = ctx.integrate_adaptive(0.0, 1.0, 0.1, max_steps=256)
        assert st["status"] == 0 and st["t"] == 1.0
        tr = ctx.read_trace()
        ctx.read_state(out)
    finally:
        ctx.close()
    got = out[ti].cpu().numpy()
    r, te, errs = orc.integrate_replay(sysd, want0, 0.0, tr[:, 0], tr[:, 2].astype(np.int32), 1e-6, 1e-6)
    dp_err = float(np.max(np.abs(got - r) / np.abs(r)))
    print("n = %d Dopri5 adaptive (%d attempts): sampled relative error %.3e" % (n, len(tr), dp_err), flush=True)
    assert te == 1.0 and dp_err <= TOL64
    assert np.all(tr[:, 2] == (tr[:, 1] <= 1.0))
    # the sampled components' error norm bounds the global one from below
    assert np.all(tr[:, 1] >= errs * (1 - 1e-9))


def _max_samples(N):
    a, b, m = 3 * N // 8, 5 * N // 8 - 1, N // 2
    zb = (1 << 31) // (N * N)  # planes past zb hold field-0 cells with flat index >= 2**31
    pts = [(a, a, a), (b, b, b), (m, m, m), (0, 0, 0), (N - 1, N - 1, N - 1), (0, N - 1, N - 1),
           (zb, 0, 0), (zb, N - 1, N - 1), (zb + 1, m, 3), (N - 1, 0, N - 21), (a - 1, b + 1, N - 1)]
    rng = np.random.default_rng(11)
    pts += [tuple(int(v) for v in rng.integers(0, N, size=3)) for _ in range(4)]
    return pts


def _ic_window(N, seed, R, c):
    """(2, W, W, W) periodic window of edge 2R + 1 around cell c of the FP32
    initial condition, as float64."""
    ax = [np.arange(ci - R, ci + R + 1) % N for ci in c]
    z, y, x = np.meshgrid(*ax, indexing="ij")
    return np.stack([inputs.gray_scott_ic_at(N, seed, f, z, y, x).astype(np.float32) for f in (0, 1)]
                    ).astype(np.float64)


def test_max_size_grayscott_fp32_1300(orc, torch_dev):
    torch, dev = torch_dev
    N, seed = 1300, 9
    n3 = N ** 3
    assert n3 > 1 << 31
    pts = _max_samples(N)
    flat = np.array([[f * n3 + x + N * (y + N * z) for (z, y, x) in pts] for f in (0, 1)], dtype=np.int64)
    ti = torch.from_numpy(flat.ravel()).to(dev)
    ic = inputs.gray_scott_ic_torch(N, seed, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    want_ic = np.array([[inputs.gray_scott_ic_at(N, seed, f, z, y, x) for (z, y, x) in pts] for f in (0, 1)])
    assert np.array_equal(ic[ti].cpu().numpy().reshape(2, -1), want_ic.astype(np.float32))
    out = torch.empty_like(ic)
    ctx = hode.Context(0)
    try:
        ctx.set_rhs(hode.RHS_GRAYSCOTT3D, PRM)
        ctx.init_state(ic, grid=N)
        print("N = %d tile (ry, zc) = %s" % (N, ctx.get_tile()), flush=True)
        steps, dt = 2, 0.02
        ctx.integrate_n_steps(hode.RK4, 0.0, dt, steps)
        ctx.read_state(out)
        g_rk4 = out[ti].cpu().numpy().reshape(2, -1)
        ctx.init_state(ic, grid=N)
        ctx.set_tolerances(1e-6, 1e-6)
        ctx.set_trace(64)
        st = ctx.integrate_adaptive(0.0, 0.1, 0.02, max_steps=64)
        assert st["status"] == 0 and st["t"] == 0.1
        tr = ctx.read_trace()
        ctx.read_state(out)
        g_dp = out[ti].cpu().numpy().reshape(2, -1)
    finally:
        ctx.close()
    del ic, out

    R = 4 * steps + 1
    W = 2 * R + 1
    sysd = orc.gs_system(W, *PRM[:4], L=PRM[4] * W / N)
    ctr = np.array([0, 1]) * W ** 3 + (R * W + R) * W + R
    worst = 0.0
    for j, c in enumerate(pts):
        yw, _ = orc.integrate_n_steps(sysd, orc.RK4, _ic_window(N, seed, R, c).ravel(), 0.0, dt, steps)
        worst = max(worst, float(np.max(np.abs(g_rk4[:, j] - yw[ctr]))))
    print("%d^3 RK4 x%d sampled max-abs vs FP64 oracle %.3e" % (N, steps, worst), flush=True)
    assert worst <= TOL32_ABS

    hs, errs, acc = tr[:, 0], tr[:, 1], tr[:, 2].astype(bool)
    assert np.all(acc == (errs <= 1.0))
    R = 6 * int(acc.sum()) + 8
    W = 2 * R + 1
    sysd = orc.gs_system(W, *PRM[:4], L=PRM[4] * W / N)
    ctr = np.array([0, 1]) * W ** 3 + (R * W + R) * W + R
    worst = 0.0
    sampled = np.zeros(len(hs))
    for j, c in enumerate(pts):
        yw = _ic_window(N, seed, R, c).ravel()
        for a, h in enumerate(hs):
            yn, _, e = orc.dopri5_attempt(sysd, yw, h)
            sampled[a] = max(sampled[a], orc.err_norm(yw[ctr], yn[ctr], e[ctr], 1e-6, 1e-6))
            if acc[a]:
                yw = yn
        worst = max(worst, float(np.max(np.abs(g_dp[:, j] - yw[ctr]))))
    print("%d^3 Dopri5 adaptive (%d attempts) sampled max-abs vs FP64 oracle %.3e"
          % (N, len(hs), worst), flush=True)
    assert worst <= TOL32_ABS
    assert np.all(errs >= sampled - 1e-2)
