"""GPU parity: 3D periodic Gray-Scott stage kernels through the C ABI against
the FP64 oracle.  FP64: 1e-12 relative per field.  FP32 state (FP64 step
control): max-abs against the FP64 oracle from the FP32-rounded initial
condition, target 1e-4.  Also: every tile shape gives bitwise-identical
results, and a circular shift of the input gives the shifted output
bitwise."""
import numpy as np
import pytest

import oracle
from paper_2309_05331_amd import hode, inputs
from gpu_util import gs_ctx, read, rel_err_fields

pytestmark = pytest.mark.gpu

TOL64 = 1e-12   # same step sequence (fixed steps, or the oracle replaying the GPU's)
FREE64 = 1e-10  # free-running adaptive: step sizes differ by error-estimate rounding
TOL32_ABS = 1e-4
PRM = dict(Du=2e-5, Dv=1e-5, F=0.053, k=0.014, L=2.5)
# stronger diffusion so the stencil matters on short runs
PRM_D = dict(Du=2e-3, Dv=1e-3, F=0.053, k=0.014, L=2.5)


@pytest.mark.parametrize("N", [1, 2, 3, 5, 8, 33, 70])
def test_rhs_matches_oracle_tiny_and_ragged(orc, N):
    y0 = inputs.gray_scott_ic(N, seed=31)
    for prm in (PRM, PRM_D):
        ctx = gs_ctx(y0, N, prm)
        f = np.empty(2 * N ** 3)
        ctx.eval_rhs(f)
        o = orc.rhs(orc.gs_system(N, **prm), y0.ravel())
        scale = np.max(np.abs(o)) + 1e-300
        assert np.max(np.abs(f - o)) / scale <= 1e-13, N


@pytest.mark.parametrize("N,tile", [(5, (1, 8)), (33, (2, 8)), (33, (4, 5)), (70, (4, 16)), (70, (1, 70))])
def test_rk4_fp64_ragged_tiles(orc, N, tile):
    y0 = inputs.gray_scott_ic(N, seed=32)
    ctx = gs_ctx(y0, N, PRM_D, tile)
    ctx.integrate_n_steps(hode.RK4, 0.0, 0.1, 20)
    g = read(ctx, np.float64, 2 * N ** 3)
    o, _ = orc.integrate_n_steps(orc.gs_system(N, **PRM_D), orc.RK4, y0, 0.0, 0.1, 20)
    assert rel_err_fields(g, o, 2) <= TOL64


def test_rk4_fp64_32cube_500_steps(orc):
    # the small parity workload: 32^3, FP64, dt 0.1, 500 steps
    N = 32
    y0 = inputs.gray_scott_ic(N, seed=1)
    ctx = gs_ctx(y0, N, PRM)
    te = ctx.integrate_n_steps(hode.RK4, 0.0, 0.1, 500)
    assert te == pytest.approx(50.0)
    g = read(ctx, np.float64, 2 * N ** 3)
    o, _ = orc.integrate_n_steps(orc.gs_system(N, **PRM), orc.RK4, y0, 0.0, 0.1, 500)
    err = rel_err_fields(g, o, 2)
    # also the element-wise figure over cells whose value is not tiny
    big = np.abs(o) > 1e-6
    elem = float(np.max(np.abs(g - o)[big] / np.abs(o)[big]))
    print("32^3 FP64 RK4 x500 relative error vs oracle: %.3e per field, %.3e element-wise (|o| > 1e-6)"
          % (err, elem))
    assert err <= TOL64
    assert elem <= 1e-9


def test_dopri5_fixed_fp64(orc):
    N = 20
    y0 = inputs.gray_scott_ic(N, seed=33)
    ctx = gs_ctx(y0, N, PRM_D)
    ctx.integrate_n_steps(hode.DOPRI5, 0.0, 0.2, 30)
    g = read(ctx, np.float64, 2 * N ** 3)
    o, _ = orc.integrate_n_steps(orc.gs_system(N, **PRM_D), orc.DOPRI5, y0, 0.0, 0.2, 30)
    assert rel_err_fields(g, o, 2) <= TOL64


@pytest.mark.parametrize("N", [16, 37])
def test_dopri5_adaptive_fp64_free_and_replay(orc, N):
    y0 = inputs.gray_scott_ic(N, seed=34)
    ctx = gs_ctx(y0, N, PRM_D)
    ctx.set_tolerances(1e-6, 1e-6)
    ctx.set_trace(100000)
    st = ctx.integrate_adaptive(0.0, 60.0, 0.1, max_steps=200000)
    g = read(ctx, np.float64, 2 * N ** 3)
    tr = ctx.read_trace()
    sysd = orc.gs_system(N, **PRM_D)
    o, ost, otr = orc.integrate_adaptive(sysd, y0, 0.0, 60.0, 0.1, 1e-6, 1e-6, trace_cap=100000)
    assert st["status"] == 0 and st["t"] == 60.0
    assert (st["accepted"], st["rejected"]) == (ost["accepted"], ost["rejected"])
    assert rel_err_fields(g, o, 2) <= FREE64
    np.testing.assert_allclose(tr[:, 0], otr[:, 0], rtol=1e-5)
    r, _, errs = orc.integrate_replay(sysd, y0, 0.0, tr[:, 0], tr[:, 2].astype(np.int32), 1e-6, 1e-6)
    assert rel_err_fields(g, r, 2) <= TOL64
    derr = np.abs(tr[:, 1] - errs)
    print("32^3 FP64 free-running Dopri5: %d attempts, error-norm trace vs oracle replay: max |d err| %.3e, "
          "max relative %.3e" % (len(errs), derr.max(), float(np.max(derr / np.maximum(np.abs(errs), 1e-300)))))
    bad = derr > 1e-9 + 1e-6 * np.abs(errs)
    for i in np.nonzero(bad)[0][:10]:
        print("attempt %d h=%.6g acc=%d err gpu=%.12g oracle=%.12g" % (i, tr[i, 0], tr[i, 2], tr[i, 1], errs[i]))
    # Near the stability edge the error norm measures a tiny high-frequency
    # component (~1e-7 of the state, amplified by |E(z)| ~ 1): with the scale
    # atol + rtol |y| ~ 1e-6, state differences of ~1e-12 move the norm by
    # ~1e-6 absolute (measured on MI355X: max |d err| 1.108e-6 over 144
    # attempts, relative 2.8e-6); elsewhere it agrees far better.  The bar is
    # 4.5x the measured value.
    np.testing.assert_allclose(tr[:, 1], errs, rtol=1e-6, atol=5e-6)


def test_dopri5_adaptive_fp32_replay(orc):
    N = 32
    y0 = inputs.gray_scott_ic(N, seed=35)
    y32 = y0.astype(np.float32)
    ctx = gs_ctx(y32, N, PRM_D)
    ctx.set_trace(100000)
    st = ctx.integrate_adaptive(0.0, 100.0, 0.1, max_steps=200000)
    assert st["status"] == 0
    g = read(ctx, np.float32, 2 * N ** 3)
    tr = ctx.read_trace()
    r, _, _ = orc.integrate_replay(orc.gs_system(N, **PRM_D), y32.astype(np.float64), 0.0, tr[:, 0],
                                   tr[:, 2].astype(np.int32), 1e-6, 1e-6)
    err = np.max(np.abs(g.astype(np.float64) - r))
    print("32^3 FP32 Dopri5 adaptive max-abs vs FP64 oracle (replay): %.3e" % err)
    assert err <= TOL32_ABS


def test_rk4_fp32_maxabs(orc):
    N = 32
    y0 = inputs.gray_scott_ic(N, seed=1)
    y32 = y0.astype(np.float32)
    ctx = gs_ctx(y32, N, PRM)
    ctx.integrate_n_steps(hode.RK4, 0.0, 0.1, 500)
    g = read(ctx, np.float32, 2 * N ** 3)
    o, _ = orc.integrate_n_steps(orc.gs_system(N, **PRM), orc.RK4, y32.astype(np.float64), 0.0, 0.1, 500)
    err = np.max(np.abs(g - o))
    print("32^3 FP32 RK4 x500 max-abs vs FP64 oracle: %.3e" % err)
    assert err <= TOL32_ABS


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_tile_shapes_bitwise_identical(dtype):
    N = 48
    y0 = inputs.gray_scott_ic(N, seed=36).astype(dtype)
    outs = []
    for tile in [(1, 8), (2, 16), (4, 48), (4, 7), (1, 1)]:
        ctx = gs_ctx(y0, N, PRM_D, tile)
        ctx.set_trace(1000)
        ctx.integrate_adaptive(0.0, 10.0, 0.1, max_steps=200000)
        outs.append((read(ctx, dtype, 2 * N ** 3), ctx.read_trace()))
    for g, tr in outs[1:]:
        assert np.array_equal(g, outs[0][0])
        assert np.array_equal(tr, outs[0][1], equal_nan=True)


def test_shift_equivariance_bitwise():
    N = 40
    y0 = inputs.gray_scott_ic(N, seed=37).reshape(2, N, N, N)
    sh = (3, -7, 11)
    ctx = gs_ctx(y0, N, PRM_D)
    ctx.integrate_n_steps(hode.RK4, 0.0, 0.2, 10)
    a = read(ctx, np.float64, 2 * N ** 3).reshape(2, N, N, N)
    ctx = gs_ctx(np.roll(y0, sh, axis=(1, 2, 3)), N, PRM_D)
    ctx.integrate_n_steps(hode.RK4, 0.0, 0.2, 10)
    b = read(ctx, np.float64, 2 * N ** 3).reshape(2, N, N, N)
    assert np.array_equal(np.roll(a, sh, axis=(1, 2, 3)), b)


def test_full_size_256_fp32_one_step(orc):
    # 256^3 FP32 in the benchmark's launch configuration: one RK4 step and one
    # Dopri5 attempt against the FP64 oracle
    N = 256
    y32 = inputs.gray_scott_ic(N, seed=3, dtype=np.float32)
    y64 = y32.astype(np.float64).ravel()
    sysd = orc.gs_system(N, **PRM)
    ctx = gs_ctx(y32, N, PRM)
    ctx.do_step(hode.RK4, 0.0, 0.1)
    g = read(ctx, np.float32, 2 * N ** 3)
    o = orc.rk4_step(sysd, y64, 0.1)
    assert np.max(np.abs(g - o)) <= 1e-6
    ctx = gs_ctx(y32, N, PRM)
    ctx.do_step(hode.DOPRI5, 0.0, 0.5)
    g = read(ctx, np.float32, 2 * N ** 3)
    yn, _, e = orc.dopri5_attempt(sysd, y64, 0.5)
    assert np.max(np.abs(g - yn)) <= 1e-6
    # one controlled attempt takes the same accept decision as the oracle
    ctx = gs_ctx(y32, N, PRM)
    t, dt, acc = ctx.try_step(0.0, 0.5)
    err = orc.err_norm(y64, yn, e, 1e-6, 1e-6)
    assert acc == (err <= 1.0)


def test_graph_and_plain_launches_bitwise():
    # the same integration replayed from captured graph chunks and enqueued
    # kernel by kernel
    N = 24
    y0 = inputs.gray_scott_ic(N, seed=38)
    outs = []
    for graphs in (True, False):
        ctx = gs_ctx(y0, N, PRM_D)
        ctx.set_graphs(graphs)
        ctx.set_tolerances(1e-8, 1e-8)
        st = ctx.integrate_adaptive(0.0, 5.0, 0.1, max_steps=100000)
        ctx.integrate_n_steps(hode.RK4, st["t"], 0.05, 7)
        outs.append((read(ctx, np.float64, 2 * N ** 3), st["accepted"], st["rejected"]))
        ctx.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1:] == outs[1][1:]



@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_eight_wavefront_tiles_bitwise(dtype):
    # tiles of eight wavefronts (one or two rows each) give every stage kind's
    # results bitwise those of four-wavefront tiles: RK4 and free-running
    # Dopri5 on ragged grids (N = 76: one partial tile per row and a partial
    # last tile row; N = 300: two or three tiles per row, the last partial)
    # (the 300^3 grid takes the workload's diffusivities: with the stronger
    # ones its explicit stability limit is below the steps taken here)
    for N, prm in ((76, PRM_D), (300, PRM)):
        y0 = inputs.gray_scott_ic(N, seed=40, dtype=dtype)
        outs = []
        for nw, ry, zc in ((4, 1, N), (8, 1, 16), (8, 2, 24), (8, 1, N)):
            ctx = gs_ctx(y0, N, prm)
            ctx.set_tile_waves(nw)
            ctx.set_tile(ry, zc)
            for k in (hode.K_D2, hode.K_D6, hode.K_R4):
                assert ctx.kind_tile(k) == (ry, zc, nw)
            ctx.integrate_n_steps(hode.RK4, 0.0, 0.05, 3)
            st = ctx.integrate_adaptive(0.15, 1.0, 0.1)
            assert st["status"] == 0
            outs.append((read(ctx, dtype, 2 * N ** 3), st["accepted"], st["rejected"]))
            ctx.close()
        for o in outs[1:]:
            assert o[1:] == outs[0][1:] and np.array_equal(o[0], outs[0][0]), N
    # kinds without eight-wavefront tiles at a row count (Fehlberg: one-row
    # strips only; Adams-Bashforth: none) keep four, and a vector width other
    # than 16-byte lanes drops the others back to four
    y0 = inputs.gray_scott_ic(64, seed=41, dtype=np.float32)
    ctx = gs_ctx(y0, 64, PRM_D)
    ctx.set_tile_waves(8)
    ctx.set_tile(1, 64)
    assert ctx.kind_tile(hode.K_D6)[2] == 8 and ctx.kind_tile(hode.K_F[0])[2] == 8
    assert ctx.kind_tile(hode.K_AB[3])[2] == 4
    ctx.set_tile(2, 64)
    assert ctx.kind_tile(hode.K_D6)[2] == 8 and ctx.kind_tile(hode.K_F[0])[2] == 4
    ctx.set_vector_width(2)
    assert ctx.kind_tile(hode.K_D6)[2] == 4 and ctx.kind_tile(hode.K_F[0])[2] == 4
    with pytest.raises(hode.HodeError):
        ctx.set_tile_waves(16)
    ctx.close()
