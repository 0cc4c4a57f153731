"""GPU: the batched ensemble (one persistent kernel stepping many Gray-Scott
instances, each with its own adaptive Dopri5 control).  Every instance must
equal, bitwise, the same instance integrated alone through the single-grid
path; FP64 instances must match the oracle replaying their step sequence to
1e-12 relative."""
import numpy as np
import pytest

import oracle
from paper_2309_05331_amd import hode, inputs
from gpu_util import rel_err_fields

pytestmark = pytest.mark.gpu


def _params(n, Du=2e-3, Dv=1e-3, seed=4):
    edges, F, k = inputs.ensemble_draws(n, seed=seed)
    return edges, [[Du, Dv, F[i], k[i], 2.5] for i in range(n)]


def _single(y0, N, prm, vw, t1, dt0, tol):
    ctx = hode.Context(0)
    ctx.set_rhs(hode.RHS_GRAYSCOTT3D, prm)
    ctx.init_state(np.ascontiguousarray(y0).ravel(), grid=N)
    ctx.set_tile(1, max(1, N // 2))
    ctx.set_vector_width(vw)
    ctx.set_tolerances(tol, tol)
    st = ctx.integrate_adaptive(0.0, t1, dt0, max_steps=100000)
    out = np.empty(2 * N ** 3, dtype=y0.dtype)
    ctx.read_state(out)
    ctx.close()
    return out, st


def _run_ensemble(edges, prms, dtype, t1, tol, vws=None, weights=None, trace=0):
    npd = np.float32 if dtype == hode.F32 else np.float64
    ens = hode.Ensemble(edges, prms, dtype=dtype)
    ys = []
    for i, N in enumerate(edges):
        y = inputs.ensemble_ic(i, N, dtype=npd)
        ys.append(y)
        ens.init_instance(i, np.ascontiguousarray(y).ravel())
        if vws:
            ens.set_instance_vector_width(i, vws[i])
    if weights is not None:
        ens.set_weights(weights)
    if trace:
        ens.set_trace(trace)
    ens.set_tolerances(tol, tol)
    stats = ens.integrate_adaptive(0.0, t1, 0.1, max_steps=100000)
    outs = []
    for i, N in enumerate(edges):
        o = np.empty(2 * N ** 3, dtype=npd)
        ens.read_instance(i, o)
        outs.append(o)
    return ens, ys, outs, stats


@pytest.mark.parametrize("dtype", [hode.F32, hode.F64])
def test_ensemble_matches_single_runs_bitwise(dtype):
    edges = [8, 16, 24, 32, 12, 20, 40]
    _, prms = _params(len(edges))
    vws = [1, 2, 1, 2, 4 if dtype == hode.F32 else 2, 2, 1]
    ens, ys, outs, stats = _run_ensemble(edges, prms, dtype, 30.0, 1e-5, vws=vws)
    for i, N in enumerate(edges):
        assert stats[i]["status"] == 0 and stats[i]["t"] == 30.0
        ref, st = _single(ys[i], N, prms[i], vws[i], 30.0, 0.1, 1e-5)
        assert (stats[i]["accepted"], stats[i]["rejected"]) == (st["accepted"], st["rejected"]), i
        assert np.array_equal(outs[i], ref), i
    ens.close()


@pytest.mark.parametrize("dtype", [hode.F32, hode.F64])
def test_ensemble_every_segment_count_bitwise(dtype):
    # 16-byte lanes: rows of nl lanes are packed into as many segments of a
    # wavefront as hold one (64/seg >= nl): seg 2, 3, 4, 5, 6, 8, 10 and 16,
    # where seg 3, 5, 6 and 10 leave lanes of the wavefront over
    vf = 4 if dtype == hode.F32 else 2
    nls = [24, 18, 14, 12, 10, 8, 6, 4]  # -> seg 2, 3, 4, 5, 6, 8, 10, 16
    edges = [vf * nl for nl in nls]
    if dtype == hode.F64:
        edges += [vf * 21, vf * 11, vf * 5]  # the widest rows of seg 3, 5 and 10
    _, prms = _params(len(edges))
    vws = [vf] * len(edges)
    ens, ys, outs, stats = _run_ensemble(edges, prms, dtype, 12.0, 1e-5, vws=vws)
    for i, N in enumerate(edges):
        assert stats[i]["status"] == 0 and stats[i]["t"] == 12.0
        ref, st = _single(ys[i], N, prms[i], 1, 12.0, 0.1, 1e-5)
        assert (stats[i]["accepted"], stats[i]["rejected"]) == (st["accepted"], st["rejected"]), i
        assert np.array_equal(outs[i], ref), (i, N)
    ens.close()


def test_ensemble_paused_launches_bitwise():
    # a few attempts per launch, so every instance is paused and resumed many
    # times (resumed instances skip stage 1: k1 is in the first-same-as-last
    # slot); work estimates that put the big instances in one queue
    edges = [48, 64, 16, 8, 33]
    _, prms = _params(len(edges))
    vws = [4, 4, 4, 4, 1]
    npd = np.float32
    ens = hode.Ensemble(edges, prms, dtype=hode.F32)
    ys = [inputs.ensemble_ic(i, N, dtype=npd) for i, N in enumerate(edges)]
    for i, N in enumerate(edges):
        ens.init_instance(i, np.ascontiguousarray(ys[i]).ravel())
        ens.set_instance_vector_width(i, vws[i])
    ens.set_weights([1e9, 1e9, 1.0, 1.0, 1.0])
    ens.set_epoch(3, 5)
    ens.set_tolerances(1e-5, 1e-5)
    stats = ens.integrate_adaptive(0.0, 20.0, 0.1, max_steps=100000)
    ms, launches = ens.timing()
    most = max(s["accepted"] + s["rejected"] for s in stats)
    assert launches == 1 + -(-(most - 3) // 5) and ms > 0
    for i, N in enumerate(edges):
        out = np.empty(2 * N ** 3, dtype=npd)
        ens.read_instance(i, out)
        ref, st = _single(ys[i], N, prms[i], vws[i], 20.0, 0.1, 1e-5)
        assert (stats[i]["accepted"], stats[i]["rejected"]) == (st["accepted"], st["rejected"]), i
        assert stats[i]["rhs_evals"] == st["rhs_evals"], i
        assert np.array_equal(out, ref), i
    ens.close()


def test_ensemble_rejects_bad_epoch():
    ens = hode.Ensemble([8], [[2e-3, 1e-3, 0.04, 0.06, 2.5]])
    with pytest.raises(hode.HodeError):
        ens.set_epoch(0, 5)
    with pytest.raises(hode.HodeError):
        ens.set_epoch(3, 5000)
    ens.set_epoch(0, 0)  # one launch for the whole integration (the default)
    with pytest.raises(hode.HodeError):
        ens.set_plane_chunk(0, -1)
    ens.close()


def test_ensemble_one_launch_and_tuned_tiles_bitwise():
    # by default the whole integration is one persistent launch (re-tiling on
    # the device as instances finish); the autotuner's per-edge tile shapes
    # and any planes-per-tile choice leave every instance bitwise equal to its
    # single-grid run
    edges = [8, 16, 24, 32, 12, 20, 40, 16]
    _, prms = _params(len(edges))
    vws = [1, 2, 1, 2, 4, 2, 1, 4]
    ens, ys, outs, stats = _run_ensemble(edges, prms, hode.F32, 30.0, 1e-5, vws=vws)
    ms, launches = ens.timing()
    assert launches == 1 and ms > 0
    most = max(s["accepted"] + s["rejected"] for s in stats)
    print("one launch: %d attempts of the longest instance in %.2f ms" % (most, ms))
    for i, N in enumerate(edges):
        ref, st = _single(ys[i], N, prms[i], vws[i], 30.0, 0.1, 1e-5)
        assert (stats[i]["accepted"], stats[i]["rejected"]) == (st["accepted"], st["rejected"]), i
        assert np.array_equal(outs[i], ref), i
    # tuned tiles: a choice per edge, reported per instance
    for i, N in enumerate(edges):
        ens.init_instance(i, np.ascontiguousarray(ys[i]).ravel())
    vw, tms = ens.autotune(2)
    tiles = [ens.instance_tile(i) for i in range(len(edges))]
    print("autotuned (vw, planes) per instance:", tiles)
    for i, N in enumerate(edges):
        # a width per edge; plane ranges stay sized from the running cells (0)
        assert tiles[i][0] == vw[i] and N % vw[i] == 0 and tiles[i][1] == 0 and tms[i] > 0
        assert tiles[i] == tiles[edges.index(N)]  # one choice per edge
    for i, N in enumerate(edges):
        ens.init_instance(i, np.ascontiguousarray(ys[i]).ravel())
        ens.set_plane_chunk(i, 1 + (i % 3) * 3)
    stats2 = ens.integrate_adaptive(0.0, 30.0, 0.1, max_steps=100000)
    for i, N in enumerate(edges):
        o = np.empty(2 * N ** 3, dtype=np.float32)
        ens.read_instance(i, o)
        ref, st = _single(ys[i], N, prms[i], tiles[i][0], 30.0, 0.1, 1e-5)
        assert (stats2[i]["accepted"], stats2[i]["rejected"]) == (st["accepted"], st["rejected"]), i
        assert np.array_equal(o, ref), i
    ens.close()


def test_ensemble_retiles_as_instances_finish_bitwise():
    # 24 instances whose attempt counts differ widely (tight and loose
    # tolerances cannot be mixed, so the spread comes from the grid edges and
    # reaction parameters): the persistent kernel re-cuts the running
    # instances into finer tiles each time their number halves, in the same
    # launch; every instance must still equal its single-grid run bitwise
    edges = [8, 12, 16, 20, 24, 28, 32, 40, 48, 56, 64, 72] * 2
    _, prms = _params(len(edges), Du=2e-4, Dv=1e-4)
    vws = [4 if N % 4 == 0 else 1 for N in edges]
    ens, ys, outs, stats = _run_ensemble(edges, prms, hode.F32, 40.0, 1e-5, vws=vws)
    ms, launches = ens.timing()
    att = sorted(s["accepted"] + s["rejected"] for s in stats)
    print("attempts per instance:", att, "launches", launches)
    assert launches == 1 and att[-1] > 2 * att[0]
    for i, N in enumerate(edges):
        ref, st = _single(ys[i], N, prms[i], vws[i], 40.0, 0.1, 1e-5)
        assert (stats[i]["accepted"], stats[i]["rejected"]) == (st["accepted"], st["rejected"]), i
        assert np.array_equal(outs[i], ref), i
    ens.close()


def test_ensemble_fp64_oracle_replay(orc):
    edges = [12, 16, 10]
    _, prms = _params(len(edges))
    ens, ys, outs, stats = _run_ensemble(edges, prms, hode.F64, 40.0, 1e-6, trace=100000)
    for i, N in enumerate(edges):
        tr = ens.read_instance_trace(i)
        assert tr.shape[0] == stats[i]["accepted"] + stats[i]["rejected"]
        sysd = orc.gs_system(N, *prms[i])
        r, te, _ = orc.integrate_replay(sysd, ys[i].ravel(), 0.0, tr[:, 0], tr[:, 2].astype(np.int32), 1e-6, 1e-6)
        assert abs(te - 40.0) < 1e-9
        assert rel_err_fields(outs[i], r, 2) <= 1e-12, i
    ens.close()


def test_ensemble_full_draws_short_horizon():
    # the 512-instance ensemble at its real sizes and parameters, over a short
    # horizon; one instance of every edge is checked bitwise against a single run
    n = 512
    edges, F, k = inputs.ensemble_draws(n, seed=4)
    prms = [[2e-5, 1e-5, F[i], k[i], 2.5] for i in range(n)]
    ens = hode.Ensemble(edges, prms, dtype=hode.F32)
    for i, N in enumerate(edges):
        ens.init_instance(i, inputs.ensemble_ic(i, N).ravel())
    ens.set_tolerances(1e-5, 1e-5)
    stats = ens.integrate_adaptive(0.0, 4.0, 0.1, max_steps=100000)
    assert all(s["status"] == 0 and s["t"] == 4.0 for s in stats)
    seen = {}
    for i, N in enumerate(edges):
        seen.setdefault(N, i)
    for N, i in sorted(seen.items()):
        out = np.empty(2 * N ** 3, dtype=np.float32)
        ens.read_instance(i, out)
        vw = 2 if N > 64 else 1
        ref, st = _single(inputs.ensemble_ic(i, N), N, prms[i], vw, 4.0, 0.1, 1e-5)
        assert np.array_equal(out, ref), (i, N)
    ens.close()


def test_ensemble_instance_failure_is_contained():
    # one instance exhausts its attempts; the others still reach t1 with the
    # same results as alone, and the call reports the failing status
    edges = [16, 12, 20]
    _, prms = _params(len(edges))
    ens = hode.Ensemble(edges, prms, dtype=hode.F64)
    ys = [inputs.ensemble_ic(i, N, dtype=np.float64) for i, N in enumerate(edges)]
    for i, N in enumerate(edges):
        ens.init_instance(i, np.ascontiguousarray(ys[i]).ravel())
    ens.set_tolerances(1e-9, 1e-9)
    ens.set_epoch(4, 4)
    # a budget between the smallest and the largest attempt count of the three
    alone = [_single(ys[i], N, prms[i], 1, 10.0, 0.1, 1e-9)[1] for i, N in enumerate(edges)]
    att = [a["accepted"] + a["rejected"] for a in alone]
    budget = (min(att) + max(att)) // 2
    assert min(att) < budget < max(att)
    stats = ens.integrate_adaptive(0.0, 10.0, 0.1, max_steps=budget, allow=(hode.EMAXSTEPS,))
    for i, N in enumerate(edges):
        if att[i] <= budget:
            assert stats[i]["status"] == 0 and stats[i]["t"] == 10.0, i
            out = np.empty(2 * N ** 3)
            ens.read_instance(i, out)
            ref, _ = _single(ys[i], N, prms[i], 1, 10.0, 0.1, 1e-9)
            assert np.array_equal(out, ref), i
        else:
            assert stats[i]["status"] == hode.EMAXSTEPS and stats[i]["t"] < 10.0, i
            assert stats[i]["accepted"] + stats[i]["rejected"] == budget, i
    ens.close()


def test_ensemble_barrier_give_up_is_reported_and_recoverable():
    # the persistent kernel's grid barriers are bounded waits; a limit of one
    # poll, set from the host, makes the first barrier give up (workgroups
    # without a tile arrive long before those with one), every workgroup
    # leaves on the error flag, and the call reports it.  Re-initialised, the
    # same ensemble then runs normally and gives a fresh ensemble's results.
    edges = [16, 24, 16, 32]
    _, prms = _params(len(edges))
    ref, ys, ref_outs, ref_stats = _run_ensemble(edges, prms, hode.F32, 5.0, 1e-5)
    ref.close()
    ens = hode.Ensemble(edges, prms, dtype=hode.F32)
    ens.set_tolerances(1e-5, 1e-5)
    with pytest.raises(hode.HodeError):
        ens.set_barrier_limit(0)
    for i in range(len(edges)):
        ens.init_instance(i, np.ascontiguousarray(ys[i]).ravel())
    ens.set_barrier_limit(1)
    with pytest.raises(hode.HodeError) as err:
        ens.integrate_adaptive(0.0, 5.0, 0.1, max_steps=100000)
    assert err.value.code == hode.EHIP and "barrier" in str(err.value)
    ens.set_barrier_limit(1 << 30)
    for i in range(len(edges)):
        ens.init_instance(i, np.ascontiguousarray(ys[i]).ravel())
    stats = ens.integrate_adaptive(0.0, 5.0, 0.1, max_steps=100000)
    for i, N in enumerate(edges):
        out = np.empty(2 * N ** 3, dtype=np.float32)
        ens.read_instance(i, out)
        assert np.array_equal(out, ref_outs[i]), i
        assert (stats[i]["accepted"], stats[i]["rejected"]) == (ref_stats[i]["accepted"], ref_stats[i]["rejected"])
    ens.close()


def test_trace_buffers_sized_from_header_constant():
    # A C caller sizes trace buffers as cap * HODE_TRACE_W doubles (the
    # header's constant, read from the header text here): the library must
    # write exactly cap records and nothing past them, for the ensemble and
    # for a single context.
    import ctypes
    import os
    import re
    hdr = os.path.join(os.path.dirname(hode.HERE), "include", "hode.h")
    W = int(re.search(r"#define\s+HODE_TRACE_W\s+(\d+)", open(hdr).read()).group(1))
    canary = np.float64(-12345.678)
    cap, tail = 3, 4 * W
    edges = [8, 16, 24]
    _, prms = _params(len(edges))
    ens, _, _, stats = _run_ensemble(edges, prms, hode.F32, 20.0, 1e-5, trace=64)
    L = hode.lib()
    for i in range(len(edges)):
        buf = np.full(cap * W + tail, canary)
        n = ctypes.c_int64()
        rc = L.hode_ensemble_read_trace(ens.h, i, buf.ctypes.data_as(ctypes.c_void_p), cap, ctypes.byref(n))
        assert rc == 0
        attempts = stats[i]["accepted"] + stats[i]["rejected"]
        assert n.value == attempts > cap
        assert np.all(buf[cap * W:] == canary), i
        rec = buf[:cap * W].reshape(cap, W)
        assert np.all(rec[:, 0] > 0) and np.all(np.isin(rec[:, 2], (0.0, 1.0))), i
        np.testing.assert_array_equal(rec, ens.read_instance_trace(i)[:cap])
    ens.close()
    ctx = hode.Context(0)
    ctx.set_rhs(hode.RHS_GRAYSCOTT3D, prms[0])
    ctx.init_state(inputs.ensemble_ic(0, 8, dtype=np.float32).ravel(), grid=8)
    ctx.set_trace(64)
    st = ctx.integrate_adaptive(0.0, 20.0, 0.1, max_steps=100000)
    buf = np.full(cap * W + tail, canary)
    n = ctypes.c_int64()
    assert L.hode_read_trace(ctx.h, buf.ctypes.data_as(ctypes.c_void_p), cap, ctypes.byref(n)) == 0
    assert n.value == st["accepted"] + st["rejected"] > cap
    assert np.all(buf[cap * W:] == canary)
    ctx.close()
