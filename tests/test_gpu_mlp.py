"""GPU: the learned step-size controller.  The library's MFMA forward and
backward kernels against the FP64 oracle on the same bf16-rounded weights and
inputs; Adam training on the GPU lowers the loss; the controller's fused
proposal matches the oracle network on the features it recorded; garbage
weights fall back to the PI controller exactly; the embedded error still
judges every step."""
import math

import numpy as np
import pytest

from oracle import mlp as omlp
from paper_2309_05331_amd import controller, hode, inputs

pytestmark = pytest.mark.gpu


def _data(B, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, 16)).astype(np.float32)
    T = rng.normal(size=B).astype(np.float32)
    W = rng.uniform(0.5, 2.0, size=B).astype(np.float32)
    return X, T, W


@pytest.mark.parametrize("B", [1, 63, 64, 1000])
def test_forward_matches_oracle(B):
    X, _, _ = _data(B)
    p = controller.init_params(seed=3)
    p[-1] = 0.3
    tr = controller.Trainer(params=p)
    y = tr.forward(X)
    pb = omlp.from_bf16_bits(tr.weights_bf16())
    yo, _ = omlp.forward(pb, X.astype(np.float64), bf16=True)
    scale = 1 + np.max(np.abs(yo))
    assert np.max(np.abs(y - yo)) <= 1e-2 * scale, np.max(np.abs(y - yo))


def test_loss_and_gradient_match_oracle():
    X, T, W = _data(700, seed=1)
    p = controller.init_params(seed=4)
    p[-1] = 0.2
    tr = controller.Trainer(params=p)
    L, g = tr.loss_grad(X, T, W)
    pb = omlp.from_bf16_bits(tr.weights_bf16())
    Lo, go = omlp.loss_and_grad(pb, X.astype(np.float64), T, W, bf16=True)
    assert abs(L - Lo) <= 1e-3 * Lo
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    cos = float(g @ go / (np.linalg.norm(g) * np.linalg.norm(go)))
    print("gradient relative error %.3e cosine %.6f" % (rel, cos))
    assert rel < 3e-2 and cos > 0.999


def test_training_reduces_loss():
    rng = np.random.default_rng(7)
    X = rng.normal(size=(8192, 16)).astype(np.float32)
    T = (0.5 * np.tanh(X[:, 12]) - 0.2 * X[:, 0] + 0.1).astype(np.float32)
    W = np.ones(8192, dtype=np.float32)
    tr = controller.Trainer(seed=1)
    hist = tr.fit(X, T, W, epochs=40, batch=1024, lr=3e-3)
    print("loss %.4f -> %.4f" % (hist[0], hist[-1]))
    assert hist[-1] < 0.1 * hist[0]
    # the oracle evaluates the trained bf16 network to the same values
    pb = omlp.from_bf16_bits(tr.weights_bf16())
    yo, _ = omlp.forward(pb, X[:512].astype(np.float64), bf16=True)
    assert np.max(np.abs(tr.forward(X[:512]) - yo)) < 1e-2


def _gs_run(ctrl, weights=None, N=24, t1=40.0, trace=True):
    prm = [2e-3, 1e-3, 0.04, 0.06, 2.5]
    y0 = inputs.gray_scott_ic(N, seed=11, dtype=np.float32).ravel()
    ctx = hode.Context(0)
    ctx.set_rhs(hode.RHS_GRAYSCOTT3D, prm)
    ctx.init_state(y0, grid=N)
    ctx.set_tolerances(1e-5, 1e-5)
    ctx.set_controller(ctrl, weights)
    if trace:
        ctx.set_trace(100000)
    st = ctx.integrate_adaptive(0.0, t1, 0.1, max_steps=100000)
    out = np.empty_like(y0)
    ctx.read_state(out)
    tr = ctx.read_trace() if trace else None
    ctx.close()
    return st, out, tr


def test_fused_proposal_matches_oracle_network():
    p = controller.init_params(seed=9)
    p[-1] = 0.15  # a mild growth bias, so proposals differ from PI
    tr = controller.Trainer(params=p)
    wb = tr.weights_bf16()
    st, _, trace = _gs_run(hode.CTRL_MLP, wb)
    assert st["status"] == 0 and st["t"] == 40.0
    rows = np.nonzero(np.isfinite(trace[:, 6]))[0]
    assert rows.size > 5
    pb = omlp.from_bf16_bits(wb)
    yo, _ = omlp.forward(pb, trace[rows, 8:24], bf16=True)
    want = np.clip(yo, math.log(0.2), math.log(5.0))
    prev_rej = np.array([r > 0 and trace[r - 1, 2] == 0 for r in rows])
    want = np.where(prev_rej, np.minimum(want, 0.0), want)
    assert np.max(np.abs(trace[rows, 6] - want)) < 1e-2
    # the proposal was applied: dt_next = h * exp(proposal)
    np.testing.assert_allclose(trace[rows, 4], trace[rows, 0] * np.exp(trace[rows, 6]), rtol=1e-12)
    # the embedded error judged every attempt
    assert np.all(trace[trace[:, 2] == 1, 1] <= 1.0) and np.all(trace[trace[:, 2] == 0, 1] > 1.0)


def test_recorded_features_match_oracle_definition(orc):
    # the features the device computes for the network (and records for
    # training) against the oracle's definition from the attempt sequence
    st, _, trace = _gs_run(hode.CTRL_PI)
    N, prm = 24, [2e-3, 1e-3, 0.04, 0.06, 2.5]
    stiff = 12.0 * max(prm[0], prm[1]) / (prm[4] / N) ** 2 + 1.0
    X = omlp.features(trace[:, 0], trace[:, 1], trace[:, 2] == 1, trace[:, 3], 40.0, 1e-5, stiff,
                      lambda e, ep, lr: orc.ctrl_decide(orc.CTRL_PI, e, ep, lr))
    acc = trace[:, 2] == 1
    assert acc.sum() > 5
    assert np.all(np.isnan(trace[~acc, 8:24]))
    got, want = trace[acc, 8:24], X[acc]
    # the device rounds each feature to fp32 once
    assert np.max(np.abs(got - want) / np.maximum(1.0, np.abs(want))) <= 1e-6, np.max(np.abs(got - want))


def test_nonfinite_network_falls_back_to_pi_exactly():
    bad = np.full(hode.MLP_NPARAM, 0x7FC0, dtype=np.uint16)  # bf16 NaN everywhere
    st_pi, y_pi, tr_pi = _gs_run(hode.CTRL_PI)
    st_ml, y_ml, tr_ml = _gs_run(hode.CTRL_MLP, bad)
    assert (st_ml["accepted"], st_ml["rejected"]) == (st_pi["accepted"], st_pi["rejected"])
    assert np.array_equal(y_ml, y_pi)
    assert np.all(np.isnan(tr_ml[:, 6]))


def test_trained_controller_beats_pi_on_held_out_instances():
    # the committed network (trained on the integrator's own traces of the
    # 512-instance workload) against PI on instances it has not seen: new
    # initial conditions, rtol 1e-6, horizon 0..400
    import os
    from paper_2309_05331_amd import train_controller as tc
    wb = np.load(os.path.join(os.path.dirname(hode.__file__), "controller_weights.npy"))
    edges, prms = tc.c4_params()
    m = 24
    he, hp = edges[:m], prms[:m]
    seeds = list(range(9500, 9500 + m))
    res = {}
    for name, kind, w in (("pi", hode.CTRL_PI, None), ("mlp", hode.CTRL_MLP, wb)):
        stats, el, _ = tc.run_ensemble(he, hp, seeds, 400.0, 1e-6, kind, weights=w)
        assert all(s["status"] == 0 and s["t"] == 400.0 for s in stats)
        res[name] = sum(s["accepted"] + s["rejected"] for s in stats)
    print("attempts PI %d learned %d" % (res["pi"], res["mlp"]))
    assert res["mlp"] < res["pi"]
