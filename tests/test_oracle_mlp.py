"""Pins for the FP64 MLP oracle of the learned step-size controller: central
finite differences for the hand-written backward pass, bf16 rounding against
torch's conversion and hand-worked ties, closed forms for degenerate
networks, and Adam's first step."""
import numpy as np
import pytest

from oracle import mlp


def _data(B=37, seed=3):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, mlp.NIN))
    t = rng.normal(size=B)
    w = rng.uniform(0.5, 2.0, size=B)
    return X, t, w


def test_gradient_matches_central_differences():
    X, t, w = _data()
    p = mlp.init_params(seed=1, scale=1.5)
    p = p + np.random.default_rng(2).normal(scale=0.05, size=p.size)  # nonzero biases too
    L, g = mlp.loss_and_grad(p, X, t, w)
    assert L == pytest.approx(mlp.loss(p, X, t, w), rel=1e-14)
    eps = 1e-6
    idx = np.random.default_rng(4).choice(p.size, size=200, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = eps
        fd = (mlp.loss(p + e, X, t, w) - mlp.loss(p - e, X, t, w)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_bf16_rounding_against_torch_and_ties():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.integers(-6, 6, size=2000),
                        [0.0, -0.0, 1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, -(1 + 2 ** -8), 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = mlp.bf16_round(x)
    assert np.array_equal(got, ref)
    assert mlp.bf16_round([1 + 2 ** -8])[0] == 1.0             # tie to even
    assert mlp.bf16_round([1 + 3 * 2 ** -9])[0] == 1 + 2 ** -7  # nearest
    bits = mlp.to_bf16_bits([1.0, -2.0])
    assert list(bits) == [0x3F80, 0xC000]
    assert np.array_equal(mlp.from_bf16_bits(bits), [1.0, -2.0])


def test_degenerate_networks_closed_form():
    X, _, _ = _data(B=5)
    P = mlp.unpack(mlp.init_params(seed=7))
    P["W2"][:] = 0.0
    P["b2"][:] = np.linspace(-1, 1, mlp.NH)
    P["b3"][:] = 0.25
    y, _ = mlp.forward(mlp.pack(P), X)
    np.testing.assert_allclose(y, P["w3"] @ np.tanh(P["b2"]) + 0.25, rtol=1e-15)
    P["W1"][:] = 0.0
    P["b1"][:] = 0.3
    P["W2"][:] = np.eye(mlp.NH)
    P["b2"][:] = 0.0
    y, _ = mlp.forward(mlp.pack(P), X)
    np.testing.assert_allclose(y, P["w3"].sum() * np.tanh(np.tanh(0.3)) + 0.25, rtol=1e-14)


def test_adam_first_step_is_signed_lr():
    p = np.zeros(10)
    g = np.linspace(-2, 3, 10)
    g[4] = 1e-3
    q, m, v = mlp.adam_step(p, g, np.zeros(10), np.zeros(10), 1, lr=0.01)
    np.testing.assert_allclose(q, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_bf16_forward_close_to_exact():
    X, _, _ = _data(B=64)
    p = mlp.init_params(seed=5)
    y, _ = mlp.forward(p, X)
    yq, _ = mlp.forward(p, X, bf16=True)
    assert np.max(np.abs(y - yq)) < 0.05 * (1 + np.max(np.abs(y)))


def test_features_history_shifts_and_special_values(orc):
    # invariants of the feature definition on a synthetic attempt sequence
    # with a reject and a NaN error: the history of attempt k is that of
    # attempt k-1 shifted by one slot (step ratios rebased to h_k), the PI
    # entry is the oracle controller's factor, and rejected rows are NaN
    hs = np.array([0.1, 0.3, 0.5, 0.2, 0.25, 0.4, 0.35])
    errs = np.array([0.2, 0.5, 3.0, float("nan"), 0.8, 0.1, 1e-40])
    accs = np.array([e <= 1.0 for e in errs])
    t_after = np.cumsum(np.where(accs, hs, 0.0))
    X = mlp.features(hs, errs, accs, t_after, 1.5, 1e-6, 7.0,
                      lambda e, ep, lr: orc.ctrl_decide(orc.CTRL_PI, e, ep, lr))
    assert np.all(np.isnan(X[~accs]))
    k_acc = np.nonzero(accs)[0]
    for k in k_acc:
        x = X[k]
        assert x[1] == 0.0 and x[2] == 1.0                       # the attempt itself
        assert x[13] == np.log(1e-6) and abs(x[15] - np.log(hs[k] * 7.0)) < 1e-15
        assert abs(x[14] - np.log(max(1.5 - t_after[k], hs[k]) / hs[k])) < 1e-15
        for i in range(1, 4):
            j = k - i
            if j < 0:
                assert np.all(x[3 * i:3 * i + 3] == 0.0)
                continue
            assert x[3 * i + 2] == (1.0 if accs[j] else 0.0)
            assert abs(x[3 * i + 1] - np.log(hs[j] / hs[k])) < 1e-14
    # NaN error counts as the upper clamp, tiny errors hit the lower clamp
    assert X[4][3] == 23.0 and X[6][0] == -23.0
    # consecutive accepted attempts: slots shift by one
    for k in (1, 5, 6):
        assert np.allclose(X[k][3:12:3], X[k - 1][0:9:3])
    # PI entry: the oracle controller's factor after attempt k
    ep, lr = 1.0, False
    for k in range(len(hs)):
        acc, fac, ep, lr = orc.ctrl_decide(orc.CTRL_PI, errs[k], ep, lr)
        if acc:
            assert X[k][12] == np.log(fac)
