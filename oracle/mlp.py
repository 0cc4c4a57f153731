"""FP64 oracle of the learned step-size controller's network (test
infrastructure only: tests, the smoke check and the benchmark's CPU-baseline
leg may use it; the HIP path shares no code with it).

Network (the method's learned controller, an addition to the paper's
controllers): x (16 features) -> h1 = tanh(W1 x + b1) (64) -> h2 = tanh(W2 h1
+ b2) (64) -> y = w3 . h2 + b3.  The device evaluates it with bf16 weights,
bf16-rounded inputs and first-layer activations, and fp32 accumulation;
``forward(..., bf16=True)`` applies exactly those roundings and then computes
in fp64, so the two differ only by accumulation order and tanh rounding.

Loss: weighted mean squared error  L = sum_b w_b (y_b - t_b)^2 / sum_b w_b.
The backward pass is written out by hand and pinned by central finite
differences in the tests.

Packed parameter layout (also the device's): W1[64][16], b1[64], W2[64][64],
b2[64], w3[64], b3.
"""
from __future__ import annotations

import numpy as np

NIN, NH = 16, 64
SHAPES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("w3", (NH,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat):
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == NPARAM
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = flat[o:o + n].reshape(shp)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init_params(seed=0, scale=1.0):
    """Glorot-uniform weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SHAPES:
        if name.startswith("b"):
            p[name] = np.zeros(shp)
        else:
            fan_in = shp[-1] if len(shp) > 1 else NH
            fan_out = shp[0] if len(shp) > 1 else 1
            lim = scale * np.sqrt(6.0 / (fan_in + fan_out))
            p[name] = rng.uniform(-lim, lim, size=shp)
    return pack(p)


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even) via float32 bit patterns;
    returns float64 values that are exactly representable in bf16."""
    f = np.asarray(a, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    r = ((bits + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    nan = np.isnan(f)
    out = r.view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def to_bf16_bits(a):
    """uint16 bit patterns of bf16_round(a)."""
    f = bf16_round(a).astype(np.float32)
    return (f.view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def from_bf16_bits(u):
    return (np.asarray(u, dtype=np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def forward(flat, X, bf16=False):
    """Returns (y, cache).  X: (B, 16)."""
    p = unpack(flat)
    X = np.asarray(X, dtype=np.float64)
    if bf16:
        p = {k: bf16_round(v) for k, v in p.items()}
        X = bf16_round(X)
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.tanh(a1)
    h1q = bf16_round(h1) if bf16 else h1
    a2 = h1q @ p["W2"].T + p["b2"]
    h2 = np.tanh(a2)
    y = h2 @ p["w3"] + p["b3"][0]
    return y, dict(X=X, h1=h1, h1q=h1q, h2=h2, p=p)


def loss(flat, X, t, w):
    y, _ = forward(flat, X)
    w = np.asarray(w, dtype=np.float64)
    return float(np.sum(w * (y - t) ** 2) / np.sum(w))


def loss_and_grad(flat, X, t, w, bf16=False):
    """Weighted MSE and its gradient w.r.t. the packed parameters (hand-written
    backward pass through the two tanh layers)."""
    y, c = forward(flat, X, bf16=bf16)
    p = c["p"]
    w = np.asarray(w, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    sw = np.sum(w)
    L = float(np.sum(w * (y - t) ** 2) / sw)
    dy = 2.0 * w * (y - t) / sw                      # (B,)
    g = {}
    g["w3"] = c["h2"].T @ dy                          # (64,)
    g["b3"] = np.array([dy.sum()])
    dh2 = np.outer(dy, p["w3"]) * (1.0 - c["h2"] ** 2)  # (B, 64)
    g["W2"] = dh2.T @ c["h1q"]                        # (64, 64)
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ p["W2"]) * (1.0 - c["h1"] ** 2)      # (B, 64)
    g["W1"] = dh1.T @ c["X"]                          # (64, 16)
    g["b1"] = dh1.sum(axis=0)
    return L, pack(g)


def adam_step(flat, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) of the fp32 master parameters."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v


def features(hs, errs, accs, t_after, t1, rtol, stiff, ctrl_decide):
    """The 16 inputs of the learned controller for every accepted attempt of
    one integration (rows of NaN for rejected ones), from the attempt
    sequence: h_n, its error norm, accept flag and the time after it.

    For an accepted attempt n, with the attempts n, n-1, n-2, n-3 as the
    history (newest first, zeros where there are fewer):
      3i+0: log of the error norm clamped to [-23, 23] (NaN counts as 23),
      3i+1: log(h_{n-i} / h_n), 3i+2: accept flag;
      12: log of the PI factor taken after attempt n (``ctrl_decide`` is the
          oracle's PI controller), 13: log(rtol),
      14: log(max(t1 - t, h_n) / h_n) with t the time after the attempt,
      15: log(h_n * stiff), stiff the scale of the System's largest Jacobian
          eigenvalue.
    """
    n = len(hs)
    X = np.full((n, NIN), np.nan)
    err_prev, last_rej = 1.0, False
    for k in range(n):
        acc, fac, err_prev, last_rej = ctrl_decide(errs[k], err_prev, last_rej)
        assert bool(acc) == bool(accs[k])
        if not acc:
            continue
        x = np.zeros(NIN)
        for i in range(4):
            j = k - i
            if j < 0:
                break
            e = errs[j]
            x[3 * i] = 23.0 if np.isnan(e) else min(23.0, max(-23.0, np.log(max(e, 1e-300))))
            x[3 * i + 1] = np.log(hs[j]) - np.log(hs[k])
            x[3 * i + 2] = 1.0 if accs[j] else 0.0
        x[12] = np.log(fac)
        x[13] = np.log(rtol)
        x[14] = np.log(max(t1 - t_after[k], hs[k]) / hs[k])
        x[15] = np.log(hs[k] * stiff)
        X[k] = x
    return X
