"""Learned step-size controller: training data from the integrator's own
attempt traces, and training on the GPU with the library's network kernels.

The network (16 -> 64 -> 64 -> 1, tanh, bf16 weights, fp32 accumulation)
proposes log(h_next / h) after an accepted attempt; the step controller
clamps it to [log 0.2, log 5], never grows after a reject, falls back to the
PI proposal on a non-finite output, retries rejected attempts with the PI
shrink, and the embedded error estimate still judges every attempt.

Training target (hindsight): for an accepted attempt n followed by attempt
n+1, the step that would have produced the error level rho under the local
model err ~ h^5 is h* = h_{n+1} (rho / err_{n+1})^(1/5); the target is
log(h* / h_n), clamped like the proposal.  Pairs whose next attempt was
rejected weigh more (a reject costs a whole attempt); rho and that weight are
chosen on held-out runs.  The 16 input features
are the ones the device computed at decision n and stored in the trace.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import hode

# the error level of the shipped network's targets (chosen on held-out runs
# among 0.3 and 0.5 by train_controller.py)
RHO = 0.5
LOG_LO, LOG_HI = math.log(0.2), math.log(5.0)


# Dopri5's stability function R5(z) = sum_{j<=5} z^j/j! + z^6/600 has modulus
# one at z = -3.30657 on the negative real axis: an explicit step longer than
# 3.30657 / lambda amplifies the System's stiffest mode (eigenvalue -lambda).
DOPRI5_REAL_STABILITY = 3.30657


def dataset_from_trace(tr, rho=RHO, reject_weight=2.0, stab_cap=0.0):
    """(X, T, W) training triples from one run's trace (rows in attempt order).

    stab_cap > 0 caps every target at stab_cap times the step where the
    method's stability function reaches modulus one for the System's
    largest eigenvalue lambda (from the recorded feature log(h (lambda + 1))):
    beyond that step the error no longer behaves like h^5, so the hindsight
    target would overshoot it."""
    tr = np.asarray(tr, dtype=np.float64)
    if tr.shape[0] < 2:
        return np.zeros((0, 16)), np.zeros(0), np.zeros(0)
    h, err, acc = tr[:, 0], tr[:, 1], tr[:, 2]
    n = np.arange(tr.shape[0] - 1)
    ok = (acc[n] == 1) & np.all(np.isfinite(tr[n, 8:24]), axis=1) & np.isfinite(err[n + 1]) & (h[n] > 0)
    n = n[ok]
    e1 = np.maximum(err[n + 1], 1e-10)
    target = np.log(h[n + 1] / h[n]) + 0.2 * np.log(rho / e1)
    if stab_cap > 0:
        lam = np.exp(tr[n, 23]) / h[n] - 1.0  # feature 15: log(h (lambda + 1))
        cap = np.log(stab_cap * DOPRI5_REAL_STABILITY / np.maximum(lam, 1e-300) / h[n])
        target = np.where(lam > 0, np.minimum(target, cap), target)
    target = np.clip(target, LOG_LO, LOG_HI)
    weight = np.where(err[n + 1] > 1.0, reject_weight, 1.0)
    return tr[n, 8:24].copy(), target, weight


def init_params(seed=0):
    """Glorot-uniform weights and zero biases (fp32 master copy), packed as
    W1[64][16], b1[64], W2[64][64], b2[64], w3[64], b3."""
    rng = np.random.default_rng(seed)

    def glorot(n_out, n_in):
        lim = math.sqrt(6.0 / (n_in + n_out))
        return rng.uniform(-lim, lim, size=n_out * n_in)

    parts = [glorot(64, 16), np.zeros(64), glorot(64, 64), np.zeros(64), glorot(1, 64) * 0.1, np.zeros(1)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == hode.MLP_NPARAM
    return p


class Trainer:
    """Adam on fp32 master weights with the library's MFMA forward/backward
    kernels; all tensors live on the GPU (torch is only the allocator)."""

    def __init__(self, params=None, seed=0, device="cuda:0"):
        import torch
        self.torch = torch
        self.dev = device
        p = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        self.Wm = torch.from_numpy(p.copy()).to(device)
        self.Wb = torch.zeros(hode.MLP_NPARAM, dtype=torch.int16, device=device)
        self.m = torch.zeros_like(self.Wm)
        self.v = torch.zeros_like(self.Wm)
        self.g = torch.zeros_like(self.Wm)
        self.acc = torch.zeros(2, dtype=torch.float64, device=device)
        self.step = 0
        self._chk(hode.lib().hode_mlp_quantize(self._p(self.Wm), self._p(self.Wb), None))

    @staticmethod
    def _p(t):
        return C.c_void_p(t.data_ptr())

    @staticmethod
    def _chk(rc):
        if rc != hode.OK:
            raise hode.HodeError(rc, "mlp kernel")

    def weights_bf16(self):
        return self.Wb.cpu().numpy().view(np.uint16).copy()

    def forward(self, X):
        X = self.torch.as_tensor(np.asarray(X, dtype=np.float32), device=self.dev).contiguous()
        Y = self.torch.empty(X.shape[0], dtype=self.torch.float32, device=self.dev)
        self._chk(hode.lib().hode_mlp_forward(self._p(self.Wb), self._p(X), self._p(Y), X.shape[0], None))
        return Y.cpu().numpy()

    def loss_grad(self, X, T, W):
        t = self.torch
        X = t.as_tensor(np.asarray(X, dtype=np.float32), device=self.dev).contiguous()
        T = t.as_tensor(np.asarray(T, dtype=np.float32), device=self.dev).contiguous()
        W = t.as_tensor(np.asarray(W, dtype=np.float32), device=self.dev).contiguous()
        loss = C.c_double()
        self._chk(hode.lib().hode_mlp_loss_grad(self._p(self.Wb), self._p(X), self._p(T), self._p(W), None,
                                                X.shape[0], self._p(self.g), self._p(self.acc), C.byref(loss), None))
        return loss.value, self.g.cpu().numpy().copy()

    def fit(self, X, T, W, epochs=200, batch=4096, lr=2e-3, seed=0, log_every=0):
        """Minibatch Adam over the dataset (kept on the GPU); returns the loss
        history (one value per epoch, mean over its batches)."""
        t = self.torch
        Xd = t.as_tensor(np.asarray(X, dtype=np.float32), device=self.dev).contiguous()
        Td = t.as_tensor(np.asarray(T, dtype=np.float32), device=self.dev).contiguous()
        Wd = t.as_tensor(np.asarray(W, dtype=np.float32), device=self.dev).contiguous()
        n = Xd.shape[0]
        rng = np.random.default_rng(seed)
        hist = []
        L = hode.lib()
        loss = C.c_double()
        perm = t.empty(n, dtype=t.int64, device=self.dev)
        for ep in range(epochs):
            # the epoch's shuffle is drawn on the host and copied in; the
            # kernels gather each minibatch's rows through its slice
            perm.copy_(t.from_numpy(rng.permutation(n).astype(np.int64)))
            tot, nb = 0.0, 0
            for b0 in range(0, n, batch):
                nbat = min(batch, n - b0)
                self.step += 1
                self._chk(L.hode_mlp_train_step(self._p(Xd), self._p(Td), self._p(Wd),
                                                C.c_void_p(perm.data_ptr() + 8 * b0), nbat, self._p(self.Wm),
                                                self._p(self.Wb), self._p(self.m), self._p(self.v), self._p(self.g),
                                                self._p(self.acc), self.step, C.c_float(lr), C.byref(loss), None))
                tot += loss.value
                nb += 1
            hist.append(tot / max(nb, 1))
            if log_every and ep % log_every == 0:
                print("epoch %d loss %.5f" % (ep, hist[-1]), flush=True)
        return hist


def collect_ensemble_traces(edges, prms, t1, rtol, dtype=hode.F32, cap=20000, seeds=None):
    """Runs an ensemble with the PI controller and returns one trace per
    instance (the integrator's own accept/reject records)."""
    from . import inputs
    ens = hode.Ensemble(edges, prms, dtype=dtype)
    npd = np.float32 if dtype == hode.F32 else np.float64
    for i, N in enumerate(edges):
        y = inputs.ensemble_ic(i if seeds is None else seeds[i], N, dtype=npd)
        ens.init_instance(i, np.ascontiguousarray(y).ravel())
    ens.set_tolerances(rtol, rtol)
    ens.set_trace(cap)
    stats = ens.integrate_adaptive(0.0, t1, 0.1, max_steps=cap)
    traces = [ens.read_instance_trace(i) for i in range(len(edges))]
    ens.close()
    return traces, stats
