"""Trains the learned step-size controller on the GPU and compares it with PI.

    python -m paper_2309_05331_amd.train_controller [--t1 2000] [--out FILE]

1. Collects accept/reject traces with the PI controller from batched-ensemble
   runs of the 512-instance Gray-Scott workload (grid edges 16..96, F and k
   drawn per instance, FP32) at rtol = atol = 1e-5 and 1e-6 (so the
   tolerance feature covers both values the controller meets).
2. Builds hindsight targets (see controller.py) and trains the network with
   the library's MFMA forward/backward kernels and Adam on the GPU.
3. Evaluates on held-out instances (other initial-condition seeds) with PI
   and with the learned controller: attempts, rejects and wall time.
4. Writes the bf16 weights (uint16 bit patterns, .npy) and a JSON summary.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import controller, hode, inputs

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "controller_weights.npy")


def c4_params(n=512, seed=4):
    edges, F, k = inputs.ensemble_draws(n, seed=seed)
    return edges, [[2e-5, 1e-5, F[i], k[i], 2.5] for i in range(n)]


def run_ensemble(edges, prms, seeds, t1, rtol, ctrl, weights=None, trace_cap=0, dtype=hode.F32):
    ens = hode.Ensemble(edges, prms, dtype=dtype)
    for i, N in enumerate(edges):
        ens.init_instance(i, inputs.ensemble_ic(seeds[i], N).ravel())
    ens.set_tolerances(rtol, rtol)
    ens.set_controller(ctrl, weights)
    if trace_cap:
        ens.set_trace(trace_cap)
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = ens.integrate_adaptive(0.0, t1, 0.1, max_steps=10 ** 6)
    el = time.perf_counter() - t0
    traces = [ens.read_instance_trace(i) for i in range(len(edges))] if trace_cap else None
    ens.close()
    return stats, el, traces


def summarize(stats, el, edges):
    acc = np.array([s["accepted"] for s in stats])
    rej = np.array([s["rejected"] for s in stats])
    cells = np.array(edges, dtype=np.float64) ** 3
    return {"wall_s": el, "accepted": int(acc.sum()), "rejected": int(rej.sum()),
            "cell_attempts": float((cells * (acc + rej)).sum()),
            "status_ok": bool(all(s["status"] == 0 for s in stats))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--t1", type=float, default=2000.0)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--holdout", type=int, default=64)
    args = ap.parse_args()
    edges, prms = c4_params()
    n = len(edges)
    X, T, W = [], [], []
    summary = {"train": {}, "eval": {}}
    for rtol in (1e-5, 1e-6):
        stats, el, traces = run_ensemble(edges, prms, list(range(4000, 4000 + n)), args.t1, rtol, hode.CTRL_PI,
                                         trace_cap=4000)
        summary["train"]["rtol=%g" % rtol] = summarize(stats, el, edges)
        for tr in traces:
            x, t, w = controller.dataset_from_trace(tr)
            X.append(x)
            T.append(t)
            W.append(w)
        print("traces rtol=%g: %s" % (rtol, summary["train"]["rtol=%g" % rtol]), flush=True)
    X, T, W = np.concatenate(X), np.concatenate(T), np.concatenate(W)
    summary["samples"] = int(X.shape[0])
    trn = controller.Trainer(seed=0)
    t0 = time.perf_counter()
    hist = trn.fit(X, T, W, epochs=args.epochs, batch=4096, lr=2e-3, log_every=10)
    summary["train_seconds"] = time.perf_counter() - t0
    summary["loss_first_last"] = [hist[0], hist[-1]]
    wb = trn.weights_bf16()
    np.save(args.out, wb)
    # held-out: same parameter draws for the first instances, new initial conditions
    m = args.holdout
    he, hp = edges[:m], prms[:m]
    seeds = list(range(9000, 9000 + m))
    for rtol in (1e-5, 1e-6):
        for name, ctrl, w in (("pi", hode.CTRL_PI, None), ("mlp", hode.CTRL_MLP, wb)):
            stats, el, _ = run_ensemble(he, hp, seeds, args.t1, rtol, ctrl, weights=w)
            summary["eval"]["%s rtol=%g" % (name, rtol)] = summarize(stats, el, he)
            print(name, rtol, summary["eval"]["%s rtol=%g" % (name, rtol)], flush=True)
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(summary, f, indent=1)
    print(json.dumps(summary))


if __name__ == "__main__":
    main()
