"""Trains the learned step-size controller on the GPU and compares it with PI.

    python -m paper_2309_05331_amd.train_controller [--t1 2000] [--out FILE]

1. Collects accept/reject traces with the PI controller from batched-ensemble
   runs of the 512-instance Gray-Scott workload (grid edges 16..96, F and k
   drawn per instance, FP32) at rtol = atol = 1e-5 and 1e-6 (so the
   tolerance feature covers both values the controller meets).
2. Builds hindsight targets (see controller.py) for each candidate target
   level rho and reject weight, and trains the network with the library's
   MFMA forward/backward kernels and Adam on the GPU.
3. Evaluates every candidate on held-out instances (other initial-condition
   seeds) against PI: attempts, rejects, wall time; keeps the candidate with
   the lowest mean wall-time ratio.
4. Writes the chosen bf16 weights (uint16 bit patterns, .npy) and a JSON
   summary of every run.
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
    ap.add_argument("--rhos", default="0.3,0.5,0.8")
    ap.add_argument("--reject-weights", default="2,5")
    args = ap.parse_args()
    edges, prms = c4_params()
    n = len(edges)
    traces = []
    summary = {"train": {}, "eval": {}, "candidates": {}}
    for rtol in (1e-5, 1e-6):
        stats, el, tr = run_ensemble(edges, prms, list(range(4000, 4000 + n)), args.t1, rtol, hode.CTRL_PI,
                                     trace_cap=4000)
        traces += tr
        summary["train"]["rtol=%g" % rtol] = summarize(stats, el, edges)
        print("traces rtol=%g: %s" % (rtol, summary["train"]["rtol=%g" % rtol]), flush=True)
    # held-out: the first instances' parameter draws with new initial conditions
    m = args.holdout
    he, hp = edges[:m], prms[:m]
    seeds = list(range(9000, 9000 + m))
    base = {}
    for rtol in (1e-5, 1e-6):
        stats, el, _ = run_ensemble(he, hp, seeds, args.t1, rtol, hode.CTRL_PI)
        base[rtol] = summarize(stats, el, he)
        summary["eval"]["pi rtol=%g" % rtol] = base[rtol]
        print("pi", rtol, base[rtol], flush=True)
    best = None
    for rho in (float(v) for v in args.rhos.split(",")):
        for rw in (float(v) for v in args.reject_weights.split(",")):
            parts = [controller.dataset_from_trace(tr, rho=rho, reject_weight=rw) for tr in traces]
            X = np.concatenate([p[0] for p in parts])
            T = np.concatenate([p[1] for p in parts])
            W = np.concatenate([p[2] for p in parts])
            trn = controller.Trainer(seed=0)
            t0 = time.perf_counter()
            hist = trn.fit(X, T, W, epochs=args.epochs, batch=4096, lr=2e-3)
            wb = trn.weights_bf16()
            res = {"samples": int(X.shape[0]), "train_seconds": time.perf_counter() - t0,
                   "loss_first_last": [hist[0], hist[-1]]}
            tot = 0.0
            for rtol in (1e-5, 1e-6):
                stats, el, _ = run_ensemble(he, hp, seeds, args.t1, rtol, hode.CTRL_MLP, weights=wb)
                res["rtol=%g" % rtol] = summarize(stats, el, he)
                tot += el / base[rtol]["wall_s"]
            res["mean_wall_ratio_vs_pi"] = tot / 2
            key = "rho=%g,reject_weight=%g" % (rho, rw)
            summary["candidates"][key] = res
            print(key, json.dumps(res), flush=True)
            if best is None or res["mean_wall_ratio_vs_pi"] < best[0]:
                best = (res["mean_wall_ratio_vs_pi"], key, wb)
    summary["chosen"] = best[1]
    np.save(args.out, best[2])
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(summary, f, indent=1)
    print("chosen", best[1], "mean wall ratio vs PI %.3f" % best[0], flush=True)


if __name__ == "__main__":
    main()
