"""Writes the stored FP64 oracle results of the long-horizon parity checks
(``oracle_*.json`` next to this file).  Calls only the oracle and the seeded
input generators; nothing here comes from the HIP path.

Each file holds, for one Gray-Scott workload integrated by the oracle in
FP64 from the FP32-rounded initial condition:
  - the workload (grid edge, parameters, seed, method, times, tolerances);
  - for adaptive runs the oracle's own step sequence (h, accepted) and its
    accepted / rejected counts, so a caller can replay exactly those steps;
  - the final state at a fixed set of sampled cells (both fields): the cube's
    corners and faces, the domain's corners (periodic wrap), a coarse lattice
    and seeded random cells;
  - per-field minimum, maximum and mean of the whole final state.

    python tests/golden/make_oracle_goldens.py [name ...]

Names: gs256-rk4-t100 (RK4, dt 0.1, 1000 steps), gs256-dp5-t100 (Dopri5,
rtol = atol = 1e-6, t 0 -> 100), gs512-dp5-t20 (Dopri5, rtol = atol = 1e-6,
t 0 -> 20; about 20 GB of host memory), ens16-dp5-t2000 (16 instances of the
512-instance ensemble covering its 11 grid edges, Dopri5, rtol = atol =
1e-5, t 0 -> 2000).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2309_05331_amd import inputs  # noqa: E402

PRM = [2e-5, 1e-5, 0.053, 0.014, 2.5]


def sample_cells(N, n_random=48, lattice=8, seed=0):
    """(z, y, x) cells: cube corners and face centres, domain corners, a
    lattice of lattice^3 cells and seeded random cells (duplicates dropped,
    order kept)."""
    a, b, m = 3 * N // 8, 5 * N // 8 - 1, N // 2
    pts = [(a, a, a), (b, b, b), (a, b, a), (b, a, b), (a, m, m), (m, m, b), (m, a, m), (m, m, m),
           (0, 0, 0), (N - 1, N - 1, N - 1), (0, N - 1, m), (m, 0, N - 1), (max(a - 1, 0), a, min(b + 1, N - 1))]
    step = max(1, N // lattice)
    pts += [(z, y, x) for z in range(0, N, step) for y in range(0, N, step) for x in range(0, N, step)]
    rng = np.random.default_rng(seed)
    pts += [tuple(int(v) for v in rng.integers(0, N, size=3)) for _ in range(n_random)]
    seen, out = set(), []
    for p in pts:
        if p not in seen:
            seen.add(p)
            out.append(p)
    return out


def summarise(y, N, cells):
    f = y.reshape(2, N, N, N)
    return {
        "cells": [list(c) for c in cells],
        "u": [float(f[0][c]) for c in cells],
        "v": [float(f[1][c]) for c in cells],
        "min": [float(f[0].min()), float(f[1].min())],
        "max": [float(f[0].max()), float(f[1].max())],
        "mean": [float(f[0].mean()), float(f[1].mean())],
    }


def gs_run(N, seed, method, prm=PRM, t1=None, dt=None, nsteps=None, tol=1e-6, dt0=0.1):
    y32 = inputs.gray_scott_ic(N, seed=seed, dtype=np.float32)
    y = y32.astype(np.float64).ravel()
    del y32
    sysd = oracle.gs_system(N, *prm)
    rec = {"N": N, "seed": seed, "params": list(prm), "start": "FP32-rounded initial condition, FP64 arithmetic"}
    t0 = time.time()
    if method == "rk4":
        y, te = oracle.integrate_n_steps(sysd, oracle.RK4, y, 0.0, dt, nsteps)
        rec.update(method="rk4", dt=dt, steps=nsteps, t_end=te)
    else:
        y, st, tr = oracle.integrate_adaptive(sysd, y, 0.0, t1, dt0, tol, tol, trace_cap=1000000)
        assert st["status"] == 0 and st["t"] == t1, st
        rec.update(method="dopri5", rtol=tol, atol=tol, t1=t1, dt0=dt0, accepted=st["accepted"],
                   rejected=st["rejected"], h=[float(v) for v in tr[:, 0]],
                   accepted_flags=[int(v) for v in tr[:, 2]], err=[float(v) for v in tr[:, 1]])
    rec["oracle_seconds"] = round(time.time() - t0, 1)
    rec["threads"] = oracle.num_threads()
    rec["final"] = summarise(y, N, sample_cells(N))
    return rec


def ensemble_subset(n_inst=512, seed=4, n_pick=16):
    """The first instance of every grid edge, then the lowest further indices,
    up to n_pick instances."""
    edges, F, k = inputs.ensemble_draws(n_inst, seed=seed)
    first = {}
    for i, N in enumerate(edges):
        first.setdefault(N, i)
    pick = sorted(first.values())
    i = 0
    while len(pick) < n_pick:
        if i not in pick:
            pick.append(i)
        i += 1
    return sorted(pick), edges, F, k


def ens_run():
    pick, edges, F, k = ensemble_subset()
    out = {"instances": [], "t1": 2000.0, "dt0": 0.1, "rtol": 1e-5, "atol": 1e-5,
           "start": "FP32-rounded initial conditions, FP64 arithmetic"}
    for i in pick:
        N = edges[i]
        prm = [PRM[0], PRM[1], float(F[i]), float(k[i]), PRM[4]]
        y = inputs.ensemble_ic(i, N).astype(np.float64).ravel()
        sysd = oracle.gs_system(N, *prm)
        t0 = time.time()
        y, st, tr = oracle.integrate_adaptive(sysd, y, 0.0, 2000.0, 0.1, 1e-5, 1e-5, trace_cap=1000000)
        assert st["status"] == 0, st
        rec = {"index": i, "N": N, "params": prm, "accepted": st["accepted"], "rejected": st["rejected"],
               "oracle_seconds": round(time.time() - t0, 1),
               "final": summarise(y, N, sample_cells(N, n_random=16, lattice=4, seed=i))}
        print("instance %d N=%d: %d accepted, %d rejected, %.1f s" % (i, N, st["accepted"], st["rejected"],
                                                                     rec["oracle_seconds"]), flush=True)
        out["instances"].append(rec)
    out["threads"] = oracle.num_threads()
    return out


RUNS = {
    "gs256-rk4-t100": lambda: gs_run(256, 3, "rk4", dt=0.1, nsteps=1000),
    "gs256-dp5-t100": lambda: gs_run(256, 3, "dp5", t1=100.0),
    "gs512-dp5-t20": lambda: gs_run(512, 5, "dp5", t1=20.0),
    "ens16-dp5-t2000": ens_run,
}


def main(names):
    for name in names or sorted(RUNS):
        t0 = time.time()
        rec = RUNS[name]()
        rec["name"] = name
        rec["generator"] = "tests/golden/make_oracle_goldens.py"
        path = os.path.join(HERE, "oracle_%s.json" % name)
        with open(path, "w") as f:
            json.dump(rec, f, indent=0, separators=(",", ":"))
            f.write("\n")
        print("wrote %s (%.0f s)" % (path, time.time() - t0), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
