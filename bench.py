"""Benchmark: cell-updates/s and HBM roofline fraction of the Runge-Kutta hot
path on one MI355X, with the FP64 CPU oracle timed beside it.

Default workload: 3D periodic Gray-Scott, 512^3 grid, FP32 state with FP64
time/step control, adaptive Dormand-Prince 5(4) with rtol = atol = 1e-6,
Du = 2e-5, Dv = 1e-5, F = 0.053, k = 0.014, box edge 2.5, initial condition a
central 128^3 cube (u = 0.5, v = 0.25) in u = 1, v = 0 plus seeded uniform
noise +-0.01 (seed 5).  One benchmark step integrates one window of `--window`
time units along the same trajectory (the next window starts where the last
ended, with the last proposed step); the value is cells x accepted steps /
wall time over the timed windows.  After the timed windows the default
workload also integrates the same grid from t = 0 to 2000 with the PI and with
the learned step-size controller (`controller_ab`: wall time to rtol 1e-6 of
each, three runs each in alternating order, mean and sd, their ratio, and
each one's final error against an FP64 run at rtol 1e-8; `--ab T1` sets
the horizon, `--ab 0` skips it).

Other workloads (--workload): gs512-dp5-fp64 (the same grid in FP64, the
paper's precision), gs256-dp5, gs256-rk4, gs512-ck54, gs512-f78,
gs512-ab4, gs32-rk4-fp64, ew24-dp5, ew24-dp5-fp32 and ens512-dp5 (the
512-instance batched ensemble, edges 16..96, rtol 1e-5, t 0 -> 2000; one
step integrates the whole horizon from the initial conditions).

Prints ONE JSON line.  Inputs are resident in HBM before timing starts.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s & %HBM peak; wall-time to rtol 1e-6, learned vs PI controller"
T_START = time.time()
PEAK_HBM_GBS = 8000.0
GS_PRM = [2e-5, 1e-5, 0.053, 0.014, 2.5]

# Algorithmic traffic: arrays (each 2 N^3 elements of the state precision)
# each Gray-Scott stage kernel must read once and write once.
#   D1: y -> k1                      R2: y,k1 -> k2     R3: y,k2 -> k3
#   R4: y,k3,k1,k2 -> ynew           D2: y,k1 -> k2     D3: y,k1,k2 -> k3
#   D4: y,k1..k3 -> k4               D5: y,k1..k4 -> k5
#   D6: y,k1..k5 -> ynew, partial error                D7: ynew,partial error,y -> k7
#   Cash-Karp: D1 D2 D3 (shared), C4: y,k1..k3 -> k4   C5: y,k1..k4 -> k5   C6: y,k1..k5 -> ynew (+ error norm)
#   Fehlberg 7(8): Fs reads y and the k_j of its tableau row (zero columns
#   skipped) and writes k_s; F13 reads y, k1, k4..k10, k12 and k11 and writes
#   ynew (82 arrays per attempt)
#   Adams-Bashforth s: y and f_{n-1} .. f_{n-s+1} -> f_n, ynew (s + 2 arrays)
GS_ARRAYS = {0: 2, 1: 3, 2: 3, 3: 5, 4: 3, 5: 4, 6: 5, 7: 6, 8: 8, 9: 4, 10: 2, 11: 5, 12: 6, 13: 7, 14: 7, 15: 2,
             16: 7,
             17: 2, 18: 3, 19: 4, 20: 4, 21: 5, 22: 5, 23: 6, 24: 6, 25: 8, 26: 9, 27: 10, 28: 8, 29: 12, 30: 11,
             31: 2, **{30 + s: s + 2 for s in range(2, 9)}, 39: 9, **{39 + s: s + 2 for s in range(1, 9)}, 48: 2, 49: 3,
             50: 3}
GS_NAMES = {0: "D1", 1: "R2", 2: "R3", 3: "R4", 4: "D2", 5: "D3", 6: "D4", 7: "D5", 8: "D6", 9: "D7", 10: "D7F",
            11: "C4", 12: "C5", 13: "C6", 14: "C6F", 15: "E1", 16: "D6F",
            **{16 + i: "F%d" % i for i in range(1, 14)}, 30: "F13F", **{30 + s: "AB%d" % s for s in range(1, 9)},
            39: "D6K", **{39 + s: "ABC%d" % s for s in range(1, 9)}, 48: "MM1", 49: "MM2", 50: "MM3"}
STAGES = {"rk4": [0, 1, 2, 3], "dp5": [4, 5, 6, 7, 8, 9], "ck54": [0, 4, 5, 11, 12, 13], "f78": list(range(17, 30)),
          "ab4": [34]}

WORKLOADS = {
    "gs512-dp5": dict(kind="gs", N=512, dtype="f32", method="dp5", window=10.0, seed=5, dt0=0.1),
    "gs256-dp5": dict(kind="gs", N=256, dtype="f32", method="dp5", window=10.0, seed=3, dt0=0.1),
    # the paper's precision on the stencil path: FP64 state and arithmetic
    "gs512-dp5-fp64": dict(kind="gs", N=512, dtype="f64", method="dp5", window=10.0, seed=5, dt0=0.1),
    "gs512-ck54": dict(kind="gs", N=512, dtype="f32", method="ck54", window=10.0, seed=5, dt0=0.1),
    "gs512-f78": dict(kind="gs", N=512, dtype="f32", method="f78", window=10.0, seed=5, dt0=0.1),
    # Adams-Bashforth 4 at h lambda_max = 0.25 (its real stability interval is 0.3)
    "gs512-ab4": dict(kind="gs", N=512, dtype="f32", method="ab4", steps_per=400, dt=0.025, seed=5),
    "gs256-rk4": dict(kind="gs", N=256, dtype="f32", method="rk4", steps_per=100, dt=0.1, seed=3),
    "gs32-rk4-fp64": dict(kind="gs", N=32, dtype="f64", method="rk4", steps_per=500, dt=0.1, seed=1,
                          compare_graphs=True),
    "ew24-dp5": dict(kind="ew", n=1 << 24, dtype="f64", method="dp5", t1=5.0, seed=2, dt0=0.01),
    "ew24-dp5-fp32": dict(kind="ew", n=1 << 24, dtype="f32", method="dp5", t1=5.0, seed=2, dt0=0.01),
    "ens512-dp5": dict(kind="ens", n=512, dtype="f32", method="dp5", t1=2000.0, seed=4, dt0=0.1, rtol=1e-5),
}
DP5_ARRAYS = 30  # arrays of 2 N^3 elements one Dopri5 attempt reads or writes


def traffic_from_profiles(kernel_tag: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "counters_%s.json" % kernel_tag)
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for nm in rec["sources"]:
            h.update(open(os.path.join(ROOT, "paper_2309_05331_amd", "csrc", nm), "rb").read())
        if h.hexdigest() != rec["sources_sha256"]:
            return None
        return rec.get("hbm_bytes_per_launch", rec.get("hbm_bytes_per_run"))
    except Exception:
        return None


def _window(y, N, R, c):
    """The (2, W, W, W) periodic window of edge W = 2R + 1 centred on cell c."""
    idx = [np.arange(ci - R, ci + R + 1) % N for ci in c]
    return y[:, idx[0]][:, :, idx[1]][:, :, :, idx[2]]


def oracle_error(oracle, wl, chk):
    """The GPU's error against the FP64 oracle on the check runs made after
    the timed region (see gs_check_runs and the element-wise and ensemble
    runners).  Gray-Scott: a cell's value after E right-hand-side
    evaluations depends only on cells within E grid steps, so the oracle
    integrates the periodic window of edge 2R + 1 (R > E) around each sampled
    cell, with the grid spacing of the full grid, replaying the GPU's steps;
    the window's centre is exact.  Element-wise: the oracle replays the whole
    run on sampled components.  Ensemble: whole instances replayed."""
    bound32 = 1e-4
    if wl["kind"] == "gs":
        N = chk["N"]
        y0 = chk["y0"].reshape(2, N, N, N)
        kind = chk["kind"]
        if kind == "rk4":
            steps = chk["steps"]
            E = 4 * steps
        elif kind == "ab4":
            steps = chk["steps"]
            E = 13 * 3 + steps
        else:
            n_acc = int(chk["acc"].sum())
            E = {"dp5": 6, "ck54": 6, "f78": 13}[kind] * n_acc + 1
        R = E + 4
        full = 2 * R + 1 >= N
        W = N if full else 2 * R + 1
        sysd = oracle.gs_system(W, GS_PRM[0], GS_PRM[1], GS_PRM[2], GS_PRM[3], GS_PRM[4] * W / N)
        om = {"dp5": oracle.DOPRI5, "ck54": oracle.CASHKARP, "f78": oracle.FEHLBERG78}
        worst = 0.0
        cells = chk["cells"]
        if full and kind == "rk4" and N <= 32:
            # the whole workload (all timed steps) on the whole grid
            o, _ = oracle.integrate_n_steps(sysd, oracle.RK4, y0.astype(np.float64), 0.0, wl["dt"], steps)
            o = o.reshape(2, N, N, N)
            rel = max(float(np.max(np.abs(chk["full"][f] - o[f])) / np.max(np.abs(o[f]))) for f in range(2))
            return {"relative_per_field": rel, "bound": 1e-12, "what": "the whole run (%d RK4 steps) on the whole "
                    "grid" % steps}
        for ci, c in enumerate(cells):
            yw = y0.astype(np.float64) if full else _window(y0, N, R, c).astype(np.float64)
            ctr = (np.array([0, 1]) * W ** 3 + (c[0] * W + c[1]) * W + c[2]) if full else \
                (np.array([0, 1]) * W ** 3 + (R * W + R) * W + R)
            if kind == "rk4":
                yw, _ = oracle.integrate_n_steps(sysd, oracle.RK4, yw, 0.0, wl["dt"], steps)
            elif kind == "ab4":
                yw, _ = oracle.integrate_n_steps(sysd, oracle.AB(4), yw, 0.0, wl["dt"], steps)
            else:
                yw, _, _ = oracle.integrate_replay(sysd, yw, 0.0, chk["hs"], chk["acc"], 1e-6, 1e-6,
                                                   method=om[kind])
            worst = max(worst, float(np.max(np.abs(chk["gpu"][:, ci] - yw.ravel()[ctr]))))
        what = ("%d %s from the initial condition, oracle on periodic windows of edge %d around %d sampled cells"
                % (steps if kind in ("rk4", "ab4") else len(chk["hs"]),
                   "steps" if kind in ("rk4", "ab4") else "attempts (GPU step sequence replayed)", W, len(cells)))
        out = {"max_abs": worst, "bound": bound32 if chk["dtype"] == "f32" else None, "what": what}
        if chk["dtype"] == "f64":
            scale = float(np.max(np.abs(chk["gpu"])))
            out["relative"] = worst / scale
            out["bound"] = 1e-12
        if "t20" in chk:
            t20 = chk["t20"]
            rec = json.load(open(t20["golden"]))
            ref = np.array([rec["final"]["u"], rec["final"]["v"]])
            out["t0_to_20"] = {
                "max_abs_replaying_oracle_steps": float(np.max(np.abs(t20["replay"] - ref))),
                "max_abs_free_running": float(np.max(np.abs(t20["free"] - ref))),
                "gpu_accepted_rejected": t20["free_counts"], "oracle_accepted_rejected": t20["oracle_counts"],
                "what": "512^3 from t = 0 to 20 against the stored FP64 oracle run (%d sampled cells)"
                        % len(rec["final"]["cells"])}
        return out
    if wl["kind"] == "ew":
        m = chk["idx"].size
        x0 = chk["x0"].astype(np.float32).astype(np.float64) if chk["dtype"] == "f32" else chk["x0"]
        o, te, _ = oracle.integrate_replay(oracle.ew_system(oracle.EXP, m), x0, 0.0, chk["hs"], chk["acc"],
                                           1e-6, 1e-6)
        d = np.abs(chk["gpu"] - o)
        out = {"max_abs": float(d.max()), "relative": float(np.max(d / np.maximum(np.abs(o), 1e-300))),
               "what": "the whole run (%d attempts) replayed by the oracle on %d sampled components (the 64 "
                       "largest initial values among them)" % (len(chk["hs"]), m)}
        if chk["dtype"] == "f32":
            # the FP32 rounding bound of the state (x(5) <= 0.5 e^5)
            out["bound"] = 2 * chk["accepted"] * 2.0 ** -24 * 0.5 * math.exp(5.0)
            out["bound_reading"] = "2 n 2^-24 max|x(t1)| for n accepted steps (states far above order one)"
        else:
            out["bound"] = 1e-12
            out["bound_applies_to"] = "relative"
        return out
    worst, parts = 0.0, []
    for r in chk["instances"]:
        N = r["N"]
        sysd = oracle.gs_system(N, *r["prm"])
        y0 = inputs_ens_ic(r["i"], N).astype(np.float64).ravel()
        o, te, _ = oracle.integrate_replay(sysd, y0, 0.0, r["hs"], r["acc"], chk["rtol"], chk["rtol"])
        d = float(np.max(np.abs(r["gpu"] - o)))
        worst = max(worst, d)
        parts.append({"instance": r["i"], "N": N, "attempts": len(r["hs"]), "max_abs": d})
    return {"max_abs": worst, "bound": bound32, "instances": parts,
            "what": "whole instances (the first of each grid edge up to 48) over t 0 -> %g, the oracle replaying "
                    "each instance's GPU step sequence" % chk["t1"]}


def inputs_ens_ic(i, N):
    from paper_2309_05331_amd import inputs
    return inputs.ensemble_ic(i, N)


def cpu_baseline_leg(wl, check=None, budget_s=10.0):
    """Times the FP64 oracle on a bounded sample of the workload, and states
    the GPU's error against it on the check runs (test infrastructure;
    nothing else in this file touches the oracle).  Returns (cpu_baseline,
    error_vs_oracle)."""
    import oracle
    from paper_2309_05331_amd import inputs
    err = None
    if check is not None:
        t0 = time.perf_counter()
        err = oracle_error(oracle, wl, check)
        err["oracle_seconds"] = round(time.perf_counter() - t0, 1)
    if wl["kind"] == "gs":
        # the workload's own grid and start, continued from call to call, k
        # steps or attempts per call (about 5e8 cell-updates, so the
        # oracle's per-call set-up of its stage arrays is shared by several;
        # Adams-Bashforth on a 128^3 grid, each call restarting a history of 3
        # Fehlberg start-up steps and 97 steps), at least two calls, each
        # timed for the spread
        Ns = wl["N"] if wl["method"] != "ab4" else min(wl["N"], 128)
        k = 100 if wl["method"] == "ab4" else max(2, -(-500000000 // Ns ** 3))
        y = inputs.gray_scott_ic(Ns, seed=wl["seed"]).ravel()
        sysd = oracle.gs_system(Ns, *GS_PRM)
        done, t0, units, t, dt, rates = 0, time.perf_counter(), 0, 0.0, wl.get("dt0", 0.1), []
        while done < 2 or time.perf_counter() - t0 < budget_s:
            tc, u = time.perf_counter(), 0
            if wl["method"] in ("rk4", "ab4"):
                y, t = oracle.integrate_n_steps(sysd, oracle.RK4 if wl["method"] == "rk4" else oracle.AB(4), y, t,
                                                wl["dt"], k)
                u = k * Ns ** 3
            else:
                om = {"ck54": oracle.CASHKARP, "f78": oracle.FEHLBERG78}.get(wl["method"], oracle.DOPRI5)
                y, st, _ = oracle.integrate_adaptive(sysd, y, t, 1e9, dt, 1e-6, 1e-6, max_steps=k, method=om)
                t, dt = st["t"], st["dt_next"]
                u = st["accepted"] * Ns ** 3
            rates.append(u / (time.perf_counter() - tc))
            units += u
            done += 1
        el = time.perf_counter() - t0
        what = {"rk4": "RK4 steps", "dp5": "adaptive Dopri5 attempts", "ck54": "adaptive Cash-Karp attempts",
                "f78": "adaptive Fehlberg 7(8) attempts",
                "ab4": "Adams-Bashforth 4 steps (each call with 3 Fehlberg start-up steps)"}[wl["method"]]
        sample = "%s, %d per call, on the %d^3 grid of the workload (same start and parameters), %d calls, %.1f s" % (
            what, k, Ns, done, el)
        unit = "cell-updates/s"
        sd = float(np.std(rates, ddof=1))
    elif wl["kind"] == "ens":
        edges, F, k = inputs.ensemble_draws(wl["n"], seed=wl["seed"])
        t0, units, i, t = time.perf_counter(), 0, 0, 0.0
        while time.perf_counter() - t0 < budget_s and i < wl["n"]:
            N = edges[i]
            y = inputs.ensemble_ic(i, N).astype(np.float64).ravel()
            sysd = oracle.gs_system(N, GS_PRM[0], GS_PRM[1], F[i], k[i], GS_PRM[4])
            _, st, _ = oracle.integrate_adaptive(sysd, y, 0.0, wl["t1"], wl["dt0"], wl["rtol"], wl["rtol"],
                                                 max_steps=20)
            units += st["accepted"] * N ** 3
            i += 1
        el = time.perf_counter() - t0
        sample = "the first %d ensemble instances, their first 20 adaptive Dopri5 attempts each, %.1f s" % (i, el)
        unit = "cell-updates/s"
    else:
        n = 1 << 20
        x0 = inputs.exp_family_x0(n, seed=wl["seed"])
        sysd = oracle.ew_system(oracle.EXP, n)
        t0, units, reps = time.perf_counter(), 0, 0
        while time.perf_counter() - t0 < budget_s:
            _, st, _ = oracle.integrate_adaptive(sysd, x0, 0.0, 5.0, 0.01, 1e-6, 1e-6)
            units += st["accepted"] * n
            reps += 1
        el = time.perf_counter() - t0
        sample = "%d adaptive Dopri5 runs t 0->5 on 2^20 components, %.1f s" % (reps, el)
        unit = "component-updates/s"
    cb = {"value": units / el, "unit": unit, "cores": oracle.num_threads(), "kind": "oracle", "sample": sample,
          "cpu_model": cpu_model()}
    if wl["kind"] == "gs":
        cb["sd_between_calls"] = sd
    return cb, err


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def timed_steps(one_step, steps):
    """Runs the timed steps between device synchronisations; returns the
    total seconds and the per-step seconds."""
    import torch
    per = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        one_step()
        torch.cuda.synchronize()
        per.append(time.perf_counter() - ts)
    return time.perf_counter() - t0, per


def run_ens(wl, steps, warmup):
    """The batched ensemble: 512 Gray-Scott instances (edges uniform over
    16..96, F and k drawn per instance), each integrated adaptively over the
    whole horizon; one step restarts every instance from its initial
    condition (device-resident, copied in inside the step)."""
    import torch
    from paper_2309_05331_amd import hode, inputs
    n = wl["n"]
    edges, F, k = inputs.ensemble_draws(n, seed=wl["seed"])
    prms = [[GS_PRM[0], GS_PRM[1], F[i], k[i], GS_PRM[4]] for i in range(n)]
    # instance i starts from the initial condition of seed 4000 + i
    ics = [torch.from_numpy(inputs.ensemble_ic(i, N).ravel()).to("cuda:0") for i, N in enumerate(edges)]
    ens = hode.Ensemble(edges, prms, dtype=hode.F32)
    ens.set_tolerances(wl["rtol"], wl["rtol"])
    ens.set_controller(hode.CTRL_PI)
    if wl.get("tiles", "auto") == "auto":
        ens.autotune(8)  # tile shape per grid edge, timed inside the whole ensemble
    if wl.get("epoch"):
        ens.set_epoch(wl["epoch"], wl["epoch"])
    tiles = {}
    for i, N in enumerate(edges):
        tiles.setdefault(str(N), list(ens.instance_tile(i)))
    cells = np.array(edges, dtype=np.float64) ** 3
    tot = {"acc": 0, "acc_inst": 0, "rej": 0, "cell_att": 0.0, "kernel_ms": 0.0, "launches": 0}

    def one_step():
        for i in range(n):
            ens.init_instance(i, ics[i])
        st = ens.integrate_adaptive(0.0, wl["t1"], wl["dt0"], max_steps=10 ** 6)
        assert all(x["status"] == 0 for x in st)
        acc = np.array([x["accepted"] for x in st])
        rej = np.array([x["rejected"] for x in st])
        kms, nl = ens.timing()
        tot["acc"] += float((cells * acc).sum())  # cell-weighted: the metric's cell updates
        tot["acc_inst"] += int(acc.sum())
        tot["rej"] += int(rej.sum())
        tot["cell_att"] += float((cells * (acc + rej)).sum())
        tot["kernel_ms"] += kms
        tot["launches"] += nl
        tot["instance_attempts"] = int((acc + rej).sum())

    for _ in range(warmup):
        one_step()
    for key in ("acc", "acc_inst", "rej", "cell_att", "kernel_ms", "launches"):
        tot[key] = 0
    el, per = timed_steps(one_step, steps)
    # oracle check (after the timed region): the same integration with every
    # instance's step sequence recorded; the first instance of each grid
    # edge up to 48 is replayed by the oracle on its whole state
    ens.set_trace(4000)
    for i in range(n):
        ens.init_instance(i, ics[i])
    st = ens.integrate_adaptive(0.0, wl["t1"], wl["dt0"], max_steps=4000)
    check = {"instances": [], "t1": wl["t1"], "rtol": wl["rtol"]}
    seen = set()
    for i, N in enumerate(edges):
        if N > 48 or N in seen:
            continue
        seen.add(N)
        tr = ens.read_instance_trace(i)
        o = np.empty(2 * N ** 3, dtype=np.float32)
        ens.read_instance(i, o)
        check["instances"].append({"i": i, "N": N, "prm": prms[i], "hs": tr[:, 0].copy(),
                                   "acc": tr[:, 2].astype(np.int32), "gpu": o.astype(np.float64),
                                   "status": st[i]["status"]})
    ens.set_trace(0)
    ens.close()
    # algorithmic bytes: 30 arrays per attempt plus the first k1 (2 arrays) per
    # instance and step
    abytes = (DP5_ARRAYS * tot["cell_att"] + 2 * steps * cells.sum()) * 2 * 4
    return dict(elapsed=el, per_step=per, cells=1, accepted=tot["acc"], rejected=tot["rej"], dom="ens_kernel",
                dom_ms=tot["kernel_ms"], dom_bytes=abytes, stage_gbs=None, check=check, tiles=tiles,
                attempt_gbs=abytes / el / 1e9, tile=None, launches=tot["launches"],
                instance_attempts=tot["instance_attempts"], accepted_steps=tot["acc_inst"])


def gs_sample_cells(N, extra=8, seed=0):
    """Cells (z, y, x) whose values the oracle checks: the cube's corners and
    faces, the domain's corners (periodic wrap), the centre, seeded random
    cells."""
    a, b, m = 3 * N // 8, 5 * N // 8 - 1, N // 2
    pts = [(a, a, a), (b, b, b), (a, b, a), (b, a, b), (a, m, m), (m, m, b), (m, a, m), (m, m, m),
           (0, 0, 0), (N - 1, N - 1, N - 1), (0, N - 1, m), (m, 0, N - 1), (max(a - 1, 0), a, min(b + 1, N - 1))]
    rng = np.random.default_rng(seed)
    return pts + [tuple(int(v) for v in rng.integers(0, N, size=3)) for _ in range(extra)]


GS_CHECK_ATTEMPTS = 4  # attempts (or steps) of the short check run from the initial condition


def gs_check_runs(ctx, wl, y0, method):
    """GPU runs for the oracle check, after the timed region, in the timed
    launch configuration: the first few attempts (steps) from the initial
    condition, with the GPU's values at sampled cells and its step sequence;
    for the 512^3 Dopri5 workload also the run to t = 20 (free-running, and
    replaying the steps of the stored FP64 oracle run) at the stored oracle
    run's sampled cells."""
    from paper_2309_05331_amd import hode
    N = wl["N"]
    ctx.init_state(y0, grid=N)
    out = {"kind": wl["method"], "y0": y0, "N": N, "dtype": wl["dtype"]}
    if wl["method"] in ("rk4", "ab4"):
        # (a grid small enough for the oracle's whole grid: the whole workload)
        out["steps"] = (wl["steps_per"] if N <= 32 else 10) if wl["method"] == "rk4" else 8
        ctx.integrate_n_steps(method, 0.0, wl["dt"], out["steps"])
    else:
        ctx.set_trace(64)
        st = ctx.integrate_adaptive(0.0, 1e9, wl.get("dt0", 0.1), max_steps=GS_CHECK_ATTEMPTS)
        assert st["status"] == hode.EMAXSTEPS, st
        tr = ctx.read_trace()
        out["hs"], out["acc"] = tr[:, 0].copy(), tr[:, 2].astype(np.int32)
        ctx.set_trace(0)
    g = np.empty(2 * N ** 3, dtype=np.float32 if wl["dtype"] == "f32" else np.float64)
    ctx.read_state(g)
    g = g.reshape(2, N, N, N)
    out["cells"] = gs_sample_cells(N)
    out["gpu"] = np.array([[g[f][c] for c in out["cells"]] for f in range(2)], dtype=np.float64)
    if N <= 32:
        out["full"] = g.astype(np.float64)
    del g
    golden = os.path.join(ROOT, "tests", "golden", "oracle_gs512-dp5-t20.json")
    if wl["method"] == "dp5" and N == 512 and wl["dtype"] == "f32" and os.path.exists(golden):
        rec = json.load(open(golden))
        cells = [tuple(c) for c in rec["final"]["cells"]]
        ctx.init_state(y0, grid=N)
        st = ctx.integrate_adaptive(0.0, rec["t1"], rec["dt0"])
        g = np.empty(2 * N ** 3, dtype=np.float32)
        ctx.read_state(g)
        g = g.reshape(2, N, N, N)
        free = np.array([[g[f][c] for c in cells] for f in range(2)], dtype=np.float64)
        ctx.init_state(y0, grid=N)
        t = 0.0
        for h, acc in zip(rec["h"], rec["accepted_flags"]):
            if acc:
                ctx.do_step(hode.DOPRI5, t, h)
                t += h
        ctx.read_state(g)
        g = g.reshape(2, N, N, N)
        replay = np.array([[g[f][c] for c in cells] for f in range(2)], dtype=np.float64)
        del g
        out["t20"] = {"golden": golden, "free": free, "replay": replay, "free_counts": [st["accepted"], st["rejected"]],
                      "oracle_counts": [rec["accepted"], rec["rejected"]]}
    return out


def run_gs(wl, steps, warmup, ctrl_kind, weights=None, tile=None):
    import torch
    from paper_2309_05331_amd import hode, inputs
    N = wl["N"]
    np_dt = np.float32 if wl["dtype"] == "f32" else np.float64
    y0 = inputs.gray_scott_ic(N, seed=wl["seed"], dtype=np_dt).ravel()
    dev = torch.from_numpy(y0).to("cuda:0")
    ctx = hode.Context(0)
    ctx.set_rhs(hode.RHS_GRAYSCOTT3D, GS_PRM)
    ctx.init_state(dev, grid=N)
    del dev
    torch.cuda.synchronize()
    ctx.set_tolerances(1e-6, 1e-6)
    ctx.set_controller(ctrl_kind, weights)
    method = {"rk4": hode.RK4, "dp5": hode.DOPRI5, "ck54": hode.CASHKARP54, "f78": hode.FEHLBERG78,
              "ab4": hode.AB(4)}[wl["method"]]
    if method in (hode.CASHKARP54, hode.FEHLBERG78):
        ctx.set_stepper(method)
    if tile is None:
        # project autotuner: fastest (ry, zc, nw) per stage for this grid;
        # with HODE_TUNE_CACHE set, a rerun of the same command (a profiled
        # one) restores the tiles of the first run without timing
        ctx.autotune_cached(method, 3)
    else:
        if len(tile) == 3:
            ctx.set_tile_waves(tile[2])
        ctx.set_tile(tile[0], tile[1])
    state = {"t": 0.0, "dt": wl.get("dt0", 0.1), "acc": 0, "rej": 0}

    def one_step():
        if wl["method"] in ("rk4", "ab4"):
            # (Adams-Bashforth: the history continues from step to step)
            ctx.integrate_n_steps(method, state["t"], wl["dt"], wl["steps_per"])
            state["t"] += wl["steps_per"] * wl["dt"]
            state["acc"] += wl["steps_per"]
        else:
            st = ctx.integrate_adaptive(state["t"], state["t"] + wl["window"], state["dt"])
            assert st["status"] == 0, st
            state["t"] = st["t"]
            state["dt"] = st["dt_next"]
            state["acc"] += st["accepted"]
            state["rej"] += st["rejected"]

    for _ in range(warmup):
        one_step()
    state["acc"] = state["rej"] = 0
    el, per = timed_steps(one_step, steps)
    no_graph = None
    if wl.get("compare_graphs"):
        # the same steps with every kernel enqueued on the stream instead of
        # replayed from captured graphs (launch overhead of a small grid)
        acc0 = state["acc"]
        ctx.set_graphs(False)
        el_ng, _ = timed_steps(one_step, steps)
        ctx.set_graphs(True)
        no_graph = {"value": N ** 3 * (state["acc"] - acc0) / el_ng, "ms_per_step": el_ng / steps * 1e3}
        state["acc"] = acc0  # the value counts the timed (graph) steps only
    # per-stage durations: HIP events around every stage kernel of attempts
    # replayed in the same order on the library's stream, right after the
    # timed region
    kinds = STAGES[wl["method"]]
    prof = ctx.profile_attempt(method, 10)  # (ends an Adams-Bashforth history: after the timed steps)
    ms = dict(zip(kinds, prof))
    dom = max(kinds, key=lambda k: ms[k])
    esz = 4 if wl["dtype"] == "f32" else 8
    arr_bytes = 2 * N ** 3 * esz
    bytes_dom = GS_ARRAYS[dom] * arr_bytes
    stage_gbs = {GS_NAMES[k]: round(GS_ARRAYS[k] * arr_bytes / (ms[k] * 1e-3) / 1e9, 1) for k in kinds}
    step_bytes = sum(GS_ARRAYS[k] for k in kinds) * arr_bytes
    attempt_ms = sum(ms.values())
    ry, zc = ctx.get_tile()
    kind_tiles = {GS_NAMES[k]: list(ctx.kind_tile(k)) for k in kinds}
    check = gs_check_runs(ctx, wl, y0, method)
    ctx.close()
    return dict(elapsed=el, per_step=per, no_graph=no_graph, cells=N ** 3, accepted=state["acc"], rejected=state["rej"],
                t_end=state["t"],
                dom=GS_NAMES[dom], dom_ms=ms[dom], dom_bytes=bytes_dom, stage_gbs=stage_gbs,
                attempt_gbs=step_bytes / (attempt_ms * 1e-3) / 1e9, tile=[ry, zc], kind_tiles=kind_tiles,
                check=check)


def run_ew(wl, steps, warmup):
    import torch
    from paper_2309_05331_amd import hode, inputs
    n = wl["n"]
    esz = 4 if wl["dtype"] == "f32" else 8
    x0 = inputs.exp_family_x0(n, seed=wl["seed"]).astype(np.float32 if esz == 4 else np.float64)
    dev = torch.from_numpy(x0).to("cuda:0")
    ctx = hode.Context(0)
    ctx.set_rhs(hode.RHS_EXP)
    acc = [0]

    def one_step():
        ctx.init_state(dev)  # device-to-device copy of the initial values
        st = ctx.integrate_adaptive(0.0, wl["t1"], wl["dt0"])
        assert st["status"] == 0
        acc[0] += st["accepted"]

    for _ in range(warmup):
        one_step()
    acc[0] = 0
    el, per = timed_steps(one_step, steps)
    ms = ctx.time_kernel(hode.DOPRI5, 20)
    # oracle check (after the timed region): the same run with its step
    # sequence recorded, the GPU's values at sampled components
    ctx.init_state(dev)
    ctx.set_trace(10000)
    st = ctx.integrate_adaptive(0.0, wl["t1"], wl["dt0"])
    tr = ctx.read_trace()
    g = np.empty(n, dtype=x0.dtype)
    ctx.read_state(g)
    rng = np.random.default_rng(0)
    idx = np.unique(np.concatenate([np.argsort(x0)[-64:], rng.integers(0, n, size=1 << 16)]))
    check = {"idx": idx, "x0": x0[idx].astype(np.float64), "gpu": g[idx].astype(np.float64), "hs": tr[:, 0].copy(),
             "acc": tr[:, 2].astype(np.int32), "t1": wl["t1"], "dtype": wl["dtype"], "accepted": st["accepted"]}
    del g
    ctx.close()
    return dict(elapsed=el, per_step=per, cells=n, accepted=acc[0], rejected=0, dom="ew_step_dp5", dom_ms=ms, check=check,
                dom_bytes=2 * n * esz, stage_gbs=None, attempt_gbs=2 * n * esz / (ms * 1e-3) / 1e9, tile=None)


def run_ab(N, t1, weights_path, dtype="f32", repeats=3, ref_rtol=1e-8, deadline=None):
    """Wall time to integrate the whole horizon with PI and with the learned
    controller (same grid, tolerances, start and autotuned tiles), `repeats`
    runs each in alternating order (PI, learned, learned, PI, ...), and each
    controller's final error against an FP64 run of the same start at rtol =
    atol = ref_rtol (0: no reference; skipped when the wall clock has passed
    `deadline`, so the whole benchmark stays within its time limit)."""
    import tempfile
    import torch
    from paper_2309_05331_amd import hode, inputs
    np_dt = np.float32 if dtype == "f32" else np.float64
    y0h = inputs.gray_scott_ic(N, seed=5, dtype=np_dt).ravel()
    y0 = torch.from_numpy(y0h).to("cuda:0")
    wb = np.load(weights_path)
    cache = os.path.join(tempfile.mkdtemp(prefix="hode_ab_"), "tune.txt")
    kinds = {"pi": (hode.CTRL_PI, None), "learned": (hode.CTRL_MLP, wb)}
    order = []
    for r in range(repeats):
        order += ["pi", "learned"] if r % 2 == 0 else ["learned", "pi"]
    runs = {"pi": [], "learned": []}
    finals = {}
    for name in order:
        kind, w = kinds[name]
        ctx = hode.Context(0)
        ctx.set_rhs(hode.RHS_GRAYSCOTT3D, GS_PRM)
        ctx.init_state(y0, grid=N)
        ctx.set_tolerances(1e-6, 1e-6)
        ctx.set_controller(kind, w)
        ctx.autotune_cached(hode.DOPRI5, 3, cache)  # the first run tunes, the others read the same tiles
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.integrate_adaptive(0.0, t1, 0.1, max_steps=10 ** 7)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        assert st["status"] == 0, st
        runs[name].append({"wall_s": el, "accepted": st["accepted"], "rejected": st["rejected"]})
        if name not in finals:
            g = np.empty(2 * N ** 3, dtype=np_dt)
            ctx.read_state(g)
            finals[name] = g
        print(json.dumps({name: runs[name][-1]}), file=sys.stderr, flush=True)
        ctx.close()
    res = {"order": order, "t1": t1, "rtol": 1e-6}
    for name in ("pi", "learned"):
        w = np.array([r["wall_s"] for r in runs[name]])
        res[name] = {"wall_s_mean": float(w.mean()), "wall_s_sd": float(w.std(ddof=1)) if w.size > 1 else None,
                     "wall_s": [round(float(v), 4) for v in w], "accepted": runs[name][0]["accepted"],
                     "rejected": runs[name][0]["rejected"],
                     "attempts": runs[name][0]["accepted"] + runs[name][0]["rejected"],
                     "cell_updates_per_s": N ** 3 * runs[name][0]["accepted"] / float(w.mean())}
    wl, wp = np.array(res["learned"]["wall_s"]), np.array(res["pi"]["wall_s"])
    res["wall_ratio_learned_over_pi"] = float(wl.mean() / wp.mean())
    # sd of the ratio from the two means' sds (first order)
    if wl.size > 1:
        res["wall_ratio_sd"] = float(res["wall_ratio_learned_over_pi"] * math.sqrt(
            (wl.std(ddof=1) / wl.mean()) ** 2 + (wp.std(ddof=1) / wp.mean()) ** 2))
    if ref_rtol > 0 and deadline is not None and time.time() > deadline:
        res["reference"] = "skipped: the time budget of the benchmark run was spent"
    elif ref_rtol > 0:
        ctx = hode.Context(0)
        ctx.set_rhs(hode.RHS_GRAYSCOTT3D, GS_PRM)
        ctx.init_state(y0h.astype(np.float64), grid=N)
        ctx.set_tolerances(ref_rtol, ref_rtol)
        ctx.autotune(hode.DOPRI5, 3)
        t0 = time.perf_counter()
        # in windows of 100 time units, one progress line each (the proposed
        # step carries over from one window to the next)
        t, dt, acc, rej = 0.0, 0.1, 0, 0
        while t < t1:
            te = min(t1, t + 100.0)
            st = ctx.integrate_adaptive(t, te, dt, max_steps=10 ** 7)
            assert st["status"] == 0, st
            t, dt, acc, rej = st["t"], st["dt_next"], acc + st["accepted"], rej + st["rejected"]
            print(json.dumps({"reference_t": t, "accepted": acc, "wall_s": round(time.perf_counter() - t0, 1)}),
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = {"accepted": acc, "rejected": rej}
        ref = np.empty(2 * N ** 3, dtype=np.float64)
        ctx.read_state(ref)
        ctx.close()
        res["reference"] = {"dtype": "f64", "rtol": ref_rtol, "accepted": st["accepted"], "rejected": st["rejected"],
                            "wall_s": round(el, 2),
                            "checked": "the FP64 stage kernels agree with the FP64 oracle to 1e-12 relative when "
                                       "both take the same steps (parity tests)"}
        for name in ("pi", "learned"):
            d = np.abs(finals[name].astype(np.float64) - ref)
            res[name]["final_max_abs_error_vs_reference"] = float(d.max())
            res[name]["final_mean_abs_error_vs_reference"] = float(d.mean())
        del ref
    return res


def run_accuracy(n=512 * 512, t1=5.0):
    """The paper's accuracy benchmark on the GPU path: every fixed-step
    method on the exponential and logistic families (n components, x0 in
    [0.01, 0.5]) against the closed forms at t1, L-inf and L2 norms of the
    error under step halving, and the observed order (log2 of successive
    L-inf ratios).  FP64."""
    import torch
    from paper_2309_05331_amd import hode, inputs
    x0 = inputs.exp_family_x0(n, seed=2)
    dev = torch.from_numpy(x0).to("cuda:0")
    methods = ([("euler", hode.EULER, 1), ("midpoint", hode.MIDPOINT, 2), ("rk4", hode.RK4, 4),
                ("cashkarp54", hode.CASHKARP54, 5), ("dopri5", hode.DOPRI5, 5), ("fehlberg78", hode.FEHLBERG78, 8)]
               + [("ab%d" % s, hode.AB(s), s) for s in range(1, 9)]
               + [("abm%d" % s, hode.ABM(s), s) for s in range(1, 9)])
    steps = [10, 20, 40, 80, 160, 320, 640, 1280]
    out = []
    for kind, kname in ((hode.RHS_EXP, "exp"), (hode.RHS_LOGISTIC, "logistic")):
        exact = x0 * np.exp(t1) if kind == hode.RHS_EXP else x0 / (x0 + (1 - x0) * np.exp(-t1))
        ctx = hode.Context(0)
        ctx.set_rhs(kind)
        y = np.empty(n)
        for name, m, p in methods:
            linf, l2 = [], []
            for ns in steps:
                ctx.init_state(dev)
                ctx.integrate_n_steps(m, 0.0, t1 / ns, ns)
                ctx.read_state(y)
                e = y - exact
                linf.append(float(np.max(np.abs(e))) if np.all(np.isfinite(e)) else float("inf"))
                l2.append(float(np.sqrt(np.sum(e * e))) if np.all(np.isfinite(e)) else float("inf"))
            orders = [round(math.log2(linf[i] / linf[i + 1]), 2) if 0 < linf[i + 1] < math.inf and linf[i] < math.inf
                      else None for i in range(len(steps) - 1)]
            rec = {"family": kname, "method": name, "expected_order": p, "steps": steps, "linf": linf, "l2": l2,
                   "observed_order": orders}
            out.append(rec)
            print(json.dumps(rec), flush=True)
        ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="gs512-dp5", choices=sorted(WORKLOADS))
    ap.add_argument("--controller", default="pi", choices=["pi", "i"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-ceiling", action="store_true",
                    help="skip timing the plain streaming copy beside the workload")
    ap.add_argument("--tile", default="auto", help="auto (autotune; through $HODE_TUNE_CACHE when set) or "
                                                   "RY,ZC[,NW]; ensemble: auto or default (the kernel's own "
                                                   "plane-chunk sizing, no autotuning)")
    ap.add_argument("--ens-epoch", type=int, default=0,
                    help="ensemble: attempts per launch (0: one launch for the whole integration)")
    ap.add_argument("--ab", type=float, default=None, metavar="T1",
                    help="also integrate the workload grid from 0 to T1 with PI and with the learned controller "
                         "(default: T1 = 2000 for the default workload, the metric's wall-time comparison over "
                         "the workload's horizon; 0 = off)")
    ap.add_argument("--ab-repeats", type=int, default=3, help="runs per controller in the comparison")
    ap.add_argument("--ab-ref-rtol", type=float, default=1e-8,
                    help="tolerance of the FP64 reference run of the comparison (0 = no reference)")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2309_05331_amd", "controller_weights.npy"))
    ap.add_argument("--accuracy", action="store_true",
                    help="print the accuracy benchmark (error norms and observed orders of every fixed-step method)")
    ap.add_argument("--copy-reference", action="store_true",
                    help="time only the plain 16-byte streaming copy of 1 GiB (bandwidth ceiling, counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; the sharding plan is documented with the design.",
              file=sys.stderr)
        sys.exit(2)
    from paper_2309_05331_amd import hode
    if args.accuracy:
        run_accuracy()
        return
    if args.copy_reference:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        ms, gbs = hode.stream_copy(dst, src, reps=max(args.steps, 1))
        print(json.dumps({"reference": "stream_copy", "bytes_read": src.numel() * 4, "bytes_written": src.numel() * 4,
                          "ms_per_copy": ms, "GBps": gbs, "frac_of_8TBps": gbs / PEAK_HBM_GBS}), flush=True)
        return
    wl = WORKLOADS[args.workload]
    ctrl = {"pi": hode.CTRL_PI, "i": hode.CTRL_I}[args.controller]
    if wl["kind"] == "gs":
        tile = None if args.tile == "auto" else tuple(int(v) for v in args.tile.split(","))
        assert tile is None or len(tile) in (2, 3), "--tile RY,ZC or RY,ZC,NW"
        r = run_gs(wl, args.steps, args.warmup, ctrl, tile=tile)
        unit = "cell-updates/s"
        cfg = {"workload": args.workload, "grid": [wl["N"]] * 3, "fields": 2,
               "method": {"dp5": "dopri5-adaptive", "ck54": "cashkarp54-adaptive", "rk4": "rk4-fixed",
                          "f78": "fehlberg78-adaptive", "ab4": "adams-bashforth4-fixed"}[wl["method"]],
               "rtol": None if wl["method"] in ("rk4", "ab4") else 1e-6, "controller": args.controller,
               "window_time_units": wl.get("window"), "dt": wl.get("dt"), "tile_ry_zc": r["tile"],
               "stage_tiles_ry_zc_nw": r["kind_tiles"],
               "params": {"Du": GS_PRM[0], "Dv": GS_PRM[1], "F": GS_PRM[2], "k": GS_PRM[3], "L": GS_PRM[4]}}
    elif wl["kind"] == "ens":
        r = run_ens(dict(wl, tiles="auto" if args.tile == "auto" else "default", epoch=args.ens_epoch), args.steps,
                    args.warmup)
        unit = "cell-updates/s"
        cfg = {"workload": args.workload, "instances": wl["n"], "edges": "uniform over 16..96 step 8", "fields": 2,
               "method": "dopri5-adaptive", "rtol": wl["rtol"], "controller": "pi", "t": [0.0, wl["t1"]],
               "launch": "one persistent kernel launch per integration, captured in a hipGraph (lock-step rounds "
                         "of stage phases over per-XCD tile queues, grid barriers)",
               "launches_per_step": r["launches"] / max(args.steps, 1), "tiles_per_edge_vw_planes": r["tiles"]}
    else:
        r = run_ew(wl, args.steps, args.warmup)
        unit = "component-updates/s"
        cfg = {"workload": args.workload, "components": wl["n"], "rhs": "exp", "method": "dopri5-adaptive",
               "rtol": 1e-6, "t": [0.0, wl["t1"]]}
    value = r["cells"] * r["accepted"] / r["elapsed"]
    achieved = r["dom_bytes"] / (r["dom_ms"] * 1e-3) / 1e9
    tag = "%s_%s" % (r["dom"], args.workload)
    per = np.array(r["per_step"]) * 1e3
    out = {
        "metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["elapsed"] / args.steps * 1e3,
        "ms_per_step_sd": round(float(per.std(ddof=1)), 3) if per.size > 1 else None,
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": wl["dtype"], "data": "synthetic", "config": cfg,
        "accepted_steps": r.get("accepted_steps", r["accepted"]), "rejected_steps": r["rejected"],
        "roofline": {"bound": "hbm", "kernel": r["dom"], "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic_from_profiles(tag)},
        "stage_gbs": r["stage_gbs"], "attempt_gbs": round(r["attempt_gbs"], 1),
    }
    if r.get("no_graph"):
        out["without_graphs"] = r["no_graph"]
    if not args.no_copy_ceiling:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        cms, cgbs = hode.stream_copy(dst, src, reps=10)
        del src, dst
        out["copy_ceiling"] = {"kernel": "hode_stream_copy", "bytes": 2 << 30, "GBps": round(cgbs, 1),
                               "frac_of_peak": round(cgbs / PEAK_HBM_GBS, 4),
                               "dominant_kernel_frac_of_copy": round(achieved / cgbs, 4)}
    ab_t1 = args.ab if args.ab is not None else (2000.0 if args.workload == "gs512-dp5" else 0.0)
    if ab_t1 > 0 and wl["kind"] == "gs":
        out["controller_ab"] = run_ab(wl["N"], ab_t1, args.weights, wl["dtype"], args.ab_repeats, args.ab_ref_rtol,
                                      deadline=T_START + 330.0)
    if not args.no_cpu_baseline:
        cb, err = cpu_baseline_leg(wl, r.get("check"))
        out["cpu_baseline"] = cb
        out["error_vs_oracle"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
