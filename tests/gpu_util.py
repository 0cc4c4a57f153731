"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare with the FP64 oracle."""
import numpy as np

from paper_2309_05331_amd import hode


def rel_err(g, o):
    """max |g - o| / max |o| (per whole array)."""
    g = np.asarray(g, dtype=np.float64).ravel()
    o = np.asarray(o, dtype=np.float64).ravel()
    den = np.max(np.abs(o))
    return float(np.max(np.abs(g - o)) / (den if den > 0 else 1.0))


def rel_err_fields(g, o, nfields):
    g = np.asarray(g, dtype=np.float64).reshape(nfields, -1)
    o = np.asarray(o, dtype=np.float64).reshape(nfields, -1)
    return max(rel_err(g[f], o[f]) for f in range(nfields))


def gs_ctx(y0, N, prm=None, tile=None):
    ctx = hode.Context(0)
    p = prm or dict(Du=2e-5, Dv=1e-5, F=0.053, k=0.014, L=2.5)
    ctx.set_rhs(hode.RHS_GRAYSCOTT3D, [p["Du"], p["Dv"], p["F"], p["k"], p["L"]])
    ctx.init_state(np.ascontiguousarray(y0).ravel(), grid=N)
    if tile:
        ctx.set_tile(*tile)
    return ctx


def ew_ctx(kind, x0):
    ctx = hode.Context(0)
    ctx.set_rhs(kind)
    ctx.init_state(np.ascontiguousarray(x0))
    return ctx


def read(ctx, dtype, n):
    out = np.empty(n, dtype=dtype)
    ctx.read_state(out)
    return out
