"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmark.

This module draws random numbers and lays out initial conditions; it holds none
of the time-stepping arithmetic.  Both sides of every parity test receive the
same bytes from here, so the initial condition never takes part in parity.

Random numbers: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), used counter-based: draw ``i`` of stream
``(seed, stream)`` is ``mix(key + (i + 1) * GAMMA)`` with
``key = mix(mix(seed + GAMMA) ^ (stream * GAMMA2))``, where ``mix`` is the
SplitMix64 finaliser.  A uniform in [0, 1) is the top 53 bits times 2**-53.

Workloads (the paper's accuracy and scalability benchmarks, "Accuracy
Benchmarks" and "Scalability Benchmarks" sections):

* element-wise families: ``x0 ~ U[0.01, 0.5]``;
* 3D Gray-Scott on an ``N^3`` periodic grid, x fastest, field u then field v:
  ``u = 1, v = 0`` except a central cube ``[3N/8, 5N/8)^3`` (edge N/4) with
  ``u = 0.5, v = 0.25``; then uniform noise ``0.01 * (2r - 1)`` is added to both
  fields at every cell from two independent streams (stream 0 for u, 1 for v);
* ensemble draws: per instance an edge from ``{16, 24, ..., 96}``,
  ``F ~ U[0.02, 0.06]``, ``k ~ U[0.045, 0.065]``.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
GAMMA2 = np.uint64(0xD1B54A32D192ED03)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Gray-Scott parameters of the scalability benchmark as used here:
# diffusivities 2e-5 / 1e-5, feed F = 0.053, kill k = 0.014, box edge 2.5.
GS_DEFAULT = dict(Du=2e-5, Dv=1e-5, F=0.053, k=0.014, L=2.5)

_CHUNK = 1 << 22


def _mix(z: np.ndarray) -> np.ndarray:
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def _key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        s = _mix(np.array([seed], dtype=np.uint64) + GAMMA)
        s ^= np.array([stream], dtype=np.uint64) * GAMMA2
        return _mix(s)[0]


def uniform(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """Draws ``start .. start+n-1`` of stream ``(seed, stream)`` as float64 in [0, 1)."""
    key = _key(seed, stream)
    out = np.empty(n, dtype=np.float64)
    scale = 2.0 ** -53
    with np.errstate(over="ignore"):
        for lo in range(0, n, _CHUNK):
            hi = min(n, lo + _CHUNK)
            idx = np.arange(start + lo + 1, start + hi + 1, dtype=np.uint64)
            z = _mix(idx * GAMMA + key)
            out[lo:hi] = (z >> np.uint64(11)).astype(np.float64) * scale
    return out


def uniform_at(seed: int, stream: int, idx) -> np.ndarray:
    """Draws at the 0-based positions ``idx`` of stream ``(seed, stream)``: the
    same values as ``uniform(seed, stream, n)[idx]``, without drawing the rest."""
    key = _key(seed, stream)
    i = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = _mix((i + np.uint64(1)) * GAMMA + key)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _signed(v) -> int:
    """A 64-bit word as the int64 value with the same bits."""
    v = int(v)
    return v - (1 << 64) if v >= 1 << 63 else v


def _mix_torch(z):
    """The SplitMix64 finaliser on int64 tensors (products wrap modulo 2**64;
    the right shifts are made logical by masking the sign extension)."""
    z = z ^ ((z >> 30) & ((1 << 34) - 1))
    z = z * _signed(_M1)
    z = z ^ ((z >> 27) & ((1 << 37) - 1))
    z = z * _signed(_M2)
    return z ^ ((z >> 31) & ((1 << 33) - 1))


def uniform_torch(seed: int, stream: int, n: int, start: int = 0, device=None):
    """``uniform(seed, stream, n, start)`` drawn on a torch device (float64),
    for inputs too large to draw on the host in reasonable time."""
    import torch

    idx = torch.arange(start + 1, start + n + 1, dtype=torch.int64, device=device)
    z = _mix_torch(idx * _signed(GAMMA) + _signed(_key(seed, stream)))
    return ((z >> 11) & ((1 << 53) - 1)).to(torch.float64) * (2.0 ** -53)


def exp_family_x0(n: int, seed: int = 2) -> np.ndarray:
    """Initial values of ``n`` independent components, ``U[0.01, 0.5]`` (float64)."""
    return 0.01 + 0.49 * uniform(seed, 0, n)


def gray_scott_ic(N: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Gray-Scott initial condition, shape ``(2, N, N, N)`` indexed ``[field, z, y, x]``.

    The returned array is C-contiguous, so its flat layout is field-major with x
    fastest: element ``(f, k, j, i)`` sits at ``f*N^3 + i + N*(j + N*k)``.
    """
    lo, hi = (3 * N) // 8, (5 * N) // 8
    u = np.ones((N, N, N), dtype=np.float64)
    v = np.zeros((N, N, N), dtype=np.float64)
    u[lo:hi, lo:hi, lo:hi] = 0.5
    v[lo:hi, lo:hi, lo:hi] = 0.25
    n3 = N * N * N
    u += (0.01 * (2.0 * uniform(seed, 0, n3) - 1.0)).reshape(N, N, N)
    v += (0.01 * (2.0 * uniform(seed, 1, n3) - 1.0)).reshape(N, N, N)
    out = np.stack([u, v])
    return out.astype(dtype, copy=False)


def exp_family_x0_torch(n: int, seed: int = 2, dtype=None, device=None, chunk: int = 1 << 26):
    """``exp_family_x0(n, seed)`` built on a torch device in chunks and stored
    as ``dtype`` (default float64)."""
    import torch

    out = torch.empty(n, dtype=dtype or torch.float64, device=device)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        out[lo:hi] = (0.01 + 0.49 * uniform_torch(seed, 0, hi - lo, lo, device)).to(out.dtype)
    return out


def gray_scott_ic_at(N: int, seed: int, f: int, z, y, x) -> np.ndarray:
    """Field ``f`` of ``gray_scott_ic(N, seed)`` at the cells ``(z, y, x)``
    (float64), without building the grid."""
    z, y, x = (np.asarray(a, dtype=np.int64) for a in (z, y, x))
    lo, hi = (3 * N) // 8, (5 * N) // 8
    inside = (z >= lo) & (z < hi) & (y >= lo) & (y < hi) & (x >= lo) & (x < hi)
    base = np.where(inside, 0.5, 1.0) if f == 0 else np.where(inside, 0.25, 0.0)
    r = uniform_at(seed, f, x + N * (y + N * z))
    return base + 0.01 * (2.0 * r - 1.0)


def gray_scott_ic_torch(N: int, seed: int, dtype=None, device=None, planes: int = 32):
    """``gray_scott_ic(N, seed)`` built on a torch device plane range by plane
    range, flat in the same layout and stored as ``dtype`` (default float64)."""
    import torch

    n3, NN = N * N * N, N * N
    lo, hi = (3 * N) // 8, (5 * N) // 8
    out = torch.empty(2 * n3, dtype=dtype or torch.float64, device=device)
    for f, (outer, inner) in enumerate(((1.0, 0.5), (0.0, 0.25))):
        for z0 in range(0, N, planes):
            z1 = min(N, z0 + planes)
            base = torch.full((z1 - z0, N, N), outer, dtype=torch.float64, device=device)
            a, b = max(lo, z0), min(hi, z1)
            if a < b:
                base[a - z0:b - z0, lo:hi, lo:hi] = inner
            r = uniform_torch(seed, f, (z1 - z0) * NN, z0 * NN, device)
            v = base.reshape(-1) + 0.01 * (2.0 * r - 1.0)
            out[f * n3 + z0 * NN:f * n3 + z1 * NN] = v.to(out.dtype)
    return out


ENSEMBLE_EDGES = tuple(range(16, 97, 8))


def ensemble_draws(n_inst: int, seed: int = 4):
    """Per-instance (edge, F, k) for the batched ensemble workload."""
    r_n = uniform(seed, 0, n_inst)
    r_f = uniform(seed, 1, n_inst)
    r_k = uniform(seed, 2, n_inst)
    edges = [ENSEMBLE_EDGES[min(int(r * len(ENSEMBLE_EDGES)), len(ENSEMBLE_EDGES) - 1)] for r in r_n]
    F = 0.02 + 0.04 * r_f
    k = 0.045 + 0.02 * r_k
    return edges, F, k


def ensemble_ic(i: int, N: int, dtype=np.float32) -> np.ndarray:
    """Initial condition of ensemble instance ``i`` (seed ``4000 + i``)."""
    return gray_scott_ic(N, 4000 + i, dtype)
