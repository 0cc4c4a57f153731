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
