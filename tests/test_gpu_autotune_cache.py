"""GPU: the autotuner's persistent cache (hode_autotune_cached): a miss
tunes and appends one entry, a hit restores every stage kind's tile without
timing, entries are keyed by method and grid, the path may come from
HODE_TUNE_CACHE, and an unwritable path is an error."""
import numpy as np
import pytest

from paper_2309_05331_amd import hode, inputs
from gpu_util import gs_ctx, read

pytestmark = pytest.mark.gpu

PRM = dict(Du=2e-5, Dv=1e-5, F=0.053, k=0.014, L=2.5)


def test_cache_miss_then_hit(tmp_path, monkeypatch):
    N = 64
    y0 = inputs.gray_scott_ic(N, seed=97, dtype=np.float32)
    path = tmp_path / "tune.txt"
    a = gs_ctx(y0, N, PRM)
    assert a.autotune_cached(hode.DOPRI5, 1, path) is False
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("hode-tune-v2 ")
    tile = a.get_tile()
    kinds = [a.kind_tile(k) for k in range(hode.K_MM[-1] + 1)]
    a.integrate_adaptive(0.0, 5.0, 0.1)
    ya = read(a, np.float32, 2 * N ** 3)
    a.close()
    b = gs_ctx(y0, N, PRM)
    assert b.autotune_cached(hode.DOPRI5, 1, path) is True
    assert b.get_tile() == tile
    assert [b.kind_tile(k) for k in range(hode.K_MM[-1] + 1)] == kinds
    b.integrate_adaptive(0.0, 5.0, 0.1)
    assert np.array_equal(read(b, np.float32, 2 * N ** 3), ya)
    # another method is another entry
    assert b.autotune_cached(hode.RK4, 1, path) is False
    assert len(path.read_text().splitlines()) == 2
    b.close()
    # the path from the environment
    env = tmp_path / "env.txt"
    monkeypatch.setenv("HODE_TUNE_CACHE", str(env))
    c = gs_ctx(y0, N, PRM)
    assert c.autotune_cached(hode.DOPRI5, 1) is False and env.exists()
    assert c.autotune_cached(hode.DOPRI5, 1) is True
    with pytest.raises(hode.HodeError):
        c.autotune_cached(hode.CASHKARP54, 1, tmp_path)  # a directory: cannot append
    c.close()


def test_ensemble_tile_cache(tmp_path, monkeypatch):
    # The ensemble's tile autotuner (timed inside the whole ensemble) appends
    # one line per grid edge to HODE_TUNE_CACHE; a second ensemble of the same
    # edge list reads the widths back without timing, and the file is
    # unchanged.  Another edge list is another key.
    edges = [16, 24, 16, 32, 24]
    prms = [[2e-3, 1e-3, 0.04 + 0.002 * i, 0.06, 2.5] for i in range(len(edges))]
    path = tmp_path / "ens.txt"
    monkeypatch.setenv("HODE_TUNE_CACHE", str(path))

    def tuned(es):
        ens = hode.Ensemble(es, prms[:len(es)], dtype=hode.F32)
        for i, N in enumerate(es):
            ens.init_instance(i, inputs.ensemble_ic(i, N).ravel())
        ens.set_tolerances(1e-5, 1e-5)
        vw, ms = ens.autotune(2)
        tiles = [ens.instance_tile(i) for i in range(len(es))]
        ens.close()
        return list(vw), tiles

    vw1, t1 = tuned(edges)
    lines = path.read_text().splitlines()
    assert len(lines) == len(set(edges)) and all(l.startswith("hode-ens-tune-v2 ") for l in lines)
    assert all(N % v == 0 for N, v in zip(edges, vw1)) and all(t[1] == 0 for t in t1)
    vw2, t2 = tuned(edges)
    assert vw2 == vw1 and t2 == t1 and path.read_text().splitlines() == lines
    tuned(edges[:3])  # edges 16, 24, 16: another instance count and edge list
    assert len(path.read_text().splitlines()) == len(lines) + 2
