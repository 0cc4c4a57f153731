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
