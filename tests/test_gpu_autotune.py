"""GPU tests of the autotuner: it picks an engine, a lockstep block size and
force-kernel lane counts (one for all replicas, then per replica size class
where that is faster) by timing throwaway runs, caches the choice in a JSON
file, and the tuned context runs exactly like one created with that choice
given explicitly."""
import json
import os

import numpy as np
import pytest

from paper_0812_1633_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def relib():
    from paper_0812_1633_amd import re as R
    R.lib()
    return R


def test_autotune_choice_cache_and_equivalence(relib, tmp_path):
    R, N = 8, 1500
    T = W.ladder(0.7, 1.5, R)
    cache = str(tmp_path / "tune.json")
    e = relib.Engine([N] * R, T, 0.8442, 2.5, 0.3, 0.005, 20, 3, autotune=True, tune_cache=cache)
    eng, tpa, team = e.query_config()
    assert eng in ("lockstep", "persistent") and tpa in (1, 2, 4, 8)
    data = json.load(open(cache))
    assert len(data) == 1
    (key, val), = data.items()
    assert "R8|" in key and val["tpa"] == tpa and val["ms_per_step"] > 0
    e.step(60)
    got = [e.get_state(r) for r in range(R)]
    e.close()
    # explicit configuration: the same run
    f = relib.Engine([N] * R, T, 0.8442, 2.5, 0.3, 0.005, 20, 3, engine=eng, threads_per_atom=tpa)
    f.step(60)
    for r in range(R):
        x, v = f.get_state(r)
        assert np.array_equal(x, got[r][0]) and np.array_equal(v, got[r][1])
    f.close()
    # a second tuned context of the same size class reads the cache
    os.utime(cache, None)
    g = relib.Engine([N] * R, T, 0.8442, 2.5, 0.3, 0.005, 20, 9, autotune=True, tune_cache=cache)
    assert g.query_config()[:2] == (eng, tpa)
    g.close()


def test_autotune_per_size_class(relib, tmp_path):
    """A ladder of replicas in four size classes (floor(log2 N) = 9 .. 12):
    the cache records the classes' lane counts, the tuned context runs them
    (re_query_lanes), and the same choice given explicitly is the same run."""
    N = [600, 700, 1500, 1800, 2500, 3000, 5000, 6000]
    R = len(N)
    T = W.ladder(0.7, 1.6, R)
    cache = str(tmp_path / "tune.json")
    e = relib.Engine(N, T, 0.8442, 2.5, 0.3, 0.005, 20, 3, autotune=True, tune_cache=cache)
    eng, tpa, team = e.query_config()
    lanes = e.query_lanes()
    data = json.load(open(cache))
    (key, val), = data.items()
    assert val["tpa"] in (1, 2, 4, 8) and val["ms_per_step"] > 0 and val["block"] in (0, 128, 256)
    cls = dict((int(k), int(t)) for k, t in (c.split(":") for c in val["classes"].split(",") if c))
    for r in range(R):
        k = int(np.floor(np.log2(N[r])))
        assert lanes[r] == cls.get(k, val["tpa"]), (r, lanes[r], cls, val)
    assert tpa == (lanes[0] if len(set(lanes.tolist())) == 1 else 0)
    e.step(60)
    got = [e.get_state(r) for r in range(R)]
    e.close()
    f = relib.Engine(N, T, 0.8442, 2.5, 0.3, 0.005, 20, 3, engine=eng, threads_per_atom_per_replica=lanes,
                     block_size=val["block"])
    f.step(60)
    for r in range(R):
        x, v = f.get_state(r)
        assert np.array_equal(x, got[r][0]) and np.array_equal(v, got[r][1])
    f.close()
