"""The autotuner's host logic (no GPU): the coordinate-descent search, the
occupancy signature, the table keys and the candidate set."""
import ctypes
import dataclasses
import json

import numpy as np
import pytest

from paper_1810_02916_amd import _lib
from paper_1810_02916_amd import tune
from paper_1810_02916_amd.nearfield import Tiles


def test_search_finds_the_minimum_of_a_separable_cost():
    want = {"dense_min": 33, "narrow_max": 16, "light_window": 2048, "narrow_window": 128,
            "flush": 64}
    calls = []

    def timer(t):
        calls.append(t)
        d = t.as_dict()
        return 1.0 + sum(abs(np.log2(d[k]) - np.log2(v)) for k, v in want.items())

    best, times = tune.search(timer)
    assert best.as_dict() == want
    # every distinct choice timed once: one pass over the candidates, a second
    # pass that changes nothing, minus repeats
    assert len(calls) == len(set(calls)) == len(times)
    assert len(calls) <= 1 + 2 * sum(len(v) for v in tune.CANDIDATES.values())
    assert times[best] == min(times.values())


def test_search_keeps_the_start_when_nothing_is_faster_and_follows_coupled_costs():
    best, times = tune.search(lambda t: 1.0 if t == tune.DEFAULTS else 2.0)
    assert best == tune.DEFAULTS
    # a cost in which the best narrow_max depends on dense_min: the second pass
    # revisits narrow_max after dense_min moved
    def coupled(t):
        return 3 * abs(t.dense_min - 57) + abs(t.narrow_max - (24 if t.dense_min > 50 else 8))
    best, _ = tune.search(coupled, order=("narrow_max", "dense_min"))
    assert (best.dense_min, best.narrow_max) == (57, 24)


def test_occupancy_signature():
    rng = np.random.default_rng(0)
    a = rng.poisson(8, 4096)
    s = tune.occupancy_signature([a])
    assert s.startswith("boxes1:")
    shares = [int(x) for x in s.split(":")[1].split("-")]
    assert len(shares) == len(tune.COUNT_BINS) - 1
    assert 7 <= sum(shares) <= 9            # eighths of all sinks, rounded per bin
    assert tune.occupancy_signature([a]) == s
    # the same shape at another size keeps its signature; a clustered box does not
    assert tune.occupancy_signature([rng.poisson(8, 40000)]) == s
    heavy = np.concatenate([a, [3000] * 40])
    assert tune.occupancy_signature([heavy]) != s
    assert tune.occupancy_signature([a] * 10).startswith("boxes64:")
    assert tune.occupancy_signature([a] * 65).startswith("boxesmany:")


def test_table_round_trip_and_stale_keys(tmp_path):
    path = str(tmp_path / "t.json")
    k1 = tune.table_key("gfx950", "7.0", "aaaa", "boxes1:0-1-2", "accel", True)
    k2 = tune.table_key("gfx950", "7.0", "bbbb", "boxes1:0-1-2", "accel", True)
    k3 = tune.table_key("gfx950", "7.0", "aaaa", "boxes1:0-1-2", "vjp", True)
    assert len({k1, k2, k3}) == 3
    assert tune.load_table(path) == {}
    t = Tiles(25, 16, 2048, 128, 64)
    tune.store(k1, {"tiles": t.as_dict(), "ms": {"x": 1.0}}, path)
    tab = tune.load_table(path)
    assert tune.tiles_from(tab[k1]["tiles"]) == t
    assert k2 not in tab                    # kernels changed: the winner is not reused
    tune.store(k3, {"tiles": Tiles().as_dict(), "ms": {}}, path)
    assert set(json.load(open(path))) == {k1, k3}
    (tmp_path / "bad.json").write_text("{not json")
    assert tune.load_table(str(tmp_path / "bad.json")) == {}


def test_every_candidate_is_accepted_by_the_library():
    """Every candidate value (others at their defaults) passes the library's
    validation; values outside the sets are refused."""
    lib = _lib.load()

    def box(t):
        return (_lib.NfBox * 1)(_lib.NfBox(1000, 8, t.dense_min, 1.0, 0.01, 0x1000, 0x1000, 0x1000,
                                           0x1000, None, t.narrow_max, t.light_window,
                                           t.narrow_window, t.flush))
    for name, vals in tune.CANDIDATES.items():
        for v in vals:
            t = dataclasses.replace(tune.DEFAULTS, **{name: v})
            assert lib.nf_workspace_bytes(1, box(t), 0) > 0, (name, v)
    for bad in (Tiles(narrow_max=65), Tiles(light_window=768), Tiles(narrow_window=64),
                Tiles(flush=257), Tiles(flush=-1), Tiles(dense_min=1)):
        assert lib.nf_workspace_bytes(1, box(bad), 0) == 0, bad
    # the windows pick kernel instances: the boxes of one call must agree
    two = (_lib.NfBox * 2)(box(Tiles())[0], box(Tiles(light_window=2048))[0])
    assert lib.nf_workspace_bytes(2, two, 0) == 0
    assert "agree" in _lib.last_error()
    same = (_lib.NfBox * 2)(box(Tiles(light_window=1024))[0], box(Tiles())[0])
    assert lib.nf_workspace_bytes(2, same, 0) > 0
