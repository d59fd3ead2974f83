"""Host checks of the forest autotuner's search and cache (no GPU): the timed
pass is replaced by a synthetic cost with a known optimum per bucket."""
import json

import numpy as np
import pytest

pytest.importorskip("torch")
import paper_2111_04182_amd.autotune as AT  # noqa: E402


class FakeXYZ:
    shape = (3, 0)


# cloud sizes spanning buckets 9 (512-1023), 10, 11 and 12
OFFSETS = np.cumsum([0, 600, 700, 1500, 1800, 3000, 5000, 5000]).astype(np.int64)
BEST_L = {9: 8, 10: 12, 11: 16, 12: 32}
BEST_WAVES = 2


def fake_cost(calls):
    def time_pass(xyz, offsets, k, leaf_sizes, reps, waves=1):
        calls.append((tuple(int(x) for x in leaf_sizes), waves))
        b = AT.size_buckets(offsets)
        cost = 100.0 + 3.0 * abs(waves - BEST_WAVES)
        for c, L in enumerate(leaf_sizes):
            cost += abs(np.log2(L) - np.log2(BEST_L[int(b[c])]))
        return cost
    return time_pass


def test_size_buckets():
    assert AT.size_buckets([0, 1000, 1024, 66560]).tolist() == [9, 4, 16]


def test_search_finds_per_bucket_leaf_sizes_and_waves(monkeypatch, tmp_path):
    calls = []
    monkeypatch.setattr(AT, "_time_pass", fake_cost(calls))
    cache = tmp_path / "tune.json"
    ls, waves, rep = AT.tune_forest(FakeXYZ(), OFFSETS, 16, reps=1, cache_path=str(cache))
    buckets = AT.size_buckets(OFFSETS)
    assert waves == BEST_WAVES
    assert [int(x) for x in ls] == [BEST_L[int(b)] for b in buckets]
    assert rep["choice"] == BEST_L and rep["query_waves"] == BEST_WAVES
    # every pass after the waves sweep runs with the chosen launch shape
    first_bucket_pass = len(AT.CANDIDATES) + len(AT.WAVES) - 1
    assert all(w == BEST_WAVES for _, w in calls[first_bucket_pass:])
    stored = json.loads(cache.read_text())
    assert stored["d3:k16:waves"] == BEST_WAVES
    assert all(stored[f"d3:k16:b{b}"] == L for b, L in BEST_L.items())
    # a second call is answered from the cache without timing anything
    calls.clear()
    ls2, waves2, rep2 = AT.tune_forest(FakeXYZ(), OFFSETS, 16, reps=1, cache_path=str(cache))
    assert calls == [] and rep2 == {"cached": True}
    assert waves2 == waves and np.array_equal(ls2, ls)
