"""The plan autotuner's cache (paper_1509_06957_amd/tuning.py), host side:
signature of a set of batches, candidate grid, JSON round trip, and a cache
hit that returns the stored choice without timing anything."""
import json
from types import SimpleNamespace

import numpy as np

from paper_1509_06957_amd import tuning


class FakeIndex:
    def __init__(self, d, T, depth):
        self.info = SimpleNamespace(d=d, T=T, depth=depth)


def test_nq_bucket():
    assert [tuning.nq_bucket(x) for x in (1, 2, 3, 4, 5, 1000, 1024, 1025)] == [1, 2, 4, 4, 8, 1024, 1024, 2048]


def test_candidates_cover_the_grid():
    c = tuning.candidates({"fused": [1], "branches": [1, 4], "proj_rows": [0], "vote_kernel": [0, 2],
                           "vote_waves": [0]})
    assert len(c) == 4 and {x["branches"] for x in c} == {1, 4} and all(x["fused"] == 1 for x in c)
    assert len(tuning.candidates()) == 2 * 4 * 2 * 2 * 2
    assert {x["vote_waves"] for x in tuning.candidates()} == {0, 16}


def test_signature_groups_batches_by_index_k_v(monkeypatch):
    monkeypatch.setattr(tuning, "arch", lambda: "gfx950")
    a, b = FakeIndex(128, 64, 10), FakeIndex(784, 64, 12)
    q = lambda m: np.zeros((m, 1), np.float32)
    s1 = tuning.signature([(a, q(100), 10, 3), (a, q(30), 10, 3), (b, q(5), 1, 3)], 1)
    s2 = tuning.signature([(b, q(5), 1, 3), (a, q(130), 10, 3)], 1)
    assert s1 == s2                                   # groups (index, k, v), nq summed then bucketed
    d = json.loads(s1)
    assert d["arch"] == "gfx950" and d["precision"] == 1
    assert d["groups"] == [[128, 64, 10, 10, 3, 256], [784, 64, 12, 1, 3, 8]]
    assert tuning.signature([(a, q(100), 10, 3)], 0) != tuning.signature([(a, q(100), 10, 3)], 1)


def test_cache_hit_returns_the_stored_choice(monkeypatch, tmp_path):
    monkeypatch.setattr(tuning, "arch", lambda: "gfx950")
    path = str(tmp_path / "t.json")
    a = FakeIndex(128, 64, 10)
    batches = [(a, np.zeros((40, 1), np.float32), 10, 3)]
    key = tuning.signature(batches, 0)
    tuning._store(path, {key: {"choice": {"fused": 1, "branches": 4, "proj_rows": 0, "vote_kernel": 0}, "ms": 1.0}})
    calls = []
    choice, timings, cached = tuning.tune(batches, 0, lambda p: calls.append(p) or 1.0, path=path)
    assert cached and timings == {} and not calls
    assert choice == {"fused": 1, "branches": 4, "proj_rows": 0, "vote_kernel": 0}
