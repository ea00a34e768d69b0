"""The on-disk oracle result cache: stored results come back bitwise, and a
change of key, of the oracle's or generators' sources, or a damaged file
computes the result again."""
import os

import numpy as np
import pytest

import oracle_cache


@pytest.fixture()
def cache(tmp_path, monkeypatch):
    monkeypatch.setenv("TRBT_ORACLE_CACHE", str(tmp_path))
    return tmp_path


def _counter():
    calls = []

    def compute():
        calls.append(1)
        rng = np.random.default_rng(len(calls))
        return {"a": rng.standard_normal((5, 3)),
                "b": rng.standard_normal(4) + 1j * rng.standard_normal(4)}
    return calls, compute


def test_round_trip_bitwise(cache):
    calls, compute = _counter()
    key = dict(cfg="C3", seed=1003, cols=np.arange(7))
    first = oracle_cache.cached("bt", key, compute)
    again = oracle_cache.cached("bt", key, compute)
    assert len(calls) == 1
    for k in first:
        assert again[k].dtype == first[k].dtype
        assert np.array_equal(again[k], first[k])
    assert len([f for f in os.listdir(cache) if f.endswith(".npz")]) == 1


def test_key_change_recomputes(cache):
    calls, compute = _counter()
    oracle_cache.cached("bt", dict(seed=1), compute)
    oracle_cache.cached("bt", dict(seed=2), compute)
    oracle_cache.cached("adj", dict(seed=1), compute)
    oracle_cache.cached("bt", dict(seed=1, cols=[0, 1]), compute)
    assert len(calls) == 4
    oracle_cache.cached("bt", dict(seed=2), compute)
    assert len(calls) == 4


def test_source_change_recomputes(cache, monkeypatch):
    calls, compute = _counter()
    oracle_cache.cached("bt", dict(seed=1), compute)
    monkeypatch.setattr(oracle_cache, "sources_hash", lambda: "another oracle")
    oracle_cache.cached("bt", dict(seed=1), compute)
    assert len(calls) == 2


def test_sources_hash_covers_the_oracle():
    h = oracle_cache.sources_hash()
    assert len(h) == 64 and h == oracle_cache.sources_hash()
    assert "oracle/oracle.c" in oracle_cache._SOURCES


def test_damaged_file_is_replaced(cache):
    calls, compute = _counter()
    first = oracle_cache.cached("bt", dict(seed=1), compute)
    (path,) = [os.path.join(cache, f) for f in os.listdir(cache)]
    with open(path, "wb") as f:
        f.write(b"not an npz file")
    again = oracle_cache.cached("bt", dict(seed=1), compute)
    assert len(calls) == 2
    assert np.array_equal(again["a"], np.random.default_rng(2).standard_normal((5, 3)))
    assert not np.array_equal(again["a"], first["a"])
    with np.load(path, allow_pickle=False) as f:   # the file was rewritten whole
        assert set(f.files) == {"a", "b"}


def test_off_stores_nothing(tmp_path, monkeypatch):
    monkeypatch.setenv("TRBT_ORACLE_CACHE", "off")
    calls, compute = _counter()
    oracle_cache.cached("bt", dict(seed=1), compute)
    oracle_cache.cached("bt", dict(seed=1), compute)
    assert len(calls) == 2
    assert oracle_cache.cache_dir() is None
