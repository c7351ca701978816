"""Autotuner host logic on the CPU: the coordinate-descent search over the
option space, and the JSON cache (write, reuse, forced re-tune, user cache
before the shipped one, corrupt files).  Timing is replaced by a stand-in
cost function of the options, so no GPU is involved."""
from __future__ import annotations

import json

import pytest

from paper_2004_13907_amd import autotune

SPACE = (
    ("a", (0, 1, 2)),
    ("b", (0, -1)),
    ("c", (0, 5, 7)),
)


def separable_cost(opts):
    """Minimum at a=2, b=-1, c=5 (each dimension independent)."""
    a, b, c = opts.get("a", 0), opts.get("b", 0), opts.get("c", 0)
    return 10.0 + {0: 3.0, 1: 2.0, 2: 0.5}[a] + {0: 1.0, -1: 0.0}[b] + {0: 2.0, 5: 0.1, 7: 1.5}[c]


def test_search_finds_separable_optimum():
    opts, secs, trials = autotune.search(separable_cost, SPACE)
    assert opts == {"a": 2, "b": -1, "c": 5}
    assert secs == pytest.approx(10.6)
    # the defaults are timed first, and no setting is timed twice
    assert trials[0]["options"] == {}
    keys = [tuple(sorted(t["options"].items())) for t in trials]
    assert len(keys) == len(set(keys))


def test_search_follows_interaction():
    """c = 7 pays off only once b = -1: a second pass must find it."""
    def cost(o):
        b, c = o.get("b", 0), o.get("c", 0)
        base = {0: 2.0, 5: 1.9, 7: 2.5}[c] + (1.0 if b == 0 else 0.0)
        if b == -1 and c == 7:
            base = 0.5
        return base
    space = (("c", (0, 5, 7)), ("b", (0, -1)))
    opts, secs, _ = autotune.search(cost, space)
    assert opts == {"b": -1, "c": 7} and secs == 0.5


def test_default_wins_when_nothing_is_faster():
    opts, secs, trials = autotune.search(lambda o: 1.0 + len(o), SPACE)
    assert opts == {} and secs == 1.0
    assert len(trials) == 1 + sum(len(v) - 1 for _, v in SPACE)


def test_library_space_is_well_formed():
    from paper_2004_13907_amd import _capi
    names = {f for f, _ in _capi.reap_options_t._fields_}
    for name, vals in autotune.SPACE:
        assert name in names and vals[0] == 0 and len(set(vals)) == len(vals)


@pytest.fixture
def fake_timing(monkeypatch):
    calls = []

    def fake(As, Bs, dtype, options, reps=2, stream=None):
        calls.append(dict(options))
        return separable_cost(options)
    monkeypatch.setattr(autotune, "time_batch", fake)
    return calls


def test_tune_writes_and_reuses_cache(tmp_path, fake_timing, monkeypatch):
    monkeypatch.setattr(autotune, "SHIPPED", str(tmp_path / "shipped.json"))
    cache = str(tmp_path / "user" / "tune.json")
    e1 = autotune.tune([], [], None, "sig-A", cache_path=cache, space=SPACE)
    assert e1["options"] == {"a": 2, "b": -1, "c": 5}
    n = len(fake_timing)
    assert n > 0
    stored = json.load(open(cache))
    assert stored["sig-A"]["options"] == e1["options"]
    # a second call is served from the cache without timing anything
    e2 = autotune.tune([], [], None, "sig-A", cache_path=cache, space=SPACE)
    assert e2["options"] == e1["options"] and len(fake_timing) == n
    # forced: timed again, entry rewritten
    autotune.tune([], [], None, "sig-A", cache_path=cache, space=SPACE, force=True)
    assert len(fake_timing) > n
    # another signature gets its own entry; the first is kept
    autotune.tune([], [], None, "sig-B", cache_path=cache, space=(("a", (0, 1)),))
    stored = json.load(open(cache))
    assert set(stored) == {"sig-A", "sig-B"} and stored["sig-B"]["options"] == {"a": 1}


def test_lookup_prefers_user_cache_over_shipped(tmp_path, monkeypatch, fake_timing):
    shipped = tmp_path / "shipped.json"
    shipped.write_text(json.dumps({"sig": {"options": {"a": 1}, "seconds": 1.0},
                                   "only-shipped": {"options": {"b": -1}, "seconds": 2.0}}))
    monkeypatch.setattr(autotune, "SHIPPED", str(shipped))
    user = tmp_path / "user.json"
    user.write_text(json.dumps({"sig": {"options": {"c": 7}, "seconds": 0.5}}))
    assert autotune.lookup("sig", str(user))["options"] == {"c": 7}
    assert autotune.lookup("only-shipped", str(user))["options"] == {"b": -1}
    assert autotune.lookup("absent", str(user)) is None
    # tune() returns the cached entries without timing
    assert autotune.tune([], [], None, "only-shipped", cache_path=str(user))["options"] == {"b": -1}
    assert fake_timing == []


def test_corrupt_cache_is_ignored_and_replaced(tmp_path, monkeypatch, fake_timing):
    monkeypatch.setattr(autotune, "SHIPPED", str(tmp_path / "none.json"))
    cache = tmp_path / "tune.json"
    cache.write_text("{not json")
    assert autotune.lookup("sig", str(cache)) is None
    e = autotune.tune([], [], None, "sig", cache_path=str(cache), space=SPACE)
    assert json.load(open(cache))["sig"]["options"] == e["options"]


def test_cache_path_from_environment(monkeypatch, tmp_path):
    monkeypatch.setenv("REAP_TUNE_CACHE", str(tmp_path / "dir"))
    assert autotune.default_cache_path() == str(tmp_path / "dir" / "autotune.json")
    monkeypatch.setenv("REAP_TUNE_CACHE", str(tmp_path / "x.json"))
    assert autotune.default_cache_path() == str(tmp_path / "x.json")
