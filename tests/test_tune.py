"""Host logic of the tile-shape autotuner (selection, size classes, cache)."""
import json

import pytest

from paper_2309_09072_amd import tune


def test_bucket_and_key():
    assert [tune.bucket(x) for x in (0, 1, 2, 3, 64, 65, 4096, 4097)] == [1, 1, 2, 4, 64, 128, 4096, 8192]
    k1 = tune.cache_key("gfx950:256", "pair", 4000, 4096, 4, 64)
    k2 = tune.cache_key("gfx950:256", "pair", 4096, 3000, 3, 64)
    assert k1 == k2 == "gfx950:256|pair|m4096|n4096|s4|h64"
    assert tune.cache_key("d", "pair", 5, 5, 20) .endswith("|hany")


def test_candidates():
    c = tune.candidates()
    assert len(c) == len(tune.BASE_ROWS) * len(tune.TILES) and tune.DEFAULT in c
    assert tune.candidates(64) == [(64, t) for t in tune.TILES]
    cp = tune.candidates(rows=tune.PAIR_BASE_ROWS)
    assert len(cp) == len(tune.PAIR_BASE_ROWS) * len(tune.TILES) and (256, 32) in cp


def test_every_candidate_is_a_valid_plan():
    from paper_2309_09072_amd import lcs
    for h, t in tune.candidates(rows=tune.PAIR_BASE_ROWS):
        p = lcs.Plan(300, 500, 4, h, t)
        assert p.workspace_for(300, 500) > 0
        p.close()


def test_pick_fastest_and_ties():
    order = [(64, 32), (64, 16), (32, 32)]
    assert tune.pick({(64, 32): 2.0, (64, 16): 1.0, (32, 32): 3.0}, order) == (64, 16)
    assert tune.pick({(64, 32): 1.0, (64, 16): 1.0}, order) == (64, 32)  # earlier wins ties
    with pytest.raises(ValueError):
        tune.pick({}, order)


def test_tune_with_fake_timer_and_cache(tmp_path):
    import torch
    path = str(tmp_path / "tune.json")
    calls = []

    def timer(c):
        calls.append(c)
        return 10.0 - c[1] * 0.1 + (0.5 if c[0] != 32 else 0.0)

    a = torch.zeros(1000, dtype=torch.uint8)
    b = torch.zeros(2000, dtype=torch.uint8)
    r = tune.tune_pair(a, b, 4, timer=timer, cache_path=path)
    assert r.best == (32, 32) and not r.cached
    assert sorted(calls) == sorted(tune.candidates(rows=tune.PAIR_BASE_ROWS))
    data = json.load(open(path))
    (key, entry), = data.items()
    assert key == "host|pair|m1024|n2048|s4|hany"
    assert entry["base_rows"] == 32 and entry["tile"] == 32
    calls.clear()
    r2 = tune.tune_pair(a, b, 4, timer=timer, cache_path=path)
    assert r2.cached and r2.best == (32, 32) and calls == []
    assert r2.ms == r.ms
    # a different size class or a fixed base_rows is a new entry
    r3 = tune.tune_pair(a, b, 4, base_rows=64, timer=timer, cache_path=path)
    assert r3.best == (64, 32) and len(json.load(open(path))) == 2


def test_corrupt_cache_is_ignored(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert tune.load_cache(str(path)) == {}
    tune.store_cache("k", {"base_rows": 16, "tile": 8}, str(path))
    assert tune.load_cache(str(path)) == {"k": {"base_rows": 16, "tile": 8}}
