"""Autotuner selection and cache logic (no GPU: the timing function is faked)."""
import json

from paper_2410_04994_amd import autotune


def test_pick_fastest_and_ties():
    costs = {(1, 256, 4, 2): 3.0, (4, 64, 4, 1): 2.0, (8, 64, 8, 2): 2.0}
    best, t = autotune.pick_fastest(list(costs), costs.__getitem__)
    assert best == (4, 64, 4, 1) and t == 2.0


def test_candidates_filter_unbuilt_schedules():
    allowed = {(1, 256, 4, 2), (8, 64, 16, 4)}
    got = autotune.candidates(lambda s: s in allowed)
    assert set(got) == allowed


def test_cache_roundtrip(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("SHG_AUTOTUNE_CACHE", str(path))
    assert autotune.load_cache() == {}
    key = autotune.cache_key("gfx950", "c64", "single", 256, 256)
    autotune.store_cache({key: [1, 256, 4, 2]})
    assert json.load(open(path)) == {key: [1, 256, 4, 2]}
    assert autotune.load_cache()[key] == [1, 256, 4, 2]
    path.write_text("{not json")
    assert autotune.load_cache() == {}
