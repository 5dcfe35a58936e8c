"""CPU tests of the autotuner's host logic: buckets, the choice rule and the cache."""
import json

from paper_2605_16058_amd import autotune as T


def test_buckets():
    assert T.ttm_bucket(8) == "n8" and T.ttm_bucket(9) == "n16" and T.ttm_bucket(96) == "n128"
    assert T.ttm_bucket(1000) == "n256"
    assert T.jacobi_bucket(512, 1024) == "r512rows"
    assert T.jacobi_bucket(300, 40) == "r64cols"
    assert T.jacobi_bucket(64, 64) == "r64cols"


def test_defaults_match_library_rules():
    assert T.default_block(255, 4000) == 16 and T.default_block(256, 256) == 32
    assert [T.default_tile(n) for n in (1, 16, 17, 32, 33, 256)] == [3, 3, 2, 2, 8, 8]
    assert [T.default_tile(n, "f32") for n in (1, 16, 17, 32, 33, 64, 65, 256)] == [3, 3, 2, 2, 4, 4, 6, 6]


def test_pick_respects_margin():
    assert T.pick({16: 10.0, 32: 9.8}, 16, margin=0.03) == 16     # 2% faster: keep
    assert T.pick({16: 10.0, 32: 9.0}, 16, margin=0.03) == 32     # 10% faster: switch
    assert T.pick({1: 5.0, 2: 4.0, 3: 6.0}, 7, margin=0.03) == 2  # unknown incumbent


def test_sample_is_even_and_deterministic():
    s = T._sample(list(range(100)), 10)
    assert s == [0, 10, 20, 30, 40, 50, 60, 70, 80, 90]
    assert T._sample([3, 4], 10) == [3, 4]


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    c = T.Cache(path)
    assert c.get("jacobi", "f32", "r512rows") is None
    c.put("jacobi", "f32", "r512rows", 32, {16: 1.5, 32: 1.25})
    c2 = T.Cache(path)
    assert c2.get("jacobi", "f32", "r512rows") == 32
    assert c2.get("jacobi", "f64", "r512rows") is None
    data = json.load(open(path))
    (entry,) = data.values()
    assert entry["choice"] == 32 and entry["ms"] == {"16": 1.5, "32": 1.25}
    # a damaged file is ignored, not fatal
    open(path, "w").write("{not json")
    assert T.Cache(path).get("jacobi", "f32", "r512rows") is None
    # in-memory cache writes nothing
    mem = T._cache(False)
    mem.put("ttm", "f32", "n8", 3, {3: 0.1})
    assert mem.get("ttm", "f32", "n8") == 3 and mem.path is None
