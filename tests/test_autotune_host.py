"""Host-side pieces of the autotuner: cache keys, subsets, cache files."""
from paper_2204_06633_amd import autotune


def test_key_buckets_and_subset(tmp_path):
    tpl = [(0, 100, 10, n, 0) for n in (1000, 3000, 2000, 5000)]
    k1 = autotune.tune_key("dev", 25, 2, "AET", 10.0, tpl)
    k2 = autotune.tune_key("dev", 25, 2, "AET", 10.0, tpl[:3] + [(0, 100, 10, 4500, 0)])
    assert k1 == k2                              # same power-of-two buckets
    assert k1 != autotune.tune_key("dev", 25, 1, "AET", 10.0, tpl)
    sub, pick = autotune.subset(tpl, 2)
    assert pick == [0, 3] and [t[3] for t in sub] == [1000, 5000]   # shortest and longest
    sub, pick = autotune.subset(tpl, 10)
    assert pick == [0, 1, 2, 3]


def test_cache_roundtrip(tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    assert autotune.load_cache(p) == {}
    autotune.save_cache({"k": {"group": 2}}, p)
    assert autotune.load_cache(p) == {"k": {"group": 2}}


def test_tile_variants():
    """Groups 1, 2, 4 at tiles of 256, 512, 1024 link samples, except the
    group of 4 at 1024 (its link rows would need 196 KB of LDS)."""
    ok = {(g, t) for g in autotune.GROUPS for t in autotune.TILES if autotune.variant_exists(g, t)}
    assert len(ok) == 8 and (4, 1024) not in ok and (4, 512) in ok and (1, 1024) in ok
    assert not autotune.variant_exists(3, 512) and not autotune.variant_exists(2, 768)
    wave = {(g, t) for g in autotune.GROUPS for t in autotune.TILES
            if autotune.variant_exists(g, t, wave=True)}
    assert wave == {(1, 512), (2, 512), (2, 1024)} and wave <= ok
