"""Autotuner host logic: cache keys, buckets and the JSON cache round trip."""
from paper_2503_11731_amd import autotune as at


def test_bucket_and_key():
    assert at.n_bucket(1) == 1
    assert at.n_bucket(1_000_000) == 1 << 20
    assert at.n_bucket(700_000) == 1 << 19
    k1 = at.cache_key("gfx950", "pinhole", 1920, 1080, 1_000_000, False)
    k2 = at.cache_key("gfx950", "pinhole", 1920, 1080, 1_100_000, False)
    k3 = at.cache_key("gfx950", "pinhole", 1920, 1080, 1_000_000, True)
    assert k1 == k2 and k1 != k3


def test_cache_round_trip(tmp_path):
    p = str(tmp_path / "sub" / "cache.json")
    c = at.TuneCache(p)
    assert c.get("x") is None
    c.put("x", {"ms": {"16x16/1024": 1.5}})
    c.save()
    c2 = at.TuneCache(p)
    assert c2.get("x") == {"ms": {"16x16/1024": 1.5}}
    assert at._parse(at._fmt((32, 8), 512)) == ((32, 8), 512)


def test_corrupt_cache_is_ignored(tmp_path):
    p = tmp_path / "c.json"
    p.write_text("{not json")
    assert at.TuneCache(str(p), seed="").data == {}


def test_pick_keeps_the_preferred_candidate_within_the_margin():
    ms = {"a": 1.00, "b": 1.02, "c": 1.10}
    assert at.pick(ms, "b", 0.03) == "b"      # within 3 % of the best: kept
    assert at.pick(ms, "c", 0.03) == "a"      # 10 % slower: the best wins
    assert at.pick(ms, None, 0.03) == "a"
    assert at.pick(ms, "zz", 0.03) == "a"     # not a candidate
    assert at.pick({2048: 5.0, 1024: 4.99}, 2048) == 2048


def test_shipped_seed_takes_precedence(tmp_path):
    user = tmp_path / "user.json"
    seed = tmp_path / "seed.json"
    user.write_text('{"k": {"ms": {"32x8/1024": 2.0}}, "u": {"ms": {}}}')
    seed.write_text('{"k": {"ms": {"16x16/4096": 1.0}}}')
    c = at.TuneCache(str(user), seed=str(seed))
    assert c.get("k") == {"ms": {"16x16/4096": 1.0}} and c.get("u") == {"ms": {}}
    assert at.TuneCache(str(user), seed="").get("k") == {"ms": {"32x8/1024": 2.0}}
