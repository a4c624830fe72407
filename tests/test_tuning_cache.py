"""On-disk cache of the level autotuner (host logic, no GPU)."""
import json

from paper_2510_13965_amd.tuning import TuningCache, cache_key

BOXES = [(16, 24, 32), (64, 64, 16), (16, 24, 32)]


def test_key_ignores_box_order_and_sees_every_input():
    k = cache_key(BOXES, 0, "MI355X", 3)
    assert k == cache_key(list(reversed(BOXES)), 0, "MI355X", 3)
    others = [cache_key(BOXES[:2], 0, "MI355X", 3),            # a box less (the multiset counts)
              cache_key([(16, 24, 48)] + BOXES[1:], 0, "MI355X", 3),
              cache_key(BOXES, 8, "MI355X", 3),                 # radiation evolved
              cache_key(BOXES, 0, "other device", 3),
              cache_key(BOXES, 0, "MI355X", 2)]
    assert len({k, *others}) == 1 + len(others)


def test_put_get_roundtrip_and_overwrite(tmp_path):
    c = TuningCache(tmp_path / "sub" / "tune.json")
    assert c.get("a") is None
    c.put("a", {"strip": 4, "block_threads": 128, "grid_per_cu": 0, "extra": 1})
    c.put("b", {"strip": 1, "block_threads": 64, "grid_per_cu": 16})
    assert TuningCache(tmp_path / "sub" / "tune.json").get("a") == {"strip": 4, "block_threads": 128, "grid_per_cu": 0}
    c.put("a", {"strip": 16, "block_threads": 256, "grid_per_cu": 4})
    assert c.get("a") == {"strip": 16, "block_threads": 256, "grid_per_cu": 4}
    assert c.get("b") == {"strip": 1, "block_threads": 64, "grid_per_cu": 16}
    assert not list((tmp_path / "sub").glob("*.tmp"))


def test_unreadable_or_malformed_cache_counts_as_empty(tmp_path):
    p = tmp_path / "tune.json"
    p.write_text("{not json")
    c = TuningCache(p)
    assert c.get("a") is None
    c.put("a", {"strip": 1, "block_threads": 64, "grid_per_cu": 0})
    assert c.get("a") == {"strip": 1, "block_threads": 64, "grid_per_cu": 0}
    p.write_text(json.dumps({"a": {"strip": "1", "block_threads": 64, "grid_per_cu": 0}, "b": [1, 2]}))
    assert c.get("a") is None and c.get("b") is None
