"""Autotuner selection and caching logic (CPU; the GPU tests run it on the
device)."""
import json

from paper_1812_06632_amd import autotune


def test_candidates_cover_space():
    space = {"block": (64, 128), "refill_min": (1, 8, 32)}
    c = list(autotune.candidates(space))
    assert len(c) == 6 and {"block": 128, "refill_min": 8} in c


def test_tune_picks_fastest_and_caches(tmp_path):
    calls = []

    def measure(cfg):
        calls.append(cfg)
        return 1.0 + abs(cfg["block"] - 256) / 256 + (0.5 if cfg["refill_min"] == 1 else 0.0)

    path = str(tmp_path / "tune.json")
    tu = autotune.Autotuner(path)
    space = {"block": (128, 256, 512), "refill_min": (1, 16)}
    key = autotune.class_key("regular", 2 ** 21, 0.04, "dust")
    best = tu.tune(key, measure, space, repeats=2)
    assert best == {"block": 256, "refill_min": 16}
    assert len(calls) == 12
    again = autotune.Autotuner(path).tune(key, measure, space)
    assert again == best and len(calls) == 12
    data = json.load(open(path))
    assert data[key]["config"] == best and len(data[key]["tried"]) == 6


def test_class_key_buckets():
    assert autotune.class_key("regular", 2 ** 21, 0.04, "dust") == autotune.class_key("regular", 2 ** 21 + 5, 0.05, "dust")
    assert autotune.class_key("octree", 100, 5.0, "bg") != autotune.class_key("octree", 100, 0.5, "bg")
