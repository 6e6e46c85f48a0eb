"""Autotuner host logic on the CPU: shape buckets, the candidate set and the
JSON cache (the timing itself needs a device)."""
import json

from paper_2008_00326_amd import autotune


def test_shape_bucket_groups_by_powers_of_two():
    a = autotune.shape_bucket(640 * 480, 9000, 2000, True)
    assert a == autotune.shape_bucket(640 * 480, 8200, 2300, True)
    assert a != autotune.shape_bucket(640 * 480, 9000, 2000, False)
    assert a != autotune.shape_bucket(320 * 240, 9000, 2000, True)
    assert a.startswith("px18-tri13-pose11-")


def test_candidates_are_valid_settings():
    defaults = {"small_block": 512, "small_words": 19440, "grid": [512, 256, 256, 64], "order": 2, "key_bands": 2}
    cands = autotune.candidates(defaults, 256)
    assert cands[0] == {"small_block": 512, "order": 2, "grid": [0, 0, 0, 0], "small_words": 0}   # the default first
    keys = {json.dumps(c, sort_keys=True) for c in cands}
    assert len(keys) == len(cands)                                                            # no duplicates
    for c in cands:
        assert c["small_block"] in (256, 512)
        assert c["order"] in (1, 2)
        assert len(c["grid"]) == 4 and all(g >= 0 for g in c["grid"])
        assert 0 <= c["small_words"] <= defaults["small_words"]
        assert c.get("key_bands", 0) in (0, 1, 2)


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert autotune.load_cache(path) == {}
    rec = {"gfx950|px18": {"tuning": {"small_block": 256}, "ms": 1.5}}
    autotune.save_cache(rec, path)
    assert autotune.load_cache(path) == rec
    (tmp_path / "sub" / "tune.json").write_text("{not json")
    assert autotune.load_cache(path) == {}


def test_a_candidate_must_beat_the_default_by_five_per_cent():
    trials = [{"tuning": "default", "ms": 100.0}, {"tuning": "a", "ms": 97.0}, {"tuning": "b", "ms": 99.0}]
    assert autotune.choose(trials)["tuning"] == "default"       # 3 % is within the spread
    trials.append({"tuning": "c", "ms": 94.0})
    assert autotune.choose(trials)["tuning"] == "c"             # 6 % faster
    assert autotune.choose(trials, min_gain=0.10)["tuning"] == "default"
