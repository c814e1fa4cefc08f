"""Host logic of the autotuning cache (no GPU): size buckets, keys and the JSON file."""
import json

import numpy as np

from paper_1405_7537_amd import tuning as T


def test_buckets_group_sizes_within_half_an_octave():
    assert T.key_single("gfx950", 32768, True, 1) == T.key_single("gfx950", 30000, True, 1)
    assert T.key_single("gfx950", 32768, True, 1) != T.key_single("gfx950", 65536, True, 1)
    assert T.key_single("gfx950", 32768, True, 1) != T.key_single("gfx950", 32768, False, 1)
    assert T.key_single("gfx950", 32768, True, 1) != T.key_single("gfx950", 32768, True, 0)
    assert T.key_single("gfx950", 32768, True, 1) != T.key_single("gfx942", 32768, True, 1)


def test_batched_key_uses_count_largest_size_and_volume():
    a = np.array([16, 100, 2048, 700])
    b = np.array([16, 101, 2048, 690])
    assert T.key_batched("gfx950", a, True, 1) == T.key_batched("gfx950", b, True, 1)
    c = np.array([16, 100, 1024, 700])
    assert T.key_batched("gfx950", a, True, 1) != T.key_batched("gfx950", c, True, 1)
    assert T.key_batched("gfx950", np.repeat(a, 4), True, 1) != T.key_batched("gfx950", a, True, 1)


def test_store_and_load_round_trip(tmp_path):
    p = str(tmp_path / "sub" / "tuning.json")
    assert T.load(p) == {}
    T.store("k1", {"split": 8, "main_passes": 2, "waves_per_simd": 8, "vwrite": 1, "ms": 4.25}, p)
    T.store("k2", {"split": 4, "main_passes": 3, "ms": 1.5}, p)
    got = T.load(p)
    assert got["k1"] == {"split": 8, "main_passes": 2, "waves_per_simd": 8, "vwrite": 1, "ms": 4.25}
    assert got["k2"]["waves_per_simd"] == 0          # absent: the library default
    assert got["k2"]["vwrite"] == 0
    assert got["k2"]["split"] == 4
    T.store("k1", {"split": 16, "main_passes": 2, "ms": 4.0}, p)
    assert T.load(p)["k1"]["split"] == 16


def test_corrupt_cache_reads_as_empty(tmp_path):
    p = tmp_path / "tuning.json"
    p.write_text("{not json")
    assert T.load(str(p)) == {}
    p.write_text(json.dumps([1, 2, 3]))
    assert T.load(str(p)) == {}


def test_cache_path_honours_environment(monkeypatch, tmp_path):
    monkeypatch.setenv("DPR1_TUNING_CACHE", str(tmp_path / "x.json"))
    assert T.cache_path() == str(tmp_path / "x.json")


def test_unwritable_cache_is_not_fatal(tmp_path):
    blocker = tmp_path / "file"
    blocker.write_text("x")
    p = str(blocker / "sub" / "tuning.json")      # a directory below a regular file cannot be made
    assert T.store("k", {"split": 8, "main_passes": 2, "ms": 1.0}, p) is False
    assert T.load(p) == {}
