"""Host logic of the convolution autotuner: the cache location and its JSON
round trip (CPU). Timing and applying shapes run on the GPU
(test_gpu_autotune.py)."""
import json

from paper_1310_7114_amd import autotune as T


def test_cache_path_order(monkeypatch, tmp_path):
    monkeypatch.delenv("ITC_TUNE_CACHE", raising=False)
    assert T.cache_path().endswith("tune.json")
    monkeypatch.setenv("ITC_TUNE_CACHE", str(tmp_path / "env.json"))
    assert T.cache_path() == str(tmp_path / "env.json")
    assert T.cache_path(str(tmp_path / "arg.json")) == str(tmp_path / "arg.json")


def test_store_and_load_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert T._load(path) == {}
    T._store(path, {"dev|images=3|weights=9|class=72": [192, 3]})
    assert T._load(path) == {"dev|images=3|weights=9|class=72": [192, 3]}
    with open(path) as f:
        assert json.load(f)["dev|images=3|weights=9|class=72"] == [192, 3]


def test_load_ignores_a_damaged_cache(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert T._load(str(path)) == {}
    path.write_text("[1, 2]")
    assert T._load(str(path)) == {}


def test_candidates_include_the_default_height():
    assert 256 in T.SEG_CANDIDATES
