"""Host logic of the autotuner: candidate filtering, cache keys and the JSON
cache round trip (no GPU)."""
import json

from paper_2403_07042_amd import autotune as A


def test_candidates_respect_ld_and_precision():
    assert A.candidates("fp32", 2048) == [(32, 32), (32, 64), (64, 32), (64, 64), (64, 128),
                                          (128, 64), (128, 128)]
    assert A.candidates("fp32", 1728) == [(32, 32), (32, 64), (64, 32), (64, 64)]
    assert A.candidates("fp64", 96) == [(32, 32)]
    assert A.candidates("bf16x3", 2048) == [(64, 64), (128, 64)]
    assert A.candidates("bf16x3", 1728) == [(64, 64)]


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert A.load_cache(path) == {}
    key = A.solver_key("gfx950", "fp32", 2048, 2048)
    A.save_cache({key: {"tiles": [64, 128]}}, path)
    assert A.load_cache(path)[key]["tiles"] == [64, 128]
    with open(path, "w") as f:
        f.write("not json")
    assert A.load_cache(path) == {}
    assert json.loads(json.dumps({key: 1}))[key] == 1


def test_cache_path_env(monkeypatch, tmp_path):
    monkeypatch.setenv(A.CACHE_ENV, str(tmp_path / "x.json"))
    assert A.cache_path() == str(tmp_path / "x.json")
