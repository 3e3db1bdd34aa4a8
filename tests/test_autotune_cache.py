"""Tile-shape autotuner cache (host logic, no GPU): a stored choice is
returned without measuring, the key separates problems that differ in any
domain, precision or option, and a corrupt cache file is ignored."""
import json

import pytest

from paper_2605_09097_amd import autotune, binding, scenes


@pytest.fixture()
def tiny():
    return scenes.workload("inclusion_tiny")


def _opts(sc, warm=False):
    return binding.schwarz_opts(sc.M, eps_tol=sc.eps_tol, warm_start=warm)


def test_cached_choice_is_returned_without_measuring(tmp_path, tiny, monkeypatch):
    path = str(tmp_path / "tiles.json")
    opts = _opts(tiny)
    cands = autotune.CANDIDATES_2D
    key = autotune.signature("batch", [tiny], opts, binding.OSMPM_MIXED, cands, 0)
    autotune._cache_put(path, key, {"tile": [16, 8], "timings": {}})

    def refuse(*a, **k):
        raise AssertionError("measured although the choice is cached")

    monkeypatch.setattr(binding, "SchwarzBatch", refuse)
    monkeypatch.setattr(binding, "SchwarzPair", refuse)
    tile, timings = autotune.tune_batch(None, [tiny], opts, binding.OSMPM_MIXED, cache=path)
    assert tile == (16, 8) and timings == {}
    kp = autotune.signature("pair", [tiny], opts, binding.OSMPM_MIXED, cands, 0)
    autotune._cache_put(path, kp, {"tile_B": [8, 8], "tile_S": [8, 4], "timings": {}})
    tB, tS, timings = autotune.tune_pair(None, tiny, opts, binding.OSMPM_MIXED, cache=path)
    assert (tB, tS, timings) == ((8, 8), (8, 4), {})
    with open(path) as f:
        assert set(json.load(f)) == {key, kp}


def test_signature_separates_problems(tiny):
    other = scenes.workload("inclusion_tiny", seed=1)
    c = autotune.CANDIDATES_2D
    base = autotune.signature("batch", [tiny], _opts(tiny), binding.OSMPM_MIXED, c, 0)
    assert base == autotune.signature("batch", [tiny], _opts(tiny), binding.OSMPM_MIXED, c, 0)
    variants = [
        autotune.signature("pair", [tiny], _opts(tiny), binding.OSMPM_MIXED, c, 0),
        autotune.signature("batch", [tiny], _opts(tiny, warm=True), binding.OSMPM_MIXED, c, 0),
        autotune.signature("batch", [tiny], _opts(tiny), binding.OSMPM_FP64, c, 0),
        autotune.signature("batch", [tiny], _opts(tiny), binding.OSMPM_MIXED, c[:2], 0),
        autotune.signature("batch", [tiny], _opts(tiny), binding.OSMPM_MIXED, c, 2),
        autotune.signature("batch", [tiny, tiny], _opts(tiny), binding.OSMPM_MIXED, c, 0),
    ]
    if len(other.B.x) != len(tiny.B.x) or len(other.S.x) != len(tiny.S.x):
        variants.append(autotune.signature("batch", [other], _opts(tiny), binding.OSMPM_MIXED, c, 0))
    assert base not in variants and len(set(variants)) == len(variants)


def test_corrupt_cache_is_ignored(tmp_path):
    path = tmp_path / "tiles.json"
    path.write_text("{not json")
    assert autotune._cache_get(str(path), "k") is None
    autotune._cache_put(str(path), "k", {"tile": [4, 4]})
    assert autotune._cache_get(str(path), "k") == {"tile": [4, 4]}
