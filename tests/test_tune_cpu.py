"""Autotuner cache and key (host only: no device is touched)."""
import json

import pytest

from paper_2303_02471_amd import _lib, api


def _opts(t_esc=128, t_dense=512, dense_rows=4096, hash_cap=2048, t_split=-1, t_block=2048):
    return _lib.Options(t_esc, t_dense, dense_rows, hash_cap, 0, t_split, t_block)


def _same(a, b):
    return all(getattr(a, f) == getattr(b, f)
               for f in ("t_esc", "t_dense", "dense_rows", "hash_cap", "t_split", "t_block"))


def test_key_buckets():
    k1 = api.tune_key([(1100, 1100, 1100, 5000, 5000)])
    assert k1 == api.tune_key([(1100, 1100, 1100, 5000, 5000)])
    # a few percent apart: same half-octave buckets
    assert k1 == api.tune_key([(1130, 1130, 1130, 5100, 5100)])
    assert k1 != api.tune_key([(4000, 4000, 4000, 5000, 5000)])
    assert k1 != api.tune_key([(1100, 1100, 1100, 5000, 5000)], dtype=api.torch.float32)
    assert k1 != api.tune_key([(1100, 1100, 1100, 5000, 5000)], device_tag="other")
    # a batch differs from a single problem of the same totals
    assert api.tune_key([(500, 500, 500, 2500, 2500)] * 2) != api.tune_key(
        [(1000, 1000, 1000, 5000, 5000)])


def test_store_load_roundtrip(tmp_path):
    path = str(tmp_path / "tune.json")
    assert api.tune_cache_load(path, "a") is None  # no file
    api.tune_cache_store(path, "a", _opts(t_esc=64), 1.5)
    api.tune_cache_store(path, "b|x\"y", _opts(t_split=2048), 2.5)
    got = api.tune_cache_load(path, "a")
    assert got is not None and _same(got, _opts(t_esc=64))
    got = api.tune_cache_load(path, "b|x\"y")
    assert got is not None and _same(got, _opts(t_split=2048))
    assert api.tune_cache_load(path, "c") is None
    # replacing an entry keeps the others; the file is plain JSON
    api.tune_cache_store(path, "a", _opts(t_esc=32), 0.5)
    doc = json.load(open(path))
    assert doc["spgemm_tune_cache"] == 1 and len(doc["entries"]) == 2
    assert _same(api.tune_cache_load(path, "a"), _opts(t_esc=32))


@pytest.mark.parametrize("text", [
    "", "garbage", "{", '{"spgemm_tune_cache": 1}', '{"entries": []}',
    '{"spgemm_tune_cache": 2, "entries": []}',
    '{"spgemm_tune_cache": 1, "entries": [{"key": "a", "t_esc": 64}',
    '{"spgemm_tune_cache": 1, "entries": [{"t_esc": 64}]}',
    '{"spgemm_tune_cache": 1, "entries": [{"key": "a", "t_esc": 6.5}]}',
    '{"spgemm_tune_cache": 1, "entries": []} trailing'])
def test_corrupt_cache_ignored_and_rewritten(tmp_path, text):
    path = str(tmp_path / "tune.json")
    with open(path, "w") as f:
        f.write(text)
    assert api.tune_cache_load(path, "a") is None
    api.tune_cache_store(path, "a", _opts(), 1.0)
    assert _same(api.tune_cache_load(path, "a"), _opts())
    json.load(open(path))


def test_out_of_range_entry_unused(tmp_path):
    path = str(tmp_path / "tune.json")
    with open(path, "w") as f:
        json.dump({"spgemm_tune_cache": 1, "entries": [
            {"key": "a", "t_esc": 3, "t_dense": 512, "dense_rows": 4096, "hash_cap": 4096,
             "t_split": 4096, "ms": 1.0},
            {"key": "b", "t_esc": 64, "t_dense": 512, "dense_rows": 4096, "hash_cap": 4096,
             "t_split": 4096, "ms": 1.0, "extra": [1, {"x": None}]}]}, f)
    assert api.tune_cache_load(path, "a") is None
    got = api.tune_cache_load(path, "b")
    assert got is not None and got.t_esc == 64


def test_lookup_only_without_entry_does_not_time():
    """Status 10 (not tuned) is distinct from real errors."""
    assert _lib.STATUS[10] == "SPGEMM_ERR_NOT_TUNED"
