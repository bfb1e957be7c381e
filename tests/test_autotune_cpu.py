"""Host logic of the autotuner's cache (no kernel runs): the JSON document
named by SWEPT_AUTOTUNE_CACHE is read on lookup, and the process table can be
cleared."""
import json

import pytest

import paper_1612_02495_amd as P
from paper_1612_02495_amd import _lib


@pytest.fixture
def cache_file(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("SWEPT_AUTOTUNE_CACHE", str(path))
    P.swept_autotune_forget()
    yield path
    P.swept_autotune_forget()


def test_lookup_reads_cache_file(cache_file):
    doc = {"swept_autotune": 1, "entries": [
        {"kind": 0, "dtype": 1, "n": 1048576, "tile_width": 1024, "steps_per_cycle": 512, "engine": 2,
         "ns_per_cell_update": 0.0003},
        {"kind": 1, "dtype": 1, "n": 65536, "tile_width": 512, "steps_per_cycle": 32, "engine": 1,
         "ns_per_cell_update": 0.002},
    ]}
    cache_file.write_text(json.dumps(doc))
    got = P.swept_autotune_lookup(1048576, "heat", "f64")
    assert got["tile_width"] == 1024 and got["steps_per_cycle"] == 512 and got["engine"] == "wave"
    got = P.swept_autotune_lookup(65536, "ks", "f64")
    assert got["tile_width"] == 512 and got["engine"] == "lds"
    assert P.swept_autotune_lookup(65536, "ks", "f32") is None


def test_lookup_without_cache(monkeypatch):
    monkeypatch.delenv("SWEPT_AUTOTUNE_CACHE", raising=False)
    P.swept_autotune_forget()
    assert P.swept_autotune_lookup(4096, "heat", "f64") is None


def test_malformed_cache_is_ignored(cache_file):
    cache_file.write_text('{"entries": [ {"kind": 0, "dtype": 1} , garbage ')
    assert P.swept_autotune_lookup(1048576, "heat", "f64") is None


def test_autotune_rejects_bad_arguments():
    lib = _lib.lib()
    assert lib.swept_autotune(1024, 9, 1, 1e-6, 1e-3, 1.0, 0, None, 0, None, None, None, None) == _lib.SWEPT_EINVAL
    assert lib.swept_autotune(1024, 0, 1, 1e-6, 1e-3, 1.0, -1, None, 0, None, None, None, None) == _lib.SWEPT_EINVAL
    assert lib.swept_autotune(1024, 0, 1, 1e-6, 1e-3, 1.0, 0, None, 4, None, None, None, None) == _lib.SWEPT_EINVAL
    assert lib.swept_autotune_lookup(1024, 5, 1, None, None, None, None) == _lib.SWEPT_EINVAL
