"""The launch configuration and the tuner's cache on the host: expm_tune_set / expm_tune_get
round trip through the C ABI, range checks, and a cache entry written, reloaded and installed
giving back exactly the configuration it holds (no GPU needed)."""
import ctypes
import json

import pytest

from paper_1710_10989_amd import _native as N
from paper_1710_10989_amd import autotune as T


def _cfg():
    return {"arrangement": [2, 1, 3], "small_kernel": 2, "per_cu": [1, 1, 2, 1, 1, 3],
            "tiles_per_launch": [1024, 4096, 2048, 1024]}


def test_set_get_round_trip():
    try:
        t = T.from_dict(_cfg())
        T.set_tune(t)
        assert T.to_dict(T.get()) == _cfg()
        T.defaults()
        assert T.to_dict(T.get()) == {"arrangement": [0, 0, 0], "small_kernel": 0, "per_cu": [0] * 6,
                                      "tiles_per_launch": [0] * 4}
    finally:
        T.defaults()


@pytest.mark.parametrize("field,value", [("arrangement", [4, 0, 0]), ("small_kernel", 3), ("per_cu", [0, -1, 0, 0, 0, 0]),
                                         ("tiles_per_launch", [0, 0, -5, 0])])
def test_out_of_range_rejected(field, value):
    d = _cfg()
    d[field] = value
    before = T.to_dict(T.get())
    assert N.lib().expm_tune_set(ctypes.byref(T.from_dict(d))) == N.EXPM_E_INVALID_ARG
    assert T.to_dict(T.get()) == before  # nothing installed


def test_cache_reload_reproduces_choices(tmp_path):
    path = str(tmp_path / "cache.json")
    entry = {"tune": _cfg(), "entries": {"arrangement/16-128/fp64/plain": {"choice": 2, "ms": {"0": 1.0, "2": 0.9}}},
             "device": "test", "quick": True, "when": "now"}
    try:
        T.save(entry, path, which="gfxTEST")
        T.save({"tune": {"arrangement": [1, 1, 1]}, "entries": {}}, path, which="gfxOTHER")
        with open(path) as fh:
            assert set(json.load(fh)) == {"gfxTEST", "gfxOTHER"}
        assert T.install(path, which="gfxTEST") == _cfg()
        assert T.to_dict(T.get()) == _cfg()
        assert T.install(path, which="gfxNONE") is None
        assert T.to_dict(T.get()) == _cfg()  # no entry: configuration unchanged
    finally:
        T.defaults()
