"""Tuning cache on the host: entries, validation and JSON persistence (no device)."""
import json
import os

import pytest

from paper_2510_20870_amd import xsec

pytestmark = pytest.mark.skipif(not os.path.exists(xsec.LIB_PATH), reason="libxsec.so not built")


@pytest.fixture(autouse=True)
def clean_cache():
    xsec.tune_cache_clear()
    yield
    xsec.tune_cache_clear()


def test_put_get_and_validation():
    assert xsec.tune_cache_get("k") is None
    xsec.tune_cache_put("k", 4, 3, 8, 1.5)
    assert xsec.tune_cache_get("k") == (4, 3, 8, 1.5)
    xsec.tune_cache_put("k", 1, 2, 1)
    assert xsec.tune_cache_get("k")[:3] == (1, 2, 1)
    assert xsec.tune_cache_size() == 1
    # occupancy options 2..6 (0, automatic, is not a shape)
    for bad in ((3, 2, 4), (2, 0, 4), (2, 7, 4), (2, 2, 0), (2, 2, 65), (16, 2, 4)):
        with pytest.raises(xsec.XsError) as e:
            xsec.tune_cache_put("x", *bad)
        assert e.value.code == xsec.XS_EINVAL
    with pytest.raises(xsec.XsError):
        xsec.tune_cache_put("", 2, 2, 4)
    assert xsec.tune_cache_size() == 1


def test_save_load_roundtrip(tmp_path):
    keys = {'gfx950:sramecc+:xnack-|cu256|fp32|fixed|d16|p1': (2, 6, 4, 12.5),
            'gfx950|cu256|fp64|fwhm|d20|pmany': (8, 4, 16, 0.25),
            'odd "quoted" \\ key': (1, 3, 2, 3.0)}
    for k, v in keys.items():
        xsec.tune_cache_put(k, *v)
    f = tmp_path / "tune.json"
    xsec.tune_cache_save(str(f))
    doc = json.loads(f.read_text())          # a valid JSON document
    assert doc["version"] == 1 and set(doc["entries"]) == set(keys)
    assert doc["entries"]['odd "quoted" \\ key']["items_per_slot"] == 2
    xsec.tune_cache_clear()
    assert xsec.tune_cache_size() == 0
    xsec.tune_cache_load(str(f))
    for k, v in keys.items():
        assert xsec.tune_cache_get(k) == v
    # loading merges: existing entries not in the file stay, file entries win
    xsec.tune_cache_put("extra", 2, 2, 4)
    xsec.tune_cache_put('gfx950|cu256|fp64|fwhm|d20|pmany', 1, 2, 1)
    xsec.tune_cache_load(str(f))
    assert xsec.tune_cache_get("extra") is not None
    assert xsec.tune_cache_get('gfx950|cu256|fp64|fwhm|d20|pmany') == (8, 4, 16, 0.25)


def test_load_accepts_extra_fields(tmp_path):
    f = tmp_path / "t.json"
    f.write_text(json.dumps({"version": 1, "note": {"a": [1, 2, {"b": None}], "c": True},
                             "entries": {"k": {"P": 4, "W": 0, "items_per_slot": 2,
                                               "probe_ms": 1.0, "comment": "x"}}}))
    xsec.tune_cache_load(str(f))
    # W 0 (no occupancy target, as files of an earlier version wrote it) is the option 2
    assert xsec.tune_cache_get("k") == (4, 2, 2, 1.0)


@pytest.mark.parametrize("text", [
    "", "{", "[]", '{"entries": {"k": {"P": 2, "W": 0}}}',           # missing field
    '{"entries": {"k": {"P": 3, "W": 0, "items_per_slot": 4}}}',     # invalid P
    '{"entries": {"k": {"P": 2, "W": 0, "items_per_slot": 4}}} x',   # trailing junk
    '{"entries": {"k": {"P": "2", "W": 0, "items_per_slot": 4}}}',   # wrong type
    '{"entries": {"k" {"P": 2, "W": 0, "items_per_slot": 4}}}',      # missing colon
])
def test_malformed_files_are_rejected(tmp_path, text):
    f = tmp_path / "bad.json"
    f.write_text(text)
    with pytest.raises(xsec.XsError) as e:
        xsec.tune_cache_load(str(f))
    assert e.value.code == xsec.XS_EINVAL
    assert xsec.tune_cache_size() == 0      # nothing merged from a bad file


def test_missing_file():
    with pytest.raises(xsec.XsError) as e:
        xsec.tune_cache_load("/nonexistent/dir/tune.json")
    assert e.value.code == xsec.XS_ENOTFOUND
