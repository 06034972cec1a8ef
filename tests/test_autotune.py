"""Host logic of the autotuner: cache keys, m buckets, knob sets and the JSON cache file."""
import json

import pytest

from paper_2510_04094_amd import autotune, nyls


def test_m_bucket_follows_the_slot_classes():
    assert [autotune.m_bucket(m) for m in (2, 32, 33, 64, 65, 128, 129, 256)] == \
        ["m<=32", "m<=32", "m<=64", "m<=64", "m<=128", "m<=128", "m<=256", "m<=256"]


def test_key_names_arch_bucket_orders_and_mode():
    assert autotune.make_key("gfx950", 50, [2, 2, 2], nyls.FP64) == "gfx950|m<=64|p2|fp64"
    assert autotune.make_key("gfx950", 100, [2, 1, 2], nyls.MIXED) == "gfx950|m<=128|p1+2|mixed"


def test_knob_values_skip_choices_that_cannot_apply():
    k = autotune.knob_values(50, 50, nyls.FP64)
    assert set(k) == {"eig_ql", "ql_lanes", "gram_valu", "tail_layout", "overlap"}
    k = autotune.knob_values(50, 50, nyls.FP64, max_n=50000)
    assert "split" in k and k["split"][0] == nyls.DEFAULT_TUNING["split"]
    k = autotune.knob_values(100, 70, nyls.FP64)
    assert "eig_ql" not in k and "gram_valu" not in k  # every basis beyond the one-wave kernels
    k = autotune.knob_values(50, 40, nyls.MIXED)
    assert "gram_valu" not in k and "overlap" not in k  # FP64-only choices, one slot class
    k = autotune.knob_values(50, 20, nyls.MIXED)
    assert "overlap" in k  # the passes of the two slot classes may run side by side
    for name, vals in autotune.knob_values(20, 20, nyls.FP64).items():
        assert vals[0] == nyls.DEFAULT_TUNING[name]  # the search starts from the defaults


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tuning.json")
    assert autotune.lookup("k", path) is None
    tun = dict(nyls.DEFAULT_TUNING, eig_ql=1)
    autotune.save_entry("k", {"tuning": tun, "ms": 1.0}, path)
    autotune.save_entry("other", {"tuning": nyls.DEFAULT_TUNING, "ms": 2.0}, path)
    assert autotune.lookup("k", path) == tun
    data = json.load(open(path))
    assert set(data) == {"k", "other"}


def test_cache_ignores_damaged_entries(tmp_path):
    path = tmp_path / "tuning.json"
    path.write_text("{not json")
    assert autotune.lookup("k", str(path)) is None
    path.write_text(json.dumps({"k": {"tuning": {"eig_ql": 1}}}))
    assert autotune.lookup("k", str(path)) is None


def test_cache_path_from_environment(monkeypatch, tmp_path):
    monkeypatch.setenv("NYLS_TUNING_CACHE", str(tmp_path / "x.json"))
    assert autotune.cache_path() == str(tmp_path / "x.json")


def test_tuning_structure_matches_the_header():
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "nyls.h")).read()
    body = re.search(r"typedef struct nyls_tuning \{(.*?)\} nyls_tuning;", hdr, re.S).group(1)
    fields = re.findall(r"(\w+)(?:,|;)", body.replace("int32_t", ""))
    assert tuple(fields) == nyls.TUNING_FIELDS
