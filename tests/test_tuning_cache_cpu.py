"""The tuning file's versioning (no GPU): a record is applied only on the
device name and library build it was written for, and a malformed record is
ignored rather than half-applied."""
import json

import paper_2108_13656_amd as P

T = {"groups": [1, 2, 2], "mixed_groups": 1, "decolor_grid_per_cu": 0, "mixed_grid_per_cu": 0,
     "pass1_grid_per_cu": 16, "pass2_grid_per_cu": 0, "tonemap_pipeline": 0}


def test_round_trip_through_json():
    rec = json.loads(json.dumps(P.tuning_record(T, "AMD Instinct MI355X", "abc")))
    assert P.tuning_from_record(rec, "AMD Instinct MI355X", "abc") == T


def test_other_device_or_build_is_ignored():
    rec = P.tuning_record(T, "AMD Instinct MI355X", "abc")
    assert P.tuning_from_record(rec, "AMD Instinct MI300X", "abc") is None
    assert P.tuning_from_record(rec, "AMD Instinct MI355X", "def") is None
    assert P.tuning_from_record(dict(rec, version=99), "AMD Instinct MI355X", "abc") is None


def test_malformed_records_are_ignored():
    ok = P.tuning_record(T, "d", "h")
    broken = dict(ok, tuning={k: v for k, v in T.items() if k != "groups"})
    for rec in ({}, [], "x", dict(ok, tuning=None), broken):
        assert P.tuning_from_record(rec, "d", "h") is None
