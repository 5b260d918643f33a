"""The binding's launch-tuning cache (a JSON file of hdg_tuning values keyed by
device, mesh, degree, flux, precision, smoother and right-hand sides): round
trip, other entries kept, unreadable or incomplete entries ignored.  Host
logic only; no library call."""
import json

from paper_2004_09389_amd.hdg import HdgTuning, tuning_cache_get, tuning_cache_put

T1 = {"mlp_samples_per_lane": 2, "rhs_block": 4, "cell_cells": 4}
T2 = {"mlp_samples_per_lane": 1, "rhs_block": 1, "cell_cells": 0}


def test_round_trip_and_other_entries_kept(tmp_path):
    path = str(tmp_path / "tuning.json")
    assert tuning_cache_get(path, "a") is None
    tuning_cache_put(path, "a", T1)
    tuning_cache_put(path, "b", T2)
    assert tuning_cache_get(path, "a") == T1
    assert tuning_cache_get(path, "b") == T2
    tuning_cache_put(path, "a", T2)
    assert tuning_cache_get(path, "a") == T2 and tuning_cache_get(path, "b") == T2
    data = json.load(open(path))
    assert data["version"] == 1 and sorted(data["entries"]) == ["a", "b"]
    assert [p.name for p in tmp_path.iterdir()] == ["tuning.json"]   # no temporary left behind


def test_every_field_is_stored():
    assert sorted(T1) == sorted(f for f, _ in HdgTuning._fields_)


def test_unreadable_or_incomplete_entries_are_ignored(tmp_path):
    path = tmp_path / "tuning.json"
    path.write_text("{ not json")
    assert tuning_cache_get(str(path), "a") is None
    tuning_cache_put(str(path), "a", T1)        # replaces the unreadable file
    assert tuning_cache_get(str(path), "a") == T1
    data = json.load(open(path))
    data["entries"]["b"] = {"rhs_block": 4}     # fields missing
    data["entries"]["c"] = {"mlp_samples_per_lane": 1, "rhs_block": "4", "cell_cells": 0}   # not an int
    path.write_text(json.dumps(data))
    assert tuning_cache_get(str(path), "b") is None
    assert tuning_cache_get(str(path), "c") is None
    assert tuning_cache_get(str(path), "a") == T1
