"""Host-side accounting of the benchmark line: algorithmic bytes per kernel
from the per-unit byte table (fixed from the state's field widths), the
whole-path bytes per track-step, the drain threshold of a session of given
size, and the lookup of committed hardware byte counts (host logic only)."""
import json
import types

import pytest

import bench


def test_field_step_bytes_add_pre_step_deposit_and_post_step():
    u = bench.UNIT_BYTES["f64"]
    assert u["field"] + u["pre"] + u["deposit"] + u["post"] == 262
    work = {"along_field": 10, "field_paused": 2}
    # 8 completed steps with their pre-step, deposit and post-step, 2 paused trips
    assert bench.kernel_bytes("along_field", work, "f64") == 8 * 262 + 2 * 112
    um = bench.UNIT_BYTES["mixed"]
    assert bench.kernel_bytes("along_field", work, "mixed") == 8 * (um["field"] + um["pre"] + um["deposit"] +
                                                                     um["post"]) + 2 * um["pause"]


def test_interaction_and_fill_bytes_count_their_units():
    work = {k: 1 for k in bench.INTERACTIONS}
    assert bench.kernel_bytes("interactions", work, "f64") == 7 * 116
    assert bench.kernel_bytes("init", {"init": 5}, "f64") == 5 * 172
    assert bench.kernel_bytes("along_neutral", {"along_neutral": 3}, "f64") == 3 * (110 + 53 + 19)
    with pytest.raises(KeyError):
        bench.kernel_bytes("sort", {}, "f64")


def test_path_bytes_per_step_include_secondary_records():
    work = {"along_field": 4, "field_paused": 0, "along_neutral": 2, "compton": 1, "init": 3, "drain": 0}
    r = bench.path_roofline(work, steps=6, rate=1e9, precision="f64", n_primaries=1)
    total = 4 * 262 + 2 * 182 + 116 + 3 * 172 + (3 - 1) * 71
    assert abs(r["bytes_per_step"] - total / 6) < 1e-9
    assert abs(r["achieved"] - 1e9 * total / 6 / 1e9) < 1e-9
    assert abs(r["frac"] - r["achieved"] / bench.HBM_PEAK_GBS) < 1e-12


def test_drain_threshold_scales_with_session_slots():
    a = types.SimpleNamespace(drain_threshold=65536)
    assert bench.drain_for(a, 1 << 20) == 65536
    assert bench.drain_for(a, 1 << 22) == 65536
    assert bench.drain_for(a, 1 << 18) == 16384
    assert bench.drain_for(a, 1 << 8) == 256
    assert bench.drain_for(types.SimpleNamespace(drain_threshold=0), 1 << 20) == 0


def test_committed_traffic_needs_the_same_sources_and_configuration(tmp_path, monkeypatch):
    key = {"workload": "w", "precision": "f64", "n_slots": 1 << 20}
    line = {"kernel": "along_field", "config": key, "sources_sha256": "abc", "bytes_per_launch": 1.0e8}
    (tmp_path / "x.md").write_text("# summary\n\ntraffic: " + json.dumps(line) + "\n")
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    monkeypatch.setattr(bench, "source_digest", lambda: "abc")
    assert bench.committed_traffic("along_field", key)["bytes_per_launch"] == 1.0e8
    assert bench.committed_traffic("interactions", key) is None
    assert bench.committed_traffic("along_field", dict(key, n_slots=1 << 21)) is None
    monkeypatch.setattr(bench, "source_digest", lambda: "def")
    assert bench.committed_traffic("along_field", key) is None
