"""Host logic of the bench and the tuner, without a GPU: the algorithmic
byte count of a row, the traffic records read from the profile summaries,
the state-update count of the headline step, the tuner's candidate space and
its cache lookups."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1005_3609_amd import tune  # noqa: E402


def test_row_bytes_formula():
    # two factors: 4 I (|S_in| + |S_out|) + 4 (|S_out| + 1) + 4 nnz each, and
    # the read-out vector (4 I |S_nc|) once with the last factor
    sizes = [(10, 12, 30), (12, 10, 25)]
    I, s_nc = 128, 7
    want = (4 * I * 22 + 4 * 13 + 4 * 30) + (4 * I * 22 + 4 * 11 + 4 * 25) + 4 * I * s_nc
    assert bench.row_bytes(sizes, I, s_nc) == want


def test_headline_step_state_updates():
    # a square m = 14 row is 787 333 state-updates per instance; the step
    # (15 rows, 14 forward rows, 640 instances) is 7.055e9
    sizes = bench.factor_sizes("square", 14)
    assert sum(s for _, s, _ in sizes) == 787333
    assert bench.updates_of("square", 14, 15, 640) == 14 * 787333 * 640


@pytest.mark.parametrize("workload", ["square_14x15", "square_18x19"])
def test_traffic_records_match_only_the_current_kernel(workload):
    # the committed record is read back only for the source hash and launch
    # shape it was measured with; after a kernel change it reads as None
    path = os.path.join(ROOT, "profiles", f"k_gather_{workload}.md")
    rec = None
    for line in open(path):
        if line.startswith("bench-traffic:"):
            rec = json.loads(line.split(":", 1)[1])
    assert rec is not None
    tuning = dict(rec["tuning"])
    got = bench.measured_traffic(rec["kernel"], tuning, workload)
    if rec["kernel_src"] == bench.kernel_source_hash():
        assert got == rec["bytes_per_launch"]
    else:
        assert got is None
    assert bench.measured_traffic(rec["kernel"], dict(tuning, streams=7), workload) is None
    other = "k_gather<1,8>" if rec["kernel"] != "k_gather<1,8>" else "k_gather<2,8>"
    assert bench.measured_traffic(other, tuning, workload) is None


def test_tuner_candidates_respect_the_rules():
    cands = tune.candidates()
    assert cands and all(c["streams"] == 1 for c in cands if c["mode"] == "grouped")
    assert not any(c["stage"] not in (0, 4, 6) and (c["mode"] == "grouped" or c["lanes_v"] > 2) for c in cands)
    assert len({json.dumps(c, sort_keys=True) for c in cands}) == len(cands)


def test_series_lanes_v():
    assert [tune.series_lanes_v(d) for d in (0, 63, 64, 127, 128, 255, 256, 511)] == [1, 1, 2, 2, 4, 4, 8, 8]


def test_tuned_table_lookups(monkeypatch, tmp_path):
    # the user cache first, then the shipped table; keys carry the gfx arch
    monkeypatch.setattr(tune, "_arch", lambda: "gfx950")
    monkeypatch.setattr(tune, "DEFAULT_CACHE", str(tmp_path / "none.json"))
    assert tune.lookup_tuned("square", 14, 640, 15)["fuse"] == 2
    assert tune.lookup_tuned_series("square", 14, 8, 79, 15)["targets_per_wave"] == 16
    assert tune.lookup_tuned_batch("square_sweep_2_14")["lanes_v"] == 2
    assert tune.lookup_tuned("square", 99, 1, 1) is None
    user = tmp_path / "user.json"
    user.write_text(json.dumps({"gfx950|square|14|640|15": {"best": {"fuse": 1, "mode": "graph"}}}))
    monkeypatch.setattr(tune, "DEFAULT_CACHE", str(user))
    assert tune.lookup_tuned("square", 14, 640, 15) == {"fuse": 1, "mode": "graph"}
    monkeypatch.setattr(tune, "_arch", lambda: "gfx942")
    monkeypatch.setattr(tune, "DEFAULT_CACHE", str(tmp_path / "none.json"))
    assert tune.lookup_tuned("square", 14, 640, 15) is None


def test_resident_candidates_fit_lds():
    # two state vectors of s_max + 1 rows per instance must fit 160 KiB:
    # square m = 13 never fits, triangular m = 12 fits up to 2 instances
    assert tune.resident_candidates("square", 13, 640, 14) == []
    tri = tune.resident_candidates("triangular", 12, 288, 13)
    assert tri and {c["lanes_v"] for c in tri} == {1, 2}
    assert all(c["mode"] == "resident" for c in tri)
    sq = tune.resident_candidates("square", 10, 320, 11)
    assert {c["lanes_v"] for c in sq} == {1, 2, 4} and {c["fuse"] for c in sq} == {1, 2, 3}
    # both arithmetic forms: exact double accumulation (0) and modular (1)
    assert {c["stage"] for c in sq} == {0, 1}


def test_written_residues_of_fused_steps():
    # a fused pair writes only the product's targets: the square 14x15 step
    # with pairs writes 14 rows x 385 911 targets x 640 instances
    assert bench.written_of("square", 14, 15, 640, 1) == bench.updates_of("square", 14, 15, 640)
    assert bench.written_of("square", 14, 15, 640, 2) == 14 * 385911 * 640


def test_lanes_v4_split_jobs():
    # lanes_v 4 runs chunks of 256 instances; the instances past the last
    # multiple of 256 form a second job at lanes_v 2 (1 for at most 64)
    assert bench.split_jobs(640, 4) == [(512, 4), (128, 2)]
    assert bench.split_jobs(300, 4) == [(256, 4), (44, 1)]
    assert bench.split_jobs(456, 4) == [(256, 4), (200, 2)]
    assert bench.split_jobs(768, 4) == [(768, 4)]
    assert bench.split_jobs(200, 4) == [(200, 4)]
    assert bench.split_jobs(640, 2) == [(640, 2)]
    assert bench.padded_instances(640, 4) == 640 and bench.padded_instances(200, 4) == 256
    assert bench.padded_instances(300, 4) == 320
    assert bench.kernel_name(640, 4, 4) == "k_gather<4,4>+k_gather<2,4>"
    assert bench.kernel_name(640, 2, 4) == "k_gather<2,4>"

