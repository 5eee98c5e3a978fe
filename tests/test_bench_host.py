"""Host logic of bench.py, on the CPU: the algorithmic work and bytes per vector the
roofline divides by, the rocprofv3 summariser (counter calibration and scaling,
the traffic record), the source-hash gate on that record, and the refusal of more
than one GPU."""

import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_counts_follow_the_operation_counts():
    """OCD: per coordinate update one B-long inner product and one B-long axpy of
    complex numbers, 4 real multiply-adds each per entry (8 flops), K U updates per
    vector; the norms, 2 multiply-adds per entry, shared by S symbols.  Bytes: H
    shared by S, y, Q FP32 LLRs and one complex z per user."""
    B, U, S, K, Q = 128, 8, 14, 3, 6
    flops, nbytes = bench.algorithmic(B, U, S, K, Q)
    assert flops == pytest.approx(K * U * (8 * B + 8 * B) + 4 * B * U / S)
    assert flops == pytest.approx(49444.571, abs=1e-3)
    assert nbytes == pytest.approx(8 * B * U / S + 8 * B + 4 * U * Q + 8 * U)
    assert nbytes == pytest.approx(1865.143, abs=1e-3)
    _, b16 = bench.algorithmic(B, U, S, K, Q, cbytes=4)
    assert nbytes - b16 == pytest.approx(4 * B * U / S + 4 * B)   # half the H and y bytes
    # explicit MMSE: Gram triangle and inverse per subcarrier, matched filter and
    # A^-1 s per vector, 8 flops per complex multiply-add
    fm, bm = bench.algorithmic_mmse(B, U, S, Q)
    assert fm == pytest.approx(8 * (U * (U + 1) // 2 * B + U ** 3) / S + 8 * (U * B + U * U))
    assert bm == pytest.approx(nbytes)


def _write_csv(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_summarize_profile_scales_counters_by_the_calibration_copy(tmp_path, capsys):
    """FETCH_SIZE of the 256 MiB copy reads 128 Mi KiB-units (scale 2), WRITE_SIZE
    256 Mi (scale 1); the detection kernel's counters are scaled by the same
    factors, and the traffic record holds their sum with the current source hash."""
    tr = tmp_path / "trace"
    tr.mkdir()
    _write_csv(tr / "x_kernel_stats.csv",
               ["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs"],
               [["void ocd::k_forward<16, 8, false, false, 8>(ocd::Params)", 3, 66000, 22000,
                 21000, 23000]])
    _write_csv(tr / "x_kernel_trace.csv",
               ["Kernel_Name", "Grid_Size_X", "Workgroup_Size_X", "Start_Timestamp",
                "End_Timestamp"],
               [["void ocd::k_forward<16, 8, false, false, 8>(ocd::Params)", 307200, 256, 0,
                 21000],
                ["void ocd::k_forward<16, 8, false, false, 8>(ocd::Params)", 307200, 256, 100000,
                 123000]])
    hdr = ["Kernel_Name", "Grid_Size", "Workgroup_Size", "Counter_Name", "Counter_Value"]
    fd, wd = tmp_path / "fetch", tmp_path / "write"
    fd.mkdir()
    wd.mkdir()
    kern = "void ocd::k_forward<16, 8, false, false, 8>(ocd::Params)"
    _write_csv(fd / "f_counter_collection.csv", hdr,
               [["__amd_rocclr_copyBuffer", 131072, 512, "FETCH_SIZE", 131072.0],
                [kern, 307200, 256, "FETCH_SIZE", 15000.0], [kern, 307200, 256, "FETCH_SIZE", 15100.0],
                [kern, 307200, 256, "FETCH_SIZE", 15200.0]])
    _write_csv(wd / "w_counter_collection.csv", hdr,
               [["__amd_rocclr_copyBuffer", 131072, 512, "WRITE_SIZE", 262144.0],
                [kern, 307200, 256, "WRITE_SIZE", 4200.0]])
    assert bench.summarize_profile([str(tr)], None, "") == 0
    out = capsys.readouterr().out
    assert "k_forward<16, 8, false, false, 8>" in out
    assert "22.000" in out and "21.000" in out            # avg (stats), mean of the trace
    rec_path = tmp_path / "traffic.json"
    plan_a = {"lanes_per_vector": 16, "vectors_per_block": 14, "xcd_remap": 1,
              "channel_in_registers": 0}
    plan_b = dict(plan_a, vectors_per_block=16)
    # a traffic record names the plan it was taken under
    assert bench.summarize_profile([str(fd), str(wd)], str(rec_path), "cmd") == 1
    capsys.readouterr()
    assert bench.summarize_profile([str(fd), str(wd)], str(rec_path), "cmd", plan_a) == 0
    out = capsys.readouterr().out
    assert "scale 2.0000" in out and "scale 1.0000" in out
    recs = json.loads(rec_path.read_text())["records"]
    assert len(recs) == 1
    rec = recs[0]
    assert rec["plan"] == [16, 14, 1, 0]
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["fetch_kib_per_launch"] == 15100.0          # the median dispatch
    assert rec["bytes_per_launch"] == pytest.approx(15100.0 * 1024 * 2 + 4200.0 * 1024)
    assert rec["source_hash"] == bench.source_hash() and rec["command"] == "cmd"
    # a second plan adds a record; the same plan again replaces its own
    assert bench.summarize_profile([str(fd), str(wd)], str(rec_path), "cmd2", plan_b) == 0
    assert bench.summarize_profile([str(fd), str(wd)], str(rec_path), "cmd3", plan_a) == 0
    recs = json.loads(rec_path.read_text())["records"]
    assert [r["plan"] for r in recs] == [[16, 14, 1, 0], [16, 16, 1, 0]]
    assert [r["command"] for r in recs] == ["cmd3", "cmd2"]


def test_summarize_profile_needs_both_counters(tmp_path):
    fd = tmp_path / "fetch"
    fd.mkdir()
    _write_csv(fd / "f_counter_collection.csv",
               ["Kernel_Name", "Grid_Size", "Workgroup_Size", "Counter_Name", "Counter_Value"],
               [["void ocd::k_forward<16, 8, false, false, 8>(ocd::Params)", 307200, 256,
                 "FETCH_SIZE", 15000.0]])
    assert bench.summarize_profile([str(fd)], str(tmp_path / "t.json"), "") == 1


def test_traffic_record_is_used_only_for_the_sources_and_plan_it_was_taken_on(tmp_path,
                                                                              monkeypatch):
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: "abc")
    path = tmp_path / "profiles" / "traffic_tag.json"
    p14 = {"lanes_per_vector": 16, "vectors_per_block": 14, "xcd_remap": 1,
           "channel_in_registers": 0, "stagger": 2}
    p16 = dict(p14, vectors_per_block=16)
    assert bench.read_traffic("tag", p14) is None            # no record
    rec = {"source_hash": "abc", "plan": [16, 14, 1, 0], "bytes_per_launch": 123.0}
    path.write_text(json.dumps({"records": [rec]}))
    assert bench.read_traffic("tag", p14) == 123.0
    assert bench.read_traffic("tag", dict(p14, stagger=0)) == 123.0   # stagger moves no bytes
    assert bench.read_traffic("tag", p16) is None            # another plan: other bytes
    path.write_text(json.dumps({"records": [rec, dict(rec, plan=[16, 16, 1, 0],
                                                      bytes_per_launch=456.0)]}))
    assert bench.read_traffic("tag", p16) == 456.0
    path.write_text(json.dumps({"records": [dict(rec, source_hash="old")]}))
    assert bench.read_traffic("tag", p14) is None            # other sources: not this kernel
    path.write_text("not json")
    assert bench.read_traffic("tag", p14) is None


def test_source_hash_covers_the_detection_kernel_sources():
    csrc = os.path.join(ROOT, "paper_1611_08779_amd", "csrc")
    for name in bench.FORWARD_SOURCES:
        assert os.path.exists(os.path.join(csrc, name)), name
    assert len(bench.source_hash()) == 16


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
