"""Host tests of the benchmark's measurement tools (no GPU): the busy time per
solve from a kernel trace, the HBM counter calibration and the kernel source
hash that keeps recorded traffic tied to the kernel it was measured on."""
import csv
import json
import os
import shutil

import pytest

import bench


def _trace(path, spans, name="void pbn::k_step_bs<false>(pbn::StepItem const*)"):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for a, b in spans:
            w.writerow({"Kernel_Name": name, "Start_Timestamp": a, "End_Timestamp": b})
        # another kernel in between counts for nothing
        w.writerow({"Kernel_Name": "pbn::k_reduce(pbn::Query const*)", "Start_Timestamp": 0, "End_Timestamp": 10 ** 9})


def test_trace_union_splits_solves_at_the_widest_gaps(tmp_path):
    ms = 1_000_000
    spans = []
    # warm-up solve: 0..20 ms busy with two overlapping dispatches
    spans += [(0, 15 * ms), (5 * ms, 20 * ms)]
    # three timed solves of 10 ms busy each, separated by 3 ms host gaps; inside
    # each a 1 ms gap (narrower) and three dispatches, two overlapping
    for k in range(3):
        t = 23 * ms + k * 14 * ms
        spans += [(t, t + 4 * ms), (t + 2 * ms, t + 5 * ms), (t + 6 * ms, t + 11 * ms)]
    trace = tmp_path / "run_kernel_trace.csv"
    _trace(trace, spans)
    out = tmp_path / "union.json"
    assert bench.trace_union(str(trace), "k_step_bs", 4, str(out)) == 0
    info = json.load(open(out))
    assert info["dispatches"] == len(spans)
    per = info["per_solve"]
    assert len(per) == 4
    assert per[0]["union_ms"] == pytest.approx(20.0)
    for p in per[1:]:
        assert p["union_ms"] == pytest.approx(10.0)
        assert p["first_to_last_ms"] == pytest.approx(11.0)
        assert p["summed_dispatch_ms"] == pytest.approx(12.0)
    assert info["timed_union_ms_per_solve"] == pytest.approx(10.0)
    assert info["timed_mean_in_flight"] == pytest.approx(1.2)


def _counters(dirpath, rows):
    os.makedirs(dirpath, exist_ok=True)
    with open(os.path.join(dirpath, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, counter, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_scale_from_the_copy_dispatches_only(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "kernel_sha", lambda: "fixed")
    step = "void pbn::k_step_bs<false>(pbn::StepItem const*)"
    fill = "void at::native::vectorized_elementwise_kernel<...>"
    copy = "__amd_rocclr_copyBuffer"
    gib_kib = 1024 * 1024
    _counters(tmp_path / "f", [(step, "FETCH_SIZE", 1000.0), (step, "FETCH_SIZE", 3000.0)])
    _counters(tmp_path / "w", [(step, "WRITE_SIZE", 500.0), (step, "WRITE_SIZE", 1500.0)])
    # the fill that makes the probe's source fetches nothing and must not count
    _counters(tmp_path / "cf", [(fill, "FETCH_SIZE", 21.0)] + [(copy, "FETCH_SIZE", gib_kib / 2)] * 4)
    _counters(tmp_path / "cw", [(fill, "WRITE_SIZE", float(gib_kib))] + [(copy, "WRITE_SIZE", float(gib_kib))] * 4)
    out = tmp_path / "traffic.json"
    assert bench.traffic_from(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                              str(tmp_path / "cw"), str(out)) == 0
    info = json.load(open(out))
    assert info["fetch_scale"] == pytest.approx(2.0)
    assert info["write_scale"] == pytest.approx(1.0)
    assert info["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 1024 * 2.0)
    assert info["write_bytes_per_launch"] == pytest.approx(1000.0 * 1024)
    assert info["dispatches"] == 2


def test_kernel_hash_ignores_comments_only(tmp_path, monkeypatch):
    src = os.path.join(bench.ROOT, "paper_1508_07828_amd", "csrc")
    dst = tmp_path / "paper_1508_07828_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in ("pbn_step_bs.hip", "pbn_device.h", "pbn_internal.h"):
        shutil.copy(os.path.join(src, f), dst / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base = bench.kernel_sha()
    k = dst / "pbn_step_bs.hip"
    text = k.read_text()
    k.write_text("// a note\n/* a block\n   comment */\n" + text.replace("\n", "\n  ", 3))
    assert bench.kernel_sha() == base
    code = "(y & 0x7F7F7F7Fu) + 0x7F7F7F7Fu"
    assert code in text
    k.write_text(text.replace(code, "(y & 0x7F7F7F7Fu) + 0x7F7F7F7Eu", 1))
    assert bench.kernel_sha() != base
