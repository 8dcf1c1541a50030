"""bench.py's profile summary on synthetic rocprofv3 CSVs (CPU only): the
time-frame dispatches are those up to the last k_output of the replays
(kernels only the per-event path runs count as "other"), and counter bytes
are scaled by the calibration copy that precedes every tracker kernel."""
import csv
import json
import os

import pytest

import bench

TRACE_HDR = ["Kind", "Agent_Id", "Queue_Id", "Stream_Id", "Thread_Id", "Dispatch_Id", "Kernel_Id",
             "Kernel_Name", "Correlation_Id", "Start_Timestamp", "End_Timestamp"]
PMC_HDR = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
           "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
           "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]

COPY = "__amd_rocclr_copyBuffer(void*)"
TF_SEQ = ["void tpcca::k_count(tpcca::Bufs, int, int)", "void tpcca::k_rowsort<1024, true>(tpcca::Bufs, int, int)",
          "void tpcca::k_kf<5>(tpcca::Bufs, tpcca::ParamsDev, int)", "void tpcca::k_output(tpcca::Bufs, int)"]
EV_SEQ = ["void tpcca::k_count(tpcca::Bufs, int, int)", "void tpcca::k_rowsort<256, false>(tpcca::Bufs, int, int)",
          "void tpcca::k_kf<5>(tpcca::Bufs, tpcca::ParamsDev, int)", "void tpcca::k_output(tpcca::Bufs, int)"]


def _dispatches():
    """(name, duration ns, FETCH KiB, WRITE KiB): a copy, 4 time-frame
    replays, then 3 per-event runs."""
    out = [(COPY, 1000, 512 * 1024, 1024 * 1024)]  # 1 GiB copy reads as 0.5 GiB of FETCH
    for _ in range(4):
        for k, n in enumerate(TF_SEQ):
            out.append((n, 10_000 * (k + 1), 100.0 * (k + 1), 10.0))
    for _ in range(3):
        for n in EV_SEQ:
            out.append((n, 500, 1.0, 1.0))
    return out


def _write(tmp, sub, rows, hdr):
    d = tmp / sub
    d.mkdir(parents=True)
    with open(d / f"{sub}_x.csv".replace("_x", "_kernel_trace" if hdr is TRACE_HDR else "_counter_collection"),
              "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(hdr)
        w.writerows(rows)
    return str(d)


@pytest.fixture()
def summary(tmp_path, monkeypatch):
    ds = _dispatches()
    trace = [["KERNEL_DISPATCH", "Agent 1", 1, 0, 1, i + 1, 0, n, i + 1, 1000 * i, 1000 * i + dur]
             for i, (n, dur, _, _) in enumerate(ds)]
    fetch = [[i + 1, i + 1, "Agent 1", 1, 1, 1, 1, 0, n, 256, 0, 0, 0, 0, 0, "FETCH_SIZE", fv, 0, 1]
             for i, (n, _, fv, _) in enumerate(ds)]
    write = [[i + 1, i + 1, "Agent 1", 1, 1, 1, 1, 0, n, 256, 0, 0, 0, 0, 0, "WRITE_SIZE", wv, 0, 1]
             for i, (n, _, _, wv) in enumerate(ds)]
    td = _write(tmp_path, "trace", trace, TRACE_HDR)
    fd = _write(tmp_path, "fetch", fetch, PMC_HDR)
    wd = _write(tmp_path, "write", write, PMC_HDR)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0123456789abcdef")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "profiles" / "traffic.json"))
    bench.summarize_profile(td, fd, wd, "the command")
    md = open(tmp_path / "profiles" / "tracker_timeframe128_kernel_trace.md").read()
    traffic = json.load(open(tmp_path / "profiles" / "traffic.json"))
    return md, traffic


def test_time_frame_dispatches_end_at_the_last_k_output_of_the_replays(summary):
    md, _ = summary
    durations = md.split("## Durations")[1].split("\n## ")[0]
    rows = {line.split("|")[1].strip(): [c.strip() for c in line.split("|")[2:-1]]
            for line in durations.splitlines() if line.startswith("| k_")}
    assert rows["k_kf<5>"][0] == "4" and rows["k_kf<5>"][3] == "3"        # 4 TF, 3 other
    assert float(rows["k_kf<5>"][1]) == pytest.approx(30.0)               # 30 us each
    assert rows["k_rowsort<1024, true>"][:1] == ["4"] and rows["k_rowsort<1024, true>"][3] == "0"
    assert "k_rowsort<256, false>" not in rows                            # per-event only: no TF row


def test_counter_bytes_are_scaled_by_the_copy(summary):
    _, traffic = summary
    assert traffic["factor"]["FETCH_SIZE"] == pytest.approx(2.0)
    assert traffic["factor"]["WRITE_SIZE"] == pytest.approx(1.0)
    kf = traffic["kernels"]["k_kf<5>"]
    assert kf["fetch_size"] == pytest.approx(300.0 * 1024 * 2.0)          # 300 KiB x scale
    assert kf["write_size"] == pytest.approx(10.0 * 1024)
    assert traffic["kernels"]["k_kf"] is not None                          # plain-name alias
    assert "k_rowsort<256, false>" not in traffic["kernels"]
