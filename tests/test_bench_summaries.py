"""The rocprofv3 summarizers behind the profiles' roofline and traffic figures, on small synthetic CSV files
with known answers: kernel-name shortening, the timed-launch average and per-pass rows of a kernel trace,
and the copy-calibrated HBM bytes of two counter runs."""
import csv
import json
import os
import re

import pytest

import bench


def _write_csv(path, fields, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def _json_line(text, tag):
    m = re.search(rf"^{tag}:\s*(\{{.*\}})\s*$", text, re.M)
    assert m, f"no {tag} line"
    return json.loads(m.group(1))


@pytest.mark.parametrize("raw, short", [
    ("void evosort::radix_pass_kernel<4, 0, 8, 768, 24, unsigned int>(evosort::RadixPassArgs, evosort::OrderMap<"
     "evosort::KeyWord<4>::U>)", "radix_pass_kernel<4, 0, 8, 768, 24, unsigned int>"),
    ("void evosort::(anonymous namespace)::merge_round_kernel<4, 0, 4096>(evosort::MergeRoundArgs)",
     "merge_round_kernel<4, 0, 4096>"),
    ("evosort::fill_zero_kernel(HIP_vector_type<unsigned int, 4u>*, unsigned long)", "fill_zero_kernel"),
])
def test_short_kernel_name(raw, short):
    assert bench.short_kernel_name(raw) == short


def test_trace_summary_averages_the_timed_launches_by_pass(tmp_path):
    name = "void evosort::radix_pass_kernel<4, 0, 8, 768, 24, unsigned int>(evosort::RadixPassArgs)"
    other = "evosort::fill_zero_kernel(HIP_vector_type<unsigned int, 4u>*, unsigned long)"
    # two warm-up launches (to be skipped), then two sorts of four passes: pass p lasts 1000 + 100 p us
    durations = [5000, 5000] + [1000 + 100 * p for _ in range(2) for p in range(4)]
    rows, t = [], 0
    for d in durations:
        rows.append({"Kernel_Name": name, "Start_Timestamp": t, "End_Timestamp": t + d * 1000})
        t += d * 1000 + 10_000
        rows.append({"Kernel_Name": other, "Start_Timestamp": t, "End_Timestamp": t + 2000})
        t += 12_000
    _write_csv(str(tmp_path / "trace" / "x_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
               rows)
    text = bench.summarize_trace(str(tmp_path / "trace"), "radix_pass_kernel<4, 0, 8, 768, 24", skip=2, passes=4,
                                 bytes_per_launch=8e9, command="cmd", title="t")
    rec = _json_line(text, "roofline_json")
    assert rec["timed_launches"] == 8
    assert rec["avg_us"] == pytest.approx(1150.0)  # mean of 1000, 1100, 1200, 1300
    assert rec["achieved_gbs"] == pytest.approx(8e9 / 1150e-6 / 1e9, abs=0.1)
    assert rec["frac"] == pytest.approx(8e9 / 1150e-6 / 1e9 / bench.HBM_PEAK_GBS, abs=1e-4)
    for p in range(4):
        assert re.search(rf"^\| {p} \| 2 \| {1000 + 100 * p:.1f} \|", text, re.M), f"pass {p} row"
    assert "| `fill_zero_kernel` | 10 |" in text


def test_trace_summary_refuses_an_ambiguous_kernel(tmp_path):
    rows = [{"Kernel_Name": f"void evosort::radix_pass_kernel<4, 0, 8, {t}, 24, unsigned int>(a)",
             "Start_Timestamp": 0, "End_Timestamp": 1000} for t in (512, 768)]
    _write_csv(str(tmp_path / "trace" / "x_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
               rows)
    with pytest.raises(SystemExit):
        bench.summarize_trace(str(tmp_path / "trace"), "radix_pass_kernel", 0, 4, 8e9, "cmd", "t")


def test_pmc_summary_scales_by_the_copy_calibration(tmp_path):
    calib = 1 << 30
    kib = 1024.0
    copy = "evosort::stream_copy_kernel(unsigned char*, unsigned char const*, unsigned long)"
    pas = "void evosort::radix_pass_kernel<4, 0, 8, 768, 24, unsigned int>(evosort::RadixPassArgs)"
    fields = ["Kernel_Name", "Dispatch_Id", "Counter_Name", "Counter_Value"]
    # the fetch counter reads half the bytes (64-byte units of 128-byte fetches), the write counter all of
    # them; a smaller copy dispatch must not be taken as the calibration
    fetch = [{"Kernel_Name": copy, "Dispatch_Id": 1, "Counter_Name": "FETCH_SIZE", "Counter_Value": calib / 2 / kib},
             {"Kernel_Name": copy, "Dispatch_Id": 2, "Counter_Name": "FETCH_SIZE", "Counter_Value": 1.0},
             {"Kernel_Name": pas, "Dispatch_Id": 3, "Counter_Name": "FETCH_SIZE", "Counter_Value": 2.0e6},
             {"Kernel_Name": pas, "Dispatch_Id": 4, "Counter_Name": "FETCH_SIZE", "Counter_Value": 2.2e6}]
    write = [{"Kernel_Name": copy, "Dispatch_Id": 1, "Counter_Name": "WRITE_SIZE", "Counter_Value": calib / kib},
             {"Kernel_Name": copy, "Dispatch_Id": 2, "Counter_Name": "WRITE_SIZE", "Counter_Value": 2.0},
             {"Kernel_Name": pas, "Dispatch_Id": 3, "Counter_Name": "WRITE_SIZE", "Counter_Value": 4.0e6},
             {"Kernel_Name": pas, "Dispatch_Id": 4, "Counter_Name": "WRITE_SIZE", "Counter_Value": 4.4e6}]
    _write_csv(str(tmp_path / "f" / "pmc_counter_collection.csv"), fields, fetch)
    _write_csv(str(tmp_path / "w" / "pmc_counter_collection.csv"), fields, write)
    text = bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"), "radix_pass_kernel<4, 0, 8, 768, 24",
                               8e9, calib, "int32", 10**9, ["cmd"], "t")
    rec = _json_line(text, "traffic_json")
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    # mean per dispatch: fetch 2.1e6 KiB x 2, write 4.2e6 KiB x 1
    assert rec["bytes_per_launch"] == round((2.1e6 * 2 + 4.2e6) * kib)
    assert rec["fetch_kib_raw"] == 2100000 and rec["write_kib_raw"] == 4200000
    assert rec["source_hash"] == bench.kernel_source_hash()
    assert f"({(2.1e6 * 2 + 4.2e6) * kib / 8e9:.3f}x)" in text


def test_counted_traffic_reads_only_a_current_matching_record(tmp_path, monkeypatch):
    rec = {"kernel": "k", "n": 10**9, "dtype": "int32", "bytes_per_launch": 8.6e9,
           "source_hash": bench.kernel_source_hash()}
    path = tmp_path / "pmc.md"
    path.write_text("# t\n\ntraffic_json: " + json.dumps(rec) + "\n")
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(path))
    assert bench.counted_traffic("int32", 10**9) == pytest.approx(8.6e9)
    assert bench.counted_traffic("int64", 10**9) is None  # another workload
    assert bench.counted_traffic("int32", 10**8) is None
    path.write_text("traffic_json: " + json.dumps(dict(rec, source_hash="0" * 16)) + "\n")
    assert bench.counted_traffic("int32", 10**9) is None  # counters taken on other kernel sources
