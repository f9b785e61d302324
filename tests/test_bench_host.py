"""Host-side logic of bench.py: the profile summaries and the traffic figure
they feed back, on synthetic rocprofv3 CSV files (no GPU)."""
import os

import pytest

import bench


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        f.write(",".join(header) + "\n")
        for r in rows:
            f.write(",".join(str(v) for v in r) + "\n")


def test_summarize_trace(tmp_path):
    d = tmp_path / "prof"
    _write(str(d / "host" / "run_kernel_stats.csv"), ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage",
                                                      "MinNs", "MaxNs"],
           [['"void hp::k_reduce_lds<1024, 2, false>(int const*, long)"', 10, 165000, 16500, 40.0, 14000, 21000],
            ['"void at::native::elementwise_kernel<128>(int)"', 3, 3000, 1000, 1.0, 900, 1100]])
    _write(str(d / "host" / "run_kernel_trace.csv"), ["Kernel_Name", "Grid_Size_X", "Workgroup_Size_X", "VGPR_Count",
                                                      "LDS_Block_Size"],
           [['"void hp::k_reduce_lds<1024, 2, false>(int const*, long)"', 262144, 1024, 20, 0]])
    text = bench.summarize_trace(str(d), "rocprofv3 ... -- python bench.py", "a title")
    assert text.startswith("# a title")
    assert "hp::k_reduce_lds<1024, 2, false>" in text and "16.50" in text and "elementwise" not in text
    assert "grid=262144 wg=1024 vgpr=20 lds=0" in text


def test_summarize_counters_and_traffic(tmp_path, monkeypatch):
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    for counter, copy_kib, red_kib in (("FETCH_SIZE", 39062.5, 40000.0), ("WRITE_SIZE", 78125.0, 4000.0)):
        rows = [['"bitwise_not_kernel"', counter, copy_kib]] * 5 + [['"hp::k_reduce_lds<1024, 2, false>"', counter,
                                                                    red_kib]] * 7
        rows.append(['"hp::k_reduce_lds<1024, 2, false>"', counter, 0.0])   # a dispatch read as 0
        _write(str(tmp_path / counter / "host" / "run_counter_collection.csv"), hdr, rows)
    text = bench.summarize_counters(str(tmp_path / "FETCH_SIZE"), str(tmp_path / "WRITE_SIZE"), 80e6,
                                    "rocprofv3 --pmc COUNTER -- python bench.py", "some_workload", 8)
    # FETCH scale 80e6 / (39062.5 KiB) = 2.0, WRITE scale 1.0
    assert "scale 2.0000" in text and "scale 1.0000" in text
    want = 40000.0 * 1024 * 2.0 + 4000.0 * 1024 * 1.0
    assert f"hbm_bytes_per_launch: {want:.0f}" in text
    assert "--pmc FETCH_SIZE" in text and "--pmc WRITE_SIZE" in text
    # the figure is read back only while the reduce sources are unchanged
    prof = tmp_path / "repo" / "profiles"
    prof.mkdir(parents=True)
    (prof / "reduce_w_counters.txt").write_text(text)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path / "repo"))
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: text.split("kernel_source_sha: ")[1].split()[0])
    assert bench.committed_traffic("w") == pytest.approx(want)
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0000")
    assert bench.committed_traffic("w") is None


def test_summarize_counters_sums_a_multi_kernel_reduce(tmp_path):
    """The binned reduce runs k_bin and k_bin_fold twice per run (rounds of
    different sizes) and k_bin_merge once: each place in the run counts with
    its own median, and the run's figure is their sum."""
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    runs = 3
    for counter in ("FETCH_SIZE", "WRITE_SIZE"):
        rows, d = [], 0
        for i in range(5):
            d += 1
            rows.append([d, '"bitwise_not_kernel"', counter, 1000.0])
        for r in range(runs):
            for name, kib in (("k_bin", 100.0), ("k_bin_fold", 10.0), ("k_bin_merge", 1.0), ("k_bin", 300.0),
                              ("k_bin_fold", 30.0), ("k_finish", 5000.0)):
                d += 1
                rows.append([d, f'"void hp::{name}(int)"', counter, kib + (r if name == "k_bin" else 0)])
        rows.reverse()       # file order need not be dispatch order
        _write(str(tmp_path / counter / "host" / "run_counter_collection.csv"), hdr, rows)
    text = bench.summarize_counters(str(tmp_path / "FETCH_SIZE"), str(tmp_path / "WRITE_SIZE"), 1000 * 1024.0,
                                    "cmd COUNTER", "w", runs)
    per_run_kib = (100 + 1) + (300 + 1) + 10 + 30 + 1      # medians over the runs; k_finish is not the reduce
    assert f"hbm_bytes_per_launch: {2 * per_run_kib * 1024:.0f}" in text
    assert "hp::k_bin " in text and "k_finish" not in text


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err
