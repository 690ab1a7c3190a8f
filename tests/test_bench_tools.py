"""bench.py's profile tooling on synthetic rocprofv3 output (CPU only): the PMC
summary attributes dispatches to the variant groups the marker dispatches
open, picks each stage's own kernel, calibrates on the copy group and keys the
traffic line to the mvm.hip digest; the kernel-statistics table sorts by total
time."""
import csv
import json
import os

import pytest

import bench


def _write_counters(folder, counter, groups):
    os.makedirs(folder, exist_ok=True)
    with open(os.path.join(folder, "p_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Correlation_Id", "Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"])
        did = 1
        # a large Rademacher launch before the first marker is not a marker
        w.writerow([did, did, 1020160, "void dski::k_rademacher<float>(unsigned long)", counter, 18.0])
        did += 1
        for kernels in groups:
            w.writerow([did, did, 256, "void dski::k_rademacher<float>(unsigned long, int)", counter, 1.0])
            did += 1
            for name, value in kernels:
                w.writerow([did, did, 5000, name, counter, value])
                did += 1


def test_pmc_summary_attributes_groups_and_calibrates(tmp_path):
    labels = ["scatter_v0", "kuu_fft", "pivchol", "pcg", "copy"]
    scat = "void dski::k_scatter_lds<2, 4, 6, float, double>(int const*)"
    fft = "void dski::k_toeplitz<9, double>(double*)"
    arg = "void dski::k_argmax_partial(double const*)"
    upd = "void dski::k_pcg_update<float, 20>(float const*)"
    cp = "__amd_rocclr_copyBuffer"
    fetch = [[(scat, 1000.0)] * 3, [(fft, 2000.0)] * 6 + [(arg, 7.0)] * 9, [(arg, 7.0)] * 50,
             [(upd, 300.0)] * 2, [(cp, 131072.0)] * 3]
    write = [[(scat, 500.0)] * 3, [(fft, 600.0)] * 6 + [(arg, 1.0)] * 9, [(arg, 1.0)] * 50,
             [(upd, 30.0)] * 2, [(cp, 262144.0)] * 3]
    _write_counters(str(tmp_path / "f"), "FETCH_SIZE", fetch)
    _write_counters(str(tmp_path / "w"), "WRITE_SIZE", write)
    log = tmp_path / "log"
    log.write_text("noise\n" + json.dumps({"pmc_mvm": "done", "copy_bytes": 256 << 20, "source": "abc123",
                                           "labels": labels}) + "\n")
    out = tmp_path / "out.md"
    t = bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"), str(log), out_path=str(out),
                          commands=["cmd"])
    # FETCH_SIZE of the copy reads half its bytes: factor 2; WRITE_SIZE all: factor 1
    assert t["scatter_v0"] == pytest.approx(1000 * 1024 * 2 + 500 * 1024)
    # the FFT group's own kernel, not the more frequent pivoted-Cholesky kernel
    assert t["kuu_fft"] == pytest.approx(2000 * 1024 * 2 + 600 * 1024)
    assert set(t) == {"scatter_v0", "kuu_fft"}
    text = out.read_text()
    assert "traffic-bytes-per-launch: scatter_v0=" in text and text.rstrip().endswith("source=abc123")
    assert "`dski::k_toeplitz<9, double>`" in text and "cmd" in text


def test_pmc_summary_rejects_marker_count_mismatch(tmp_path):
    _write_counters(str(tmp_path / "f"), "FETCH_SIZE", [[("k", 1.0)]])
    _write_counters(str(tmp_path / "w"), "WRITE_SIZE", [[("k", 1.0)]])
    log = tmp_path / "log"
    log.write_text(json.dumps({"pmc_mvm": "done", "copy_bytes": 1, "source": "x", "labels": ["a", "copy"]}) + "\n")
    with pytest.raises(ValueError):
        bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"), str(log), out_path=str(tmp_path / "o.md"))


def test_stats_table_sorted_by_total(tmp_path):
    p = tmp_path / "run_kernel_stats.csv"
    with open(p, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        w.writerow(["void dski::small(int)", 10, 1000, 100, 10.0, 90, 110, 1])
        w.writerow(["void dski::big<3>(double*)", 4, 9000, 2250, 90.0, 2000, 2500, 10])
    rows = bench.stats_table(str(p)).splitlines()
    assert rows[2].startswith("| `dski::big<3>` | 4 | 0.0 | 2.25 | 90.0 |")
    assert rows[3].startswith("| `dski::small` | 10 |")


def test_fastest_variant_skips_untimed():
    # -1 marks a variant the tuner did not time (the grouped 3-D scatter on a 2-D plan)
    assert bench._fastest([13.3, 144.9, 100.4, 13.2, 14.4, 29.3, -1.0]) == 3
    assert bench._fastest([-1.0, 5.0, 4.0]) == 2
    tune = {"scatter_us": [2.0, -1.0, 1.5], "gather_us": [1.0, 0.5, 0.7], "kuu_us": [[8.8, 24.9], [7.2, -1.0]]}
    v = bench.tuned_variants(tune)
    assert v["scatter"] == 2 and v["gather"] == 1 and v["kuu"] == [0, 0]
