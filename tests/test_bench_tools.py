"""Host-side tools of the benchmark (no GPU): the counter and kernel-time
summaries written from rocprofv3 CSV files, and the refusal of more than one
GPU."""

import csv
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

KA = "void sbbf::(anonymous namespace)::part_count_kernel(unsigned long const*, unsigned int)"
KB = "void sbbf::(anonymous namespace)::lookup_kernel<2, false, 0u, 8u>(unsigned long const*)"
KT = "void at::native::elementwise_kernel<128, 2>(int)"


def _counters_csv(path, rows):
    cols = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for d, k, c, v in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": k, "Grid_Size": 1024, "Counter_Name": c, "Counter_Value": v})


def test_counter_summary_means_and_derived_rates(tmp_path):
    a, b = tmp_path / "a.csv", tmp_path / "b.csv"
    # two dispatches of KA (means 30 hits / 10 misses), one of KB; a torch kernel that must be left out
    _counters_csv(a, [(1, KA, "TCC_HIT", 20), (1, KA, "TCC_MISS", 5), (2, KA, "TCC_HIT", 40), (2, KA, "TCC_MISS", 15),
                      (3, KB, "TCC_HIT", 1), (3, KB, "TCC_MISS", 3), (4, KT, "TCC_HIT", 99), (4, KT, "TCC_MISS", 1)])
    _counters_csv(b, [(1, KB, "TCC_EA0_RDREQ", 200), (1, KB, "TCC_EA0_RDREQ_32B", 50)])
    out = tmp_path / "s.md"
    assert bench.main(["--counter-summary", str(out), str(a), str(b), "--summary-title", "T",
                       "--summary-command", "cmd one", "--summary-command", "cmd two"]) == 0
    text = out.read_text()
    assert text.startswith("# T\n") and "cmd one\ncmd two" in text
    rows = {r.split("|")[1].strip(): [c.strip() for c in r.split("|")[2:-1]]
            for r in text.splitlines() if r.startswith("| `")}
    assert set(rows) == {"`part_count_kernel`", "`lookup_kernel<2, false, 0u, 8u>`"}
    ka = rows["`part_count_kernel`"]
    kb = rows["`lookup_kernel<2, false, 0u, 8u>`"]
    # columns: TCC_HIT, TCC_MISS, TCC_EA0_RDREQ, TCC_EA0_RDREQ_32B, L2 hit, 32B rd
    assert ka[:2] == ["30", "10"] and ka[2:4] == ["-", "-"] and ka[4] == "0.750" and ka[5] == "-"
    assert kb[:4] == ["1", "3", "200", "50"] and kb[4] == "0.250" and kb[5] == "0.250"


def test_kernel_summary_keeps_library_kernels(tmp_path):
    stats = tmp_path / "k.csv"
    with open(stats, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs"])
        w.writeheader()
        w.writerow({"Name": KA, "Calls": 3, "TotalDurationNs": 900000, "AverageNs": 300000, "MinNs": 250000,
                    "MaxNs": 350000})
        w.writerow({"Name": KT, "Calls": 1, "TotalDurationNs": 5, "AverageNs": 5, "MinNs": 5, "MaxNs": 5})
    out = tmp_path / "k.md"
    assert bench.main(["--kernel-summary", str(stats), str(out), "--summary-title", "K",
                       "--summary-command", "rocprofv3 ..."]) == 0
    lines = [r for r in out.read_text().splitlines() if r.startswith("| `")]
    assert lines == ["| `part_count_kernel` | 3 | 300.0 | 250.0 | 350.0 | 0.90 |"]


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err
