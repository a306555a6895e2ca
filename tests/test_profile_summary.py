"""The profile summary that bench.py writes from rocprofv3 output folders.

Synthetic CSV files in the rocprofv3 layout check the arithmetic: HBM bytes per
dispatch scaled by the copy calibration, the VALU issue utilisation, and that a
stored figure is used only while the kernel sources match the summary's digest.
"""

import csv
import os

import pytest

import bench


def write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


SEARCH = "void frnn::(anonymous namespace)::k_search<8, false>(float const*, unsigned int const*)"
COPY = "__amd_rocclr_copyBuffer"


@pytest.fixture
def dirs(tmp_path):
    d = {k: str(tmp_path / k) for k in ("trace", "fetch", "write", "cfetch", "cwrite", "sq")}
    write_csv(os.path.join(d["trace"], "run_kernel_stats.csv"), ["Name", "Calls", "AverageNs", "MinNs", "MaxNs"],
              [[SEARCH, 10, 50000, 40000, 60000], [COPY, 5, 1000, 900, 1100]])

    def counters(folder, rows):
        write_csv(os.path.join(d[folder], "run_counter_collection.csv"),
                  ["Kernel_Name", "Counter_Name", "Counter_Value"], rows)

    # Two dispatches of the search: averages 1000 and 3000 KiB.
    counters("fetch", [[SEARCH, "FETCH_SIZE", 900], [SEARCH, "FETCH_SIZE", 1100]])
    counters("write", [[SEARCH, "WRITE_SIZE", 3000], [SEARCH, "WRITE_SIZE", 3000]])
    # The 256 MiB copy reads as half its size and writes as its size.
    counters("cfetch", [[COPY, "FETCH_SIZE", 128 * 1024]])
    counters("cwrite", [[COPY, "WRITE_SIZE", 256 * 1024]])
    valu = 0.25 * 50e-6 * 2.4e9 * 1024 / 4  # a quarter of the SIMD cycles
    counters("sq", [[SEARCH, "SQ_WAVES", 8192], [SEARCH, "SQ_INSTS_VALU", valu], [SEARCH, "SQ_INSTS_SALU", 7],
                    [SEARCH, "SQ_INSTS_LDS", 3], [SEARCH, "SQ_INSTS_SMEM", 2]])
    return d


def test_bytes_are_scaled_by_the_copy_calibration(dirs):
    text = bench.summarize(dirs["trace"], dirs["fetch"], dirs["write"], dirs["cfetch"], dirs["cwrite"],
                           commands=["c"] * 5)
    assert "scale factors fetch x2.000, write x1.000" in text
    # (1000 KiB x 2 + 3000 KiB x 1) x 1024 bytes
    assert "traffic k_search<8, false> bytes per launch: 5120000" in text
    assert "| k_search<8, false> | 10 | 50.00 | 40.00 | 60.00 |" in text
    assert "VALU issue" not in text


def test_valu_issue_utilisation(dirs):
    text = bench.summarize(dirs["trace"], dirs["fetch"], dirs["write"], dirs["cfetch"], dirs["cwrite"],
                           commands=["c"] * 6, sq_dir=dirs["sq"])
    assert "valu k_search<8, false> issue utilisation: 0.2500" in text


def test_stored_figures_follow_the_source_digest(dirs, tmp_path, monkeypatch):
    text = bench.summarize(dirs["trace"], dirs["fetch"], dirs["write"], dirs["cfetch"], dirs["cwrite"],
                           commands=["c"] * 6, sq_dir=dirs["sq"])
    path = tmp_path / "summary.md"
    path.write_text(text)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.stored_traffic("k_search<8, false>") == 5120000
    assert bench.stored_valu("k_search<8, false>") == pytest.approx(0.25)
    path.write_text(text.replace(bench.kernel_source_digest(), "0000000000000000"))
    assert bench.stored_traffic("k_search<8, false>") is None
    assert bench.stored_valu("k_search<8, false>") is None


def test_trace_only_summary(dirs):
    text = bench.summarize_trace("a workload", dirs["trace"], "the command")
    assert text.startswith("# rocprofv3 summary: a workload")
    assert f"kernel sources sha256/16: {bench.kernel_source_digest()}" in text
    assert "command: `the command`" in text
    assert "| k_search<8, false> | 10 | 50.00 | 40.00 | 60.00 |" in text
    assert "copyBuffer" not in text  # only the library's kernels are listed
