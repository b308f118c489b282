"""Host-side checks of the counter summaries (paper_1601_01237_amd.profiling):
the copy-calibrated traffic arithmetic, the derived counter ratios and the
comment-blind source hash, on small synthetic counter files."""

import csv
import json
import os

import pytest

from paper_1601_01237_amd import profiling

STEP = "void lbm::march_kernel<(lbm::Storage)0, false, (lbm::Mode)0, 128, 4, 3, 0>(lbm::Grid)"
FIELDS = "void lbm::march_kernel<(lbm::Storage)0, false, (lbm::Mode)2, 128, 4, 3, 0>(lbm::Grid)"
COPY = "lbm::(anonymous namespace)::stream_copy_kernel(unsigned int __vector(4) const*)"
REVERSE = "void lbm::(anonymous namespace)::adjoint_march_kernel<false, false, true, 32, 8, 2>(lbm::Grid)"


def _write(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(("Kernel_Name", "Counter_Name", "Counter_Value"), r)))


def test_traffic_is_scaled_by_the_reference_copy(tmp_path):
    gib = 1.0
    known = profiling.copy_bytes(gib)
    cells = 128 ** 3
    algo = 304 * cells
    # the counter reads half the copy's bytes (scale 2) on reads and all of
    # them on writes; the step reads 1.1x and writes 1.0x its algorithmic half
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    _write(fetch, [(COPY, "FETCH_SIZE", known / 2 / 1024), (COPY, "FETCH_SIZE", known / 2 / 1024),
                   (STEP, "FETCH_SIZE", 1.1 * algo / 2 / 2 / 1024)])
    _write(write, [(COPY, "WRITE_SIZE", known / 1024), (STEP, "WRITE_SIZE", algo / 2 / 1024)])
    js, out = tmp_path / "t.json", tmp_path / "t.txt"
    profiling.main(["traffic", "--fetch", str(fetch), "--write", str(write), "--workload", "128",
                    "--workload-key", "128^3", "--storage", "fp32", "--copy-gib", str(gib), "--json", str(js),
                    "--out", str(out), "--command", "x"])
    e = json.load(open(js))["128^3:fp32"]
    assert e["fetch_scale"] == pytest.approx(2.0) and e["write_scale"] == pytest.approx(1.0)
    assert e["read_bytes_per_launch"] == pytest.approx(1.1 * algo / 2, abs=1.0)
    assert e["write_bytes_per_launch"] == pytest.approx(algo / 2, abs=1.0)
    assert e["traffic_over_algorithmic"] == pytest.approx(1.05, abs=1e-4)
    assert e["kernel_hash"] == profiling.kernel_source_hash("step")
    assert e["copy_dispatches"] == 2 and e["step_dispatches"] == 1


def test_reverse_traffic_picks_the_reverse_march(tmp_path):
    known = profiling.copy_bytes(1.0)
    cells = 96 ** 3
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    # forward steps in the same run must not be counted
    _write(fetch, [(COPY, "FETCH_SIZE", known / 2 / 1024), (FIELDS, "FETCH_SIZE", 1e9),
                   (REVERSE, "FETCH_SIZE", 304 * cells / 2 / 1024)])
    _write(write, [(COPY, "WRITE_SIZE", known / 1024), (FIELDS, "WRITE_SIZE", 1e9),
                   (REVERSE, "WRITE_SIZE", 152 * cells / 1024)])
    js, out = tmp_path / "t.json", tmp_path / "t.txt"
    profiling.main(["traffic", "--fetch", str(fetch), "--write", str(write), "--workload", "adjoint96",
                    "--workload-key", "r", "--storage", "fp32", "--copy-gib", "1.0", "--json", str(js),
                    "--out", str(out)])
    e = json.load(open(js))["r:fp32"]
    assert e["algorithmic_bytes_per_launch"] == 456 * cells
    assert e["traffic_over_algorithmic"] == pytest.approx(1.0, abs=1e-6)
    assert e["kernel_hash"] == profiling.kernel_source_hash("reverse")


def test_derived_ratios():
    cyc = 1000.0
    m = {"GRBM_GUI_ACTIVE": 8 * cyc, "SQ_ACTIVE_INST_VALU": 0.5 * cyc * 1024 / 4,
         "TA_ADDR_STALLED_BY_TC_CYCLES_sum": 0.25 * cyc * 256, "TCP_TCC_READ_REQ_sum": 20.0 * cyc,
         "TCP_TCC_READ_REQ_LATENCY_sum": 20.0 * cyc * 900.0, "TCC_HIT_sum": 3.0, "TCC_MISS_sum": 1.0}
    d = "; ".join(profiling._derived(m))
    assert "VALU busy 50.0%" in d
    assert "TA address stalled by L1 25.0%" in d
    assert "mean L1->L2 read latency 900 cycles" in d
    assert "L1->L2 reads in flight 1.8e+04" in d
    assert "L2 hit rate 75.0%" in d


def test_kernel_classes():
    assert profiling._kernel_class(STEP) == "step"
    assert profiling._kernel_class(FIELDS) == "step+fields"
    assert profiling._kernel_class(COPY) == "lbm_stream_copy"
    assert profiling._kernel_class(REVERSE) == "reverse"
    assert profiling._kernel_class("void at::native::elementwise") is None


def test_source_hash_ignores_comments():
    a = "int f(int x) { // a comment\n  return x + 1; /* and\n another */ }\n"
    b = "int f(int x) {\n\n  return x + 1;   }"
    assert profiling._code_only(a) == profiling._code_only(b)
    assert profiling._code_only("a + b") != profiling._code_only("a - b")
    for kind in ("step", "reverse"):
        for name in profiling.KERNEL_SOURCES[kind]:
            assert os.path.exists(os.path.join(profiling.HERE, "csrc", name)), name
