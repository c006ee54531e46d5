"""bench.py's reading of committed rocprofv3 summaries: a figure is used only
while the kernel source it was measured on is unchanged."""
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def write(path, text):
    with open(path, "w") as f:
        f.write(text)


def test_summary_values_follow_the_source(tmp_path):
    src = tmp_path / "kernel.hip"
    write(src, "__global__ void k() {}\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    summary = tmp_path / "summary.md"
    write(summary, f"# k\n\n- traffic_bytes_per_launch: 1.5e+11\n- kernel_source_sha256: `{sha}`\n"
                   "- SQ_INSTS_VALU: 6.144e+11\n")
    assert bench.measured_traffic(str(summary), str(src)) == 1.5e11
    vals = bench.summary_values(str(summary), str(src))
    assert float(vals["SQ_INSTS_VALU"]) == 6.144e11
    write(src, "__global__ void k() { }\n")  # the kernel changed: no figure
    assert bench.measured_traffic(str(summary), str(src)) is None
    assert bench.summary_values(str(summary), str(src)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.md"), str(src)) is None


def test_source_digest_of_several_files(tmp_path):
    a, b = tmp_path / "a", tmp_path / "b"
    write(a, "x")
    write(b, "y")
    assert bench.source_digest([str(a), str(b)]) == hashlib.sha256(b"xy").hexdigest()
    assert bench.source_digest(str(a)) == hashlib.sha256(b"x").hexdigest()


def test_valu_issue_rate(tmp_path, monkeypatch):
    # 256 CUs x 2.4e9 cycles of one wave instruction each, over a 1 s kernel:
    # one per CU per cycle; against a ceiling of twice the derived rate, half
    src = tmp_path / "exact.hip"
    write(src, "kernel source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    summary = tmp_path / "counters.md"
    write(summary, f"- kernel_source_sha256: `{sha}`\n- SQ_INSTS_VALU: 6.144e+11\n")
    monkeypatch.setattr(bench, "COUNTERS_SUMMARY", str(summary))
    monkeypatch.setattr(bench, "PAIR_KERNEL_SRC", str(src))
    out = bench.valu_issue(1000.0, 2 * bench.VALU_PEAK_DERIVED)
    assert abs(out["per_cu_per_cycle"] - 1.0) < 1e-12 and abs(out["calibrated_per_cu_per_cycle"] - 2.0) < 1e-12
    assert abs(out["frac"] - 0.5) < 1e-12
    write(summary, f"- kernel_source_sha256: `{sha}`\n- SQ_INSTS_VALU: 3.072e+11\n")
    assert abs(bench.valu_issue(2000.0, bench.VALU_PEAK_DERIVED)["per_cu_per_cycle"] - 0.25) < 1e-12
    write(src, "changed\n")
    assert bench.valu_issue(1000.0, bench.VALU_PEAK_DERIVED) is None


def test_derived_valu_peak():
    # 256 CUs x 64 lanes x 2.4 GHz
    assert abs(bench.VALU_PEAK_DERIVED - 39.3216e12) < 1e6


def test_cpu_baseline_sample_is_stratified(monkeypatch):
    # a small graph, a short budget: every octave with centres is represented
    # in proportion, and the record names the host
    from workloads import make_config
    monkeypatch.setenv("OMP_NUM_THREADS", "2")
    h = make_config("medium", scale=0.02)
    out = bench.cpu_baseline(h, 0.5)
    assert out["kind"] == "oracle" and out["cores"] <= 2 and out["value"] > 0
    assert out["cpu_model"] and out["nproc"] >= 1
    assert out["tiny_one_thread"]["threads"] == 1 and out["tiny_one_thread"]["connected_triples"] > 0
    shares = [r["workload_share"] for r in out["octaves"]]
    assert abs(sum(shares) - 1.0) < 1e-9
    assert sum(r["centres"] for r in out["octaves"]) > 0
