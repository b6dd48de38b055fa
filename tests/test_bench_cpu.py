"""Host-side checks of bench.py's contract (no GPU): it refuses more than one GPU, prices against
the published MI355X peaks, and takes a kernel's HBM traffic from the counter summary only while
that kernel's source is the one the counters were taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402  (module level holds constants and helpers only; no torch import)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_published_peaks():
    assert bench.HBM_PEAK_GBS == 8000.0
    assert bench.BF16_PEAK_TFLOPS == 2500.0
    assert bench.FP32_PEAK_TFLOPS == 157.3
    assert bench.FP64_PEAK_TFLOPS == 78.6


def _summary_with(entries):
    return "# counters\n\n```json\n" + json.dumps(entries) + "\n```\n"


def test_traffic_figure_needs_matching_source_and_problem_count(tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_text("// kernel source\n")
    import hashlib
    sha = hashlib.sha1(src.read_bytes()).hexdigest()
    summary = tmp_path / "traffic.md"
    entry = {"source": str(src), "sha1": sha, "problems_per_launch": 2, "read_bytes": 1000, "write_bytes": 24}
    summary.write_text(_summary_with({"k_x": entry}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(summary))
    # os.path.join keeps an absolute source path as it is
    assert bench.measured_traffic("k_x", 2.0) == 1024.0
    assert bench.measured_traffic("k_x", 1.0) is None          # another grouping
    assert bench.measured_traffic("k_y", 2.0) is None          # no entry
    src.write_text("// kernel source, edited since the counters were taken\n")
    assert bench.measured_traffic("k_x", 2.0) is None


def test_traffic_figure_needs_matching_launch_files(tmp_path, monkeypatch):
    # the pass's figures also depend on the split-K table that shapes its launch
    import hashlib
    src = tmp_path / "kernel.hip"
    src.write_text("// kernel source\n")
    table = tmp_path / "table.inc"
    table.write_text("{2, 14, 224, 4},\n")
    entry = {"source": str(src), "sha1": hashlib.sha1(src.read_bytes()).hexdigest(),
             "also": [[str(table), hashlib.sha1(table.read_bytes()).hexdigest()]],
             "problems_per_launch": 2, "read_bytes": 1000, "write_bytes": 24}
    summary = tmp_path / "traffic.md"
    summary.write_text(_summary_with({"k_x": entry}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(summary))
    assert bench.measured_traffic("k_x", 2.0) == 1024.0
    table.write_text("{2, 14, 224, 8},\n")
    assert bench.measured_traffic("k_x", 2.0) is None


def test_committed_summary_parses():
    # every committed entry either applies to the current source or is skipped, never an error
    for kernel, ppl in (("k_pass", 2.0), ("k_gemv", 1.0), ("k_rebuild", 2.0)):
        v = bench.measured_traffic(kernel, ppl)
        assert v is None or v > 0


def test_parity_tolerances():
    # the split-BF16 form is held to the FP32 bar: the same stated accuracy
    assert bench.PARITY_TOL == {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-5}
