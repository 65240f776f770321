"""Host-side checks of bench.py: the one-GPU guard and the reading of the
committed counter summary (traffic is reported only for the kernel sources the
counters were taken on)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_summary_is_tied_to_kernel_sources(tmp_path, monkeypatch):
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    src = tmp_path / "paper_2302_08341_amd" / "csrc"
    src.mkdir(parents=True)
    for p in bench.KERNEL_SOURCES:
        (tmp_path / p).write_text("kernel source " + p)
    (tmp_path / "profiles").mkdir()
    f = tmp_path / "profiles" / "k_marchv_urban8x8x2_traffic.md"
    f.write_text("# summary\n- kernel_sources_sha256: `%s`\n- traffic_bytes_per_launch: 1234.5\n"
                 "- algorithmic_bytes_per_launch: 1000\n" % bench.kernel_source_hash())
    assert bench.measured_traffic("k_marchv", "urban8x8x2") == pytest.approx(1234.5)
    # only for the launches the counters were taken on (same algorithmic bytes per launch)
    assert bench.measured_traffic("k_marchv", "urban8x8x2", 1003.0) == pytest.approx(1234.5)
    assert bench.measured_traffic("k_marchv", "urban8x8x2", 1100.0) is None
    assert bench.measured_traffic("k_marchv", "urban8x8x4") is None
    # comments and layout are not the kernel
    (tmp_path / bench.KERNEL_SOURCES[0]).write_text("// a note\nkernel  /* more */ source\n  "
                                                    + bench.KERNEL_SOURCES[0] + "  // end\n")
    assert bench.measured_traffic("k_marchv", "urban8x8x2") == pytest.approx(1234.5)
    (tmp_path / bench.KERNEL_SOURCES[0]).write_text("changed kernel")
    assert bench.measured_traffic("k_marchv", "urban8x8x2") is None
