"""Host logic of bench.py that needs no GPU: the one-GPU guard, the
committed counter summary's validity rule, and the per-unit work figures
that the roofline multiplies."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_counter_summary_is_used_only_for_its_sources_and_size(tmp_path, monkeypatch):
    assert bench.measured_traffic(4095) is None            # another batch size
    summary = tmp_path / "traffic.txt"
    summary.write_text(f"# header\nscenarios = 10\nhbm_bytes_per_launch = 1.5e9\n"
                       f"source_sha256 = {bench.source_digest()}\n")
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(summary))
    assert bench.measured_traffic(10) == 1.5e9
    assert bench.measured_traffic(11) is None
    summary.write_text("scenarios = 10\nhbm_bytes_per_launch = 1.5e9\nsource_sha256 = 0123\n")
    assert bench.measured_traffic(10) is None              # older than the kernel sources
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic(10) is None


def test_source_digest_follows_the_kernel_sources():
    d = bench.source_digest()
    assert len(d) == 64 and d == bench.source_digest()


@pytest.mark.parametrize("dp", [2, 3])
def test_per_unit_work_figures(dp):
    """The pair-step's algorithmic bytes are the collapsed dual's read and
    write (4 + 4 bytes); the flop counts are positive and the 3-D pair step
    costs more than the 2-D one."""
    assert bench.BYTES_PER_UNIT[dp]["pair"] == 8.0
    assert all(v > 0 for v in bench.FLOPS_PER_UNIT[dp].values())
    assert bench.FLOPS_PER_UNIT[3]["pair"] > bench.FLOPS_PER_UNIT[2]["pair"]
