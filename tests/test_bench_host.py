"""Host-side tests of bench.py's plumbing (no GPU is touched).

* More than one GPU is refused with a message before anything is imported
  or allocated.
* The roofline's `traffic` is read from the committed counter summary only
  for the configuration it was taken on and the current kernel source.
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2505_06022_amd.profile_run import kernel_source_hash  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and f"--gpus {n}" in r.stderr
    assert r.stdout == ""


def _summary(path, depth, rows, kernel_hash, nbytes):
    doc = {"kernel": "wave2d_kernel", "depth": depth, "tile_rows": rows,
           "kernel_hash": kernel_hash, "bytes_per_launch": nbytes}
    with open(path, "a") as f:
        f.write("# a section\n\ntraffic-json: " + json.dumps(doc) + "\n\n")


def test_traffic_taken_on_this_config_and_source(tmp_path):
    p = str(tmp_path / "traffic.md")
    _summary(p, 8, 32, "0" * 16, 111)             # another kernel source
    _summary(p, 8, 64, kernel_source_hash(), 222)  # another tile height
    _summary(p, 8, 32, kernel_source_hash(), 333)
    assert bench.load_traffic(8, 32, p) == 333
    assert bench.load_traffic(8, 64, p) == 222
    assert bench.load_traffic(7, 32, p) is None
    assert bench.load_traffic(8, 16, p) is None


def test_traffic_absent_or_stale(tmp_path):
    assert bench.load_traffic(8, 32, str(tmp_path / "missing.md")) is None
    p = str(tmp_path / "stale.md")
    _summary(p, 8, 32, "f" * 16, 444)
    assert bench.load_traffic(8, 32, p) is None

