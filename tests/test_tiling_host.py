"""Host-side invariants of the row-per-lane tilings (tests/cpp/ell_check.cpp),
compiled with the host compiler against the library's mesh and tiling sources:
row ownership, entry order and positions, LDS slot targets, padding and bounds
for unit squares of 3, 12 and 128 cells and the step channel, every tile shape
and member width the autotuner offers."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2108_05110_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_row_per_lane_tilings(tmp_path):
    exe = str(tmp_path / "ell_check")
    cmd = ["g++", "-O1", "-std=c++17", "-I", CSRC, os.path.join(ROOT, "tests", "cpp", "ell_check.cpp"),
           os.path.join(CSRC, "tiling.cpp"), os.path.join(CSRC, "mesh.cpp"), "-o", exe]
    subprocess.run(cmd, check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "FAIL" not in out.stdout
    lines = [l for l in out.stdout.splitlines() if l.startswith("M ")]
    assert len(lines) == 4 * 6   # meshes x (shape, member width)
