"""The site-coordinate division of the one-lane-per-site kernels (a multiply
and a shift, csrc/common.h) equals integer division: the header's own code,
compiled for the host and checked exhaustively over small divisors and at
the edge numerators of large ones (no GPU needed)."""
import os
import subprocess

import pytest

from paper_1007_3432_amd import build

HERE = os.path.dirname(os.path.abspath(__file__))


def test_fastdiv_matches_integer_division(tmp_path):
    exe = str(tmp_path / "fastdiv_check")
    cmd = [build.HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(build.ROOT, "include"), "-I", build.CSRC,
           os.path.join(HERE, "native", "fastdiv_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail("hipcc failed:\n" + r.stderr[-2000:])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok"), out.stdout
