"""The pencil lane order (a compile-time table in the kernels) is a
permutation of the pencil tasks and keeps the 3D Euler N=4 float64 pencil
accesses within the LDS's conflict-free rules (8- and 16-lane write groups,
16-lane reads of 16-byte words).  Host code only: the check includes the
kernel header and evaluates the same constexpr order."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None,
                    reason="hipcc not available")
def test_lane_order_is_conflict_free(tmp_path):
    exe = str(tmp_path / "lane_order_check")
    src = os.path.join(ROOT, "tests", "lane_order_check.hip")
    cmd = [HIPCC if os.path.exists(HIPCC) else "hipcc", "-std=c++17", "-O1", "-x", "hip",
           "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"), src, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    print(r.stdout)
    assert "permutation=0" not in r.stdout
    assert r.returncode == 0, r.stdout
