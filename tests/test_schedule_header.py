"""The public device-side schedule header (include/lb_schedule.hpp) stands
alone: a user's kernels that include only it compile for gfx950."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_user_kernels_compile_against_the_public_header(tmp_path):
    src = os.path.join(ROOT, "tests", "schedule_user_kernel.hip")
    out = tmp_path / "user.o"
    cmd = [HIPCC, "-x", "hip", "-O2", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-c", src, "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    assert out.stat().st_size > 0
