"""Host-side check of the force-pass plan arithmetic of the HIP library
(csrc/common.h, plan_layout): compiled for the CPU with hipcc and run.  It
covers cluster sizes the GPU tests cannot reach (up to the library's limit
of 2^30 particles; from 2^26 on the plan uses 64-bit integers)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0711_0643_amd", "csrc")


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_plan_layout_invariants(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = tmp_path / "plan_check"
    src = os.path.join(ROOT, "tests", "native", "plan_check.cpp")
    # host-only compilation of the header's plan functions (no device code)
    subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "--offload-arch=gfx950", "-O1", "-std=c++17",
                    f"-I{CSRC}", "-o", str(exe), src], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok"), r.stdout
