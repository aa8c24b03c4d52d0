"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle is rebuilt with -fsanitize=address,undefined and every pin runs
against that build in a child interpreter (the sanitizer runtime preloaded,
leak checking off: the interpreter itself is not instrumented).  The plan
arithmetic of the HIP library's header is compiled for the host with the
same sanitizers and its invariant check run.  Any report fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]

CHILD = r"""
import sys
sys.path.insert(0, {root!r})
import oracle
oracle.use_library({lib!r})
from tests import oracle_pins
for pin in oracle_pins.ALL_PINS:
    pin()
print("pins ok", len(oracle_pins.ALL_PINS))
"""


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_asan_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if shutil.which("gcc") is None or asan is None or ubsan is None:
        pytest.skip("gcc sanitizer runtimes not available")
    sys.path.insert(0, ROOT)
    import oracle

    lib = tmp_path / "liboracle_san.so"
    flags = [f for f in oracle.CFLAGS if f != "-O2"] + ["-O1"] + SAN
    subprocess.run(["gcc", *flags, "-o", str(lib), os.path.join(ROOT, "oracle", "oracle.c"), "-lm"], check=True)
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=str(lib))], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    report = r.stdout + r.stderr
    assert r.returncode == 0 and "pins ok" in r.stdout, report[-4000:]
    assert "runtime error" not in report and "AddressSanitizer" not in report, report[-4000:]


def test_plan_check_under_asan_ubsan(tmp_path):
    hipcc = next((c for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc"))
                  if c and os.path.exists(c)), None)
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = tmp_path / "plan_check_san"
    src = os.path.join(ROOT, "tests", "native", "plan_check.cpp")
    csrc = os.path.join(ROOT, "paper_0711_0643_amd", "csrc")
    host_san = []
    for f in SAN:  # host-side flags only: no device code is compiled here
        host_san += ["-Xarch_host", f]
    subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "--offload-arch=gfx950", "-O1", "-std=c++17",
                    *host_san, f"-I{csrc}", "-o", str(exe), src], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.startswith("ok"), (r.stdout + r.stderr)[-4000:]
    assert "runtime error" not in r.stderr
