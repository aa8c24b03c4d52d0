"""Build libnbody.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB = PKG / "libnbody.so"
SOURCES = ["force.hip", "force_tuned.hip", "force_tuned_t128.hip", "step.hip", "perturbers.hip", "api.hip"]
BUILD = PKG / "_build"

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 (v_pk_*_f32) stays off: scalar FP32 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden",
    "-Wall",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and Path(cand).exists():
            return cand
    return "hipcc"


def _run(cmd) -> str:
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{err}")
    return err


def build(verbose: bool = False) -> Path:
    """Compile every source for gfx950 (one hipcc per source, in parallel)
    and link them into paper_0711_0643_amd/libnbody.so."""
    from concurrent.futures import ThreadPoolExecutor

    BUILD.mkdir(exist_ok=True)
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    objs = [BUILD / (s + ".o") for s in SOURCES]
    cmds = [[hipcc(), *compile_flags, f"-I{ROOT / 'include'}", f"-I{CSRC}", "-c", "-o", str(o), str(CSRC / s)]
            for s, o in zip(SOURCES, objs)]
    with ThreadPoolExecutor(max_workers=len(cmds)) as pool:
        errs = list(pool.map(_run, cmds))
    tmp = LIB.with_suffix(".so.tmp")
    errs.append(_run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", str(tmp), *map(str, objs)]))
    if verbose:
        for e in errs:
            if e.strip():
                print(e, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


def asm(source: str = "force.hip") -> str:
    """Device assembly of one source (for inspection)."""
    out = PKG / "csrc" / (source + ".s")
    cmd = [hipcc(), *[f for f in HIPCC_FLAGS if f not in ("-shared", "-fPIC")], "--cuda-device-only", "-S",
           f"-I{ROOT / 'include'}", f"-I{CSRC}", "-o", str(out), str(CSRC / source)]
    subprocess.run(cmd, check=True, capture_output=True)
    return str(out)


if __name__ == "__main__":
    print(build(verbose=True))
