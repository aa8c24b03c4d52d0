"""The C ABI library on the CPU: it loads, exports every declared symbol,
and its host-side validation rejects bad arguments before touching a GPU."""
import ctypes
import re
import subprocess
from pathlib import Path

import numpy as np
import pytest

import paper_0711_0643_amd as nb
from paper_0711_0643_amd import nbody as nbmod

ROOT = Path(__file__).resolve().parent.parent
HEADER = ROOT / "include" / "nbody.h"


def declared_symbols():
    text = HEADER.read_text()
    return sorted(set(re.findall(r"NBODY_API\s+[\w\s\*]+?\b(nbody_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("nbody_init", "nbody_predict", "nbody_force", "nbody_correct", "nbody_step",
                     "nbody_sync", "nbody_energy", "nbody_destroy", "nbody_strerror"):
        assert required in names
    assert names == sorted(nbmod.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = nb.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", str(nb.library_path())], capture_output=True, text=True,
                         check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    for name in declared_symbols():
        assert name in exported, name
        assert hasattr(lib, name)
    # nothing else leaks out of the library's C++ internals
    assert {e for e in exported if e.startswith("nbody_")} == set(declared_symbols())


def test_header_compiles_as_c():
    src = '#include "nbody.h"\nint main(void){nbody_params p; nbody_default_params(&p); return p.precision;}\n'
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", f"-I{ROOT / 'include'}", "-x", "c",
                        "-"], input=src, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_default_params_and_strerror():
    p = nbmod.default_params()
    assert p.eta == 0.01 and p.eta_init == 0.01 and p.dt_max == 0.125 and p.dt_min == 2.0**-40
    assert p.precision == nb.FP64 and p.compute_pot == 0
    for code in range(-7, 1):
        assert nb.lib().nbody_strerror(code)
    assert nb.lib().nbody_strerror(-99) == b"unknown status"


def test_workspace_bytes_validation():
    L = nb.lib()
    p = nbmod.default_params()
    sz = ctypes.c_size_t(0)
    assert L.nbody_workspace_bytes(1000, 1, ctypes.byref(p), ctypes.byref(sz)) == 0 and sz.value > 0
    small = sz.value
    assert L.nbody_workspace_bytes(2000, 1, ctypes.byref(p), ctypes.byref(sz)) == 0 and sz.value > small
    assert L.nbody_workspace_bytes(0, 1, ctypes.byref(p), ctypes.byref(sz)) == -1
    assert L.nbody_workspace_bytes(10, 0, ctypes.byref(p), ctypes.byref(sz)) == -1
    assert L.nbody_workspace_bytes(10, 11, ctypes.byref(p), ctypes.byref(sz)) == -1
    assert L.nbody_workspace_bytes(1 << 31, 1, ctypes.byref(p), ctypes.byref(sz)) == -1
    # the particle limit, 2^30: accepted at the limit, rejected above it
    assert L.nbody_workspace_bytes(1 << 30, 1, ctypes.byref(p), ctypes.byref(sz)) == 0 and sz.value > 0
    assert L.nbody_workspace_bytes((1 << 30) + 1, 1, ctypes.byref(p), ctypes.byref(sz)) == -1


def _init(n=8, nc=1, coff=None, eps=None, ws_bytes=1 << 30, workspace=256, params=None, **pk):
    L = nb.lib()
    p = params or nbmod.default_params(**pk)
    m = np.full(n, 1.0 / n)
    x = np.random.default_rng(0).standard_normal((3, n))
    v = np.zeros((3, n))
    coff = np.array(coff if coff is not None else [0, n], dtype=np.int64)
    eps = np.array(eps if eps is not None else [0.01] * nc, dtype=np.float64)
    ctx = ctypes.c_void_p(None)
    r = L.nbody_init(ctypes.byref(ctx), n, nc, coff.ctypes.data, m.ctypes.data, x.ctypes.data, v.ctypes.data,
                     eps.ctypes.data, ctypes.byref(p), workspace, ws_bytes, None)
    return r, ctx


@pytest.mark.parametrize("case", [
    dict(coff=[0, 4]),               # offsets do not end at n
    dict(coff=[1, 8]),               # offsets do not start at 0
    dict(n=8, nc=2, coff=[0, 0, 8]),  # empty cluster
    dict(eps=[-1.0]),                # negative softening
    dict(workspace=257),             # misaligned workspace
    dict(eta=0.0),                   # eta must be positive
    dict(dt_max=0.1),                # dt_max must be a power of two
    dict(dt_min=1.0),                # dt_min above dt_max
    dict(precision=7),               # unknown precision
])
def test_init_rejects_bad_arguments_on_the_host(case):
    r, ctx = _init(**case)
    assert r == -1 and not ctx.value


def test_init_reports_small_workspace():
    r, ctx = _init(ws_bytes=16)
    assert r == -2 and not ctx.value


def test_null_context_calls_are_rejected():
    L = nb.lib()
    assert L.nbody_sync(None) == -1
    assert L.nbody_step(None, 1, 0.125) == -1
    assert L.nbody_force(None, None, None, 1, None, None, None) == -1
    assert L.nbody_destroy(None) == 0


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    monkeypatch.setattr(nbmod, "_LIB_PATH", tmp_path / "missing.so")
    monkeypatch.setattr(nbmod, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        nbmod.lib()
