"""Helpers shared by the GPU tests: case banners and error measures."""
from __future__ import annotations

import sys

import numpy as np


def banner(msg: str) -> None:
    """Name the case on stdout before a GPU step runs (survives a crash)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def rel_err(got, ref):
    """Per-particle |got - ref| / |ref| for (3, n) vectors or (n,) scalars."""
    got, ref = np.asarray(got), np.asarray(ref)
    if got.ndim == 2:
        return np.linalg.norm(got - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)
    return np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)


def normwise_err(got, ref, scale):
    """|got - ref| measured against the sum of the absolute pair terms."""
    got, ref = np.asarray(got), np.asarray(ref)
    if got.ndim == 2:
        return np.linalg.norm(got - ref, axis=0) / np.maximum(scale, 1e-300)
    return np.abs(got - ref) / np.maximum(scale, 1e-300)
