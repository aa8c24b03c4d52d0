"""Seeded synthetic initial conditions for direct N-body runs.

This module is shared by the CPU oracle, the HIP path, the tests and the
benchmark.  It only draws random numbers and turns them into particle
distributions; it holds none of the integrator's or the force's arithmetic.

Every model is returned as ``(m, x, v)`` with ``m`` of shape ``(N,)`` and
``x``, ``v`` of shape ``(3, N)`` (structure-of-arrays: the three Cartesian
components are separate contiguous rows), all float64, in N-body units
(G = 1, total mass 1, total energy -1/4 in expectation), centre-of-mass frame.

Only uniform draws from numpy's PCG64 generator are used; all transforms are
written out here, so a seed fixes the bytes on every machine.
"""
from __future__ import annotations

import hashlib
import math

import numpy as np

__all__ = [
    "plummer",
    "ensemble_sizes",
    "ensemble",
    "active_subset",
    "state_digest",
    "PLUMMER_SCALE",
]

# Plummer's model with scale radius 1 and G = M = 1 has total energy -3*pi/64.
# Standard N-body units ask for E = -1/4, reached by stretching lengths by
# 3*pi/16 and slowing velocities by sqrt(16/(3*pi)) (virial equilibrium is
# kept because v^2 scales as 1/length).
PLUMMER_SCALE = 3.0 * math.pi / 16.0


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _isotropic(rng: np.random.Generator, radius: np.ndarray) -> np.ndarray:
    """Vectors of the given lengths with directions uniform on the sphere."""
    n = radius.shape[0]
    u = rng.random(n)
    w = rng.random(n)
    cos_t = 1.0 - 2.0 * u
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    phi = 2.0 * math.pi * w
    out = np.empty((3, n))
    out[0] = radius * sin_t * np.cos(phi)
    out[1] = radius * sin_t * np.sin(phi)
    out[2] = radius * cos_t
    return out


def plummer(n: int, seed: int, mass_cut: float = 0.999):
    """Equal-mass Plummer sphere (Aarseth, Henon & Wielen 1974 sampling).

    Radii come from inverting the cumulative mass M(<r) = r^3 / (1 + r^2)^(3/2)
    for a uniform mass fraction X <= ``mass_cut`` (the cut removes the few
    particles that would land at very large radius).  Speeds are
    q * sqrt(2) * (1 + r^2)^(-1/4), the escape speed times q, with q drawn by
    von Neumann rejection from the density q^2 (1 - q^2)^(7/2) on [0, 1]
    (its maximum is below 0.1, which bounds the rejection envelope).
    Directions are isotropic.  The sample is moved to its centre-of-mass frame
    and scaled to N-body units by PLUMMER_SCALE.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = _rng(seed)
    mfrac = rng.random(n) * mass_cut
    # X = r^3/(1+r^2)^{3/2}  <=>  r = (X^{-2/3} - 1)^{-1/2}
    with np.errstate(divide="ignore"):
        r = 1.0 / np.sqrt(np.power(np.maximum(mfrac, 1e-300), -2.0 / 3.0) - 1.0)
    x = _isotropic(rng, r)

    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        cand = rng.random(todo.size)
        height = 0.1 * rng.random(todo.size)
        ok = height < cand * cand * np.power(1.0 - cand * cand, 3.5)
        q[todo[ok]] = cand[ok]
        todo = todo[~ok]
    speed = q * math.sqrt(2.0) * np.power(1.0 + r * r, -0.25)
    v = _isotropic(rng, speed)

    m = np.full(n, 1.0 / n)
    x -= (x @ m)[:, None] / m.sum()
    v -= (v @ m)[:, None] / m.sum()
    x *= PLUMMER_SCALE
    v /= math.sqrt(PLUMMER_SCALE)
    return m, np.ascontiguousarray(x), np.ascontiguousarray(v)


def ensemble_sizes(n_clusters: int, seed: int, n_lo: int = 256, n_hi: int = 8192) -> np.ndarray:
    """Cluster sizes drawn log-uniformly in [n_lo, n_hi] (rounded to integers)."""
    rng = _rng(seed)
    u = rng.random(n_clusters)
    sizes = np.rint(np.exp(math.log(n_lo) + u * (math.log(n_hi) - math.log(n_lo))))
    return np.clip(sizes, n_lo, n_hi).astype(np.int64)


def ensemble(n_clusters: int, seed: int, n_lo: int = 256, n_hi: int = 8192):
    """Independent Plummer clusters, concatenated.

    Cluster c uses seed ``seed * 10**6 + c``.  Returns
    ``(m, x, v, offsets, eps)`` where cluster c owns particles
    ``offsets[c]:offsets[c+1]`` and has softening ``eps[c] = 1/N_c``.
    """
    sizes = ensemble_sizes(n_clusters, seed, n_lo, n_hi)
    offsets = np.zeros(n_clusters + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    total = int(offsets[-1])
    m = np.empty(total)
    x = np.empty((3, total))
    v = np.empty((3, total))
    for c, nc in enumerate(sizes):
        mc, xc, vc = plummer(int(nc), seed * 10**6 + c)
        s = slice(offsets[c], offsets[c + 1])
        m[s], x[:, s], v[:, s] = mc, xc, vc
    eps = 1.0 / sizes.astype(np.float64)
    return m, x, v, offsets, eps


def active_subset(n: int, n_act: int, seed: int = 7) -> np.ndarray:
    """The first ``n_act`` entries of a seeded permutation of range(n), sorted."""
    if not 0 <= n_act <= n:
        raise ValueError("need 0 <= n_act <= n")
    perm = _rng(seed).permutation(n)
    return np.sort(perm[:n_act]).astype(np.int32)


def state_digest(*arrays: np.ndarray) -> str:
    """SHA-256 over the raw little-endian bytes of the given arrays."""
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).astype(a.dtype.newbyteorder("<"), copy=False).tobytes())
    return h.hexdigest()
