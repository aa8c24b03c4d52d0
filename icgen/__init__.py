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
    "king",
    "king_profile",
    "salpeter_masses",
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


def salpeter_masses(n: int, rng: np.random.Generator, slope: float = 2.35, m_lo: float = 0.1,
                    m_hi: float = 100.0) -> np.ndarray:
    """Masses from dN/dm ~ m^-slope on [m_lo, m_hi] by inverting the
    cumulative distribution, normalised to a total of 1."""
    a = 1.0 - slope
    u = rng.random(n)
    m = np.power(m_lo**a + u * (m_hi**a - m_lo**a), 1.0 / a)
    return m / m.sum()


def _king_rho(w):
    """King (1966) density in units of the value it would have at W -> inf
    scale: exp(W) erf(sqrt W) - sqrt(4W/pi) (1 + 2W/3)."""
    w = np.maximum(w, 0.0)
    from scipy.special import erf

    return np.exp(w) * erf(np.sqrt(w)) - np.sqrt(4.0 * w / math.pi) * (1.0 + 2.0 * w / 3.0)


def king_profile(w0: float, dr: float = 1e-3):
    """Solve King's equation (1/r^2) d/dr (r^2 dW/dr) = -9 rho(W)/rho(W0) in
    core-radius units (sigma = 1, G = 1, 4 pi G rho0 = 9) from W(0) = w0,
    W'(0) = 0 outward to the tidal radius where W = 0 (classical RK4).

    Returns (r, W, M) tabulated from 0 to the tidal radius (M = enclosed
    mass in the same units)."""
    rho0 = _king_rho(np.array([w0]))[0]

    def rhs(r, y):
        w, dw = y
        lap = -9.0 * _king_rho(np.array([w]))[0] / rho0
        return np.array([dw, lap - (2.0 / r) * dw if r > 0 else lap / 3.0])

    # start slightly off the centre with the series W = w0 - (3/2) r^2 rho/rho0 ...
    r = dr
    y = np.array([w0 - 1.5 * r * r, -3.0 * r])
    rs, ws = [0.0, r], [w0, y[0]]
    while y[0] > 0.0 and r < 1e4:
        k1 = rhs(r, y)
        k2 = rhs(r + dr / 2, y + dr / 2 * k1)
        k3 = rhs(r + dr / 2, y + dr / 2 * k2)
        k4 = rhs(r + dr, y + dr * k3)
        y_new = y + dr / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        if y_new[0] <= 0.0:  # tidal radius inside this step: interpolate W = 0
            f = y[0] / (y[0] - y_new[0])
            r += f * dr
            rs.append(r)
            ws.append(0.0)
            break
        r += dr
        y = y_new
        rs.append(r)
        ws.append(y[0])
    r = np.array(rs)
    w = np.array(ws)
    rho = 9.0 / (4.0 * math.pi) * _king_rho(w) / rho0  # rho0 = 9 / (4 pi) in these units
    dm = 4.0 * math.pi * r * r * rho
    M = np.concatenate([[0.0], np.cumsum(0.5 * (dm[1:] + dm[:-1]) * np.diff(r))])
    return r, w, M


def king(n: int, w0: float, seed: int, masses: str = "salpeter"):
    """King (1966) model with central potential w0, n particles.

    Radii follow the enclosed-mass profile of king_profile (inverse CDF by
    linear interpolation); speeds at radius r are drawn by rejection from
    v^2 (exp(W(r) - v^2/2) - 1) on [0, sqrt(2 W(r))]; directions isotropic.
    Masses are Salpeter (slope 2.35 on [0.1, 100]) assigned independently of
    position, or equal.  The model is scaled to N-body units with its
    analytic energy (virial: E = U/2 with U the smooth-model potential
    energy), so E = -1/4 and Q = 1/2 hold in expectation."""
    rng = _rng(seed)
    r_tab, w_tab, m_tab = king_profile(w0)
    mtot = m_tab[-1]
    # radii
    u = rng.random(n) * mtot
    r = np.interp(u, m_tab, r_tab)
    w = np.interp(r, r_tab, w_tab)
    x = _isotropic(rng, r)
    # speeds by rejection, per-particle envelope from a grid maximum
    vmax = np.sqrt(2.0 * w)
    grid = np.linspace(0.0, 1.0, 65)[None, :] * vmax[:, None]
    pdf_grid = grid**2 * (np.exp(w[:, None] - grid**2 / 2.0) - 1.0)
    pmax = 1.1 * pdf_grid.max(axis=1) + 1e-300
    speed = np.zeros(n)
    todo = np.arange(n)
    while todo.size:
        cand = rng.random(todo.size) * vmax[todo]
        h = rng.random(todo.size) * pmax[todo]
        p = cand**2 * (np.exp(w[todo] - cand**2 / 2.0) - 1.0)
        ok = h < p
        speed[todo[ok]] = cand[ok]
        todo = todo[~ok]
    v = _isotropic(rng, speed)
    if masses == "salpeter":
        m = salpeter_masses(n, rng)
    elif masses == "equal":
        m = np.full(n, 1.0 / n)
    else:
        raise ValueError("masses must be 'salpeter' or 'equal'")
    # analytic energy of the smooth model: phi = -W - M/r_t (sigma = 1, G = 1)
    rt = r_tab[-1]
    rho = np.gradient(m_tab, r_tab) / np.maximum(4.0 * math.pi * r_tab**2, 1e-300)
    rho[0] = rho[1]
    phi = -w_tab - mtot / rt
    dU = 0.5 * 4.0 * math.pi * r_tab**2 * rho * phi
    U = float(np.sum(0.5 * (dU[1:] + dU[:-1]) * np.diff(r_tab)))
    E_model = 0.5 * U
    # to total mass 1 (v scales as sqrt(M)), then to E = -1/4 (length lambda)
    v /= math.sqrt(mtot)
    E1 = E_model / mtot**2
    lam = E1 / -0.25
    x -= (x @ m)[:, None]
    v -= (v @ m)[:, None]
    x *= lam
    v /= math.sqrt(lam)
    return m, np.ascontiguousarray(x), np.ascontiguousarray(v)
