"""The seeded initial-condition generators (CPU)."""
import math

import numpy as np
import pytest
from scipy import stats

import icgen
import oracle


def test_plummer_is_seeded_and_centred():
    m1, x1, v1 = icgen.plummer(2000, 7)
    m2, x2, v2 = icgen.plummer(2000, 7)
    assert np.array_equal(x1, x2) and np.array_equal(v1, v2)
    assert not np.array_equal(x1, icgen.plummer(2000, 8)[1])
    assert abs(m1.sum() - 1.0) < 1e-14
    assert np.abs(x1 @ m1).max() < 1e-14 and np.abs(v1 @ m1).max() < 1e-14


def test_plummer_mass_profile_and_energy():
    """M(<r) follows r^3/(r^2 + a^2)^(3/2) (a = 3 pi / 16, truncated at 0.999
    of the mass; KS test), and E = -1/4, Q = 1/2 within sampling noise."""
    m, x, v = icgen.plummer(4096, 11)
    r = np.sqrt((x * x).sum(0))
    a = icgen.PLUMMER_SCALE

    def cdf(rr):
        return np.minimum(rr**3 / (rr * rr + a * a) ** 1.5 / 0.999, 1.0)

    # the centre-of-mass shift moves radii by O(1e-2 / sqrt(N)); KS is insensitive to it
    assert stats.kstest(r, cdf).pvalue > 0.01
    d = oracle.diagnostics(m, x, v, 0.0)
    assert abs(d["E"] + 0.25) < 0.02
    assert abs(d["KE"] / -d["PE"] - 0.5) < 0.03


def test_king_w0_6_concentration():
    """King W0 = 6 has concentration c = log10(r_t / r_c) ~ 1.25."""
    r, w, M = icgen.king_profile(6.0)
    assert w[0] == 6.0 and abs(w[-1]) < 1e-12
    assert 1.23 < math.log10(r[-1]) < 1.28
    assert np.all(np.diff(M) >= 0)


def test_king_sampling_and_units():
    n = 4096
    m, x, v = icgen.king(n, 6.0, 5, masses="equal")
    r_tab, w_tab, m_tab = icgen.king_profile(6.0)
    # radii follow the enclosed mass (scale-free test: compare r / r_half)
    r = np.sqrt((x * x).sum(0))
    rh_model = np.interp(0.5 * m_tab[-1], m_tab, r_tab)
    scaled = r / np.median(r) * rh_model
    assert stats.kstest(scaled, lambda q: np.interp(q, r_tab, m_tab) / m_tab[-1]).pvalue > 0.01
    d = oracle.diagnostics(m, x, v, 0.0)
    assert abs(d["E"] + 0.25) < 0.02
    assert abs(d["KE"] / -d["PE"] - 0.5) < 0.03


def test_salpeter_slope_by_maximum_likelihood():
    rng = np.random.Generator(np.random.PCG64(3))
    m = icgen.salpeter_masses(200000, rng) 
    m = m / m.min() * 0.1  # back to solar units: lower bound 0.1
    # truncated power law MLE for the slope, numerically
    lo, hi = 0.1, m.max()
    mean_log = np.mean(np.log(m))

    def score(s):
        a = 1 - s
        # d/ds log-likelihood of p(m) = m^-s / Z(s), Z = (hi^a - lo^a)/a
        za = (hi**a * np.log(hi) - lo**a * np.log(lo)) / (hi**a - lo**a) - 1 / a
        return -mean_log + za

    from scipy.optimize import brentq

    s_hat = brentq(score, 1.5, 3.5)
    assert abs(s_hat - 2.35) < 0.02


def test_ensemble_sizes_log_uniform():
    sizes = icgen.ensemble_sizes(256, 4)
    assert sizes.min() >= 256 and sizes.max() <= 8192
    u = (np.log(sizes) - math.log(256)) / (math.log(8192) - math.log(256))
    assert stats.kstest(u, "uniform").pvalue > 0.01
    m, x, v, off, eps = icgen.ensemble(5, 4, 256, 600)
    assert off[0] == 0 and off[-1] == m.size and np.all(np.diff(off) > 0)
    assert np.allclose(eps, 1.0 / np.diff(off))
    for c in range(5):
        s = slice(off[c], off[c + 1])
        assert abs(m[s].sum() - 1.0) < 1e-14


def test_active_subset():
    a = icgen.active_subset(1000, 37)
    assert a.dtype == np.int32 and a.size == 37 and np.all(np.diff(a) > 0)
    assert np.array_equal(a, icgen.active_subset(1000, 37))
    assert np.array_equal(icgen.active_subset(10, 10), np.arange(10))
    with pytest.raises(ValueError):
        icgen.active_subset(10, 11)
