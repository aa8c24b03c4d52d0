"""The threshold test of the perturber kernel decides m / R^2 > t (the
rounded FP64 quotient, Sect. 3.1) without dividing where the outcome is
certain: with t and p = fl(t R^2) between 2^-1000 and 2^1000, m > fl(p (1 +
2^-40)) means pass and m < fl(p (1 - 2^-40)) means fail; every other case
takes the quotient.  This CPU test applies that rule in IEEE float64
(numpy, no fused operations) to adversarial inputs (ties within a few units
in the last place and at the band's edge, exponents across the whole
range, subnormals, zeros, infinities, NaN) and checks that wherever the
rule claims certainty it agrees with the rounded quotient.  The kernel's
own code is compared with the oracle on the GPU, at one pair's term and
one unit either side of it."""
import numpy as np

LO, HI = 2.0**-1000, 2.0**1000
UP, DOWN = 1.0 + 2.0**-40, 1.0 - 2.0**-40


def rule(m, r2, t):
    """(certain, decision): the product test as the kernel takes it."""
    with np.errstate(all="ignore"):
        p = t * r2
        ok = (p > LO) & (p < HI) & (t > LO) & (t < HI)
        sure_pass = ok & (m > p * UP)
        sure_fail = ok & (m < p * DOWN)
    return sure_pass | sure_fail, sure_pass


def quotient(m, r2, t):
    with np.errstate(all="ignore"):
        return (m / r2) > t


def _check(m, r2, t):
    certain, dec = rule(m, r2, t)
    exact = quotient(m, r2, t)
    bad = certain & (dec != exact)
    assert not bad.any(), (m[bad][:5], r2[bad][:5], t[bad][:5])
    return certain.mean()


def test_rule_agrees_with_the_quotient_on_random_exponents():
    rng = np.random.default_rng(1)
    n = 400_000
    r2 = 2.0 ** rng.uniform(-1070, 1020, n) * rng.uniform(1, 2, n)
    t = 2.0 ** rng.uniform(-1074, 1020, n) * rng.uniform(1, 2, n)
    m = 2.0 ** rng.uniform(-1074, 1023, n) * rng.uniform(1, 2, n)
    _check(m, r2, t)


def test_rule_agrees_near_ties():
    """m placed at t r2 times 1 + k 2^-52 for small k, and at the edges of
    the 2^-40 band, over a wide range of scales (subnormal t included)."""
    rng = np.random.default_rng(2)
    n = 300_000
    r2 = 2.0 ** rng.uniform(-600, 600, n) * rng.uniform(1, 2, n)
    t = 2.0 ** rng.uniform(-1074, 600, n) * rng.uniform(1, 2, n)
    k = rng.integers(-8, 9, n).astype(np.float64)
    edge = rng.choice([2.0**-40, -(2.0**-40), 2.0**-39, -(2.0**-39), 2.0**-41, -(2.0**-41)], n)
    scale = np.where(rng.random(n) < 0.5, 1.0 + k * 2.0**-52, 1.0 + edge + k * 2.0**-52)
    with np.errstate(all="ignore"):
        m = (t * r2) * scale
    frac = _check(m, r2, t)
    assert frac > 0.2  # the band edges are mostly decided without division
    # exact ties: m / r2 == t in floating point
    with np.errstate(all="ignore"):
        m2 = t * r2
    _check(m2, r2, t)


def test_rule_special_values():
    vals = np.array([0.0, -0.0, 5e-324, 2.0**-1022, 1.0, 2.0**1000, 1.7e308, np.inf, -1.0, np.nan])
    m, r2, t = np.meshgrid(vals, vals, vals, indexing="ij")
    _check(m.ravel(), r2.ravel(), t.ravel())
