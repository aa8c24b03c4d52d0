"""Pins for the FP64 oracle: checks against facts the paper and the mathematics fix.

None of these re-types the oracle's pair formula.  Each compares the oracle
with something independent: a closed form (two bodies, a cube, a ring), an
invariant (Newton's third law, Euler's theorem for the -1-homogeneous
potential, the gradient of the potential energy, the time derivative of the
acceleration), an exactness property of the Hermite scheme on polynomial
trajectories, Kepler's solution of the two-body problem, the order of the
scheme, or the energy conservation of a Plummer cluster.

Every ``pin_*`` function raises AssertionError on failure.  The mutation test
runs all of them against deliberately broken builds of the oracle and expects
each break to trip at least one pin.
"""
from __future__ import annotations

import math

import numpy as np

import icgen
import oracle


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# --------------------------------------------------------------------------
# Force, jerk, potential: closed forms (Sect. 2.1, Eq. Force with the
# attractive sign; softening and potential as read in the oracle header).

def pin_two_body_closed_form():
    """Two bodies on the x axis: a = m_j d / (d^2+eps^2)^(3/2) toward j."""
    for eps in (0.0, 0.3):
        d, m1, m2 = 1.5, 0.25, 0.75
        m = np.array([m1, m2])
        x = np.array([[0.125, 0.125 + d], [0.0, 0.0], [-0.5, -0.5]])
        v = np.zeros((3, 2))
        acc, jerk, pot = oracle.force(m, x, v, eps)
        R2 = d * d + eps * eps
        assert _rel(acc[:, 0], [m2 * d / R2**1.5, 0, 0]) < 1e-15
        assert _rel(acc[:, 1], [-m1 * d / R2**1.5, 0, 0]) < 1e-15
        assert abs(pot[0] + m2 / math.sqrt(R2)) < 1e-15
        assert abs(pot[1] + m1 / math.sqrt(R2)) < 1e-15
        assert np.all(jerk == 0.0)


def pin_cube_closed_form():
    """Equal masses on the corners of a cube of side s: each acceleration
    points at the centre; per axis it is -m s [1/(s^2+e^2)^1.5 +
    2/(2s^2+e^2)^1.5 + 1/(3s^2+e^2)^1.5] (neighbours differing in 1, 2, 3
    coordinates); the potential is -m [3/sqrt(s^2+e^2) + 3/sqrt(2s^2+e^2) +
    1/sqrt(3s^2+e^2)]."""
    s, mm, eps = 0.75, 0.125, 0.1
    corners = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], float)
    x = (0.5 * s * corners).T.copy()
    m = np.full(8, mm)
    acc, _, pot = oracle.force(m, x, np.zeros((3, 8)), eps)
    e2 = eps * eps
    per_axis = mm * s * (1 / (s * s + e2) ** 1.5 + 2 / (2 * s * s + e2) ** 1.5 + 1 / (3 * s * s + e2) ** 1.5)
    expect = -np.sign(x) * per_axis
    assert _rel(acc, expect) < 1e-14
    phi = -mm * (3 / math.sqrt(s * s + e2) + 3 / math.sqrt(2 * s * s + e2) + 1 / math.sqrt(3 * s * s + e2))
    assert _rel(pot, np.full(8, phi)) < 1e-14


def _ring(n, R, omega, mm):
    th = 2 * math.pi * np.arange(n) / n
    x = np.vstack([R * np.cos(th), R * np.sin(th), np.zeros(n)])
    v = np.vstack([-omega * R * np.sin(th), omega * R * np.cos(th), np.zeros(n)])
    return np.full(n, mm), x, v, th


def pin_rotating_ring():
    """A rigidly rotating ring of n equal masses.  The acceleration of each body
    points at the centre with magnitude sum_k m 2R s_k^2 / (4R^2 s_k^2+e^2)^1.5,
    s_k = sin(pi k/n); rigid rotation at rate omega turns it, so the jerk is
    omega z x a (the exact time derivative), and the potential is
    -sum_k m / sqrt(4R^2 s_k^2 + e^2)."""
    for n, eps in ((7, 0.0), (12, 0.05)):
        R, om, mm = 1.25, 0.8, 1.0 / n
        m, x, v, th = _ring(n, R, om, mm)
        acc, jerk, pot = oracle.force(m, x, v, eps)
        sk = np.sin(math.pi * np.arange(1, n) / n)
        mag = np.sum(mm * 2 * R * sk**2 / (4 * R * R * sk**2 + eps * eps) ** 1.5)
        expect_a = -mag * np.vstack([np.cos(th), np.sin(th), np.zeros(n)])
        assert _rel(acc, expect_a) < 1e-14
        expect_k = om * np.vstack([-expect_a[1], expect_a[0], np.zeros(n)])
        assert _rel(jerk, expect_k) < 1e-13
        phi = -np.sum(mm / np.sqrt(4 * R * R * sk**2 + eps * eps))
        assert _rel(pot, np.full(n, phi)) < 1e-14


def _random_system(n, seed, unequal=True):
    rng = np.random.Generator(np.random.PCG64(seed))
    m = rng.random(n) + 0.2 if unequal else np.full(n, 1.0 / n)
    m /= m.sum()
    x = rng.standard_normal((3, n))
    v = rng.standard_normal((3, n)) * 0.5
    return m, x, v


def pin_newton_third_law():
    """Pairwise antisymmetry: sum m a = 0, sum m k = 0, sum m x cross a = 0."""
    m, x, v = _random_system(97, 11)
    for eps in (0.0, 0.05):
        acc, jerk, _ = oracle.force(m, x, v, eps)
        scale_a = np.sum(m * np.linalg.norm(acc, axis=0))
        scale_k = np.sum(m * np.linalg.norm(jerk, axis=0))
        assert np.max(np.abs(acc @ m)) < 1e-14 * scale_a
        assert np.max(np.abs(jerk @ m)) < 1e-14 * scale_k
        torque = np.cross(x.T, acc.T) * m[:, None]
        assert np.max(np.abs(torque.sum(0))) < 1e-14 * np.sum(m * np.linalg.norm(x, axis=0) * np.linalg.norm(acc, axis=0))


def pin_euler_virial_identity():
    """For the unsoftened 1/r potential (homogeneous of degree -1),
    sum_i m_i x_i . a_i equals the potential energy (1/2) sum_i m_i phi_i."""
    m, x, v = _random_system(64, 5)
    acc, _, pot = oracle.force(m, x, v, 0.0)
    lhs = float(np.sum(m * np.einsum("ij,ij->j", x, acc)))
    rhs = 0.5 * float(np.sum(m * pot))
    assert abs(lhs - rhs) < 1e-13 * abs(rhs)


def pin_gradient_of_potential_energy():
    """a_i = -(1/m_i) dW/dx_i with W = (1/2) sum m phi (softened), by central
    differences of the oracle's own potential energy."""
    m, x, v = _random_system(24, 8)
    eps, h = 0.07, 1e-5
    acc, _, _ = oracle.force(m, x, v, eps)

    def W(xx):
        return 0.5 * float(np.sum(m * oracle.force(m, xx, v, eps)[2]))

    for i in (0, 7, 23):
        g = np.zeros(3)
        for d in range(3):
            xp, xm = x.copy(), x.copy()
            xp[d, i] += h
            xm[d, i] -= h
            g[d] = (W(xp) - W(xm)) / (2 * h)
        assert _rel(-g / m[i], acc[:, i]) < 1e-6


def pin_jerk_is_time_derivative():
    """k = d a / dt along straight-line motion x(t) = x + v t, by a
    Richardson-extrapolated central difference."""
    m, x, v = _random_system(40, 3)
    eps = 0.02
    _, jerk, _ = oracle.force(m, x, v, eps)

    def cd(h):
        ap = oracle.force(m, x + v * h, v, eps)[0]
        am = oracle.force(m, x - v * h, v, eps)[0]
        return (ap - am) / (2 * h)

    rich = (4 * cd(5e-4) - cd(1e-3)) / 3
    assert _rel(rich, jerk) < 1e-8


def pin_active_subset_matches_full():
    """Forces on an active subset equal the matching rows of the all-active call
    (the block only selects rows; Sect. 2.1 item list)."""
    m, x, v = _random_system(50, 21)
    act = np.array([0, 3, 4, 17, 49], dtype=np.int32)
    a_all, k_all, p_all = oracle.force(m, x, v, 0.01)
    a_s, k_s, p_s = oracle.force(m, x, v, 0.01, act)
    assert np.array_equal(a_s, a_all[:, act])
    assert np.array_equal(k_s, k_all[:, act])
    assert np.array_equal(p_s, p_all[act])


# --------------------------------------------------------------------------
# Sums of absolute pair terms (the error scale of the force gates): closed
# forms and the triangle inequality, with equality where every term points
# the same way.

def pin_force_abs_two_body():
    """One pair, r = (d, 0, 0), relative velocity (u, w, 0): the acceleration
    term has length m d / R^3, the jerk term is m/R^3 (u (1 - 3 d^2/R^2), w, 0)
    and the potential term m / R, with R^2 = d^2 + eps^2."""
    d, u, w, m1, m2, eps = 1.25, 0.5, -0.75, 0.375, 0.625, 0.2
    m = np.array([m1, m2])
    x = np.array([[0.5, 0.5 + d], [0.25, 0.25], [0.0, 0.0]])
    v = np.array([[0.125, 0.125 + u], [1.0, 1.0 + w], [-0.5, -0.5]])
    out = oracle.force_abs(m, x, v, eps)
    R2 = d * d + eps * eps
    R3 = R2**1.5
    for i, mj in ((0, m2), (1, m1)):
        assert abs(out[0, i] - mj * d / R3) < 1e-15 * mj * d / R3
        kj = mj / R3 * math.hypot(u * (1 - 3 * d * d / R2), w)
        assert abs(out[1, i] - kj) < 1e-14 * kj
        assert abs(out[2, i] - mj / math.sqrt(R2)) < 1e-15 * mj / math.sqrt(R2)


def pin_force_abs_rotating_ring():
    """Rigid rotation at rate omega: every relative velocity is omega z x r,
    perpendicular to r with length omega |r|, so each jerk term has length
    omega times its acceleration term and the jerk sum is omega times the
    acceleration sum, sum_k m c_k / (c_k^2 + eps^2)^1.5 with chords
    c_k = 2 R sin(pi k / n); the potential sum is sum_k m / sqrt(c_k^2 + eps^2)."""
    for n, eps in ((9, 0.0), (16, 0.1)):
        R, om, mm = 0.8, 1.3, 1.0 / n
        m, x, v, _ = _ring(n, R, om, mm)
        out = oracle.force_abs(m, x, v, eps)
        ck = 2 * R * np.sin(math.pi * np.arange(1, n) / n)
        sa = np.sum(mm * ck / (ck**2 + eps * eps) ** 1.5)
        sp = np.sum(mm / np.sqrt(ck**2 + eps * eps))
        assert _rel(out[0], np.full(n, sa)) < 1e-14
        assert _rel(out[1], np.full(n, om * sa)) < 1e-13
        assert _rel(out[2], np.full(n, sp)) < 1e-14


def pin_force_abs_collinear_equality():
    """Particle 0 at the end of a line of particles on the x axis, all others
    receding along the line (u_j > u_0): every acceleration term points along
    +x and (for |r| > eps / sqrt 2) every jerk term along -x, so the sums of
    term lengths equal the lengths of the sums; every potential term is
    negative, so the potential sum is -phi."""
    rng = np.random.Generator(np.random.PCG64(31))
    n, eps = 12, 0.05
    m = rng.random(n) + 0.1
    x = np.zeros((3, n))
    x[0] = np.concatenate([[0.0], np.sort(rng.random(n - 1)) * 3 + 0.2])
    v = np.zeros((3, n))
    v[0] = np.concatenate([[-0.3], rng.random(n - 1) + 0.05])
    acc, jerk, pot = oracle.force(m, x, v, eps)
    out = oracle.force_abs(m, x, v, eps)
    assert abs(out[0, 0] - np.linalg.norm(acc[:, 0])) < 1e-14 * out[0, 0]
    assert abs(out[1, 0] - np.linalg.norm(jerk[:, 0])) < 1e-14 * out[1, 0]
    assert _rel(out[2], -pot) < 1e-14


def pin_force_abs_bounds():
    """Triangle inequality on a random system: |a_i| <= A_i, |k_i| <= K_i, and
    the potential sum is -phi_i (all terms of one sign)."""
    m, x, v = _random_system(80, 17)
    acc, jerk, pot = oracle.force(m, x, v, 0.03)
    out = oracle.force_abs(m, x, v, 0.03)
    assert np.all(np.linalg.norm(acc, axis=0) <= out[0] * (1 + 1e-14))
    assert np.all(np.linalg.norm(jerk, axis=0) <= out[1] * (1 + 1e-14))
    assert _rel(out[2], -pot) < 1e-14
    # and the bound is not slack everywhere: cancellation is partial
    assert np.min(out[0] / np.linalg.norm(acc, axis=0)) < 3.0


# --------------------------------------------------------------------------
# Diagnostics: Galilean invariance fixes how energy, momentum and angular
# momentum change under a shift of origin and a boost.

def pin_diagnostics_galilean_boost():
    """A system with sum m x = 0 and sum m v = 0, shifted by C and boosted by
    V: P = M V, L = L0 + M C x V, KE = KE0 + M |V|^2 / 2, PE unchanged."""
    m, x, v = _random_system(60, 23)
    M = m.sum()
    x = x - (x @ m)[:, None] / M
    v = v - (v @ m)[:, None] / M
    eps = 0.02
    d0 = oracle.diagnostics(m, x, v, eps)
    C = np.array([0.75, -1.5, 0.25])
    V = np.array([0.3, -0.2, 0.7])
    d1 = oracle.diagnostics(m, x + C[:, None], v + V[:, None], eps)
    assert _rel(d1["P"], M * V) < 1e-13
    assert np.max(np.abs(d0["P"])) < 1e-15
    assert _rel(d1["L"], d0["L"] + M * np.cross(C, V)) < 1e-13
    assert abs(d1["KE"] - (d0["KE"] + 0.5 * M * V @ V)) < 1e-13 * d1["KE"]
    assert abs(d1["PE"] - d0["PE"]) < 1e-13 * abs(d0["PE"])


def pin_diagnostics_two_body_closed_form():
    """Two bodies at x = -/+ (d/2) e_x with velocities -/+ (w/2) e_y:
    L = 2 m (d/2)(w/2) e_z, P = 0, KE = m w^2 / 4, PE = -m^2 / sqrt(d^2+eps^2)."""
    mm, d, w, eps = 0.5, 1.5, 0.8, 0.1
    m = np.array([mm, mm])
    x = np.array([[-d / 2, d / 2], [0.0, 0.0], [0.0, 0.0]])
    v = np.array([[0.0, 0.0], [-w / 2, w / 2], [0.0, 0.0]])
    dg = oracle.diagnostics(m, x, v, eps)
    assert _rel(dg["L"], [0.0, 0.0, mm * d * w / 2]) < 1e-15
    assert np.all(dg["P"] == 0.0)
    assert abs(dg["KE"] - mm * w * w / 4) < 1e-16
    assert abs(dg["PE"] + mm * mm / math.sqrt(d * d + eps * eps)) < 1e-15


def pin_boosted_kepler_momentum():
    """The e = 0.5 Kepler pair boosted by V: the block-step run keeps
    P = M V and moves the centre of mass as X(t) = X(0) + V t."""
    m, x, v = _kepler_state()
    V = np.array([0.25, -0.5, 0.125])
    v = v + V[:, None]
    sim = oracle.Sim(m, x, v, eps=0.0)
    d0 = sim.diagnostics()
    assert _rel(d0["P"], V * m.sum()) < 1e-15
    sim.run(1.0, max_steps=20000)
    d1 = sim.diagnostics()
    assert _rel(d1["P"], d0["P"]) < 1e-12
    com = (sim.x @ m) / m.sum()
    assert np.max(np.abs(com - V * 1.0)) < 1e-12


def pin_j_slices_sum_to_total():
    """The paper's j-parallel partition: partial sums over contiguous j-slices,
    added in slice order, give the full sum up to FP64 rounding (Sect. 3)."""
    m, x, v = icgen.plummer(300, 9)
    a0, k0, p0 = oracle.force(m, x, v, 1 / 300)
    A = oracle.force(np.abs(m), x, np.zeros_like(v), 1 / 300)  # scale for the tolerance
    for p in (1, 2, 3, 7, 64, 300):
        a, k, ph = oracle.force(m, x, v, 1 / 300, slices=p)
        assert np.max(np.abs(a - a0)) < 1e-13 * np.max(np.abs(a0))
        assert np.max(np.abs(k - k0)) < 1e-13 * np.max(np.abs(k0))
        assert np.max(np.abs(ph - p0)) < 1e-13 * np.max(np.abs(p0))
    del A


# --------------------------------------------------------------------------
# Hermite predictor and corrector (Sect. 2.1): exactness on polynomials.

def pin_predictor_exact_on_cubic():
    """x(t) = x0 + v0 t + a0 t^2/2 + k0 t^3/6 is reproduced exactly from its
    value and first three derivatives at an earlier time."""
    rng = np.random.Generator(np.random.PCG64(2))
    n = 6
    x0, v0, a0, k0 = (rng.integers(-8, 8, (3, n)) / 8.0 for _ in range(4))
    t0 = np.array([0.0, 0.25, 0.5, 0.125, 0.375, 0.0])
    tp = 0.75

    def at(t):
        xt = x0 + v0 * t + a0 * t**2 / 2 + k0 * t**3 / 6
        vt = v0 + a0 * t + k0 * t**2 / 2
        return xt, vt, a0 + k0 * t, k0

    xs, vs, as_, ks = (np.empty((3, n)) for _ in range(4))
    for i in range(n):
        xi, vi, ai, ki = at(t0[i])
        xs[:, i], vs[:, i], as_[:, i], ks[:, i] = xi[:, i], vi[:, i], ai[:, i], ki[:, i]
    xp, vp = oracle.predict(xs, vs, as_, ks, t0, tp)
    xe, ve, _, _ = at(tp)
    assert _rel(xp, xe) < 1e-15 and _rel(vp, ve) < 1e-15


def pin_corrector_exact_on_quintic():
    """For a quintic trajectory (cubic acceleration) the corrector recovers the
    second and third derivatives of a at the start of the step exactly and
    lands on the exact position and velocity at the end."""
    rng = np.random.Generator(np.random.PCG64(4))
    x0, v0, a0, k0, s, c = (rng.standard_normal(3) for _ in range(6))
    h = 0.0625

    def traj(t):
        x = x0 + v0 * t + a0 * t**2 / 2 + k0 * t**3 / 6 + s * t**4 / 24 + c * t**5 / 120
        v = v0 + a0 * t + k0 * t**2 / 2 + s * t**3 / 6 + c * t**4 / 24
        a = a0 + k0 * t + s * t**2 / 2 + c * t**3 / 6
        k = k0 + s * t + c * t**2 / 2
        return x, v, a, k

    xp = x0 + v0 * h + a0 * h**2 / 2 + k0 * h**3 / 6
    vp = v0 + a0 * h + k0 * h**2 / 2
    x1, v1, a1, k1 = traj(h)
    xc, vc, a2, a3 = oracle.correct_one(h, a0, k0, a1, k1, xp, vp)
    assert _rel(a2, s) < 1e-10
    assert _rel(a3, c) < 1e-9
    assert _rel(xc, x1) < 1e-14
    assert _rel(vc, v1) < 1e-14


# --------------------------------------------------------------------------
# Time steps (Sect. 2.1, Eq. timestep and the block rule).

def pin_aarseth_circular_motion():
    """On circular motion at rate w every derivative of a has length |a| w^n, so
    the criterion is sqrt(eta) / w exactly."""
    w, A, eta = 1.7, 2.3, 0.01
    e1, e2 = np.array([1.0, 0, 0]), np.array([0, 1.0, 0])
    a = -A * e1
    k = -A * w * e2
    a2 = A * w * w * e1
    a3 = A * w**3 * e2
    dt = oracle.aarseth_dt(eta, a, k, a2, a3, 0.0)
    assert abs(dt - math.sqrt(eta) / w) < 1e-15
    # the second derivative is propagated to the end of the step: a2 + a3 h
    h = 0.01
    dt_h = oracle.aarseth_dt(eta, a, k, a2 - a3 * h, a3, h)
    assert abs(dt_h - math.sqrt(eta) / w) < 1e-15


def pin_aarseth_hand_vector():
    """sqrt(nu (|a||a2| + |k|^2) / (|k||a3| + |a2|^2)) on hand-picked vectors
    (nu = 0.01): |a| = 3, |k| = 5, |a2| = 2, |a3| = 4 -> sqrt(0.01 * 31 / 24)."""
    a = np.array([3.0, 0, 0])
    k = np.array([0, 3.0, 4.0])
    a2 = np.array([0, 0, 2.0])
    a3 = np.array([0, 4.0, 0])
    dt = oracle.aarseth_dt(0.01, a, k, a2, a3, 0.0)
    assert abs(dt - math.sqrt(0.01 * 31.0 / 24.0)) < 1e-16


QUANT_TABLE = "tests/golden/quantize_rules.txt"


def pin_quantize_rule_table():
    """Power-of-two block steps: the table in tests/golden lists hand-worked
    cases of the rule (shrink freely, double at most once and only on a
    commensurate time, cap at dt_max, error below dt_min)."""
    import os

    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), QUANT_TABLE)
    rows = 0
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            raw, old, t, dmax, dmin, expect, est = line.split()
            got, st = oracle.quantize(float(raw), float(old), float(t), float(dmax), float(dmin))
            if est == "ok":
                assert st == 0 and got == float(expect), (line, got, st)
            else:
                code = {"dtmin": oracle.E_DTMIN, "nonfinite": oracle.E_NONFINITE}[est]
                assert st == code, (line, got, st)
            rows += 1
    assert rows >= 10


def pin_pow2_floor():
    for x, e in ((1.0, 1.0), (0.75, 0.5), (0.5, 0.5), (1e-3, 2.0**-10), (3.0, 2.0), (2.0**-40 * 1.5, 2.0**-40)):
        assert oracle.pow2_floor(x) == e


def pin_initial_dt():
    """eta_s |a|/|k| rounded down to a power of two, capped at dt_max."""
    dt, st = oracle.initial_dt(0.01, [3.0, 4.0, 0.0], [0.0, 0.0, 0.1], 0.125, 2.0**-40)
    assert st == 0 and dt == 0.125  # 0.01*5/0.1 = 0.5 -> capped at 0.125
    dt, st = oracle.initial_dt(0.01, [3.0, 4.0, 0.0], [0.0, 0.0, 10.0], 0.125, 2.0**-40)
    assert st == 0 and dt == 2.0**-8  # 0.005 -> 2^-8 = 0.00390625


# --------------------------------------------------------------------------
# Integrator: Kepler problem, order of accuracy, cluster energy.

def _kepler_state(e=0.5, a=1.0, m1=0.5, m2=0.5):
    """Two bodies at pericentre in the COM frame."""
    M = m1 + m2
    rp = a * (1 - e)
    vp = math.sqrt(M * (1 + e) / (a * (1 - e)))
    r = np.array([rp, 0.0, 0.0])
    w = np.array([0.0, vp, 0.0])
    x = np.vstack([-m2 / M * r, m1 / M * r]).T.copy()
    v = np.vstack([-m2 / M * w, m1 / M * w]).T.copy()
    return np.array([m1, m2]), x, v


def _kepler_separation(t, e=0.5, a=1.0, M=1.0):
    """Relative position at time t after pericentre (Kepler's equation)."""
    n = math.sqrt(M / a**3)
    Mmean = n * t
    E = Mmean
    for _ in range(60):
        E -= (E - e * math.sin(E) - Mmean) / (1 - e * math.cos(E))
    return np.array([a * (math.cos(E) - e), a * math.sqrt(1 - e * e) * math.sin(E), 0.0])


def pin_kepler_orbit_block_steps():
    """e = 0.5, a = 1, eps = 0, eta = 0.01, block steps: after 8 time units the
    separation matches Kepler's solution and energy, angular momentum and the
    eccentricity are conserved."""
    m, x, v = _kepler_state()
    sim = oracle.Sim(m, x, v, eps=0.0, eta=0.01, eta_s=0.01, dt_max=2.0**-3)
    d0 = sim.diagnostics()
    sim.run(8.0, max_steps=20000)
    d1 = sim.diagnostics()
    sep = sim.x[:, 1] - sim.x[:, 0]
    assert np.max(np.abs(sep - _kepler_separation(8.0))) < 2e-5
    assert abs((d1["E"] - d0["E"]) / d0["E"]) < 2e-6
    assert _rel(d1["L"], d0["L"]) < 2e-6
    w = sim.v[:, 1] - sim.v[:, 0]
    r = np.linalg.norm(sep)
    evec = np.cross(w, np.cross(sep, w)) / 1.0 - sep / r
    assert abs(np.linalg.norm(evec) - 0.5) < 1e-6


def _shared_step_error(dt):
    m, x, v = _kepler_state()
    sim = oracle.Sim(m, x, v, eps=0.0, eta=1e30, eta_s=1e30, dt_max=dt)
    sim.run(2.0, max_steps=int(4.0 / dt))
    assert np.all(sim.dt == dt)
    sep = sim.x[:, 1] - sim.x[:, 0]
    return float(np.linalg.norm(sep - _kepler_separation(2.0)))


def pin_fourth_order_convergence():
    """With one shared fixed step, halving the step divides the error by about
    2^4 = 16: the scheme is fourth order (Sect. 2.1)."""
    e1 = _shared_step_error(2.0**-6)
    e2 = _shared_step_error(2.0**-7)
    order = math.log2(e1 / e2)
    assert 3.7 < order < 4.3, order


def pin_plummer_energy_conservation():
    """A 256-body Plummer sphere (eps = 1/256, eta = 0.01) to t = 1/2 keeps
    |dE/E| below 1e-5 and its block times on the power-of-two grid."""
    m, x, v = icgen.plummer(256, 12)
    eps = 1.0 / 256
    sim = oracle.Sim(m, x, v, eps=eps)
    E0 = sim.diagnostics()["E"]
    sim.run(0.5, max_steps=50000)
    E1 = sim.diagnostics()["E"]
    assert abs((E1 - E0) / E0) < 1e-5
    assert np.all(sim.t == 0.5)
    mant, _ = np.frexp(sim.dt)
    assert np.all(mant == 0.5)  # powers of two
    assert np.all(np.fmod(sim.t, sim.dt) == 0.0)


def pin_perturbers_lattice_closed_form():
    """Perturber lists (Sect. 3.1) on a line of equal masses m at integer
    positions, ids permuted against positions, eps = 0 and threshold m / 9:
    a star's perturbers are the stars one or two places away (m/1, m/4 pass,
    m/9 equals the threshold and does not), listed by ascending id (the
    order a serial sweep finds them), not by position."""
    n, mm = 40, 0.025
    rng = np.random.default_rng(5)
    place = rng.permutation(n)  # id -> position on the line
    x = np.zeros((3, n))
    x[0] = place.astype(float)
    m = np.full(n, mm)
    lists, counts = oracle.perturbers(m, x, 0.0, mm / 9.0, cap=8)
    for i in range(n):
        want = sorted(j for j in range(n) if j != i and abs(int(place[j]) - int(place[i])) <= 2)
        assert counts[i] == len(want), (i, counts[i], want)
        assert list(lists[i, :len(want)]) == want, (i, lists[i], want)
        assert np.all(lists[i, len(want):] == -1)


def pin_perturbers_cap_keeps_first_in_id_order():
    """With every other star passing (threshold 0), the list holds the first
    cap ids in ascending order (skipping the star itself) and the count all
    n - 1 of them."""
    n, cap = 300, 256
    rng = np.random.default_rng(6)
    x = rng.standard_normal((3, n))
    m = np.full(n, 1.0 / n)
    act = np.array([0, 7, 299], dtype=np.int32)
    lists, counts = oracle.perturbers(m, x, 0.01, 0.0, active=act, cap=cap)
    for q, i in enumerate(act):
        want = [j for j in range(n) if j != i][:cap]
        assert counts[q] == n - 1
        assert list(lists[q]) == want


def pin_perturbers_mass_not_distance():
    """A heavy star far away passes where a light near one does not (the
    force, not the distance, decides): m = 1e-3 at R = 0.1 gives 0.1, m = 10
    at R = 5 gives 0.4, threshold 0.2."""
    m = np.array([1.0, 1e-3, 10.0])
    x = np.zeros((3, 3))
    x[0] = [0.0, 0.1, 5.0]
    lists, counts = oracle.perturbers(m, x, 0.0, 0.2, active=np.array([0], dtype=np.int32), cap=4)
    assert counts[0] == 1 and list(lists[0]) == [2, -1, -1, -1]


def pin_perturbers_softened_distance():
    """Plummer softening enters the test as in the force: m / (R^2 + eps^2).
    Two stars at R = 1, m = 1, threshold 0.9: they perturb each other with
    eps = 0 (1 > 0.9) and not with eps = 0.5 (1 / 1.25 = 0.8)."""
    m = np.ones(2)
    x = np.zeros((3, 2))
    x[1, 1] = 1.0
    _, c0 = oracle.perturbers(m, x, 0.0, 0.9, cap=2)
    _, c1 = oracle.perturbers(m, x, 0.5, 0.9, cap=2)
    assert list(c0) == [1, 1] and list(c1) == [0, 0]


ALL_PINS = [
    pin_two_body_closed_form,
    pin_cube_closed_form,
    pin_rotating_ring,
    pin_newton_third_law,
    pin_euler_virial_identity,
    pin_gradient_of_potential_energy,
    pin_jerk_is_time_derivative,
    pin_active_subset_matches_full,
    pin_force_abs_two_body,
    pin_force_abs_rotating_ring,
    pin_force_abs_collinear_equality,
    pin_force_abs_bounds,
    pin_perturbers_lattice_closed_form,
    pin_perturbers_cap_keeps_first_in_id_order,
    pin_perturbers_mass_not_distance,
    pin_perturbers_softened_distance,
    pin_diagnostics_galilean_boost,
    pin_diagnostics_two_body_closed_form,
    pin_boosted_kepler_momentum,
    pin_j_slices_sum_to_total,
    pin_predictor_exact_on_cubic,
    pin_corrector_exact_on_quintic,
    pin_aarseth_circular_motion,
    pin_aarseth_hand_vector,
    pin_quantize_rule_table,
    pin_pow2_floor,
    pin_initial_dt,
    pin_kepler_orbit_block_steps,
    pin_fourth_order_convergence,
    pin_plummer_energy_conservation,
]
