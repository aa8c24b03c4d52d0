"""The performance model's fit and total (Sect. 4.1, Eq. tsnb) on synthetic
block-step timings, CPU only: the fit recovers the per-step constants it
was given, and the model total is T_adv of the mean block times the number
of steps."""
import numpy as np

import bench


def _rows(taus, seed, noise):
    rng = np.random.default_rng(seed)
    rows = []
    for n in (1024, 4096, 16384, 65536):
        # block sizes spread over powers of two, as block steps produce them
        for s in 2.0 ** rng.integers(0, int(np.log2(n)) + 1, size=400):
            t = bench.model_total(taus, n, s, 1) * (1.0 + noise * rng.standard_normal())
            rows.append((n, float(s), t))
    return rows


def test_fit_recovers_the_step_constants():
    taus = (3.1e-5, 4.0e-11, 7.5e-9, 1.0e-12)
    got = bench.fit_step_model(_rows(taus, 1, 0.0))
    np.testing.assert_allclose(got, taus, rtol=1e-8)
    # with 2 % noise per step the interaction cost and the fixed cost stay within a few percent
    got = bench.fit_step_model(_rows(taus, 2, 0.02))
    assert abs(got[0] / taus[0] - 1) < 0.05
    assert abs(got[3] / taus[3] - 1) < 0.05


def test_model_total_is_mean_step_times_steps():
    taus = (2e-5, 1e-10, 1e-8, 1e-12)
    n, s, k = 16384, 200.0, 3000
    direct = k * (taus[0] + taus[1] * n + taus[2] * s + taus[3] * n * s)
    assert bench.model_total(taus, n, s, k) == direct
    # the fixed cost dominates a run of small blocks at small N
    assert taus[0] * k > 0.5 * bench.model_total(taus, 1024, 4.0, k)
