"""The autotuner: every configuration it returns passes the parity gate
against the oracle, and its cache round-trips (GPU)."""
import json

import numpy as np
import pytest

import icgen
import oracle
from tests.gpu_util import banner, rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [1, 0], ids=["mixed", "fp64"])
def test_tuner_picks_a_parity_passing_config(precision, tmp_path, monkeypatch):
    import torch

    import paper_0711_0643_amd as nb
    from paper_0711_0643_amd import tune

    monkeypatch.setenv("NBODY_TUNE_CACHE", str(tmp_path / "tune.json"))
    n = 16384
    m, x, v = icgen.plummer(n, 17)
    eps = 1.0 / n
    banner(f"tune N={n} precision={precision}")
    sim = nb.Sim(m, x, v, eps, precision=precision)
    cfg = tune.tune(sim, ladder=[1, 64, 1024, 4096, n])
    assert cfg == sim.get_tuning()
    data = json.loads((tmp_path / "tune.json").read_text())
    key = tune.cache_key(sim)
    assert key in data and data[key]["tuning"] == cfg
    assert any(r["ok"] for r in data[key]["records"])
    # the chosen configuration against the oracle on several block sizes:
    # acceleration and potential per particle, jerk per particle where its
    # terms do not cancel by more than a factor 10
    for na in (1, 100, n):
        act = icgen.active_subset(n, na)
        a, k, _ = sim.force(act)
        _, _, phi = sim.force(act, pot=True)
        torch.cuda.synchronize()
        ra, rk, rphi = oracle.force(m, x, v, eps, act)
        tol = 1e-6 if precision == 1 else 1e-12
        assert rel_err(a.cpu().numpy(), ra).max() <= tol
        assert rel_err(phi.cpu().numpy(), rphi).max() <= tol
        kappa = oracle.force_abs(m, x, v, eps, act)[1] / np.linalg.norm(rk, axis=0)
        ek = rel_err(k.cpu().numpy(), rk)
        assert ek[kappa <= 10].max() <= tol
    recs = data[key]["records"]
    assert all({"err", "err_jerk_p999", "err_pot", "ok"} <= set(r) for r in recs)
    if precision == 1:
        if min(cfg["min_block"][:2]) <= n:  # the full block runs a one-lane-per-i layout: builds searched
            assert {(r["tile"], r["window"], r["waves"]) for r in recs if "window" in r} == {
                tune._key(b) for b in tune.BUILDS}
    # a second call is served from the cache
    sim2 = nb.Sim(m, x, v, eps, precision=precision)
    assert tune.tune(sim2) == cfg
    sim.close()
    sim2.close()


def test_batch_tuner_restores_state_and_passes_parity(tmp_path, monkeypatch):
    """tune_batch times block steps from the batch's current state: it must
    leave that state as it found it (bitwise), return a configuration that
    passes the parity gate, and cache it."""
    import torch

    import paper_0711_0643_amd as nb
    from paper_0711_0643_amd import tune

    monkeypatch.setenv("NBODY_TUNE_CACHE", str(tmp_path / "tune.json"))
    m, x, v, coff, eps = icgen.ensemble(6, 12, 256, 1500)
    banner("tune_batch 6 clusters")
    sim = nb.Sim(m, x, v, eps, cluster_offsets=coff, precision=1)
    sim.step(20, 0.25)
    before = sim.host_state()
    prog = sim.progress()
    cfg = tune.tune_batch(sim, replays=20)
    assert cfg == sim.get_tuning()
    after = sim.host_state()
    for key in before:
        assert np.array_equal(before[key], after[key]), key
    for u, w in zip(prog, sim.progress()):
        assert np.array_equal(u, w)
    data = json.loads((tmp_path / "tune.json").read_text())
    assert data[tune.batch_key(sim)]["tuning"] == cfg
    # the chosen configuration on the first cluster's predicted state against the oracle
    b, e = int(coff[0]), int(coff[1])
    act = np.arange(b, e, dtype=np.int32)
    aoff = np.array([0] + [e - b] * len(eps), dtype=np.int64)
    sim.predict(None)
    a, _, _ = sim.force(act, aoff)
    torch.cuda.synchronize()
    xs = sim.xp.cpu().numpy()[:, b:e]
    vs = sim.vp.cpu().numpy()[:, b:e]
    ra, _, _ = oracle.force(m[b:e], xs, vs, eps[0])
    assert rel_err(a.cpu().numpy(), ra).max() <= 1e-6
    sim.close()


@pytest.mark.parametrize("tile,window", [(256, 16), (256, 32), (256, 64), (128, 16), (128, 32)])
def test_every_kernel_build_matches_oracle(tile, window):
    """Each build of the lean tile-relative kernel the tuner may choose
    (j-tiles of 256 or 128 records; FP32 window 16, 32, 64, or 16, 32 on
    128-record tiles; 2 to 5 waves per SIMD) against the oracle:
    acceleration per particle, jerk per particle where kappa_k <= 10."""
    import torch

    import paper_0711_0643_amd as nb

    n = 6000
    m, x, v = icgen.plummer(n, 23)
    eps = 1.0 / n
    sim = nb.Sim(m, x, v, eps, precision=1)
    for na in (n, 2000):
        act = icgen.active_subset(n, na, seed=5)
        ra, rk, _ = oracle.force(m, x, v, eps, act)
        kappa = oracle.force_abs(m, x, v, eps, act)[1] / np.linalg.norm(rk, axis=0)
        for waves in (2, 3, 4, 5):
            banner(f"kernel build tile={tile} window={window} waves={waves} n_act={na}")
            sim.set_tuning(tile=tile, window=window, waves=waves, small_cluster_n=0)
            a, k, _ = sim.force(act)
            torch.cuda.synchronize()
            assert sim.status() == 0
            assert rel_err(a.cpu().numpy(), ra).max() <= 1e-6
            assert rel_err(k.cpu().numpy(), rk)[kappa <= 10].max() <= 1e-6
    sim.close()
