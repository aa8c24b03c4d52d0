"""Parity of the HIP predictor, corrector, block selection and block-step
pipeline with the FP64 oracle (GPU)."""
import numpy as np
import pytest

import icgen
import oracle
from tests.gpu_util import banner, rel_err

pytestmark = pytest.mark.gpu


def _sim(m, x, v, eps, precision=0, coff=None, **kw):
    import paper_0711_0643_amd as nb

    return nb.Sim(m, x, v, eps, cluster_offsets=coff, precision=precision, **kw)


def test_startup_matches_oracle():
    """a, k at t = 0 and the initial power-of-two steps."""
    n = 1500
    m, x, v = icgen.plummer(n, 31)
    eps = 1.0 / n
    banner("startup")
    sim = _sim(m, x, v, eps)
    st = sim.host_state()
    a, k, _ = oracle.force(m, x, v, eps)
    assert rel_err(st["a"], a).max() <= 1e-12
    assert rel_err(st["k"], k).max() <= 1e-12
    ref_dt = np.array([oracle.initial_dt(0.01, a[:, i], k[:, i], 0.125, 2.0**-40)[0] for i in range(n)])
    assert np.all(st["t"] == 0.0)
    # a power-of-two boundary can flip on a last-bit difference; none is expected here
    assert np.mean(st["dt"] == ref_dt) >= 0.999
    sim.close()


def test_predictor_matches_oracle():
    n = 2000
    m, x, v = icgen.plummer(n, 32)
    banner("predictor")
    sim = _sim(m, x, v, 1.0 / n)
    st = sim.host_state()
    for tp in (0.0, 2.0**-7, 0.1):
        sim.predict(tp)
        import torch

        torch.cuda.synchronize()
        xp, vp = sim.xp.cpu().numpy(), sim.vp.cpu().numpy()
        rx, rv = oracle.predict(st["x"], st["v"], st["a"], st["k"], st["t"], tp)
        assert np.max(np.abs(xp - rx)) <= 4e-16 * max(1.0, np.abs(rx).max())
        assert np.max(np.abs(vp - rv)) <= 4e-16 * max(1.0, np.abs(rv).max())
        if tp == 0.0:
            assert np.array_equal(xp, st["x"]) and np.array_equal(vp, st["v"])
    sim.close()


def test_corrector_matches_oracle():
    """One block step driven through the separate entry points
    (predict -> force -> correct) against the oracle's corrector, Aarseth
    criterion and quantisation applied to the same inputs."""
    import torch

    n = 1024
    m, x, v = icgen.plummer(n, 33)
    eps = 1.0 / n
    banner("corrector")
    sim = _sim(m, x, v, eps)
    s0 = sim.host_state()
    t_sys = float(np.min(s0["t"] + s0["dt"]))
    block = np.nonzero(s0["t"] + s0["dt"] == t_sys)[0].astype(np.int32)
    sim.predict(t_sys)
    acc, jerk, _ = sim.force(block)
    sim.correct(block, acc, jerk)
    torch.cuda.synchronize()
    assert sim.status() == 0
    s1 = sim.host_state()
    a1, k1 = acc.cpu().numpy(), jerk.cpu().numpy()
    xp, vp = oracle.predict(s0["x"], s0["v"], s0["a"], s0["k"], s0["t"], t_sys)
    same_dt = 0
    for q, i in enumerate(block):
        h = t_sys - s0["t"][i]
        xn, vn, a2, a3 = oracle.correct_one(h, s0["a"][:, i], s0["k"][:, i], a1[:, q], k1[:, q], xp[:, i], vp[:, i])
        assert rel_err(s1["x"][:, i:i + 1], xn[:, None]).max() <= 1e-14
        assert rel_err(s1["v"][:, i:i + 1], vn[:, None]).max() <= 1e-14
        raw = oracle.aarseth_dt(0.01, a1[:, q], k1[:, q], a2, a3, h)
        dtn, st = oracle.quantize(raw, s0["dt"][i], t_sys, 0.125, 2.0**-40)
        assert st == 0
        same_dt += int(dtn == s1["dt"][i])
        assert s1["t"][i] == t_sys
        assert np.array_equal(s1["a"][:, i], a1[:, q])
    assert same_dt >= len(block) - 1
    # particles outside the block are untouched
    rest = np.setdiff1d(np.arange(n), block)
    assert np.array_equal(s1["x"][:, rest], s0["x"][:, rest])
    assert np.array_equal(s1["dt"][rest], s0["dt"][rest])
    sim.close()


def test_block_steps_follow_oracle_n256():
    """Plummer N = 256 to t = 1/4 in FP64 through the captured step graph,
    against the oracle integrator from the same initial conditions: same
    block structure while the dt decisions agree, and close trajectories."""
    n = 256
    m, x, v = icgen.plummer(n, 41)
    eps = 1.0 / n
    banner("block steps N=256 fp64")
    sim = _sim(m, x, v, eps)
    ref = oracle.Sim(m, x, v, eps)
    E0 = ref.diagnostics()["E"]
    steps = 0
    while True:
        blk = ref.block_step()
        sim.step(1, 0.25)
        steps += 1
        t_gpu, _, _ = sim.progress()
        assert t_gpu[0] == ref.time, (steps, t_gpu[0], ref.time)
        if ref.time >= 0.25:
            break
        assert steps < 100000
    st = sim.host_state()
    assert sim.status() == 0
    assert np.all(st["t"] == 0.25)
    assert np.max(np.abs(st["x"] - ref.x)) < 1e-9
    assert np.max(np.abs(st["v"] - ref.v)) < 1e-9
    assert np.mean(st["dt"] == ref.dt) > 0.99
    E = sim.energy()[0]
    assert abs(E - ref.diagnostics()["E"]) < 1e-12 * abs(E0)
    _, gsteps, inter = sim.progress()
    assert gsteps[0] == steps
    assert inter[0] == ref.interactions
    sim.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_plummer_n1024_to_t1_conserves_energy(precision):
    """Plummer N = 1024, eps = 1/1024, eta = 0.01, block steps to t = 1:
    relative energy drift below 1e-5 (FP64 and mixed force)."""
    n = 1024
    m, x, v = icgen.plummer(n, 1)
    eps = 1.0 / 1024
    banner(f"C1 run to t=1 precision={precision}")
    sim = _sim(m, x, v, eps, precision=precision)
    E0 = sim.energy()[0]
    ref_E0 = oracle.diagnostics(m, x, v, eps)["E"]
    assert abs(E0 - ref_E0) <= 1e-13 * abs(ref_E0)
    sim.run(1.0, chunk=256)
    E1 = sim.energy()[0]
    assert sim.status() == 0
    assert abs((E1 - E0) / E0) < 1e-5, (E1 - E0) / E0
    st = sim.host_state()
    assert np.all(st["t"] == 1.0)
    # individual block steps conserve momentum only to the integration error
    P = st["v"] @ st["m"]
    assert np.max(np.abs(P)) < 1e-7
    sim.close()


def test_checkpoint_restart_is_bitwise():
    n = 512
    m, x, v = icgen.plummer(n, 51)
    banner("checkpoint")
    sim = _sim(m, x, v, 1.0 / n)
    sim.step(40, 0.5)
    blob = sim.get_state()
    sim.step(60, 0.5)
    a = sim.host_state()
    ta = sim.progress()
    sim.set_state(blob)
    sim.step(60, 0.5)
    b = sim.host_state()
    tb = sim.progress()
    for key in a:
        assert np.array_equal(a[key], b[key]), key
    for u, w in zip(ta, tb):
        assert np.array_equal(u, w)
    sim.close()


@pytest.mark.parametrize("clusters", [1, 3], ids=["one_cluster", "three_clusters"])
def test_step_calls_of_any_length_give_the_same_run(clusters):
    """Block steps alternate between two halves of the selection buffers
    (the step parity), and runs of 32 steps replay one graph that starts at
    parity 0.  Splitting 101 steps into calls of odd and even lengths, which
    changes which graphs run, must give the same bits as one call."""
    if clusters == 1:
        m, x, v = icgen.plummer(700, 61)
        eps, coff = 1.0 / 700, None
    else:
        m, x, v, coff, eps = icgen.ensemble(3, 15, 300, 900)
    banner(f"step call lengths, {clusters} cluster(s)")
    ref = _sim(m, x, v, eps, precision=1, coff=coff)
    ref.step(101, 0.5)
    a = ref.host_state()
    sim = _sim(m, x, v, eps, precision=1, coff=coff)
    for k in (1, 7, 33, 2, 32, 1, 25):
        sim.step(k, 0.5)
    b = sim.host_state()
    assert sim.status() == 0
    for key in a:
        assert np.array_equal(a[key], b[key]), key
    for u, w in zip(ref.progress(), sim.progress()):
        assert np.array_equal(u, w)
    ref.close()
    sim.close()


@pytest.mark.parametrize("clusters", [1, 3], ids=["one_cluster", "three_clusters"])
def test_tuning_change_between_step_calls(clusters):
    """A run whose slicing target and layout thresholds change between two
    step calls continues exactly as a run restarted from a checkpoint with
    the new tuning (the carried-over selection state must not assume the
    old plan)."""
    if clusters == 1:
        m, x, v = icgen.plummer(4096, 62)
        eps, coff = 1.0 / 4096, None
    else:
        m, x, v, coff, eps = icgen.ensemble(3, 16, 300, 900)
    banner(f"tuning change, {clusters} cluster(s)")
    # fewer j-slices per block (so the reduction's units change) and other
    # layouts; the change comes right after the block at t = 1/8, where every
    # particle is active, so the carried-over state spans many reduce units
    new = dict(target_items=8, min_block=[8192, 8192, 8, 2], small_cluster_n=0)
    probe = _sim(m, x, v, eps, precision=1, coff=coff)
    probe.run(0.125)
    k = int(probe.progress()[1].max())  # replays up to and including the block at t = 1/8
    probe.close()
    a = _sim(m, x, v, eps, precision=1, coff=coff)
    a.step(k, 0.125)
    blob = a.get_state()
    a.set_tuning(**new)
    a.step(60, 0.25)
    b = _sim(m, x, v, eps, precision=1, coff=coff)
    b.set_state(blob)
    b.set_tuning(**new)
    b.step(60, 0.25)
    sa, sb = a.host_state(), b.host_state()
    assert a.status() == 0 and b.status() == 0
    for key in sa:
        assert np.array_equal(sa[key], sb[key]), key
    for u, w in zip(a.progress(), b.progress()):
        assert np.array_equal(u, w)
    a.close()
    b.close()


def test_batched_clusters_match_single_runs():
    """Four clusters advanced together: every cluster is bit-identical to the
    same cluster integrated alone (plans depend only on a cluster's own sizes)."""
    m, x, v, coff, eps = icgen.ensemble(4, 6, 256, 1200)
    banner("batched vs single")
    both = _sim(m, x, v, eps, coff=coff)
    both.run(0.25, chunk=128)
    sb = both.host_state()
    tb, nb_steps, _ = both.progress()
    assert np.all(tb == 0.25)
    for c in range(4):
        b, e = int(coff[c]), int(coff[c + 1])
        one = _sim(m[b:e], x[:, b:e], v[:, b:e], eps[c])
        one.run(0.25, chunk=128)
        so = one.host_state()
        for key in ("x", "v", "a", "k"):
            assert np.array_equal(sb[key][:, b:e], so[key]), (c, key)
        assert np.array_equal(sb["dt"][b:e], so["dt"])
        assert one.progress()[1][0] == nb_steps[c]
        one.close()
    both.close()


def test_batched_mixed_clusters_match_single_runs():
    """Mixed precision with the one-lane-per-i layout from blocks of 256 on:
    in the batch every selection counts block sizes and forms the tile frames
    of the blocks that take that layout, while the 200-particle cluster run
    alone never reaches it (split-only build, no counting).  Every cluster
    stays bit-identical to the same cluster integrated alone."""
    sizes = (200, 700, 1200)
    parts = [icgen.plummer(n, 70 + n) for n in sizes]
    m = np.concatenate([p[0] for p in parts])
    x = np.concatenate([p[1] for p in parts], axis=1)
    v = np.concatenate([p[2] for p in parts], axis=1)
    coff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    eps = np.array([1.0 / n for n in sizes])
    tuning = dict(small_cluster_n=0, min_block=[1 << 30, 256, 48, 12])
    banner("batched vs single, mixed, one lane per i from 256")
    both = _sim(m, x, v, eps, precision=1, coff=coff)
    both.set_tuning(**tuning)
    both.run(0.25, chunk=128)
    assert both.status() == 0
    sb = both.host_state()
    _, nb_steps, _ = both.progress()
    for c in range(len(sizes)):
        b, e = int(coff[c]), int(coff[c + 1])
        one = _sim(m[b:e], x[:, b:e], v[:, b:e], eps[c], precision=1)
        one.set_tuning(**tuning)
        one.run(0.25, chunk=128)
        assert one.status() == 0
        so = one.host_state()
        for key in ("x", "v", "a", "k"):
            assert np.array_equal(sb[key][:, b:e], so[key]), (c, key)
        assert np.array_equal(sb["dt"][b:e], so["dt"])
        assert one.progress()[1][0] == nb_steps[c]
        one.close()
    both.close()


def test_finished_batch_idles_then_continues():
    """Clusters of a batch that have reached the end time take no step: more
    step calls leave every bit of the state and the step counts alone, and a
    later call with a larger end time carries on exactly as a run that never
    stopped (t = 1/4 is a multiple of dt_max = 1/8, so every particle lands on
    it in both runs)."""
    m, x, v, coff, eps = icgen.ensemble(5, 21, 64, 700)
    banner("finished batch idles then continues")
    sim = _sim(m, x, v, eps, coff=coff)
    sim.run(0.25, chunk=64)
    a = sim.host_state()
    pa = [np.array(u, copy=True) for u in sim.progress()]
    assert np.all(pa[0] == 0.25)
    for n_steps in (1, 7, 64):
        sim.step(n_steps, 0.25)
    b = sim.host_state()
    for key in a:
        assert np.array_equal(a[key], b[key]), key
    for u, w in zip(pa, sim.progress()):
        assert np.array_equal(u, w)
    sim.run(0.5, chunk=64)
    ref = _sim(m, x, v, eps, coff=coff)
    ref.run(0.5, chunk=64)
    c, d = sim.host_state(), ref.host_state()
    for key in c:
        assert np.array_equal(c[key], d[key]), key
    for u, w in zip(sim.progress(), ref.progress()):
        assert np.array_equal(u, w)
    sim.close()
    ref.close()


def test_status_reports_step_underflow():
    """Two bodies 1e-9 apart with no softening need steps far below dt_min = 2^-20."""
    m = np.array([0.5, 0.5])
    x = np.array([[0.0, 1e-9], [0.0, 0.0], [0.0, 0.0]])
    v = np.array([[0.0, 0.0], [-1e-3, 1e-3], [0.0, 0.0]])
    banner("dt underflow")
    sim = _sim(m, x, v, 0.0, dt_min=2.0**-20)
    assert sim.status() == -5
    sim.close()


@pytest.mark.parametrize("case", ["single_mixed", "batch_fp64"])
def test_device_error_freezes_the_state(case):
    """After a new step falls below dt_min, later block steps change nothing.
    A run stepped one block step at a time finds the failing step; the state
    after it is bitwise the state after many more steps enqueued at once,
    before the host has read the error (the device freezes itself), and
    nbody_step returns the error once nbody_sync has read it.  Restoring an
    earlier checkpoint clears the error and the run continues."""
    import paper_0711_0643_amd as nb

    if case == "single_mixed":
        m, x, v = icgen.plummer(1024, 41)
        eps, coff, prec = 1.0 / 1024, None, 1
    else:
        m, x, v, coff, eps = icgen.ensemble(3, 14, 300, 900)
        prec = 0
    t_end = 0.25
    banner(f"device error freezes the state {case}")

    def prefix():
        sim = _sim(m, x, v, eps, precision=prec, coff=coff)
        sim.step(150, t_end)
        assert sim.status() == 0
        good = sim.get_state()
        dt_floor = float(sim.host_state()["dt"].min())
        # every particle with a step this small fails at its next correction
        sim.set_params(dt_min=4.0 * dt_floor)
        return sim, good

    a, good = prefix()
    k = 0
    while k < 4000:
        a.step(1, t_end)
        k += 1
        if a.status() != 0:
            break
    assert a.status() == nb.NBODY_E_DTMIN, k
    frozen = a.get_state()
    prog = a.progress()
    with pytest.raises(nb.NBodyError) as err:
        a.step(8, t_end)
    assert err.value.code == nb.NBODY_E_DTMIN
    assert a.get_state() == frozen

    b, _ = prefix()
    b.step(k + 70, t_end)  # the error has not been read yet: enqueued
    assert b.status() == nb.NBODY_E_DTMIN
    assert b.get_state() == frozen
    for u, w in zip(prog, b.progress()):
        assert np.array_equal(u, w)

    # recovery: the checkpoint before the failure, the original floor
    b.set_state(good)
    b.set_params(dt_min=2.0**-40)
    b.step(20, t_end)
    assert b.status() == 0
    ref = _sim(m, x, v, eps, precision=prec, coff=coff)
    ref.step(150, t_end)
    ref.step(20, t_end)
    assert ref.get_state() == b.get_state()
    for s_ in (a, b, ref):
        s_.close()


def test_api_calls_between_steps_leave_the_run_unchanged():
    """The step pipeline carries the next block time over from one step to
    the next; calls that replace the plan or read the state in between
    (force on some list, energy, predict, checkpoint) must not change the
    trajectory: the run is bit-identical to one without them."""
    import torch

    m, x, v, coff, eps = icgen.ensemble(3, 14, 300, 900)
    banner("api calls between steps")
    ref = _sim(m, x, v, eps, precision=1, coff=coff)
    ref.step(50, 0.25)
    ref.step(50, 0.25)
    a = ref.host_state()
    sim = _sim(m, x, v, eps, precision=1, coff=coff)
    sim.step(50, 0.25)
    act = np.concatenate([np.arange(int(coff[c]), int(coff[c]) + 5, dtype=np.int32) for c in range(3)])
    sim.force(act, np.array([0, 5, 10, 15], dtype=np.int64))
    sim.energy()
    sim.predict(None)
    blob = sim.get_state()
    sim.set_state(blob)
    torch.cuda.synchronize()
    sim.step(50, 0.25)
    b = sim.host_state()
    for key in a:
        assert np.array_equal(a[key], b[key]), key
    for u, w in zip(ref.progress(), sim.progress()):
        assert np.array_equal(u, w)
    ref.close()
    sim.close()


def test_diagnostics_match_oracle():
    """Kinetic and potential energy, momentum and angular momentum of every
    cluster at a synchronised time against the oracle's diagnostics of the
    same state."""
    m, x, v, coff, eps = icgen.ensemble(3, 21, 300, 1200)
    banner("diagnostics")
    sim = _sim(m, x, v, eps, precision=1, coff=coff)
    sim.run(0.125, chunk=128)
    d = sim.diagnostics()
    st = sim.host_state()
    assert np.all(st["t"] == 0.125)
    for c in range(3):
        b, e = int(coff[c]), int(coff[c + 1])
        ref = oracle.diagnostics(m[b:e], st["x"][:, b:e], st["v"][:, b:e], eps[c])
        for key in ("KE", "PE", "E"):
            assert abs(d[key][c] - ref[key]) <= 1e-13 * abs(ref[key]), (c, key, d[key][c], ref[key])
        scale_p = float(np.sum(m[b:e] * np.linalg.norm(st["v"][:, b:e], axis=0)))
        scale_l = float(np.sum(m[b:e] * np.linalg.norm(st["x"][:, b:e], axis=0) * np.linalg.norm(st["v"][:, b:e], axis=0)))
        assert np.max(np.abs(d["P"][c] - ref["P"])) <= 1e-14 * scale_p
        assert np.max(np.abs(d["L"][c] - ref["L"])) <= 1e-14 * scale_l
    assert np.allclose(sim.energy(), d["E"], rtol=0, atol=0)
    sim.close()


def test_batch_with_tiny_clusters_follows_oracle():
    """A batch with clusters of 1, 2 and 3 particles beside larger ones
    (one cluster per selection chunk and one spanning several): every
    cluster, integrated in FP64 through the step graph to t = 1/4, takes
    the oracle's block steps and ends at the oracle's state."""
    rng = np.random.default_rng(77)
    sizes = [1, 2, 3, 700, 1, 2500]
    ms, xs, vs, eps = [], [], [], []
    for n in sizes:
        if n < 10:  # a few softened bodies
            m = rng.random(n) + 0.5
            m /= m.sum()
            xc, vc = rng.standard_normal((3, n)), rng.standard_normal((3, n)) * 0.3
            eps.append(0.05)
        else:
            m, xc, vc = icgen.plummer(n, 90 + n)
            eps.append(1.0 / n)
        ms.append(m)
        xs.append(xc)
        vs.append(vc)
    m = np.concatenate(ms)
    x = np.concatenate(xs, axis=1)
    v = np.concatenate(vs, axis=1)
    coff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    banner("tiny clusters in a batch")
    sim = _sim(m, x, v, np.array(eps), coff=coff)
    sim.run(0.25, chunk=256)
    assert sim.status() == 0
    st = sim.host_state()
    t, steps, inter = sim.progress()
    assert np.all(t == 0.25)
    for c, n in enumerate(sizes):
        b, e = int(coff[c]), int(coff[c + 1])
        ref = oracle.Sim(ms[c], xs[c], vs[c], eps[c])
        ref.run(0.25)
        assert steps[c] == ref.steps, (c, steps[c], ref.steps)
        assert inter[c] == ref.interactions
        assert np.max(np.abs(st["x"][:, b:e] - ref.x)) < 1e-9
        assert np.max(np.abs(st["v"][:, b:e] - ref.v)) < 1e-9
    sim.close()


def test_many_tiny_clusters():
    """2000 clusters of 3 .. 30 softened bodies (more clusters than the plan
    kernel's workgroup has threads, one selection chunk each) to t = 1/8 in
    FP64: six clusters checked against the oracle run alone."""
    rng = np.random.default_rng(5)
    sizes = rng.integers(3, 31, size=2000)
    ms, xs, vs = [], [], []
    for n in sizes:
        m = rng.random(n) + 0.5
        ms.append(m / m.sum())
        xs.append(rng.standard_normal((3, n)))
        vs.append(rng.standard_normal((3, n)) * 0.3)
    m = np.concatenate(ms)
    x = np.concatenate(xs, axis=1)
    v = np.concatenate(vs, axis=1)
    coff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    eps = np.full(sizes.size, 0.1)
    banner("2000 tiny clusters")
    sim = _sim(m, x, v, eps, coff=coff)
    sim.run(0.125, chunk=256)
    assert sim.status() == 0
    st = sim.host_state()
    t, steps, inter = sim.progress()
    assert np.all(t == 0.125)
    for c in (0, 1, 777, 1500, 1998, 1999):
        b, e = int(coff[c]), int(coff[c + 1])
        ref = oracle.Sim(ms[c], xs[c], vs[c], 0.1)
        ref.run(0.125)
        assert steps[c] == ref.steps and inter[c] == ref.interactions, c
        assert np.max(np.abs(st["x"][:, b:e] - ref.x)) < 1e-11
    sim.close()
