"""Parity of the HIP force pass with the FP64 oracle (GPU).

Inputs are seeded Plummer spheres (equal masses, eps = 1/N) and random
systems; the oracle recomputes a, k, phi from the same FP64 predicted state.

Tolerances:
  FP64 kernel  -- per particle |da|/|a|, |dk|/|k|, |dphi|/|phi| <= 1e-12
                  (summation order and FMA differ from the oracle's plain
                  j-ascending loop; 1e-12 leaves room for cancellation).
  mixed kernel -- acceleration and potential: per particle relative error
                  <= 1e-6 (the force-error bar).  Jerk: per particle relative
                  error <= 1e-6 for every particle whose jerk cancellation
                  kappa_k = K_i/|k_i| (K_i = sum of |jerk term|) is at most
                  10; every particle, whatever its kappa_k, within 1e-6 K_i.
                  FP32 pair terms carry a few units of u = 2^-24 each, so
                  the relative jerk error of a particle with strong
                  cancellation scales with kappa_k, which reaches a few
                  hundred in a Plummer sphere; those particles are counted
                  and reported by the benchmark rather than held to the
                  relative bar.
"""
import numpy as np
import pytest

import icgen
import oracle
from tests.gpu_util import banner, normwise_err, rel_err

pytestmark = pytest.mark.gpu


def _sim(m, x, v, eps, precision, coff=None, **kw):
    import paper_0711_0643_amd as nb

    sim = nb.Sim(m, x, v, eps, cluster_offsets=coff, precision=precision, **kw)
    if precision == 1:
        # every block in the one-lane-per-i layout, the one that runs the
        # tile-relative arithmetic (the split layouts run the FP64 one)
        sim.set_tuning(min_block=[1 << 30, 1, 1, 1], small_cluster_n=0)
    return sim


def _gpu_force(sim, act, aoff=None, pot=True):
    import torch

    acc, jerk, ph = sim.force(act, aoff, pot=pot)
    torch.cuda.synchronize()
    assert sim.status() == 0
    return acc.cpu().numpy(), jerk.cpu().numpy(), (ph.cpu().numpy() if ph is not None else None)


def _check_fp64(got, ref):
    a, k, p = got
    ra, rk, rp = ref
    assert rel_err(a, ra).max() <= 1e-12, rel_err(a, ra).max()
    assert rel_err(k, rk).max() <= 1e-12, rel_err(k, rk).max()
    if p is not None:
        assert rel_err(p, rp).max() <= 1e-12, rel_err(p, rp).max()


def _check_mixed(got, ref, absum):
    a, k, p = got
    ra, rk, rp = ref
    ea = rel_err(a, ra)
    assert ea.max() <= 1e-6, ea.max()
    ek_norm = normwise_err(k, rk, absum[1])
    assert ek_norm.max() <= 1e-6, ek_norm.max()
    kappa = absum[1] / np.maximum(np.linalg.norm(rk, axis=0), 1e-300)
    ek = rel_err(k, rk)
    low = kappa <= 10
    assert not low.any() or ek[low].max() <= 1e-6, (ek[low].max(), int((ek[low] > 1e-6).sum()))
    if p is not None:
        assert rel_err(p, rp).max() <= 1e-6, rel_err(p, rp).max()


SIZES = [(3, [1, 3]), (64, [1, 7, 40, 64]), (1000, [1, 13, 100, 256, 1000]), (3000, [50, 700, 3000])]


@pytest.mark.parametrize("n,acts", SIZES, ids=[f"N{n}" for n, _ in SIZES])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_force_plummer_matches_oracle(n, acts, precision):
    m, x, v = icgen.plummer(n, 100 + n)
    eps = 1.0 / n
    banner(f"force plummer N={n} precision={precision}")
    sim = _sim(m, x, v, eps, precision)
    for na in acts:
        act = icgen.active_subset(n, na, seed=7)
        banner(f"  n_act={na}")
        got = _gpu_force(sim, act)
        ref = oracle.force(m, x, v, eps, act)
        if precision == 0:
            _check_fp64(got, ref)
        else:
            _check_mixed(got, ref, oracle.force_abs(m, x, v, eps, act))
    sim.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_force_without_softening(precision):
    """eps = 0: the self pair must be dropped exactly (masked tiles)."""
    rng = np.random.default_rng(5)
    n = 700
    m = rng.random(n) + 0.5
    m /= m.sum()
    x = rng.standard_normal((3, n))
    v = rng.standard_normal((3, n)) * 0.3
    banner(f"force eps=0 N={n} precision={precision}")
    sim = _sim(m, x, v, 0.0, precision)
    act = icgen.active_subset(n, 333, seed=3)
    got = _gpu_force(sim, act)
    ref = oracle.force(m, x, v, 0.0, act)
    if precision == 0:
        _check_fp64(got, ref)
    else:
        _check_mixed(got, ref, oracle.force_abs(m, x, v, 0.0, act))
    sim.close()


def test_two_body_closed_form_on_gpu():
    m = np.array([0.25, 0.75])
    x = np.array([[0.0, 1.5], [0.0, 0.0], [0.0, 0.0]])
    v = np.zeros((3, 2))
    banner("two body fp64")
    sim = _sim(m, x, v, 0.0, 0)
    a, k, p = _gpu_force(sim, np.array([0, 1], dtype=np.int32))
    assert abs(a[0, 0] - 0.75 / 1.5**2) < 1e-16 and abs(a[0, 1] + 0.25 / 1.5**2) < 1e-16
    assert abs(p[0] + 0.75 / 1.5) < 1e-16
    assert np.all(k == 0)
    sim.close()


def test_single_particle_cluster_has_no_force():
    banner("single particle")
    sim = _sim(np.array([1.0]), np.zeros((3, 1)), np.ones((3, 1)), 0.01, 0)
    a, k, p = _gpu_force(sim, np.array([0], dtype=np.int32))
    assert np.all(a == 0) and np.all(k == 0) and np.all(p == 0)
    sim.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_clusters_are_independent(precision):
    """Several clusters in one pass: each matches the oracle run on that
    cluster alone, including an empty block in one cluster."""
    m, x, v, coff, eps = icgen.ensemble(5, 4, 256, 1500)
    banner(f"ensemble of 5 precision={precision}")
    sim = _sim(m, x, v, eps, precision, coff=coff)
    acts, aoff = [], [0]
    picks = [37, 0, 300, 1, 256]
    for c in range(5):
        nc = int(coff[c + 1] - coff[c])
        sub = icgen.active_subset(nc, min(picks[c], nc), seed=11 + c) + int(coff[c])
        acts.append(sub)
        aoff.append(aoff[-1] + sub.size)
    act = np.concatenate(acts).astype(np.int32)
    got = _gpu_force(sim, act, np.array(aoff, dtype=np.int64))
    for c in range(5):
        b, e = int(coff[c]), int(coff[c + 1])
        s = slice(aoff[c], aoff[c + 1])
        if aoff[c + 1] == aoff[c]:
            continue
        loc = acts[c] - b
        ref = oracle.force(m[b:e], x[:, b:e], v[:, b:e], eps[c], loc)
        part = (got[0][:, s], got[1][:, s], got[2][s])
        if precision == 0:
            _check_fp64(part, ref)
        else:
            _check_mixed(part, ref, oracle.force_abs(m[b:e], x[:, b:e], v[:, b:e], eps[c], loc))
    sim.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_force_is_deterministic(precision):
    m, x, v = icgen.plummer(4096, 9)
    banner(f"determinism precision={precision}")
    sim = _sim(m, x, v, 1 / 4096, precision)
    act = icgen.active_subset(4096, 1500)
    g1 = _gpu_force(sim, act)
    g2 = _gpu_force(sim, act)
    for u, w in zip(g1, g2):
        assert np.array_equal(u, w)
    sim.close()


def test_j_split_changes_only_rounding():
    """The paper's independence of the processor count: other slicings of j
    (target_items) agree to FP64 rounding, and the FP64 results stay on the
    oracle."""
    n = 5000
    m, x, v = icgen.plummer(n, 21)
    banner("j-split invariance")
    sim = _sim(m, x, v, 1 / n, 0)
    act = icgen.active_subset(n, 900)
    ref = oracle.force(m, x, v, 1 / n, act)
    base = None
    for target in (1, 7, 64, 2048, 16384):
        sim.set_tuning(target_items=target)
        got = _gpu_force(sim, act)
        _check_fp64(got, ref)
        if base is None:
            base = got
        else:
            assert rel_err(got[0], base[0]).max() < 1e-13
    sim.close()


def test_layout_variants_agree():
    """Every i x j layout (2 i per lane; 1, 4, 16, 64 lanes per i) gives the
    oracle's sums."""
    n = 2000
    m, x, v = icgen.plummer(n, 22)
    act = icgen.active_subset(n, 300)
    ref = oracle.force(m, x, v, 1 / n, act)
    sim = _sim(m, x, v, 1 / n, 0)
    big = 100000
    for mb in ([1, 1, 1, 1], [big, 1, 1, 1], [big, big, 1, 1], [big, big, big, 1], [big, big, big, big]):
        banner(f"layout min_block={mb}")
        sim.set_tuning(min_block=mb, small_cluster_n=0)
        _check_fp64(_gpu_force(sim, act), ref)
    sim.close()


def test_double_single_format_matches_oracle():
    """The mixed kernel with double-single positions (mixed_format = 0:
    dr = (hi_j - hi_i) + (lo_j - lo_i) in FP32) passes the mixed gate in
    every layout, in both kernel builds."""
    n = 3000
    m, x, v = icgen.plummer(n, 24)
    eps = 1.0 / n
    act = icgen.active_subset(n, 700, seed=9)
    ref = oracle.force(m, x, v, eps, act)
    absum = oracle.force_abs(m, x, v, eps, act)
    sim = _sim(m, x, v, eps, 1)
    big = 100000
    for mb in ([1, 1, 1, 1], [big, 1, 1, 1], [big, big, 1, 1], [big, big, big, 1], [big, big, big, big]):
        banner(f"double-single min_block={mb}")
        sim.set_tuning(min_block=mb, small_cluster_n=0, mixed_format=0)
        _check_mixed(_gpu_force(sim, act), ref, absum)
    sim.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_split_layout_kernel_matches_full_kernel_bitwise(precision):
    """When no cluster can reach a one-lane-per-i layout the library runs a
    kernel holding only the j-split layouts (higher occupancy).  For the same
    layout it must give the same bits as the kernel with every layout."""
    n = 2000
    m, x, v = icgen.plummer(n, 23)
    act = icgen.active_subset(n, 300)
    sim = _sim(m, x, v, 1 / n, precision)
    out = []
    for mb in ([100000, 100000, 1, 1], [n, n, 1, 1]):  # block of 300 -> 4 lanes per i in both
        banner(f"precision {precision} min_block={mb}")
        sim.set_tuning(min_block=mb, small_cluster_n=0)
        acc, jerk, _ = _gpu_force(sim, act, pot=False)
        out.append((acc, jerk))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    sim.close()


def test_empty_block_is_a_no_op():
    import paper_0711_0643_amd as nb

    m, x, v = icgen.plummer(100, 1)
    sim = _sim(m, x, v, 0.01, 0)
    banner("empty block")
    acc, jerk, _ = sim.force(np.zeros(0, dtype=np.int32))
    assert acc.shape == (3, 0)
    assert sim.status() == 0
    with pytest.raises(nb.NBodyError):
        sim.force(np.zeros(200, dtype=np.int32))  # more entries than particles
    sim.close()


def test_index_outside_cluster_is_reported():
    m, x, v, coff, eps = icgen.ensemble(2, 8, 256, 300)
    banner("bad index")
    sim = _sim(m, x, v, eps, 0, coff=coff)
    # entry of cluster 0 pointing into cluster 1
    act = np.array([0, int(coff[1]) + 3], dtype=np.int32)
    import torch

    acc, jerk, _ = sim.force(act, np.array([0, 2, 2], dtype=np.int64))
    torch.cuda.synchronize()
    assert sim.status() == -7
    assert np.all(acc.cpu().numpy()[:, 1] == 0)
    sim.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_full_size_n65536_all_particles(precision):
    """Plummer N = 65536, eps = 1/N, every particle active (the launch the
    benchmark times); every one of the 65536 results against the oracle."""
    n = 65536
    m, x, v = icgen.plummer(n, 3)
    eps = 1.0 / n
    banner(f"full size N=65536 precision={precision}")
    sim = _sim(m, x, v, eps, precision)
    act = np.arange(n, dtype=np.int32)
    got = _gpu_force(sim, act)
    ref = oracle.force(m, x, v, eps)
    if precision == 0:
        _check_fp64(got, ref)
    else:
        _check_mixed(got, ref, oracle.force_abs(m, x, v, eps))
    # Newton's third law over the whole system (equal masses): sum a = 0
    a = got[0]
    scale = np.abs(a).sum()
    assert np.abs(a.sum(axis=1)).max() <= (1e-13 if precision == 0 else 1e-6) * scale
    sim.close()


def test_mixed_near_pairs_in_fp64_fix_close_neighbours():
    """With the FP64 treatment of near pairs off, the FP32 error of a single
    dominant close-neighbour term exceeds 1e-6 relative for a few particles
    of the N = 65536 Plummer sphere; with it on (default) none does."""
    n = 65536
    m, x, v = icgen.plummer(n, 3)
    eps = 1.0 / n
    banner("near pairs on/off")
    sim = _sim(m, x, v, eps, 1)
    act = np.arange(n, dtype=np.int32)
    ref = oracle.force(m, x, v, eps)
    ea_on = rel_err(_gpu_force(sim, act)[0], ref[0])
    sim.set_tuning(near_tau=0.0)
    ea_off = rel_err(_gpu_force(sim, act)[0], ref[0])
    assert ea_on.max() <= 1e-6
    assert ea_off.max() > ea_on.max()
    sim.close()


def test_mixed_mid_pairs_fix_pairs_close_against_their_tile():
    """A pair much closer than its tile is large loses part of its distance
    in tile-relative FP32 coordinates (error about u L / R) although its term
    is below the near threshold.  On the N = 65536 Plummer sphere, with the
    mid replacement off (mid_tau huge) jerks with kappa_k <= 10 miss 1e-6;
    with it on (default), and with the close pairs of nearly every window
    replaced (mid_tau = 0.01), acceleration and those jerks pass."""
    n = 65536
    m, x, v = icgen.plummer(n, 3)
    eps = 1.0 / n
    banner("mid pairs on/off")
    sim = _sim(m, x, v, eps, 1)
    act = np.arange(n, dtype=np.int32)
    ref = oracle.force(m, x, v, eps)
    kappa = oracle.force_abs(m, x, v, eps)[1] / np.linalg.norm(ref[1], axis=0)
    errs = {}
    for tau in (4.0, 0.01, 1e30):
        sim.set_tuning(mid_tau=tau)
        a, k, _ = _gpu_force(sim, act)
        assert sim.status() == 0
        errs[tau] = (rel_err(a, ref[0]).max(), rel_err(k, ref[1])[kappa <= 10].max())
    for tau in (4.0, 0.01):
        assert errs[tau][0] <= 1e-6 and errs[tau][1] <= 1e-6, (tau, errs[tau])
    assert errs[1e30][1] > 1e-6, errs[1e30]
    sim.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_king_salpeter_n262144_full_block_sampled(precision):
    """King W0 = 6 with Salpeter masses, N = 262144, eps = 1/N, every
    particle active (the largest workload, default launch configuration):
    2048 seeded sample particles against the oracle, one by one.  Unequal
    masses exercise the near-pair window test with a spread of m_j."""
    n = 262144
    m, x, v = icgen.king(n, 6.0, 5)
    eps = 1.0 / n
    banner(f"King+Salpeter N={n} full block precision={precision}")
    sim = _sim(m, x, v, eps, precision)
    got = _gpu_force(sim, np.arange(n, dtype=np.int32))
    sample = np.sort(np.random.default_rng(3).choice(n, 2048, replace=False)).astype(np.int32)
    ref = oracle.force(m, x, v, eps, sample)
    part = (got[0][:, sample], got[1][:, sample], got[2][sample])
    if precision == 0:
        _check_fp64(part, ref)
    else:
        _check_mixed(part, ref, oracle.force_abs(m, x, v, eps, sample))
    sim.close()


def test_plummer_n1048576_sampled():
    """The largest single cluster tested: Plummer N = 2^20, eps = 1/N, a
    block of 4096 active particles (2 i per lane, 1024 tiles per slice row);
    256 seeded entries of it against the oracle, one by one, in both
    precisions, plus a few block steps that must stay error free."""
    n = 1 << 20
    m, x, v = icgen.plummer(n, 8)
    eps = 1.0 / n
    act = icgen.active_subset(n, 4096, seed=11)
    pick = np.sort(np.random.default_rng(4).choice(act.size, 256, replace=False))
    sample = act[pick]
    ref = oracle.force(m, x, v, eps, sample)
    absum = oracle.force_abs(m, x, v, eps, sample)
    for precision in (0, 1):
        banner(f"Plummer N={n} block 4096 precision={precision}")
        sim = _sim(m, x, v, eps, precision)
        got = _gpu_force(sim, act)
        part = (got[0][:, pick], got[1][:, pick], got[2][pick])
        if precision == 0:
            _check_fp64(part, ref)
        else:
            _check_mixed(part, ref, absum)
        sim.step(3, 0.125)
        assert sim.status() == 0
        sim.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_batch_of_256_clusters_ragged_blocks(precision):
    """The 256-cluster batch (N log-uniform in [256, 8192], sum 673038), a
    ragged block in every cluster (1 .. N_c entries; cluster 5 has none), in
    one force pass; 24 seeded clusters checked entry by entry against the
    oracle run on that cluster alone."""
    m, x, v, coff, eps = icgen.ensemble(256, 4)
    nc = 256
    rng = np.random.default_rng(17)
    acts, aoff = [], [0]
    for c in range(nc):
        nn = int(coff[c + 1] - coff[c])
        na = 0 if c == 5 else int(rng.integers(1, nn + 1))
        sub = icgen.active_subset(nn, na, seed=1000 + c) + int(coff[c]) if na else np.zeros(0, np.int32)
        acts.append(sub.astype(np.int32))
        aoff.append(aoff[-1] + na)
    act = np.concatenate(acts).astype(np.int32)
    banner(f"batch of 256 clusters, {act.size} active, precision={precision}")
    sim = _sim(m, x, v, eps, precision, coff=coff)
    got = _gpu_force(sim, act, np.array(aoff, dtype=np.int64))
    for c in sorted(rng.choice(nc, 24, replace=False)):
        b, e = int(coff[c]), int(coff[c + 1])
        s = slice(aoff[c], aoff[c + 1])
        if aoff[c + 1] == aoff[c]:
            continue
        loc = acts[c] - b
        ref = oracle.force(m[b:e], x[:, b:e], v[:, b:e], eps[c], loc)
        part = (got[0][:, s], got[1][:, s], got[2][s])
        if precision == 0:
            _check_fp64(part, ref)
        else:
            _check_mixed(part, ref, oracle.force_abs(m[b:e], x[:, b:e], v[:, b:e], eps[c], loc))
    sim.close()


def test_split_layouts_of_the_mixed_mode_run_the_fp64_arithmetic():
    """In the tile-relative format the layouts that split j over lanes
    (blocks below min_block[1], 1024 by default) run the FP64 arithmetic:
    the same bits as the FP64 precision, in a single cluster and in a batch
    beside a cluster whose block runs the mixed arithmetic."""
    import torch

    import paper_0711_0643_amd as nb

    n = 20000
    m, x, v = icgen.plummer(n, 44)
    eps = 1.0 / n
    banner("mixed small blocks in FP64")
    mixed = nb.Sim(m, x, v, eps, precision=1)
    fp64 = nb.Sim(m, x, v, eps, precision=0)
    assert mixed.get_tuning()["min_block"][1] == 1024
    for na in (1, 7, 30, 200, 1023):
        act = icgen.active_subset(n, na, seed=na)
        got = mixed.force(act, pot=True)
        ref = fp64.force(act, pot=True)
        torch.cuda.synchronize()
        for u, w in zip(got, ref):
            assert torch.equal(u, w), na
    act = icgen.active_subset(n, 1024, seed=3)
    got = [t.cpu().numpy() for t in mixed.force(act, pot=True)]
    ref = [t.cpu().numpy() for t in fp64.force(act, pot=True)]
    assert not np.array_equal(got[0], ref[0])  # the mixed arithmetic from 1024 on
    assert rel_err(got[0], ref[0]).max() <= 1e-6
    mixed.close()
    fp64.close()

    # a batch: a cluster of 20000 with a block of 4096 (mixed arithmetic)
    # beside clusters of 300 and 900 with small blocks (FP64 arithmetic)
    parts = [icgen.plummer(k, 50 + k) for k in (20000, 300, 900)]
    m = np.concatenate([p[0] for p in parts])
    x = np.concatenate([p[1] for p in parts], axis=1)
    v = np.concatenate([p[2] for p in parts], axis=1)
    coff = np.array([0, 20000, 20300, 21200], dtype=np.int64)
    eps = np.array([1.0 / 20000, 1.0 / 300, 1.0 / 900])
    act = np.concatenate([np.arange(4096), 20000 + np.arange(5), 20300 + np.arange(300)]).astype(np.int32)
    aoff = np.array([0, 4096, 4101, 4401], dtype=np.int64)
    mixed = nb.Sim(m, x, v, eps, cluster_offsets=coff, precision=1)
    fp64 = nb.Sim(m, x, v, eps, cluster_offsets=coff, precision=0)
    got = [t.cpu().numpy() for t in mixed.force(act, aoff)[:2]]
    ref = [t.cpu().numpy() for t in fp64.force(act, aoff)[:2]]
    for u, w in zip(got, ref):
        assert np.array_equal(u[:, 4096:], w[:, 4096:])  # the small blocks: FP64 bits
    assert not np.array_equal(got[0][:, :4096], ref[0][:, :4096])
    assert rel_err(got[0][:, :4096], ref[0][:, :4096]).max() <= 1e-6
    mixed.close()
    fp64.close()
