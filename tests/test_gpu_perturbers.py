"""Perturber lists (Sect. 3.1) from the HIP path against the oracle, bit for
bit: the same ids in the same (serial identification) order and the same
counts (GPU).  Every case runs on the initial state, where the predicted
positions are the given ones on both sides."""
import numpy as np
import pytest

import icgen
import oracle
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu


def _mean_acc(m, x, v, eps):
    a = oracle.force(m, x, v, eps)[0]
    return float(np.linalg.norm(a, axis=0).mean())


@pytest.mark.parametrize("frac,cap", [(1e-2, 256), (1e-4, 256), (1e-2, 16), (3.0, 256)])
def test_perturbers_match_oracle_one_cluster(frac, cap):
    import paper_0711_0643_amd as nb

    n = 4096
    m, x, v = icgen.plummer(n, 77)
    eps = 1.0 / n
    thr = frac * _mean_acc(m, x, v, eps)
    banner(f"perturbers N={n} threshold={frac}<|a|> cap={cap}")
    sim = nb.Sim(m, x, v, eps, precision=1)
    act = icgen.active_subset(n, 700, seed=3)
    lists, counts = sim.perturbers(act, [thr], max_pert=cap)
    rl, rc = oracle.perturbers(m, x, eps, thr, act, cap)
    assert sim.status() == 0
    assert np.array_equal(counts.cpu().numpy(), rc)
    assert np.array_equal(lists.cpu().numpy(), rl)
    sim.close()


def test_perturbers_batch_with_ragged_blocks():
    """Five clusters, each with its own threshold and active subset (one
    empty): each cluster's lists are the oracle's on that cluster alone,
    shifted by the cluster's first id."""
    import paper_0711_0643_amd as nb

    m, x, v, coff, eps = icgen.ensemble(5, 8, 256, 1500)
    banner("perturbers batch of 5")
    sim = nb.Sim(m, x, v, eps, cluster_offsets=coff, precision=0)
    acts, aoff, thr = [], [0], []
    picks = [40, 0, 300, 1, 256]
    for c in range(5):
        b, e = int(coff[c]), int(coff[c + 1])
        sub = icgen.active_subset(e - b, min(picks[c], e - b), seed=20 + c) + b
        acts.append(sub)
        aoff.append(aoff[-1] + sub.size)
        thr.append(0.05 * _mean_acc(m[b:e], x[:, b:e], v[:, b:e], eps[c]))
    act = np.concatenate(acts).astype(np.int32)
    lists, counts = sim.perturbers(act, thr, active_offsets=np.array(aoff, dtype=np.int64), max_pert=64)
    lists, counts = lists.cpu().numpy(), counts.cpu().numpy()
    assert sim.status() == 0
    for c in range(5):
        b, e = int(coff[c]), int(coff[c + 1])
        s = slice(aoff[c], aoff[c + 1])
        rl, rc = oracle.perturbers(m[b:e], x[:, b:e], eps[c], thr[c], acts[c] - b, 64)
        assert np.array_equal(counts[s], rc), c
        assert np.array_equal(np.where(lists[s] >= 0, lists[s] - b, -1), rl), c
    sim.close()


def test_perturbers_full_block_n65536_sampled():
    """Plummer N = 65536, every particle listed (the full block): 512 seeded
    sample entries against the oracle one by one."""
    import paper_0711_0643_amd as nb

    n = 65536
    m, x, v = icgen.plummer(n, 3)
    eps = 1.0 / n
    thr = 0.01 * _mean_acc(m, x, v, eps)
    banner("perturbers N=65536 full block")
    sim = nb.Sim(m, x, v, eps, precision=1)
    act = np.arange(n, dtype=np.int32)
    lists, counts = sim.perturbers(act, [thr])
    lists, counts = lists.cpu().numpy(), counts.cpu().numpy()
    assert sim.status() == 0
    sample = np.sort(np.random.default_rng(9).choice(n, 512, replace=False)).astype(np.int32)
    rl, rc = oracle.perturbers(m, x, eps, thr, sample, 256)
    assert np.array_equal(counts[sample], rc)
    assert np.array_equal(lists[sample], rl)
    assert counts.max() > 0
    sim.close()


def test_perturbers_edge_cases():
    """An empty active list is a no-op; max_pert outside 1..256 is rejected
    on the host; an id outside its cluster is reported and gets an empty
    list."""
    import torch

    import paper_0711_0643_amd as nb

    m, x, v, coff, eps = icgen.ensemble(2, 9, 100, 300)
    sim = nb.Sim(m, x, v, eps, cluster_offsets=coff, precision=0)
    thr = [0.1, 0.1]
    lists, counts = sim.perturbers(np.zeros(0, dtype=np.int32), thr, active_offsets=np.zeros(3, dtype=np.int64))
    assert lists.shape == (0, 256) and counts.shape == (0,)
    for bad in (0, 257):
        with pytest.raises(nb.NBodyError):
            sim.perturbers(np.array([0], dtype=np.int32), thr, active_offsets=np.array([0, 1, 1]), max_pert=bad)
    # id of cluster 1 listed under cluster 0
    wrong = np.array([int(coff[1])], dtype=np.int32)
    lists, counts = sim.perturbers(wrong, thr, active_offsets=np.array([0, 1, 1], dtype=np.int64), max_pert=8)
    torch.cuda.synchronize()
    assert sim.status() == nb.NBODY_E_INDEX
    assert counts.cpu().numpy()[0] == 0 and np.all(lists.cpu().numpy() == -1)
    sim.close()


def test_perturbers_offsets_ending_before_the_list():
    """Active offsets whose last entry is below n_active: the entries past
    it belong to no cluster, are reported and get empty lists; the one
    entry inside matches the oracle."""
    import torch

    import paper_0711_0643_amd as nb

    m, x, v, coff, eps = icgen.ensemble(2, 9, 100, 300)
    sim = nb.Sim(m, x, v, eps, cluster_offsets=coff, precision=0)
    act = np.array([3, 5, 7], dtype=np.int32)
    lists, counts = sim.perturbers(act, [0.05, 0.05], active_offsets=np.array([0, 1, 1], dtype=np.int64),
                                   max_pert=32)
    torch.cuda.synchronize()
    assert sim.status() == nb.NBODY_E_INDEX
    lists, counts = lists.cpu().numpy(), counts.cpu().numpy()
    b, e = int(coff[0]), int(coff[1])
    rl, rc = oracle.perturbers(m[b:e], x[:, b:e], eps[0], 0.05, np.array([3 - b], dtype=np.int32), 32)
    assert counts[0] == rc[0] and np.array_equal(np.where(lists[0] >= 0, lists[0] - b, -1), rl[0])
    assert np.all(counts[1:] == 0) and np.all(lists[1:] == -1)
    sim.close()


def test_perturbers_thresholds_at_a_pairs_term():
    """Thresholds at one pair's own term m_j / R^2 (formed in the same
    operation order), one unit in the last place either side, and just
    inside and outside a relative band of 2^-40 around it: the lists match
    the oracle's bit for bit, the pair is left out at equality and listed
    one unit below (the test is a strict inequality on the rounded
    quotient)."""
    import paper_0711_0643_amd as nb

    n = 512
    m, x, v = icgen.plummer(n, 31)
    eps = 1.0 / n
    i = 7
    d = x - x[:, i:i + 1]
    r2 = ((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]) + eps * eps
    terms = m / r2
    terms[i] = -np.inf
    j = int(np.argsort(terms)[-3])  # a pair near the top of i's list
    t0 = float(m[j] / r2[j])
    act = np.array([i, j, 0, n - 1], dtype=np.int32)
    sim = nb.Sim(m, x, v, eps, precision=0)
    cases = [t0, np.nextafter(t0, 0.0), np.nextafter(t0, np.inf), t0 * (1 + 2.0**-41), t0 * (1 - 2.0**-41),
             t0 * (1 + 2.0**-39), t0 * (1 - 2.0**-39)]
    banner(f"perturbers threshold at the term of pair ({i}, {j})")
    for thr in cases:
        lists, counts = sim.perturbers(act, [thr], max_pert=64)
        rl, rc = oracle.perturbers(m, x, eps, thr, act, 64)
        assert sim.status() == 0
        assert np.array_equal(counts.cpu().numpy(), rc), thr
        assert np.array_equal(lists.cpu().numpy(), rl), thr
    row = lambda thr: sim.perturbers(act, [thr], max_pert=64)[0].cpu().numpy()[0]
    assert j not in row(t0)
    assert j in row(np.nextafter(t0, 0.0))
    sim.close()
