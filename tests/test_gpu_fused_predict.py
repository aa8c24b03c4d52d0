"""Prediction in the force pass (Sect. 2.1: the prediction may run on the
accelerator; tuning switch pred_in_force): block steps whose block fills a
single i-chunk of a j-split layout predict only the block's members in the
selection, and the force pass predicts its j-records itself with the same
arithmetic.  The integration must be bitwise the one with the switch off
(GPU); the stored prediction of the non-members, left at an earlier time
by such steps, shows that they ran."""
import numpy as np
import pytest

import icgen
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu


def _pair(make, precision):
    import paper_0711_0643_amd as nb

    a = make(nb, precision)
    b = make(nb, precision)
    b.set_tuning(pred_in_force=1)
    assert b.get_tuning()["pred_in_force"] == 1 and a.get_tuning()["pred_in_force"] == 0
    return a, b


def _run_pair(a, b, steps, t_end):
    import torch

    fused = 0
    for s in range(steps):
        a.step(1, t_end)
        b.step(1, t_end)
        torch.cuda.synchronize()
        if not torch.equal(a.xp, b.xp):
            fused += 1
        assert a.get_state() == b.get_state(), f"state differs after step {s}"
    assert a.status() == 0 and b.status() == 0
    return fused


def _single(n, pot=False):
    def make(nb, precision):
        m, x, v = icgen.plummer(n, 41)
        return nb.Sim(m, x, v, 1.0 / n, precision=precision, compute_pot=pot)
    return make


@pytest.mark.parametrize("n,precision,pot", [(4096, 0, False), (4096, 1, False), (20000, 1, False),
                                             (20000, 0, False), (20000, 1, True), (4096, 0, True)])
def test_fused_prediction_single_cluster_is_bitwise(n, precision, pot):
    """One Plummer cluster, FP64 and mixed, with and without the potential:
    N = 20000 runs the full kernels (one-lane-per-i and j-split layouts),
    N = 4096 the j-split-only builds, so every fused build runs.  60 single
    block steps, the state compared after each; then a direct force call on
    the stepped state."""
    import torch

    banner(f"fused prediction N={n} precision={precision} pot={pot}")
    a, b = _pair(_single(n, pot), precision)
    fused = _run_pair(a, b, 60, 1.0)
    assert fused > 0, "no step took the fused predictor"
    act = a.storage_active(300)
    fa, fb = a.force(act, pot=True), b.force(act, pot=True)
    torch.cuda.synchronize()
    for u, w in zip(fa, fb):
        assert torch.equal(u, w)
    assert a.status() == 0 and b.status() == 0
    a.close()
    b.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_fused_prediction_batch_is_bitwise(precision):
    """A ragged batch of six clusters (some small enough that most of their
    blocks fill one i-chunk): 40 replays of the step graph, state compared
    after each, and the run continued in 32-step graphs to t = 1/8."""
    def make(nb, prec):
        m, x, v, coff, eps = icgen.ensemble(6, 17, 64, 3000)
        return nb.Sim(m, x, v, eps, cluster_offsets=coff, precision=prec)

    banner(f"fused prediction batch precision={precision}")
    a, b = _pair(make, precision)
    fused = _run_pair(a, b, 40, 1.0)
    assert fused > 0, "no step took the fused predictor"
    a.run(0.125)
    b.run(0.125)
    assert a.get_state() == b.get_state()
    assert a.status() == 0 and b.status() == 0
    a.close()
    b.close()


def test_pred_in_force_switch_validation():
    import paper_0711_0643_amd as nb

    m, x, v = icgen.plummer(256, 5)
    sim = nb.Sim(m, x, v, 1.0 / 256, precision=0)
    for bad in (-1, 2):
        with pytest.raises(nb.NBodyError):
            sim.set_tuning(pred_in_force=bad)
    assert sim.get_tuning()["pred_in_force"] == 0
    sim.close()
