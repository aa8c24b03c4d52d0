"""nbody_force_noalloc (the force pass with its slice partials in the
library's static device scratch, for callers that cannot allocate) against
nbody_force on the same context: two calls in a row, the second with a
smaller active list, must give the same bits as nbody_force gives for each
list; a call whose pass could outgrow the scratch is refused."""
import numpy as np
import pytest

import icgen
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu


def _lists(sim, coff, sizes, seed):
    """Active lists of `sizes[c]` particles of each cluster c, and offsets."""
    import torch

    rng = np.random.default_rng(seed)
    ids = [int(coff[c]) + np.sort(rng.choice(int(coff[c + 1] - coff[c]), size=k, replace=False))
           for c, k in enumerate(sizes)]
    act = np.concatenate(ids).astype(np.int32)
    aoff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return torch.as_tensor(act, device=sim.device), torch.as_tensor(aoff, device=sim.device)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("case", ["plummer_n65536", "batch_of_3"])
def test_noalloc_force_matches_force(case, precision):
    import torch

    import paper_0711_0643_amd as nb

    if case == "plummer_n65536":
        n = 65536
        m, x, v = icgen.plummer(n, 3)
        coff, eps = np.array([0, n]), 1.0 / n
        big, small = [n], [1000]
    else:
        m, x, v, coff, eps = icgen.ensemble(3, 14, 300, 900)
        sizes = np.diff(coff)
        big, small = [int(k) for k in sizes], [5, 1, 37]
    banner(f"no-alloc force {case} precision={precision}")
    sim = nb.Sim(m, x, v, eps, cluster_offsets=coff if case != "plummer_n65536" else None, precision=precision)
    sim.step(20, 0.125)  # a state after block steps (partial prediction)
    lists = [_lists(sim, coff, big, 1), _lists(sim, coff, small, 2)]
    if case == "plummer_n65536":
        lists[0] = (sim.storage_active(), lists[0][1])  # the full block in storage order, as the bench times it
    ref = [sim.force(a, o, pot=True) for a, o in lists]
    got = [sim.force_noalloc(a, o, pot=True) for a, o in lists]  # two calls in a row, the second smaller
    torch.cuda.synchronize()
    assert sim.status() == 0
    for r, g in zip(ref, got):
        for u, w in zip(r, g):
            assert torch.equal(u, w)
    sim.close()


def test_noalloc_force_refuses_a_pass_beyond_the_scratch():
    import paper_0711_0643_amd as nb

    n = 65536
    m, x, v = icgen.plummer(n, 3)
    banner("no-alloc force over the scratch limit")
    sim = nb.Sim(m, x, v, 1.0 / n, precision=1)
    sim.set_tuning(target_items=16384)  # up to 2^21 partial rows for the full block
    act = sim.storage_active()
    with pytest.raises(nb.NBodyError) as err:
        sim.force_noalloc(act, None)
    assert err.value.code == nb.NBODY_E_INVAL
    # nbody_force still runs the same pass from the workspace
    sim.force(act, None)
    assert sim.status() == 0
    sim.close()
