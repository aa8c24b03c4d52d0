"""Full integrations on the GPU against stored oracle runs (GPU).

tests/golden/oracle_runs.json holds the FP64 oracle's integration of the
seeded Plummer workloads (written by tests/golden/make_oracle_runs.py, which
calls only the oracle): N = 1024 to t = 1, N = 16384 and N = 65536 to t = 1/4
(eps = 1/N, eta = 0.01, dt_max = 1/8), with the energy at every multiple of
1/8, the number of block steps and of pairwise interactions.

FP64 kernel: the block structure is deterministic given the forces, and the
GPU forces differ from the oracle's only at rounding level, so the block
steps and interaction counts are expected to be equal and the energies to
agree to ~1e-12.  Mixed kernel: forces differ at ~1e-7 relative, so only the
energy drift is compared (|dE/E| below 1e-5, and within 1e-8 of the
oracle's drift).
"""
import json
import os

import numpy as np
import pytest

import icgen
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_runs.json")


def _golden(name):
    with open(GOLDEN) as f:
        return json.load(f)[name]


def _run_traced(sim, t_end):
    trace = [sim.energy()[0]]
    t = 0.0
    while t < t_end:
        t += 0.125
        sim.run(t, chunk=512)
        trace.append(sim.energy()[0])
    assert sim.status() == 0
    return np.array(trace)


@pytest.mark.parametrize("case", ["C1", "C2", "C3"])
def test_fp64_run_matches_oracle_run(case):
    import paper_0711_0643_amd as nb

    g = _golden(case)
    m, x, v = icgen.plummer(g["n"], g["seed"])
    banner(f"fp64 run {case} N={g['n']}")
    sim = nb.Sim(m, x, v, g["eps"], precision=nb.FP64)
    trace = _run_traced(sim, g["t_end"])
    ref = np.array([e for _, e in g["energy_trace"]])
    assert np.max(np.abs(trace - ref)) <= 1e-12 * abs(ref[0])
    _, steps, inter = sim.progress()
    assert int(steps[0]) == g["block_steps"]
    assert float(inter[0]) == g["interactions"]
    sim.close()


@pytest.mark.parametrize("case", ["C1", "C3"])
def test_mixed_run_energy_drift_matches_oracle(case):
    import paper_0711_0643_amd as nb

    g = _golden(case)
    m, x, v = icgen.plummer(g["n"], g["seed"])
    banner(f"mixed run {case} N={g['n']}")
    sim = nb.Sim(m, x, v, g["eps"], precision=nb.MIXED)
    trace = _run_traced(sim, g["t_end"])
    ref = np.array([e for _, e in g["energy_trace"]])
    drift = (trace[-1] - trace[0]) / abs(trace[0])
    ref_drift = (ref[-1] - ref[0]) / abs(ref[0])
    assert abs(drift) < 1e-5
    assert abs(drift - ref_drift) < 1e-8
    sim.close()


def test_mixed_run_switching_layouts_matches_oracle():
    """C1 with the one-lane-per-i layout from blocks of 64 on: most steps
    switch between the j-split layouts (FP64 arithmetic, no tile frames) and
    the tile-relative one, whose frames the selection forms only when the
    block size it derives from the chunk and reduce-unit minima reaches that
    threshold.  A frame read at another time than it was formed for raises
    the state status; the run must end with none and follow the oracle run."""
    import paper_0711_0643_amd as nb

    g = _golden("C1")
    m, x, v = icgen.plummer(g["n"], g["seed"])
    banner(f"mixed run C1 N={g['n']}, one lane per i from 64")
    sim = nb.Sim(m, x, v, g["eps"], precision=nb.MIXED)
    sim.set_tuning(min_block=[1 << 30, 64, 48, 12], small_cluster_n=0)
    trace = _run_traced(sim, g["t_end"])
    ref = np.array([e for _, e in g["energy_trace"]])
    drift = (trace[-1] - trace[0]) / abs(trace[0])
    ref_drift = (ref[-1] - ref[0]) / abs(ref[0])
    assert abs(drift - ref_drift) < 1e-8
    sim.close()


def _batch_traces(sim, t_end):
    traces = [sim.energy()]
    t = 0.0
    while t < t_end:
        t += 0.125
        sim.run(t, chunk=512)
        traces.append(sim.energy())
    assert sim.status() == 0
    return np.array(traces)  # (times, clusters)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_batch_of_256_clusters_matches_oracle_runs(precision):
    """The 256-cluster ensemble (N log-uniform in [256, 8192]) advanced as one
    batch to t = 1/2; six clusters (two smallest, two of median size, two
    largest) against the oracle integrating each of them alone.  FP64: block
    steps and interactions exactly, energies to 1e-12.  Mixed: the energy
    drift of each cluster within 1e-7 of the oracle's."""
    import paper_0711_0643_amd as nb

    g = _golden("C4")
    m, x, v, coff, eps = icgen.ensemble(g["n_clusters"], g["master_seed"])
    banner(f"batch of {g['n_clusters']} clusters precision={precision}")
    sim = nb.Sim(m, x, v, eps, cluster_offsets=coff, precision=precision)
    traces = _batch_traces(sim, g["t_end"])
    _, steps, inter = sim.progress()
    for key, rec in g["clusters"].items():
        c = int(key)
        assert int(coff[c + 1] - coff[c]) == rec["n"]
        ref = np.array([e for _, e in rec["energy_trace"]])
        tr = traces[:, c]
        if precision == 0:
            assert int(steps[c]) == rec["block_steps"], (c, int(steps[c]), rec["block_steps"])
            assert float(inter[c]) == rec["interactions"]
            assert np.max(np.abs(tr - ref)) <= 1e-12 * abs(ref[0])
        else:
            drift = (tr[-1] - tr[0]) / abs(tr[0])
            ref_drift = (ref[-1] - ref[0]) / abs(ref[0])
            assert abs(drift - ref_drift) < 1e-7, (c, drift, ref_drift)
    sim.close()
