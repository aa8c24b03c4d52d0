"""Writes tests/golden/oracle_runs.json: reference integrations by the FP64
oracle (block-step Hermite scheme of Sect. 2.1) of the seeded Plummer
spheres used as workloads -- N = 1024 to t = 1, N = 16384 and N = 65536 to
t = 1/4 (eps = 1/N, eta = 0.01, dt_max = 1/8), and six clusters of the
256-cluster ensemble (master seed 4: the two smallest, two of median size,
the two largest) to t = 1/2, each integrated alone (clusters of a batch
never interact).  Records per run: energy at every multiple of 1/8, block
steps, pairwise interactions.  Calls only the oracle and the input
generator.  The N = 65536 run takes about 15 minutes on 8 cores, the
ensemble clusters about a minute.

Usage: python tests/golden/make_oracle_runs.py [C1 C2 C3 C4]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import icgen  # noqa: E402
import oracle  # noqa: E402

CASES = {"C1": (1024, 1, 1.0), "C2": (16384, 2, 0.25), "C3": (65536, 3, 0.25)}
# ensemble clusters integrated alone: indices into icgen.ensemble(256, 4)
C4_CLUSTERS = (116, 176, 53, 9, 226, 178)
C4_T_END = 0.5
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_runs.json")


def run_system(m, x, v, eps, t_end):
    t0 = time.time()
    sim = oracle.Sim(m, x, v, eps)
    trace = [[0.0, sim.diagnostics()["E"]]]
    t = 0.0
    while t < t_end:
        t += 0.125
        sim.run(t)
        trace.append([t, sim.diagnostics()["E"]])
    return {"n": int(m.shape[0]), "eps": eps, "t_end": t_end, "eta": 0.01, "dt_max": 0.125,
            "energy_trace": trace, "block_steps": sim.steps, "interactions": sim.interactions,
            "wall_s": round(time.time() - t0, 1), "threads": oracle.threads()}


def run_ensemble():
    m, x, v, coff, eps = icgen.ensemble(256, 4)
    out = {"master_seed": 4, "n_clusters": 256, "t_end": C4_T_END, "clusters": {}}
    for c in C4_CLUSTERS:
        b, e = int(coff[c]), int(coff[c + 1])
        out["clusters"][str(c)] = run_system(m[b:e], x[:, b:e], v[:, b:e], float(eps[c]), C4_T_END)
    return out


def run(name):
    if name == "C4":
        return run_ensemble()
    n, seed, t_end = CASES[name]
    m, x, v = icgen.plummer(n, seed)
    eps = 1.0 / n
    t0 = time.time()
    sim = oracle.Sim(m, x, v, eps)
    trace = [[0.0, sim.diagnostics()["E"]]]
    t = 0.0
    while t < t_end:
        t += 0.125
        sim.run(t)
        trace.append([t, sim.diagnostics()["E"]])
    return {"n": n, "seed": seed, "eps": eps, "t_end": t_end, "eta": 0.01, "dt_max": 0.125,
            "energy_trace": trace, "block_steps": sim.steps, "interactions": sim.interactions,
            "wall_s": round(time.time() - t0, 1), "threads": oracle.threads()}


def main():
    which = sys.argv[1:] or list(CASES) + ["C4"]
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in which:
        data[name] = run(name)
        print(name, json.dumps(data[name]), flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1)


if __name__ == "__main__":
    main()
