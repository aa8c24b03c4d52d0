"""Throughput of the Hermite block-step hot path on one MI355X.

A step is one full block step of the integrator on a Plummer sphere of
N = 65536 equal masses (eps = 1/N) with every particle in the block: block
selection, Hermite prediction of all particles, the pairwise acceleration +
jerk pass of the mixed-precision kernel over all N x N pairs, the reduction
of slice partials, and the Hermite correction with new time steps.  Shared
steps (dt = dt_max = 2^-10 for every particle) keep every block full, so a
step does N^2 interactions.  Inputs are resident in HBM before timing.

Printed: one JSON line with the metric (Ginteractions/s of acc + jerk), the
roofline of the dominant kernel (the mixed force kernel, timed with HIP
events around its own launches), the same workload with the FP64 kernel,
the force error of the mixed kernel against the FP64 kernel, and the FP64
CPU oracle timed on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic flops per acc + jerk interaction, counting an FMA as 2 and the
# reciprocal square root as 1: dr 3, dv 3, R^2 6, rsqrt 1, R^-2 / m R^-1 /
# m R^-3 3, r.v 5, -3 r.v / R^2 2, a 6, k 12 = 41; the potential adds 1.
# The timed kernel computes no potential, so the roofline counts 41.
FLOPS_ACC_JERK = 41
FLOPS_WITH_POT = 42
FLOPS_PER_INTERACTION = FLOPS_ACC_JERK
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector peak (published; counts packed FP32)
PEAK_FP64_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-integrations", action="store_true",
                    help="skip the integration workloads (N=65536 run, 256-cluster batch, performance model)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target duration of the CPU sample")
    ap.add_argument("--kernel-reps", type=int, default=10, help="timed launches of the force kernel alone")
    ap.add_argument("--no-sweep", action="store_true",
                    help="full-block runs only (no n_act sweep, no alternative kernels): clean profiles")
    ap.add_argument("--workload", choices=["c1", "c2", "c3", "c4", "c5", "model"], default=None,
                    help="instead of the headline line, run one of the integration workloads and print its record")
    ap.add_argument("--profile-window", action="store_true",
                    help="open the rocprofv3 --selected-regions window around the timed force launches only")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run 5 plain device copies of 256 MiB (reference for HBM byte counters)")
    return ap.parse_args()


def calibrate_copy():
    """Five device-to-device copies of 256 MiB: the hardware byte counters of
    this known transfer scale the counters read for the force kernel."""
    import torch

    nbytes = 256 << 20
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "copies": 5}), flush=True)


# the sources the force kernel is compiled from
FORCE_SOURCES = ("force.hip", "force_impl.h", "force_tuned.hip", "force_tuned_t128.hip", "common.h", "kernels.h")


def recorded_traffic():
    """HBM bytes per launch of the mixed force kernel from the committed
    rocprofv3 counter summary -- only if the force kernel's sources are the
    ones that were profiled (else None)."""
    import hashlib

    prof = os.path.join(ROOT, "profiles", "force_mixed_n65536_hbm_counters.txt")
    try:
        text = open(prof).read()
        for name in FORCE_SOURCES:
            src = os.path.join(ROOT, "paper_0711_0643_amd", "csrc", name)
            digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
            if f"{name} sha256: {digest}" not in text:
                return None
    except OSError:
        return None
    for line in text.splitlines():
        if line.startswith("traffic_bytes_per_launch:"):
            return float(line.split(":", 1)[1])
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


PROFILE_WINDOW = False
_roctx = None


def profile_window(open_: bool) -> None:
    """With --profile-window: open (resume) or close (pause) the region a
    profiler started with rocprofv3 --selected-regions records, so that its
    kernel statistics cover exactly the timed launches."""
    global _roctx
    if not PROFILE_WINDOW:
        return
    import ctypes

    if _roctx is None:
        lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib", "librocprofiler-sdk-roctx.so")
        _roctx = ctypes.CDLL(lib)
    fn = _roctx.roctxProfilerResume if open_ else _roctx.roctxProfilerPause
    fn(ctypes.c_uint64(0))


def time_steps(sim, steps, warmup, dt):
    import torch

    t_end = (warmup + steps) * dt
    sim.step(warmup, t_end)
    sim.sync()
    torch.cuda.synchronize()
    t_start, _, _ = sim.progress()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(sim.stream)
    sim.step(steps, t_end)
    ev1.record(sim.stream)
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    sim.sync()
    t_now, steps_done, _ = sim.progress()
    assert t_now[0] == t_end, (t_now, t_end)
    return (w1 - w0), ev0.elapsed_time(ev1) / 1e3


def kernel_time(sim, act, aoff, reps, warm=3):
    """Median duration of one force-kernel launch (HIP events around the
    launch, on the stream it runs on) for the active list `act`, after
    `warm` untimed calls (the clock settles over the first launches)."""
    acc, jerk, _ = sim.force(act, aoff)
    for _ in range(warm):
        sim.force(act, aoff, out=(acc, jerk, None))
    sim.sync()
    sim.profile_force(True)
    sim.profile_read()
    times = []
    profile_window(True)
    for _ in range(reps):
        sim.force(act, aoff, out=(acc, jerk, None))
        ms, launches = sim.profile_read()
        times.append(ms / launches)
    profile_window(False)
    sim.profile_force(False)
    sim.sync()
    return float(np.median(times)) / 1e3, acc, jerk


def call_time(sim, act, aoff, reps):
    """Median duration of a whole nbody_force call (plan + force + reduce),
    inputs and outputs already on the device."""
    import torch

    acc, jerk, _ = sim.force(act, aoff)
    sim.sync()
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        sim.force(act, aoff, out=(acc, jerk, None))
        e1.record(sim.stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times)) / 1e3


def run_workload(name, args):
    """Integration workloads: block-step runs with energy drift and step statistics.

    c1: Plummer N=1024, eps=1/1024, FP64 force, to t=1
    c2: Plummer N=16384, eps=1/N, FP64 force, to t=1/4
    c3: Plummer N=65536, eps=1/N, mixed force (and FP64 for comparison), to t=1/4
    c4: 256 Plummer clusters, N log-uniform in [256, 8192], eps=1/N each, mixed, to t=1/2
    c5: King W0=6 with Salpeter masses, N=262144, eps=1/N, mixed: full-block force
        throughput and 100 block steps
    """
    import torch

    import icgen
    import paper_0711_0643_amd as nb

    def drift_run(sim, t_end, chunk):
        d0 = sim.diagnostics()
        E0 = d0["E"]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        sim.run(t_end, chunk=chunk)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        d1 = sim.diagnostics()
        E1 = d1["E"]
        t, steps, inter = sim.progress()
        drift = (E1 - E0) / np.abs(E0)
        # momentum and angular momentum change, relative to sum m |v| and sum m |x||v| at the start
        st = sim.host_state()
        sc_p, sc_l = [], []
        for c in range(sim.nc):
            b, e = int(sim.cluster_offsets[c]), int(sim.cluster_offsets[c + 1])
            mv = st["m"][b:e] * np.linalg.norm(st["v"][:, b:e], axis=0)
            sc_p.append(mv.sum())
            sc_l.append((mv * np.linalg.norm(st["x"][:, b:e], axis=0)).sum())
        dP = float(np.max(np.linalg.norm(d1["P"] - d0["P"], axis=1) / np.array(sc_p)))
        dL = float(np.max(np.linalg.norm(d1["L"] - d0["L"], axis=1) / np.array(sc_l)))
        return {"_drift": drift, "wall_s": round(wall, 4), "block_steps": [int(x) for x in steps][:4] if steps.size > 4 else
                [int(x) for x in steps], "interactions": float(inter.sum()),
                "Ginteractions_per_s": round(float(inter.sum()) / wall / 1e9, 3),
                "mean_block": float(inter.sum() / max(1, steps.sum())) / float(sim.n / sim.nc),
                "max_abs_rel_energy_drift": float(np.abs(drift).max()),
                "max_rel_momentum_change": dP, "max_rel_angular_momentum_change": dL,
                "rel_energy_drift": [float(d) for d in drift[:4]], "t_end": t_end}

    out = {"workload": name}
    if name == "model":
        out.update(perf_model())
        print(json.dumps(out), flush=True)
        return
    if name in ("c1", "c2", "c3"):
        n, seed, t_end = {"c1": (1024, 1, 1.0), "c2": (16384, 2, 0.25), "c3": (65536, 3, 0.25)}[name]
        eps = 1.0 / n
        m, x, v = icgen.plummer(n, seed)
        precs = [("fp64", nb.FP64)] if name != "c3" else [("mixed", nb.MIXED), ("fp64", nb.FP64)]
        for label, prec in precs:
            sim = nb.Sim(m, x, v, eps, precision=prec)
            out[label] = drift_run(sim, t_end, 256)
            out[label].pop("_drift")
            log(f"{name} {label}: {out[label]}")
            sim.close()
        out["config"] = f"Plummer N={n}, eps=1/N, eta=0.01, dt_max=1/8, to t={t_end}"
    elif name == "c4":
        from paper_0711_0643_amd import tune

        m, x, v, coff, eps = icgen.ensemble(256, 4)
        # layouts for this batch: tune_batch from the initial state (search timed apart)
        probe = nb.Sim(m, x, v, eps, cluster_offsets=coff, precision=nb.MIXED)
        w0 = time.perf_counter()
        tuned = tune.tune_batch(probe, use_cache=False)
        out["tune_batch"] = {"search_s": round(time.perf_counter() - w0, 2), "tuning": tuned}
        probe.close()
        sim = nb.Sim(m, x, v, eps, cluster_offsets=coff, precision=nb.MIXED)
        out["mixed_default_tuning"] = {k: v_ for k, v_ in drift_run(sim, 0.5, 256).items() if not k.startswith("_")}
        sim.close()
        sim = nb.Sim(m, x, v, eps, cluster_offsets=coff, precision=nb.MIXED)
        sim.set_tuning(**tuned)
        rec = drift_run(sim, 0.5, 256)
        t, steps, inter = sim.progress()
        rec["block_steps_per_cluster"] = {"min": int(steps.min()), "median": int(np.median(steps)),
                                          "max": int(steps.max())}
        rec["graph_replays"] = int(steps.max())
        rec["per_cluster_drift"] = [float(d) for d in rec.pop("_drift")]
        sizes = np.diff(coff)
        worst = int(np.argmax(np.abs(rec["per_cluster_drift"])))
        rec["worst_cluster"] = {"index": worst, "n": int(sizes[worst]), "drift": rec["per_cluster_drift"][worst]}
        out["mixed"] = rec
        out["config"] = (f"256 Plummer clusters, N log-uniform in [256, 8192] (sum {int(coff[-1])}), "
                         "eps=1/N_c, mixed, to t=1/2, one graph replay = one block step of every cluster; "
                         "'mixed' runs with the tune_batch layouts")
        sim.close()
    else:
        n = 262144
        m, x, v = icgen.king(n, 6.0, 5)
        eps = 1.0 / n
        sim = nb.Sim(m, x, v, eps, precision=nb.MIXED)
        act = sim.storage_active()  # the full block in storage order, as the block steps list it
        aoff = torch.tensor([0, n], dtype=torch.int64, device=sim.device)
        kt, _, _ = kernel_time(sim, act, aoff, 5, warm=3)
        out["force_full_block"] = {"kernel_ms": round(kt * 1e3, 3),
                                   "Ginteractions_per_s": round(n * float(n) / kt / 1e9, 2),
                                   "TFLOP_s": round(FLOPS_ACC_JERK * n * float(n) / kt / 1e12, 2)}
        # 100 block steps one at a time, recording the block sizes
        sizes = []
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        prev = 0.0
        for _ in range(100):
            sim.step(1, 1.0)
            _, _, inter = sim.progress()
            sizes.append(int(round((inter[0] - prev) / n)))
            prev = inter[0]
        wall = time.perf_counter() - w0
        t, steps, inter = sim.progress()
        hist, edges = np.histogram(np.log2(np.maximum(sizes, 1)), bins=np.arange(0, 20))
        out["block_steps"] = {"steps": int(steps[0]), "t_reached": float(t[0]), "wall_s": round(wall, 4),
                              "interactions": float(inter[0]), "mean_block": float(np.mean(sizes)),
                              "max_block": int(max(sizes)), "min_block": int(min(sizes)),
                              "log2_block_histogram": [int(h) for h in hist]}
        out["config"] = "King W0=6, Salpeter masses (slope 2.35, 0.1-100, total 1), N=262144, eps=1/N, mixed"
        sim.close()
    print(json.dumps(out), flush=True)


def fit_step_model(rows):
    """Least-squares fit of T_adv(s) = tau_0 + tau_pr N + tau_cr s + tau_f N s
    to measured block steps, rows of (N, s, seconds); relative residuals, so
    that every step counts by its relative misfit.  Returns (tau_0, tau_pr,
    tau_cr, tau_f)."""
    A = np.array([[1.0, n, s_, n * s_] for n, s_, _ in rows])
    y = np.array([t_ for _, _, t_ in rows])
    w = 1.0 / y
    coef, *_ = np.linalg.lstsq(A * w[:, None], y * w, rcond=None)
    return tuple(float(c) for c in coef)


def model_total(taus, n, mean_block, steps):
    """Eq. tsnb on one GPU: the time of a run of `steps` block steps of mean
    size `mean_block` in a system of n, T_N = T_adv(s_mean) n_steps."""
    tau0, tau_pr, tau_cr, tau_f = taus
    return (tau0 + tau_pr * n + tau_cr * mean_block + tau_f * n * mean_block) * steps


def perf_model():
    """The paper's performance model on one MI355X (Sect. 4.1, Eq. tsnb).

    Per block step of size s in a system of N:  T_adv(s) = tau_0 + tau_pr N +
    tau_cr s + tau_f N s  (tau_0: the fixed cost of one step -- launches and
    latency -- which the paper's host model does not have; no communication
    term on one GPU).  Every block step of Plummer runs to t = 1/8 (the
    paper's integration time) is timed with HIP events; the taus come from a
    least-squares fit over all steps of all N; the model total T_N =
    T_adv(s_mean) n_steps (Eq. tsnb) is compared with the measured total."""
    import torch

    import icgen
    import paper_0711_0643_amd as nb

    rows = []
    per_n = {}
    for n in (1024, 4096, 16384, 65536):
        m, x, v = icgen.plummer(n, 100 + n)
        sim = nb.Sim(m, x, v, 1.0 / n, precision=nb.MIXED)
        times, sizes = [], []
        prev = 0.0
        t = 0.0
        guard = 0
        while t < 0.125 and guard < 200000:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(sim.stream)
            sim.step(1, 0.125)
            e1.record(sim.stream)
            e1.synchronize()
            tt, _, inter = sim.progress()
            t = float(tt[0])
            s_blk = (inter[0] - prev) / n
            prev = inter[0]
            times.append(e0.elapsed_time(e1) * 1e-3)
            sizes.append(s_blk)
            guard += 1
        sim.close()
        times = np.array(times)
        sizes = np.array(sizes)
        per_n[n] = {"steps": int(times.size), "mean_block": float(sizes.mean()), "measured_s": float(times.sum())}
        for tt_, ss in zip(times, sizes):
            rows.append((n, ss, tt_))
    tau0, tau_pr, tau_cr, tau_f = fit_step_model(rows)
    for n, rec in per_n.items():
        rec["model_s"] = model_total((tau0, tau_pr, tau_cr, tau_f), n, rec["mean_block"], rec["steps"])
        rec["model_over_measured"] = rec["model_s"] / rec["measured_s"]
    return {"fit": {"tau_0_s": tau0, "tau_pr_s": tau_pr, "tau_cr_s": tau_cr, "tau_f_s": tau_f,
                    "interactions_per_s_from_tau_f": 1.0 / tau_f if tau_f > 0 else None},
            "per_N": {str(k): v for k, v in per_n.items()},
            "paper_LISA": {"tau_pr_s": 5.6e-8, "tau_cr_s": 1.0e-6, "tau_f_s": 1.2e-7},
            "config": "Plummer N in {1024, 4096, 16384, 65536}, eps=1/N, mixed force, eta=0.01, every block step "
                      "to t=1/8 timed with HIP events"}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def golden_runs():
    path = os.path.join(ROOT, "tests", "golden", "oracle_runs.json")
    with open(path) as f:
        return json.load(f)


def integration_evidence():
    """The workloads beside the headline, measured in the same run:
    the N = 65536 Plummer run to t = 1/4 (mixed), the 256-cluster batch to
    t = 1/2 (mixed), and the paper's performance model fitted to every block
    step of Plummer runs to t = 1/8 (Sect. 4.1, Eq. tsnb).  Drifts are
    compared with the FP64 oracle's integration of the same inputs
    (tests/golden/oracle_runs.json)."""
    import torch

    import icgen
    import paper_0711_0643_amd as nb

    g = golden_runs()
    out = {}

    def timed_run(sim, t_end):
        E0 = sim.energy()
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        sim.run(t_end, chunk=512)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        E1 = sim.energy()
        _, steps, inter = sim.progress()
        return wall, (E1 - E0) / np.abs(E0), steps, inter

    # C3: Plummer N = 65536, eps = 1/N, mixed, to t = 1/4
    c3 = g["C3"]
    m, x, v = icgen.plummer(c3["n"], c3["seed"])
    sim = nb.Sim(m, x, v, c3["eps"], precision=nb.MIXED)
    wall, drift, steps, inter = timed_run(sim, c3["t_end"])
    sim.close()
    ref = [e for _, e in c3["energy_trace"]]
    ref_drift = (ref[-1] - ref[0]) / abs(ref[0])
    out["c3_plummer_n65536_mixed_to_t0.25"] = {
        "wall_s": round(wall, 4), "block_steps": int(steps[0]), "us_per_block_step": round(wall / steps[0] * 1e6, 2),
        "Ginteractions_per_s": round(float(inter[0]) / wall / 1e9, 2), "rel_energy_drift": float(drift[0]),
        "oracle_rel_energy_drift": ref_drift, "oracle_block_steps": c3["block_steps"]}
    log(f"c3 run: {out['c3_plummer_n65536_mixed_to_t0.25']}")

    # the same run with the switch pred_in_force off and on (the force pass
    # predicts the j-records of one-chunk blocks): time per block step, and
    # whether the two final states are bitwise equal
    walls, states = {}, {}
    for pif in (0, 1):
        sim = nb.Sim(m, x, v, c3["eps"], precision=nb.MIXED)
        sim.set_tuning(pred_in_force=pif)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        sim.run(c3["t_end"], chunk=512)
        torch.cuda.synchronize()
        walls[pif] = time.perf_counter() - w0
        _, fsteps, _ = sim.progress()
        states[pif] = sim.get_state()
        sim.close()
    same = states[0] == states[1]
    out["c3_pred_in_force"] = {
        "us_per_block_step_off": round(walls[0] / fsteps[0] * 1e6, 2),
        "us_per_block_step_on": round(walls[1] / fsteps[0] * 1e6, 2), "state_bitwise_equal": bool(same)}
    log(f"c3 pred_in_force: {out['c3_pred_in_force']}")

    # C4: the 256-cluster ensemble, mixed, to t = 1/2 (default tuning)
    c4 = g["C4"]
    m, x, v, coff, eps = icgen.ensemble(c4["n_clusters"], c4["master_seed"])
    sim = nb.Sim(m, x, v, eps, cluster_offsets=coff, precision=nb.MIXED)
    wall, drift, steps, inter = timed_run(sim, c4["t_end"])
    sim.close()
    vs = {}
    for key, rec in c4["clusters"].items():
        r = [e for _, e in rec["energy_trace"]]
        vs[key] = {"n": rec["n"], "rel_energy_drift": float(drift[int(key)]),
                   "oracle_rel_energy_drift": (r[-1] - r[0]) / abs(r[0])}
    worst = int(np.argmax(np.abs(drift)))
    out["c4_batch256_mixed_to_t0.5"] = {
        "wall_s": round(wall, 4), "graph_replays": int(steps.max()), "sum_n": int(coff[-1]),
        "Ginteractions_per_s": round(float(inter.sum()) / wall / 1e9, 2),
        "worst_rel_energy_drift": {"cluster": worst, "n": int(coff[worst + 1] - coff[worst]),
                                   "drift": float(drift[worst])},
        "clusters_vs_oracle": vs}
    log(f"c4 batch: wall {wall:.3f} s, {out['c4_batch256_mixed_to_t0.5']['Ginteractions_per_s']} Ginteractions/s")

    out["performance_model"] = perf_model()
    out["perturber_lists_n65536"] = perturber_timing()
    return out


def perturber_timing():
    """Perturber lists (Sect. 3.1) for every particle of the N = 65536
    Plummer sphere: nbody_perturbers with a threshold of 1 % of the mean |a|
    and lists of up to 256, timed with HIP events on the library's stream."""
    import torch

    import icgen
    import paper_0711_0643_amd as nb

    n = 65536
    m, x, v = icgen.plummer(n, 3)
    sim = nb.Sim(m, x, v, 1.0 / n, precision=nb.MIXED)
    thr = [0.01 * float(np.linalg.norm(sim.host_state()["a"], axis=0).mean())]
    act = torch.arange(n, dtype=torch.int32, device=sim.device)
    for _ in range(2):
        lists, counts = sim.perturbers(act, thr)
    ts = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        lists, counts = sim.perturbers(act, thr)
        e1.record(sim.stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    c = counts.cpu().numpy()
    sim.close()
    t = float(np.median(ts))
    return {"ms_per_call": round(t * 1e3, 3), "pair_tests_per_s": round(n * float(n) / t, 1),
            "mean_list_length": round(float(c.mean()), 2), "max_list_length": int(c.max()),
            "config": "every particle listed, threshold 0.01 <|a|>, at most 256 per list, ascending ids"}


def main():
    global PROFILE_WINDOW
    args = parse()
    PROFILE_WINDOW = args.profile_window
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.workload:
        run_workload(args.workload, args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch

    import icgen
    import paper_0711_0643_amd as nb

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(2)
    n = args.n
    eps = 1.0 / n
    dt = 2.0**-10
    m, x, v = icgen.plummer(n, 3)
    log(f"Plummer N={n} eps=1/N, shared steps dt={dt}")

    results = {}
    # name, precision, tuning overrides, full sweep + steps
    variants = [("mixed", nb.MIXED, {}, True), ("fp64", nb.FP64, {}, True),
                ("mixed_no_near_fp64", nb.MIXED, {"near_tau": 0.0}, False),
                ("mixed_fp64_differences", nb.MIXED, {"mixed_format": 1}, False),
                ("mixed_double_single", nb.MIXED, {"mixed_format": 0}, False)]
    if args.no_sweep:
        variants = [("mixed", nb.MIXED, {}, False)]
    for name, prec, tune, full in variants:
        # eta huge: every step is dt_max, so every block holds all N particles
        sim = nb.Sim(m, x, v, eps, precision=prec, eta=1e30, eta_init=1e30, dt_max=dt)
        if tune:
            sim.set_tuning(**tune)
        sim.sync()
        # force kernel alone on the t = 0 state (x_p = x), full block, the
        # active list in the library's storage order (as the block steps use it)
        act = sim.storage_active()
        order = sim.order.cpu().numpy()
        aoff = torch.tensor([0, n], dtype=torch.int64, device=sim.device)
        kt, acc, jerk = kernel_time(sim, act, aoff, args.kernel_reps, warm=10)
        a_id = np.empty((3, n)); a_id[:, order] = acc.cpu().numpy()
        k_id = np.empty((3, n)); k_id[:, order] = jerk.cpu().numpy()
        res = dict(kernel_s=kt, acc=a_id, jerk=k_id)
        if args.no_sweep:
            wall, evs = time_steps(sim, args.steps, args.warmup, dt)
            res.update(wall=wall, ev=evs)
            log(f"{name}: {args.steps} steps {wall * 1e3:.2f} ms wall, force kernel {kt * 1e3:.3f} ms/launch")
        elif full:
            sweep = {}
            for na in (1, 64, 1024, 16384, n):
                # a random subset of the slots, listed in storage order (the
                # order in which the block selection lists its members)
                slots = np.sort(np.random.Generator(np.random.PCG64(7)).permutation(n)[:na])
                sub = torch.as_tensor(order[slots].astype(np.int32), device=sim.device)
                soff = torch.tensor([0, na], dtype=torch.int64, device=sim.device)
                kts, _, _ = kernel_time(sim, sub, soff, 5)
                ct = call_time(sim, sub, soff, 5)
                sweep[str(na)] = {"kernel_ms": round(kts * 1e3, 4), "call_ms": round(ct * 1e3, 4),
                                  "Ginteractions_per_s": round(na * float(n) / kts / 1e9, 2)}
            res["sweep"] = sweep
            wall, evs = time_steps(sim, args.steps, args.warmup, dt)
            res.update(wall=wall, ev=evs)
            log(f"{name}: {args.steps} steps {wall * 1e3:.2f} ms wall ({evs * 1e3:.2f} ms events), "
                f"force kernel {kt * 1e3:.3f} ms/launch")
        else:
            log(f"{name}: force kernel {kt * 1e3:.3f} ms/launch")
        results[name] = res
        sim.close()
        del sim

    inter_step = float(n) * float(n)
    if args.no_sweep:
        mx = results["mixed"]
        print(json.dumps({"metric": "Ginteractions/s acc+jerk at N=65536 (profiling run, no comparisons)",
                          "value": round(args.steps * inter_step / mx["wall"] / 1e9, 3),
                          "unit": "Ginteractions/s", "kernel_ms": round(mx["kernel_s"] * 1e3, 4)}), flush=True)
        return
    mx, fp = results["mixed"], results["fp64"]
    value = args.steps * inter_step / mx["wall"] / 1e9
    # both kernels on the same t = 0 state
    ea = np.linalg.norm(mx["acc"] - fp["acc"], axis=0) / np.linalg.norm(fp["acc"], axis=0)
    ek = np.linalg.norm(mx["jerk"] - fp["jerk"], axis=0) / np.linalg.norm(fp["jerk"], axis=0)
    alt = {}
    for name in ("mixed_no_near_fp64", "mixed_fp64_differences", "mixed_double_single"):
        r = results[name]
        e = np.linalg.norm(r["acc"] - fp["acc"], axis=0) / np.linalg.norm(fp["acc"], axis=0)
        ej = np.linalg.norm(r["jerk"] - fp["jerk"], axis=0) / np.linalg.norm(fp["jerk"], axis=0)
        alt[name] = {"kernel_ms": round(r["kernel_s"] * 1e3, 4),
                     "Ginteractions_per_s": round(n * float(n) / r["kernel_s"] / 1e9, 2),
                     "acc_max_rel_vs_fp64": float(e.max()), "n_acc_above_1e-6": int((e > 1e-6).sum()),
                     "jerk_max_rel_vs_fp64": float(ej.max())}

    achieved = FLOPS_ACC_JERK * inter_step / mx["kernel_s"] / 1e12
    out = {
        "metric": "Ginteractions/s acc+jerk at N=65536 (mixed vs FP64, <=1e-6 rel force err)",
        "value": round(value, 3),
        "unit": "Ginteractions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mx["wall"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "mixed",
        "data": "synthetic",
        "config": {
            "workload": f"Plummer sphere N={n}, equal masses, eps=1/N, full-block Hermite block steps "
                        f"(select, predict, mixed force, reduce, correct), shared dt=2^-10",
            "n": n,
            "n_active": n,
            "precision": "mixed: FP64 positions and velocities; FP32 coordinates relative to each 256-particle "
                         "tile's frame (Morton storage order); FP32 pair terms; near pairs (acceleration term > "
                         "|a|/4, jerk term > |k|) in FP64; pairs much closer than their tile with FP64 "
                         "differences; FP64 totals",
        },
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "traffic": recorded_traffic(),
            "kernel": "nb::force_kernel<3, false, true, false, true, 32, 4, 256, false> (mixed tile-relative, no potential, "
                      "near pairs, lean; FP32 window 32, 4 waves per SIMD, 256-record j-tiles)",
            "flops_per_interaction": FLOPS_ACC_JERK,
            "flop_count_rule": "algorithmic acc + jerk without the potential (FMA = 2, rsqrt = 1); 42 with it",
            "interactions_per_launch": inter_step,
            "kernel_ms": round(mx["kernel_s"] * 1e3, 4),
            # labelled context, not used for frac: the 60-flop acc+jerk count common in
            # the GPU Hermite literature
            "context": {
                "frac_at_60_flops_per_interaction": round(60 * inter_step / mx["kernel_s"] / 1e12 / PEAK_FP32_TFLOPS, 4),
            },
        },
        "fp64": {
            "value": round(args.steps * inter_step / fp["wall"] / 1e9, 3),
            "ms_per_step": round(fp["wall"] / args.steps * 1e3, 4),
            "kernel_ms": round(fp["kernel_s"] * 1e3, 4),
            "kernel_tflops": round(FLOPS_ACC_JERK * inter_step / fp["kernel_s"] / 1e12, 3),
            "frac_of_fp64_peak": round(FLOPS_ACC_JERK * inter_step / fp["kernel_s"] / 1e12 / PEAK_FP64_TFLOPS, 4),
            "force_sweep": fp["sweep"],
        },
        "mixed_force_sweep": mx["sweep"],
        "force_sweep_note": ("a force call whose active list is below the one-lane-per-i threshold (1024) launches "
                             "the same j-split FP64 kernel in both precisions (bitwise equal results); the two "
                             "sweeps there differ by run-to-run noise only"),
        "mixed_alternatives": alt,
        "mixed_vs_fp64_error": {
            "acc_max_rel": float(ea.max()),
            "acc_median_rel": float(np.median(ea)),
            "jerk_max_rel": float(ek.max()),
            "jerk_median_rel": float(np.median(ek)),
            "n_acc_above_1e-6": int((ea > 1e-6).sum()),
        },
    }

    if not args.no_cpu:
        import oracle

        # the oracle on the same t = 0 state, for a sample of active particles
        # sized to take about args.cpu_seconds on the host cores
        probe = icgen.active_subset(n, 256, seed=7)
        t0 = time.perf_counter()
        oracle.force(m, x, v, eps, probe)
        t1 = time.perf_counter()
        per_i = (t1 - t0) / probe.size
        n_s = int(min(n, max(256, args.cpu_seconds / max(per_i, 1e-9))))
        sample = icgen.active_subset(n, n_s, seed=7)
        t0 = time.perf_counter()
        ra, rk, _ = oracle.force(m, x, v, eps, sample)
        t1 = time.perf_counter()
        cpu_rate = n_s * float(n) / (t1 - t0) / 1e9
        out["cpu_baseline"] = {
            "value": round(cpu_rate, 5),
            "unit": "Ginteractions/s",
            "cores": oracle.threads(),
            "cpu_model": cpu_model(),
            "kind": "oracle",
            "sample": f"FP64 oracle acc+jerk+pot on {n_s} active particles x {n} (same Plummer state), "
                      f"{t1 - t0:.1f} s",
        }
        # one host thread, on a smaller sample
        cores = oracle.threads()
        oracle.set_threads(1)
        one = icgen.active_subset(n, 512, seed=7)
        t0 = time.perf_counter()
        oracle.force(m, x, v, eps, one)
        t2 = time.perf_counter()
        oracle.set_threads(cores)
        out["cpu_baseline"]["single_thread"] = {"value": round(one.size * float(n) / (t2 - t0) / 1e9, 5),
                                                "sample": f"{one.size} active x {n}, {t2 - t0:.1f} s"}
        # both kernels against the oracle on that sample (same t = 0 state);
        # the jerk gate is per particle for jerk cancellation kappa_k <= 10
        # (kappa_k = sum of |jerk terms| / |k|); the others are counted
        absum = oracle.force_abs(m, x, v, eps, sample)
        kap = absum[1] / np.linalg.norm(rk, axis=0)
        ea_o = np.linalg.norm(mx["acc"][:, sample] - ra, axis=0) / np.linalg.norm(ra, axis=0)
        ef_o = np.linalg.norm(fp["acc"][:, sample] - ra, axis=0) / np.linalg.norm(ra, axis=0)
        ek_o = np.linalg.norm(mx["jerk"][:, sample] - rk, axis=0) / np.linalg.norm(rk, axis=0)
        en_o = np.linalg.norm(mx["jerk"][:, sample] - rk, axis=0) / absum[1]
        low = kap <= 10
        above = np.nonzero(ek_o > 1e-6)[0]
        out["vs_oracle"] = {
            "sample": int(n_s),
            "mixed_acc_max_rel": float(ea_o.max()), "fp64_acc_max_rel": float(ef_o.max()),
            "mixed_n_acc_above_1e-6": int((ea_o > 1e-6).sum()),
            "mixed_jerk_max_rel_kappa_le_10": float(ek_o[low].max()) if low.any() else None,
            "mixed_n_jerk_above_1e-6_kappa_le_10": int((ek_o[low] > 1e-6).sum()),
            "mixed_jerk_max_normwise": float(en_o.max()),
            "n_kappa_above_10": int((~low).sum()),
            "mixed_jerk_above_1e-6": {"count": int(above.size),
                                      "kappa": [round(float(kap[i]), 1) for i in above[:20]],
                                      "rel_err": [float(ek_o[i]) for i in above[:20]]},
        }
        log(f"cpu oracle: {cpu_rate:.4f} Ginteractions/s on {oracle.threads()} threads")

    if not args.no_integrations:
        out["integrations"] = integration_evidence()

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
