"""Autotuner for the force pass: searches the launch tuning of libnbody
(nbody_set_tuning) on the caller's own system and caches the result.

What is searched (all runtime knobs of the library):
  * the i x j layout per block size -- the smallest block for the layouts
    with 2 i per lane, 1 i per lane, 4, 16 lanes per i (min_block, applied
    to every cluster: small_cluster_n = 0), chosen by timing every layout at
    a ladder of block sizes;
  * (mixed) the build of the lean tile-relative kernel: j-tiles of 256 or
    128 records, FP32 window of 16, 32 or 64 pairs (16 or 32 on 128-record
    tiles) and 2 to 5 waves per SIMD (tile, window, waves), on the full
    block, among the builds no slower than the default on the smallest
    block (a build that spills registers costs microseconds per launch);
  * the j-slicing target (target_items) and the persistent grid size (grid)
    for the full block;
  * the position format of the mixed kernel (mixed_format).

Every candidate must pass a parity gate before it may be timed: its
acceleration, jerk and potential on the same predicted state must agree with
the FP64 kernel's in its default configuration.  Mixed: per particle,
relative acceleration and potential errors <= 1e-6, and the relative jerk
error <= 1e-6 for 99.9 % of the particles (the others are particles whose
jerk terms cancel strongly, where the FP32 rounding of the terms shows) and
<= 1e-4 for all; FP64: <= 1e-12 for all three.  Timings are medians of
HIP-event kernel times.  Results are cached as JSON keyed by GPU architecture, HIP
runtime version, precision and the power-of-two bucket of N; the cache file
is $NBODY_TUNE_CACHE or ~/.cache/nbody_tune.json.

For a batch of clusters, tune_batch() times whole block steps (graph
replays) from the batch's current state instead: there the best layout
thresholds and slicing depend on how much work every step offers across the
whole batch, not on one cluster's block.

Usage:
    sim = paper_0711_0643_amd.Sim(...)
    cfg = tune.tune(sim)          # single cluster: searches (or loads) and applies
    cfg = tune.tune_batch(sim)    # batch of clusters
"""
from __future__ import annotations

import json
import math
import os
from pathlib import Path

import numpy as np

BIG = 1 << 30
GATE_MIXED = 1e-6
GATE_MIXED_JERK_MAX = 1e-4

# the builds of the lean tile-relative kernel (force_tuned.hip, force_tuned_t128.hip)
BUILDS = [dict(tile=tile, window=window, waves=waves)
          for tile in (256, 128) for window in (16, 32, 64) for waves in (2, 3, 4, 5)
          if not (tile == 128 and window == 64)]


def _key(cfg):
    return (cfg["tile"], cfg["window"], cfg["waves"])
GATE_FP64 = 1e-12


def cache_path() -> Path:
    p = os.environ.get("NBODY_TUNE_CACHE")
    return Path(p) if p else Path.home() / ".cache" / "nbody_tune.json"


def cache_key(sim) -> str:
    import torch

    props = torch.cuda.get_device_properties(sim.device)
    arch = getattr(props, "gcnArchName", props.name)
    hip = getattr(torch.version, "hip", None) or "unknown"
    nbucket = 1 << int(math.ceil(math.log2(max(2, sim.n // max(1, sim.nc)))))
    prec = "mixed" if sim.params.precision == 1 else "fp64"
    return f"{arch}|hip{hip}|{prec}|N{nbucket}|C{sim.nc}"


def _load_cache() -> dict:
    try:
        return json.loads(cache_path().read_text())
    except (OSError, ValueError):
        return {}


def _save_cache(data: dict) -> None:
    p = cache_path()
    p.parent.mkdir(parents=True, exist_ok=True)
    tmp = p.with_suffix(".tmp")
    tmp.write_text(json.dumps(data, indent=1, sort_keys=True))
    os.replace(tmp, p)


def _kernel_ms(sim, act, aoff, reps=5, warm=2):
    acc, jerk, _ = sim.force(act, aoff)
    for _ in range(warm):
        sim.force(act, aoff, out=(acc, jerk, None))
    sim.sync()
    sim.profile_force(True)
    sim.profile_read()
    t = []
    for _ in range(reps):
        sim.force(act, aoff, out=(acc, jerk, None))
        ms, k = sim.profile_read()
        t.append(ms / k)
    sim.profile_force(False)
    sim.sync()
    return float(np.median(t)), acc


def _rel(a, ref):
    a = a.cpu().numpy()
    ref = ref.cpu().numpy()
    return float(np.max(np.linalg.norm(a - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)))


def _rel_all(a, ref):
    """Per-particle relative errors of (3, n) vectors or (n,) scalars."""
    a = a.cpu().numpy()
    ref = ref.cpu().numpy()
    if a.ndim == 2:
        return np.linalg.norm(a - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)
    return np.abs(a - ref) / np.maximum(np.abs(ref), 1e-300)


def _forces(sim, act, aoff):
    """Acceleration and jerk from the pass without the potential (the one
    the tuned kernel builds serve) and the potential from the pass with it."""
    acc, jerk, _ = sim.force(act, aoff)
    _, _, pot = sim.force(act, aoff, pot=True)
    sim.sync()
    return acc.clone(), jerk.clone(), pot.clone()


def gate_check(got, ref, prec) -> dict:
    """The parity gate on acceleration, jerk and potential (see the module
    text); returns the errors and whether they pass."""
    ea, ek, ep = (_rel_all(g, r) for g, r in zip(got, ref))
    if prec == 1:
        ok = ea.max() <= GATE_MIXED and ep.max() <= GATE_MIXED and \
            np.quantile(ek, 0.999) <= GATE_MIXED and ek.max() <= GATE_MIXED_JERK_MAX
    else:
        ok = max(ea.max(), ek.max(), ep.max()) <= GATE_FP64
    return {"err": float(ea.max()), "err_jerk_p999": float(np.quantile(ek, 0.999)), "err_jerk_max": float(ek.max()),
            "err_pot": float(ep.max()), "ok": bool(ok)}


def tune(sim, use_cache: bool = True, ladder=None, verbose: bool = False) -> dict:
    """Search (or load) the best tuning for `sim` (single cluster) and apply it."""
    import torch

    if sim.nc != 1:
        raise ValueError("tune() works on a single-cluster Sim; apply its result to batches with set_tuning")
    key = cache_key(sim)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        cfg = cache[key]["tuning"]
        sim.set_tuning(**cfg)
        return cfg

    n = sim.n
    dev = sim.device
    base = sim.get_tuning()
    prec = sim.params.precision
    log = print if verbose else (lambda *a, **k: None)

    order = sim.order.cpu().numpy()

    def active(na):
        # a random subset of the slots in storage order, the order in which
        # the block selection lists its members
        rng = np.random.Generator(np.random.PCG64(7))
        slots = np.sort(rng.permutation(n)[:na])
        idx = order[slots].astype(np.int32)
        return (torch.as_tensor(idx, device=dev), torch.tensor([0, na], dtype=torch.int64, device=dev))

    # FP64 reference (default FP64 configuration) for the gate
    def reference(act, aoff):
        sim.set_precision(0)
        sim.set_tuning(**base)
        ref = _forces(sim, act, aoff)
        sim.set_precision(prec)
        return ref

    def trial(cfg, act, aoff, ref, **rec):
        sim.set_tuning(**cfg)
        g = gate_check(_forces(sim, act, aoff), ref, prec)
        ms = _kernel_ms(sim, act, aoff)[0] if g["ok"] else float("inf")
        records.append(dict(rec, ms=ms, **g))
        log(f"{rec}: {ms:.4f} ms err a {g['err']:.2e} k {g['err_jerk_p999']:.2e}/{g['err_jerk_max']:.2e} "
            f"phi {g['err_pot']:.2e} ok {g['ok']}")
        return ms

    ladder = ladder or sorted({1, 4, 16, 64, 256, 1024, 4096, n} & set(range(1, n + 1)))
    records = []
    best_variant = {}
    for na in ladder:
        act, aoff = active(na)
        ref = reference(act, aoff)
        times = {}
        for v in range(5):
            # min_block forcing layout v for every block size (non-increasing)
            cfg = dict(base, min_block=[BIG if i < v else 1 for i in range(4)], small_cluster_n=0)
            ms = trial(cfg, act, aoff, ref, n_act=na, variant=v)
            if ms < float("inf"):
                times[v] = ms
        best_variant[na] = min(times, key=times.get) if times else 1
    # thresholds: variant v is used from the smallest ladder size where a
    # variant <= v wins onwards (monotone by construction)
    min_block = []
    for v in range(4):
        sizes = [na for na in ladder if best_variant[na] <= v]
        min_block.append(min(sizes) if sizes else BIG)
    for i in range(1, 4):
        min_block[i] = min(min_block[i], min_block[i - 1])
    tuned = dict(base, min_block=min_block, small_cluster_n=0)

    # full block: kernel build (mixed), slicing target, grid and mixed format
    act, aoff = active(n)
    ref = reference(act, aoff)
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    best = None
    if prec == 1 and base["mixed_format"] == 2 and min(min_block[0], min_block[1]) <= n:
        # the full block runs a one-lane-per-i layout: the kernel build matters.
        # A build must also be no slower than the default one on the smallest
        # block of the ladder: builds that spill registers need scratch
        # memory, which costs microseconds per launch at every block size.
        small_act, small_aoff = active(ladder[0])
        small_ref = reference(small_act, small_aoff)
        t_small = {}
        for build in BUILDS:
            cfg = dict(tuned, **build)
            t_small[_key(build)] = trial(cfg, small_act, small_aoff, small_ref, n_act=ladder[0], **build)
        limit = 1.05 * t_small[_key(base)]
        for build in BUILDS:
            cfg = dict(tuned, **build)
            ms = trial(cfg, act, aoff, ref, n_act=n, **build)
            if t_small[_key(build)] <= limit and (best is None or ms < best[0]):
                best = (ms, cfg)
        if best is not None:
            tuned = best[1]
    best = None
    formats = (0, 1, 2) if prec == 1 else (base["mixed_format"],)
    for fmt in formats:
        for target in (2 * cus, 4 * cus, 8 * cus, 16 * cus):
            for grid in (4 * cus, 8 * cus, 16 * cus):
                cfg = dict(tuned, target_items=target, grid=grid, mixed_format=fmt)
                ms = trial(cfg, act, aoff, ref, n_act=n, target_items=target, grid=grid, mixed_format=fmt)
                if ms < float("inf") and (best is None or ms < best[0]):
                    best = (ms, cfg)
    cfg = best[1] if best else tuned
    sim.set_tuning(**cfg)
    cfg = sim.get_tuning()
    if use_cache:
        cache = _load_cache()
        cache[key] = {"tuning": cfg, "records": records}
        _save_cache(cache)
    return cfg


def batch_key(sim) -> str:
    import torch

    props = torch.cuda.get_device_properties(sim.device)
    arch = getattr(props, "gcnArchName", props.name)
    hip = getattr(torch.version, "hip", None) or "unknown"
    nbucket = 1 << int(math.ceil(math.log2(max(2, sim.n))))
    prec = "mixed" if sim.params.precision == 1 else "fp64"
    return f"{arch}|hip{hip}|{prec}|batch|Nsum{nbucket}|C{sim.nc}"


def batch_candidates(cus: int):
    """Layout thresholds and slicing targets searched by tune_batch."""
    mbs = ([1024, 1024, 48, 12], [384, 192, 48, 12], [BIG, 768, 96, 12], [BIG, BIG, 48, 12], [BIG, BIG, 96, 24],
           [BIG, BIG, 24, 6], [BIG, BIG, BIG, 12])
    # the default (size-dependent thresholds) first, then one threshold set for every cluster
    return [{}] + [{"min_block": list(mb), "small_cluster_n": 0, "target_items": t} for mb in mbs
                   for t in (8 * cus, 16 * cus)]


def tune_batch(sim, replays: int = 200, t_end: float = None, use_cache: bool = True, verbose: bool = False) -> dict:
    """Search (or load) min_block and target_items for a batch of clusters and apply them.

    Every candidate starts from the batch's current state (restored from a
    state blob) and is timed over `replays` block steps (HIP events on the
    library's stream); the state is restored afterwards.  Parity gate: one
    force pass over a fixed sample of every cluster must match the FP64
    kernel in acceleration, jerk and potential (gate_check)."""
    import torch

    key = batch_key(sim)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        cfg = cache[key]["tuning"]
        sim.set_tuning(**cfg)
        return cfg
    log = print if verbose else (lambda *a, **k: None)
    base = sim.get_tuning()
    prec = sim.params.precision
    blob = sim.get_state()
    dev = sim.device
    coff = sim.cluster_offsets
    t_now, _, _ = sim.progress()
    if t_end is None:
        t_end = float(np.ceil((t_now.max() + 1e-300) / sim.params.dt_max) + 1) * sim.params.dt_max
    # gate sample: every 7th particle of every cluster
    idx, aoff = [], [0]
    for c in range(sim.nc):
        sub = np.arange(int(coff[c]), int(coff[c + 1]), 7, dtype=np.int32)
        idx.append(sub)
        aoff.append(aoff[-1] + sub.size)
    act = torch.as_tensor(np.concatenate(idx), device=dev)
    aoff_t = torch.as_tensor(np.array(aoff, dtype=np.int64), device=dev)
    sim.predict(None)
    sim.set_precision(0)
    sim.set_tuning(**base)
    ref = _forces(sim, act, aoff_t)
    sim.set_precision(prec)
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    records, best = [], None
    for cand in batch_candidates(cus):
        cfg = dict(base, **cand)
        sim.set_state(blob)
        sim.set_tuning(**cfg)
        g = gate_check(_forces(sim, act, aoff_t), ref, prec)
        ok = g["ok"]
        ms = float("inf")
        if ok:
            sim.step(1, t_end)  # builds the graph for this configuration
            sim.sync()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(sim.stream)
            sim.step(replays, t_end)
            e1.record(sim.stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / replays
        records.append(dict(cand, ms_per_step=ms, **g))
        log(f"batch {cand}: {ms:.4f} ms/step {g}")
        if ok and (best is None or ms < best[0]):
            best = (ms, cfg)
    sim.set_state(blob)
    cfg = best[1] if best else base
    sim.set_tuning(**cfg)
    cfg = sim.get_tuning()
    if use_cache:
        cache = _load_cache()
        cache[key] = {"tuning": cfg, "records": records}
        _save_cache(cache)
    return cfg
