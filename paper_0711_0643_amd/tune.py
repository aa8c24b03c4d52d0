"""Autotuner for the force pass: searches the launch tuning of libnbody
(nbody_set_tuning) on the caller's own system and caches the result.

What is searched (all runtime knobs of the library):
  * the i x j layout per block size -- the smallest block for the layouts
    with 2 i per lane, 1 i per lane, 4, 16 lanes per i (min_block, applied
    to every cluster: small_cluster_n = 0), chosen by timing every layout at
    a ladder of block sizes;
  * the j-slicing target (target_items) and the persistent grid size (grid)
    for the full block;
  * the position format of the mixed kernel (mixed_format).

Every candidate must pass a parity gate before it may be timed: its forces on
a sample of the active set must agree with the FP64 kernel's on the same
predicted state (mixed: per-particle relative acceleration error <= 1e-6;
FP64: <= 1e-12 against the FP64 default).  Timings are medians of HIP-event
kernel times.  Results are cached as JSON keyed by GPU architecture, HIP
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
    gate = GATE_MIXED if prec == 1 else GATE_FP64
    log = print if verbose else (lambda *a, **k: None)

    def active(na):
        rng = np.random.Generator(np.random.PCG64(7))
        idx = np.sort(rng.permutation(n)[:na]).astype(np.int32)
        return (torch.as_tensor(idx, device=dev), torch.tensor([0, na], dtype=torch.int64, device=dev))

    # FP64 reference forces for the gate (default FP64 configuration)
    def reference(act, aoff):
        sim.set_precision(0)
        sim.set_tuning(**base)
        acc, _, _ = sim.force(act, aoff)
        sim.sync()
        ref = acc.clone()
        sim.set_precision(prec)
        return ref

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
            sim.set_tuning(**cfg)
            ms, acc = _kernel_ms(sim, act, aoff)
            err = _rel(acc, ref)
            ok = err <= gate
            records.append({"n_act": na, "variant": v, "ms": ms, "err": err, "ok": ok})
            log(f"n_act={na} variant={v}: {ms:.4f} ms err {err:.2e}")
            if ok:
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

    # full block: slicing target, grid and mixed format
    act, aoff = active(n)
    ref = reference(act, aoff)
    best = None
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    formats = (0, 1, 2) if prec == 1 else (base["mixed_format"],)
    for fmt in formats:
        for target in (2 * cus, 4 * cus, 8 * cus, 16 * cus):
            for grid in (4 * cus, 8 * cus, 16 * cus):
                cfg = dict(tuned, target_items=target, grid=grid, mixed_format=fmt)
                sim.set_tuning(**cfg)
                ms, acc = _kernel_ms(sim, act, aoff)
                err = _rel(acc, ref)
                ok = err <= gate
                records.append({"n_act": n, "target_items": target, "grid": grid, "mixed_format": fmt, "ms": ms,
                                "err": err, "ok": ok})
                log(f"full block fmt={fmt} target={target} grid={grid}: {ms:.4f} ms err {err:.2e}")
                if ok and (best is None or ms < best[0]):
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
    kernel (mixed: 1e-6 per particle; FP64: 1e-12)."""
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
    gate = GATE_MIXED if prec == 1 else GATE_FP64
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
    ref, _, _ = sim.force(act, aoff_t)
    sim.sync()
    ref = ref.clone()
    sim.set_precision(prec)
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    records, best = [], None
    for cand in batch_candidates(cus):
        cfg = dict(base, **cand)
        sim.set_state(blob)
        sim.set_tuning(**cfg)
        acc, _, _ = sim.force(act, aoff_t)
        sim.sync()
        err = _rel(acc, ref)
        ok = err <= gate
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
        records.append(dict(cand, ms_per_step=ms, err=err, ok=ok))
        log(f"batch {cand}: {ms:.4f} ms/step err {err:.2e}")
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
