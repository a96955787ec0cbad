"""Launch-configuration autotuner for crp_propagate.

Searches the crp_tuning knobs (block size, persistent blocks per CU, refill
threshold, cell cache, longest-first order) on the particles (a random subset
of ``sample`` of them when there are more), one knob at a time (coordinate
descent from the defaults), timing each candidate with HIP events on the
launch stream.  A launch is often set by its longest trajectories, which a
subset may not hold, so the default sample covers whole workloads of up to a
million particles.  The winner is cached
per device architecture and workload signature.  For the FP64 path every
configuration must give bit-identical results; the winner is checked against
the defaults on the subset before it is returned.
"""
from __future__ import annotations

import hashlib
import json
import os

from . import crp

SPACE = {
    "block_size": [256, 128, 64],
    "blocks_per_cu": [4, 2, 8],
    "refill_threshold": [32, 8, 64, 1],
    "cache_cells": [0, 1, -1],
    "order_by_rigidity": [1, 0],
}
_FIELDS = ["block_size", "blocks_per_cu", "refill_threshold", "order_by_rigidity", "cache_cells"]


def default_cache_path() -> str:
    base = os.environ.get("CRP_AUTOTUNE_CACHE")
    if base:
        return base
    root = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(root, "crp", "autotune.json")


def signature(fields, params, n: int, precision: int) -> str:
    f = fields[0].desc
    sig = {"n_fields": len(fields), "grid": [int(f.n[0]), int(f.n[1]), int(f.n[2])], "dtype": int(f.dtype),
           "layout": int(f.layout), "n_params": len(params), "n_log2": int(n).bit_length(),
           "precision": int(precision), "tol": [p.tol for p in params[:1]]}
    return hashlib.sha1(json.dumps(sig, sort_keys=True).encode()).hexdigest()[:16]


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{getattr(p, 'gcnArchName', p.name)}:{p.multi_processor_count}"


def _subset(particles: dict, idx):
    return {k: (v[idx].contiguous() if v is not None else None) for k, v in particles.items()}


def _time(fields, params, pristine, precision, tuning, reps):
    import torch
    best = float("inf")
    state = None
    for _ in range(reps):
        state = crp.clone_particles(pristine)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        crp.crp_propagate(fields, params, state, precision=precision, tuning=tuning)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best, state


def autotune(fields, params, particles: dict, precision: int = crp.CRP_PREC_FP64, sample: int = 1_000_000,
             reps: int = 1, use_cache: bool = True, cache_path: str | None = None, seed: int = 0,
             log=None) -> crp.crp_tuning:
    """Return the fastest crp_tuning found for this workload (cached)."""
    import torch
    n = int(particles["energy"].numel())
    key = f"{_arch()}|{signature(fields, params, n, precision)}"
    path = cache_path or default_cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return crp.make_tuning(**cache[key]["tuning"])

    g = torch.Generator(device="cpu").manual_seed(seed)
    m = min(sample, n)
    idx = torch.randperm(n, generator=g)[:m].sort().values.to(particles["energy"].device)
    pristine = _subset(particles, idx)

    cur = {"block_size": 256, "blocks_per_cu": 4, "refill_threshold": 32, "order_by_rigidity": 1, "cache_cells": 0}
    t_best, ref_state = _time(fields, params, pristine, precision, crp.make_tuning(**cur), reps)
    trials = [(dict(cur), t_best)]
    for knob, values in SPACE.items():
        for v in values:
            if v == cur[knob]:
                continue
            cand = dict(cur)
            cand[knob] = v
            t, _ = _time(fields, params, pristine, precision, crp.make_tuning(**cand), reps)
            trials.append((cand, t))
            if log:
                log(f"autotune: {cand} {t:.2f} ms")
            if t < t_best:
                t_best, cur = t, cand
    best = crp.make_tuning(**cur)
    if precision == crp.CRP_PREC_FP64:
        _, st = _time(fields, params, pristine, precision, best, 1)
        for k in ("x", "y", "z", "ux", "uy", "uz", "length", "status", "n_accepted", "n_rejected"):
            if not torch.equal(st[k], ref_state[k]):
                raise RuntimeError(f"autotune: configuration {cur} changed FP64 results ({k})")
    cache[key] = {"tuning": cur, "ms_on_subset": t_best, "subset": m,
                  "trials": [{"tuning": c, "ms": t} for c, t in trials]}
    if use_cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path + ".tmp", "w") as fh:
                json.dump(cache, fh, indent=1)
            os.replace(path + ".tmp", path)
        except OSError:
            pass
    return best
