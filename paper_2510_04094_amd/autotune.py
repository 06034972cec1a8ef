"""Autotuner over the library's launch choices (nyls_tuning), with a JSON cache.

Every choice computes the same method (the parity tests run each of them against the
oracle); they differ in speed on a given GPU and batch shape.  The tuner times `nyls_solve`
on the caller's batch for a small set of candidates, coordinate by coordinate from the
defaults, keeps the fastest, and records it under the batch's key

    (GPU architecture, m bucket, ODE orders, mode)

where the m bucket is the slot class of the largest basis (m <= 32, <= 64, <= 128, <= 256).
A later plan with the same key can start from the cached choice (`Batch(..., tuning="cached")`).

Cache file: $NYLS_TUNING_CACHE, else ~/.cache/nyls/tuning.json.  Timing uses HIP events on
torch's current stream; nothing here computes any part of the method.
"""
import json
import os
import time

import numpy as np
import torch

from . import nyls

MODE_NAMES = {nyls.FP64: "fp64", nyls.MIXED: "mixed", nyls.FP64_EXPLICIT: "fp64_explicit"}


def cache_path():
    p = os.environ.get("NYLS_TUNING_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "nyls", "tuning.json")


def m_bucket(m):
    """Slot class of the one-wave passes for an m-landmark basis."""
    m = int(m)
    if m <= 32:
        return "m<=32"
    if m <= 64:
        return "m<=64"
    if m <= 128:
        return "m<=128"
    return "m<=256"


def arch_name(device=None):
    props = torch.cuda.get_device_properties(device if device is not None else torch.cuda.current_device())
    return str(getattr(props, "gcnArchName", props.name)).split(":")[0]


def make_key(arch, max_m, orders, mode):
    """Cache key of a batch: architecture, m bucket of its largest basis, its ODE orders
    (sorted, '+'-joined) and the mode's name."""
    ords = "+".join(str(int(p)) for p in sorted(set(int(p) for p in orders)))
    return "%s|%s|p%s|%s" % (arch, m_bucket(max_m), ords, MODE_NAMES.get(mode, str(mode)))


def batch_key(batch, arch=None):
    return make_key(arch or arch_name(batch.device), int(np.max(batch.m)), batch.p, batch.mode)


def load_cache(path=None):
    path = path or cache_path()
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return {}
    return data if isinstance(data, dict) else {}


def save_entry(key, entry, path=None):
    """Merge one entry into the cache file (written atomically: temp file + rename)."""
    path = path or cache_path()
    data = load_cache(path)
    data[key] = entry
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = "%s.tmp%d" % (path, os.getpid())
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(key, path=None):
    """The cached tuning dict for `key`, or None."""
    entry = load_cache(path).get(key)
    if not entry or "tuning" not in entry:
        return None
    tun = entry["tuning"]
    if not all(k in tun for k in nyls.TUNING_FIELDS):
        return None
    return {k: int(tun[k]) for k in nyls.TUNING_FIELDS}


def _slot_class(m):
    """Landmark-slot class of the one-wave passes (their launches run side by side)."""
    return 0 if m <= 32 else (1 if m <= 64 else 2)


def knob_values(max_m, min_m, mode, max_n=0):
    """The values worth trying per knob for a batch (others are no-ops there)."""
    knobs = {}
    if min_m <= 64:
        knobs["eig_ql"] = [0, 1]
        knobs["ql_lanes"] = [64, 32, 16]
    if mode == nyls.FP64 and min_m + 2 <= 64:
        knobs["gram_valu"] = [0, 1]
    knobs["tail_layout"] = [1, 0]
    if mode == nyls.FP64 or _slot_class(min_m) != _slot_class(max_m):
        knobs["overlap"] = [1, 0]  # (mixed mode: only the passes of different slot classes)
    if mode == nyls.FP64:
        if max_n >= 4096:
            knobs["split"] = [-1, 0, 2048, 512]
    return knobs


def _time_solve(batch, refine, reps):
    """Median ms of `reps` nyls_solve calls after one warm-up."""
    batch.solve(refine)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        batch.solve(refine)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    return float(np.median(times))


def autotune(batch, refine=4, reps=3, save=True, path=None, log=None, min_gain=0.02):
    """Coordinate search over the knobs from the library defaults: each knob in turn takes
    the value with the lowest median solve time, the others held at the best so far; a
    change must beat the best so far by the fraction `min_gain` (run-to-run noise of a
    solve is about 1%).
    Returns dict(key, tuning, ms, default_ms, tried=[(tuning, ms), ...]); the batch is left
    with the chosen tuning applied, and (with save) the choice is written to the cache."""
    best = dict(nyls.DEFAULT_TUNING)
    batch.set_tuning(**best)
    tried = []
    best_ms = _time_solve(batch, refine, reps)
    tried.append((dict(best), best_ms))
    default_ms = best_ms
    knobs = knob_values(int(np.max(batch.m)), int(np.min(batch.m)), batch.mode, int(np.max(batch.n)))
    for name, values in knobs.items():
        if name == "ql_lanes" and best.get("eig_ql", 0) == 1:
            continue  # the lane-parallel QL is not used then
        for v in values:
            if v == best[name]:
                continue
            cand = dict(best, **{name: v})
            batch.set_tuning(**cand)
            ms = _time_solve(batch, refine, reps)
            tried.append((dict(cand), ms))
            if log:
                log("autotune %s=%d: %.3f ms (best %.3f)" % (name, v, ms, best_ms))
            if ms < (1.0 - min_gain) * best_ms:
                best, best_ms = cand, ms
    batch.set_tuning(**best)
    key = batch_key(batch)
    out = dict(key=key, tuning=best, ms=best_ms, default_ms=default_ms, tried=tried)
    if save:
        save_entry(key, {"tuning": best, "ms": best_ms, "default_ms": default_ms,
                         "batch": int(batch.batch), "max_n": int(np.max(batch.n)),
                         "refine": int(refine), "when": time.strftime("%Y-%m-%d %H:%M:%S")}, path)
    return out
