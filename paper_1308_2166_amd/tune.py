"""Autotuner of the step's launch shapes (tc_tuning) for a workload.

The shapes -- radix digit width where the vertex bound allows a choice,
radix tiles per chunk of the reduce-then-scan, waiting estimators per Step-3
join partition, batch edges per join block, the largest chunk that takes the
fused single-launch step -- change no result, only the
time a step takes, and the best ones depend on the step's batch sizes and
bank sizes and on the width of the vertex ids.  `tune` times candidate shapes
on the caller's own steps by coordinate descent (one field at a time, every
value of it, keeping the fastest) and the result is cached in a JSON file
keyed by (GPU architecture, w bucket, r bucket, key bits): the buckets are
the floor of log2 of the mean batch size and of the mean bank size, the key
bits those of the largest vertex id allowed.

Timing runs the library's kernels; nothing here computes a step.
"""
from __future__ import annotations

import json
import math
import os
import tempfile
import time

import torch

from . import DEFAULT_TUNING, TUNING_FIELDS

CANDIDATES = {
    "digit_bits": (0, 8),
    "chunk_tiles": (8, 16, 32),
    "part_estimators": (1024, 2048, 4096),
    "join_edges": (4096, 8192, 16384),
    "fused_edges": (0, 2048),
}


def bucket(x: float) -> int:
    """floor(log2(x)) for x >= 1 (0 below)."""
    return int(math.floor(math.log2(x))) if x >= 1 else 0


def key(arch: str, mean_w: float, mean_r: float, key_bits: int) -> str:
    return f"{arch}|w2^{bucket(mean_w)}|r2^{bucket(mean_r)}|b{int(key_bits)}"


def arch() -> str:
    """Architecture name of the current GPU (e.g. gfx950)."""
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def default_cache_path() -> str:
    return os.environ.get("TC_TUNING_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_1308_2166_amd", "tuning.json")


def load(path: str | None = None) -> dict:
    path = path or default_cache_path()
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def save(entries: dict, path: str | None = None) -> str:
    """Merge entries into the cache file (atomic replace); returns its path."""
    path = path or default_cache_path()
    d = load(path)
    d.update(entries)
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(os.path.abspath(path)), suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return path


def lookup(k: str, path: str | None = None) -> dict | None:
    """The cached tuning for key k (a tc_tuning dict), or None."""
    e = load(path).get(k)
    if not e or set(e.get("tuning", {})) != set(TUNING_FIELDS):
        return None
    return dict(e["tuning"])


def tune(run, apply, repeats: int = 2, candidates: dict = CANDIDATES,
         start: dict | None = None):
    """Coordinate descent over `candidates`: apply(tuning) sets the shapes,
    run() performs the timed work (it must leave the device idle: it is
    bracketed by synchronisations here).  Every configuration is run once
    untimed, then `repeats` times; its time is the fastest.  Returns (best
    tuning, its seconds, {str(tuning): seconds} of every configuration)."""
    trials = {}

    def timed(cfg):
        k = json.dumps(cfg, sort_keys=True)
        if k in trials:
            return trials[k]
        apply(cfg)
        run()
        torch.cuda.synchronize()
        best = None
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        trials[k] = best
        return best

    cur = dict(start or DEFAULT_TUNING)
    cur_t = timed(cur)
    for field, values in candidates.items():
        for v in values:
            if v == cur[field]:
                continue
            cand = dict(cur)
            cand[field] = v
            t = timed(cand)
            if t < cur_t:
                cur, cur_t = cand, t
    apply(cur)
    return cur, cur_t, trials
