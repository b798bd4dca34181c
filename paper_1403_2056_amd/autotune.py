"""Autotuner for the sorter's tuning (splitters v, keys per thread, base-case
threshold).

The sorted output does not depend on the tuning (the result is unique), only
the time does.  `tune` times every candidate on a caller-supplied device
input and returns the fastest; results are cached per (GPU architecture,
workload class, size class) in tuning_cache.json next to this file.
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning_cache.json")

V_CHOICES = (63, 127, 255)
K_CHOICES = (4, 8)
TB_CHOICES = (64, 128, 256, 512, 1024)


def size_class(n: int) -> str:
    return f"2^{max(0, int(math.log2(max(n, 1))))}"


def load_cache() -> dict:
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def lookup(arch: str, workload: str, n: int):
    return load_cache().get(f"{arch}/{workload}/{size_class(n)}")


def store(arch: str, workload: str, n: int, entry: dict):
    c = load_cache()
    c[f"{arch}/{workload}/{size_class(n)}"] = entry
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def candidates(vs=V_CHOICES, ks=K_CHOICES, tbs=TB_CHOICES):
    return [dict(v=v, keys_per_thread=k, base_threshold=tb) for v, k, tb in itertools.product(vs, ks, tbs)]


def tune(run_factory, cands=None, reps: int = 3, warmup: int = 1, log=None):
    """run_factory(tuning_dict) -> callable that performs one timed unit of
    work and synchronises.  Returns (best tuning, [(tuning, ms), ...])."""
    cands = cands or candidates()
    table = []
    for c in cands:
        fn = run_factory(c)
        for _ in range(warmup):
            fn()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        ms = (time.perf_counter() - t0) * 1000.0 / reps
        table.append((c, ms))
        if log:
            log(f"[tune] {c} {ms:.3f} ms")
        del fn
    best = min(table, key=lambda x: x[1])[0]
    return best, table
