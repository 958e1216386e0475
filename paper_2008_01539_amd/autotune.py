"""Schedule choice per model class by measurement.

The kernels' tiles are fixed at compile time (256-row tiles, 64-row
slices, operand chunks sized to a register budget); what varies with the
model is the schedule around them: how many BiCGStab iterations are queued
between host checks, and whether the fracture-block preconditioner pays
for its extra kernels on a given fracture network.  ``tune`` times a short
probe of each candidate on the model itself (after one warm-up timestep)
and keeps the fastest, cached per model class (block size, precision,
cell-count bucket), so that the models of an ensemble or a serving pool
pay for the probe once per class.

    opts = tune(model, Options(precision=MIXED), cache_path="tune.json")
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import replace

DEFAULT_CANDIDATES = (
    {"check_every": 4, "precond": 1},
    {"check_every": 8, "precond": 1},
    {"check_every": 16, "precond": 1},
    {"check_every": 8, "precond": 0},
)


def model_class(model, options) -> str:
    """Cache key: block size, Krylov precision and the power-of-two bucket
    of the cell count."""
    bucket = 1 << int(math.floor(math.log2(max(1, int(model.n)))))
    return f"b{int(model.b)}-prec{int(options.precision)}-n{bucket}"


def _probe(model, options, steps, mode):
    """Wall time of `steps` timesteps after one warm-up timestep."""
    import torch
    from .fim import FimModel
    fm = FimModel(model, options)
    try:
        fm.set_state(model.u0, model.status0)
        sched = list(model.schedule)
        fm.solve_timestep(sched[0], mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for dt in sched[1:1 + steps]:
            fm.solve_timestep(dt, mode)
        torch.cuda.synchronize()
        return time.perf_counter() - t0
    finally:
        fm.close()


def tune(model, options, candidates=DEFAULT_CANDIDATES, probe_steps=2, mode=1,
         cache_path=None, probe=None):
    """Options with the fastest candidate settings for this model's class.

    probe(model, options, steps, mode) -> seconds may replace the GPU
    timing (tests).  The cache (a JSON file, optional) maps the class key
    to the chosen settings and the measured times."""
    probe = probe or _probe
    key = model_class(model, options)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
    if key in cache:
        return replace(options, **cache[key]["choice"])
    times = []
    for cand in candidates:
        times.append(probe(model, replace(options, **cand), probe_steps, mode))
    best = min(range(len(candidates)), key=lambda i: times[i])
    cache[key] = {"choice": dict(candidates[best]),
                  "times_s": [float(t) for t in times],
                  "candidates": [dict(c) for c in candidates]}
    if cache_path:
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    return replace(options, **candidates[best])
