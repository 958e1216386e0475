"""Schedule autotuner (CPU): picks the fastest candidate by the probe, and
a second model of the same class reuses the cached choice without probing."""
from dataclasses import dataclass

import numpy as np

from paper_2008_01539_amd import MIXED, Options
from paper_2008_01539_amd.autotune import model_class, tune


@dataclass
class _M:
    n: int
    b: int
    schedule: np.ndarray = None


def test_tune_picks_fastest_and_caches(tmp_path):
    calls = []

    def probe(model, opts, steps, mode):
        calls.append((opts.check_every, opts.precond))
        return {4: 3.0, 8: 1.0, 16: 2.0}[opts.check_every] + (5.0 if opts.precond == 0 else 0.0)

    cache = str(tmp_path / "tune.json")
    base = Options(precision=MIXED)
    o = tune(_M(n=5000, b=2), base, cache_path=cache, probe=probe)
    assert (o.check_every, o.precond) == (8, 1)
    assert o.precision == MIXED and len(calls) == 4
    # same class (same b, precision, size bucket): cached, no probe
    o2 = tune(_M(n=6000, b=2), base, cache_path=cache, probe=probe)
    assert (o2.check_every, o2.precond) == (8, 1) and len(calls) == 4
    # another bucket probes again
    tune(_M(n=70000, b=2), base, cache_path=cache, probe=probe)
    assert len(calls) == 8


def test_model_class_buckets():
    base = Options(precision=MIXED)
    assert model_class(_M(n=4096, b=1), base) == model_class(_M(n=8191, b=1), base)
    assert model_class(_M(n=4096, b=1), base) != model_class(_M(n=8192, b=1), base)
    assert model_class(_M(n=4096, b=1), base) != model_class(_M(n=4096, b=2), base)
