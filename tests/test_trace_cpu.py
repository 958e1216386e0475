"""Instrumentation log (CPU): run-length encoding round trip, JSONL records
and the M_A total/average as the paper's tables define them (total = sum
over iterations of n_A / n, average = total / iterations)."""
import json

import numpy as np

from paper_2008_01539_amd.trace import IterationLog, rle, unrle


def test_rle_round_trip():
    rng = np.random.default_rng(3)
    for n in (0, 1, 7, 1000):
        a = (rng.random(n) < 0.1).astype(np.uint8) * rng.integers(1, 8, n).astype(np.uint8)
        a[: n // 3] = 0
        assert np.array_equal(unrle(rle(a)), a)
    assert rle(np.array([5, 5, 5, 0, 0, 7], np.uint8)) == [5, 3, 0, 2, 7, 1]


def test_jsonl_records_and_m_a(tmp_path):
    p = tmp_path / "run.jsonl"
    log = IterationLog(str(p), n_cells=1000, classes_every=2)
    n_a = [100, 150, 50, 400]
    for i, na in enumerate(n_a):
        st = {"n_active": na, "n_boundary": 10, "is_expand": 0, "converged": int(i % 2),
              "krylov_iters": 7, "dp_max": 0.5}
        cls = np.zeros(1000, np.uint8)
        cls[:na] = 1
        log.add(i // 2, 86400.0, st, cls if i % 2 == 0 else None)
    log.close()
    lines = [json.loads(s) for s in p.read_text().splitlines()]
    assert [r["iteration"] for r in lines] == [0, 1, 2, 3]
    assert [r["m_a"] for r in lines] == [na / 1000 for na in n_a]
    assert "classes_rle" in lines[0] and "classes_rle" not in lines[1]
    assert int(unrle(lines[2]["classes_rle"]).sum()) == 50
    s = log.summary()
    assert s["iterations"] == 4
    assert abs(s["m_a_total"] - 0.7) < 1e-12
    assert abs(s["m_a_average"] - 0.175) < 1e-12
    assert s["krylov_iters"] == 28
