"""Per-iteration instrumentation of a run (Sections 5.2.1 and 5.2.3 report
the active-cell ratio M_A = n_A / n per Newton iteration, its total and
average over a run, and plot four cell classes per iteration).

``IterationLog`` writes one JSON object per Newton iteration (a JSONL
file) and, when asked, the cell classes of selected iterations as
run-length-encoded arrays in the same record; ``summary`` returns the
run's M_A total and average the way the paper's tables count them (total =
sum over iterations, average = total / iterations).

    log = IterationLog("run.jsonl", n_cells=model.n, classes_every=5)
    log.run(fm, model.schedule, LOCAL)
    print(log.summary())

The cell classes (bit 0 active, bit 1 boundary, bit 2 |dp| >= eps) come
from the library (``fim_get_flags``); this module only formats them.
"""
from __future__ import annotations

import json

import numpy as np


def rle(a: np.ndarray) -> list:
    """Run-length encoding [value, count, value, count, ...] of a 1-D
    array (compact for the large uniform regions of class maps)."""
    a = np.asarray(a).ravel()
    if a.size == 0:
        return []
    edge = np.flatnonzero(np.diff(a)) + 1
    starts = np.concatenate(([0], edge))
    counts = np.diff(np.concatenate((starts, [a.size])))
    out = []
    for s, c in zip(starts, counts):
        out += [int(a[s]), int(c)]
    return out


def unrle(pairs: list, dtype=np.uint8) -> np.ndarray:
    v = np.asarray(pairs[0::2], dtype=dtype)
    c = np.asarray(pairs[1::2], dtype=np.int64)
    return np.repeat(v, c)


class IterationLog:
    """JSONL log of Newton iterations.

    n_cells: cells of the model (M_A denominator, all cells, matrix and
    fracture); classes_every: attach the cell classes to every k-th
    iteration (0: never); path may be None (records kept in memory)."""

    def __init__(self, path, n_cells: int, classes_every: int = 0):
        self.path = path
        self.n = int(n_cells)
        self.classes_every = int(classes_every)
        self.records = []
        self._fh = open(path, "w") if path else None
        self._iter = 0

    def add(self, step: int, dt: float, stats: dict, classes=None):
        """One Newton iteration: stats is the library's iteration record
        (IterStats.as_dict()); classes the u8 class map or None."""
        rec = {"step": int(step), "iteration": self._iter, "dt": float(dt),
               "m_a": stats["n_active"] / self.n}
        rec.update({k: (float(v) if isinstance(v, float) else int(v)) for k, v in stats.items()})
        if classes is not None:
            rec["classes_rle"] = rle(classes)
        self.records.append(rec)
        if self._fh:
            self._fh.write(json.dumps(rec) + "\n")
        self._iter += 1
        return rec

    def run(self, fm, schedule, mode):
        """Advance fm through schedule one Newton iteration at a time,
        logging each; returns the records."""
        if self.classes_every:
            fm.record_flags(True)
        for k, dt in enumerate(schedule):
            while True:
                it = fm.newton_step(dt, mode)
                cls = None
                if self.classes_every and self._iter % self.classes_every == 0:
                    cls = fm.flags()
                self.add(k, dt, it.as_dict(), cls)
                if it.converged:
                    break
        if self.classes_every:
            fm.record_flags(False)
        return self.records

    def summary(self) -> dict:
        """M_A total (sum over iterations) and average (total / iterations),
        as in the paper's tables, plus iteration and Krylov counts."""
        ma = [r["m_a"] for r in self.records]
        return {"iterations": len(ma), "m_a_total": float(sum(ma)),
                "m_a_average": float(sum(ma) / len(ma)) if ma else 0.0,
                "krylov_iters": int(sum(r.get("krylov_iters", 0) for r in self.records))}

    def close(self):
        if self._fh:
            self._fh.close()
            self._fh = None
