"""The discrete problem handed to the oracle and to the HIP library.

Layout (structure of arrays, SI units):

* cells ``0 .. n_matrix-1`` are matrix cells in natural (x fastest) order,
  cells ``n_matrix .. n-1`` are fracture cells;
* ``pv_ref``   reference pore volume V*phi_ref per cell (m^3);
* ``depth``    cell-centre depth, positive downward (m);
* ``kind``     0 = matrix, 1 = fracture;
* ``always_active`` 1 for cells that every active set contains (fracture and
  perforated cells: the paper does not localize fracture cells);
* connections ``conn_i < conn_j`` with transmissibility ``conn_T`` (m^3);
* perforations ``perf_cell``, well index ``perf_wi`` (m^3), bottom-hole
  pressure ``perf_bhp`` (Pa);
* ``u0`` initial state, shape (b, n): pressure, then water saturation, then
  the third variable (gas saturation or dissolved-gas ratio) for black oil;
* ``status0`` per-cell phase status (black oil: 1 = saturated, X = S_g;
  0 = undersaturated, X = R_s);
* ``schedule`` timestep sizes in seconds.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

FLUID_SINGLE = 1     # single-phase slightly compressible liquid, b = 1
FLUID_DEADOIL = 2    # water + dead oil, b = 2 (p, S_w)
FLUID_BLACKOIL = 3   # water + oil + gas with dissolution, b = 3 (p, S_w, X)


@dataclass
class Model:
    name: str
    n_matrix: int
    pv_ref: np.ndarray
    depth: np.ndarray
    kind: np.ndarray
    always_active: np.ndarray
    conn_i: np.ndarray
    conn_j: np.ndarray
    conn_T: np.ndarray
    perf_cell: np.ndarray
    perf_wi: np.ndarray
    perf_bhp: np.ndarray
    fluid: dict
    rock: dict
    gravity: float
    u0: np.ndarray
    status0: np.ndarray
    schedule: np.ndarray
    grid: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pv_ref.shape[0])

    @property
    def nc(self) -> int:
        return int(self.conn_i.shape[0])

    @property
    def b(self) -> int:
        return int(self.fluid["kind"])

    def validate(self) -> None:
        n = self.n
        assert self.depth.shape == (n,) and self.kind.shape == (n,)
        assert self.always_active.shape == (n,)
        assert np.all(self.pv_ref > 0)
        assert np.all(self.conn_i < self.conn_j)
        assert np.all(self.conn_i >= 0) and np.all(self.conn_j < n)
        assert np.all(self.conn_T >= 0)
        assert self.u0.shape == (self.b, n)
        assert self.status0.shape == (n,)
        key = self.conn_i.astype(np.int64) * n + self.conn_j
        assert np.unique(key).size == key.size, "duplicate connection"

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.pv_ref, self.depth, self.conn_i, self.conn_j,
                  self.conn_T, self.perf_cell, self.perf_wi, self.perf_bhp,
                  self.u0, self.status0, self.schedule):
            h.update(np.ascontiguousarray(a).tobytes())
        h.update(repr(sorted(self.fluid.items())).encode())
        h.update(repr(sorted(self.rock.items())).encode())
        return h.hexdigest()[:16]

    def copy_with(self, **kw) -> "Model":
        d = dict(self.__dict__)
        d.update(kw)
        return Model(**d)
