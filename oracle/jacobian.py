"""Jacobian J = dF/du of the discrete residual (oracle; test infrastructure).

Section 4.1 defines J(u) as the derivative of the residual with respect to
the unknowns.  The oracle takes it literally: each column block is obtained
by complex-step differentiation of ``physics.residual``,

    dF/du_k = Im F(u + i h e_k) / h,

which is exact to rounding (no subtractive cancellation).  Columns whose
cells are at graph distance > 2 never share a row, so one residual
evaluation serves a whole colour class of a greedy distance-2 colouring.
This is slow and plain by design; no derivative formula is written out here,
so the oracle's Jacobian and the HIP library's hand-derived one are
independent derivations.

Unknowns are ordered cell-major: global index i*b + v.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .physics import residual


def adjacency(model):
    """Symmetric CSR adjacency (row_ptr, nbr) of the connection graph,
    neighbours sorted ascending."""
    n = model.n
    a = np.concatenate([model.conn_i, model.conn_j]).astype(np.int64)
    b = np.concatenate([model.conn_j, model.conn_i]).astype(np.int64)
    order = np.lexsort((b, a))
    a, b = a[order], b[order]
    row_ptr = np.zeros(n + 1, np.int64)
    np.add.at(row_ptr, a + 1, 1)
    return np.cumsum(row_ptr), b


def distance2_colouring(model):
    """Greedy colouring in which cells within graph distance 2 differ."""
    n = model.n
    rp, nb = adjacency(model)
    colour = np.full(n, -1, np.int64)
    for i in range(n):
        used = set()
        for j in nb[rp[i]:rp[i + 1]]:
            if colour[j] >= 0:
                used.add(colour[j])
            for k in nb[rp[j]:rp[j + 1]]:
                if colour[k] >= 0:
                    used.add(colour[k])
        c = 0
        while c in used:
            c += 1
        colour[i] = c
    return colour


class JacobianBuilder:
    def __init__(self, model):
        self.model = model
        self.n = model.n
        self.b = model.b
        self.colour = distance2_colouring(model)
        self.ncol = int(self.colour.max()) + 1 if self.n else 0
        rp, nb = adjacency(model)
        # closed neighbourhood pairs (row cell i, column cell j)
        rows = np.repeat(np.arange(self.n), np.diff(rp))
        self.pair_i = np.concatenate([np.arange(self.n), rows])
        self.pair_j = np.concatenate([np.arange(self.n), nb])
        self.by_colour = [np.nonzero(self.colour[self.pair_j] == c)[0]
                          for c in range(self.ncol)]

    def build(self, u, status, m_old, dt, h=1e-30, variables=None):
        """Return (R, J): R (b, n) real, J scipy CSR (b n x b n).
        ``variables``: the unknowns (0 = pressure, ...) whose columns are
        formed; the other columns are left empty (default: all)."""
        b, n = self.b, self.n
        R = residual(self.model, u, status, m_old, dt)
        rr, cc, vv = [], [], []
        for c in range(self.ncol):
            sel = self.by_colour[c]
            pi, pj = self.pair_i[sel], self.pair_j[sel]
            cells = np.nonzero(self.colour == c)[0]
            for v in (range(b) if variables is None else variables):
                scale = np.maximum(1.0, np.abs(u[v][cells]))
                uc = u.astype(np.complex128)
                uc[v, cells] += 1j * h * scale
                Rc = residual(self.model, uc, status, m_old, dt)
                col_scale = np.ones(n)
                col_scale[cells] = scale
                for e in range(b):
                    rr.append(pi * b + e)
                    cc.append(pj * b + v)
                    vv.append(np.imag(Rc[e][pi]) / (h * col_scale[pj]))
        J = sp.csr_matrix((np.concatenate(vv), (np.concatenate(rr),
                                                 np.concatenate(cc))),
                          shape=(b * n, b * n))
        return np.real(R), J
