"""Cartesian matrix grid with two-point transmissibilities.

Matrix-matrix transmissibility is the harmonic two-point form
T = A / (d_i/k_i + d_j/k_j) with half-cell distances d and isotropic
permeability (the paper names TPFA in its Appendix A without giving the
coefficient, so this textbook form is used).
"""
from __future__ import annotations

import numpy as np


def lognormal_perm(rng, n, median, sigma):
    """ln k ~ N(ln median, sigma^2): ``median`` is the geometric mean."""
    return median * np.exp(sigma * rng.standard_normal(n))


def cartesian_connections(nx, ny, nz, dx, dy, dz, perm):
    """Return (ci, cj, T) for the 7-point stencil, ci < cj, natural order."""
    idx = np.arange(nx * ny * nz).reshape(nz, ny, nx)
    k = perm.reshape(nz, ny, nx)
    ci, cj, tt = [], [], []

    def add(a, b, ka, kb, area, half):
        t = area / (half / ka + half / kb)
        ci.append(a.ravel())
        cj.append(b.ravel())
        tt.append(t.ravel())

    if nx > 1:
        add(idx[:, :, :-1], idx[:, :, 1:], k[:, :, :-1], k[:, :, 1:],
            dy * dz, 0.5 * dx)
    if ny > 1:
        add(idx[:, :-1, :], idx[:, 1:, :], k[:, :-1, :], k[:, 1:, :],
            dx * dz, 0.5 * dy)
    if nz > 1:
        add(idx[:-1, :, :], idx[1:, :, :], k[:-1, :, :], k[1:, :, :],
            dx * dy, 0.5 * dz)
    if not ci:
        return (np.zeros(0, np.int32), np.zeros(0, np.int32),
                np.zeros(0, np.float64))
    return (np.concatenate(ci).astype(np.int32),
            np.concatenate(cj).astype(np.int32),
            np.concatenate(tt).astype(np.float64))


def layer_depths(nz, dz, top):
    """Cell-centre depths of the layers, positive downward."""
    return top + dz * (np.arange(nz) + 0.5)
