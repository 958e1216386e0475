"""Embedded discrete fractures (vertical planar fractures in a layered grid).

The paper embeds its fractures with EDFM and gives no formulas, so the
connection factors below are the common textbook choices:

* a fracture cell is the part of one fracture plane inside one matrix cell
  (in-plane length L_s times the layer thickness h);
* matrix-fracture: T = 2 A_s k_m / <d>, A_s = L_s h and <d> the mean normal
  distance from the matrix cell to the fracture plane (midpoint quadrature
  on a 16 x 16 map-view sub-grid; exactly dx/4 for a plane through the
  cell centre parallel to a face);
* fracture-fracture along one fracture: harmonic mean of the half-cell
  conductances k_f w h / (L/2) (in plane) and k_f w L / (h/2) (vertical);
* fracture-fracture at an intersection: T_a T_b / (T_a + T_b) with
  T_x = k_f w h / d_x and d_x the mean distance from fracture cell x to the
  intersection line, (a^2 + (L - a)^2) / (2 L).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Fracture:
    x0: float
    y0: float
    x1: float
    y1: float
    k0: int        # first layer (inclusive)
    k1: int        # last layer (inclusive)
    w: float       # aperture (m)
    kf: float      # permeability (m^2)
    phi: float = 1.0


def _clip(x0, y0, x1, y1, lx, ly):
    """Liang-Barsky clip of a segment to [0,lx]x[0,ly]; None if outside."""
    dx, dy = x1 - x0, y1 - y0
    t0, t1 = 0.0, 1.0
    for p, q in ((-dx, x0), (dx, lx - x0), (-dy, y0), (dy, ly - y0)):
        if p == 0.0:
            if q < 0.0:
                return None
            continue
        r = q / p
        if p < 0.0:
            t0 = max(t0, r)
        else:
            t1 = min(t1, r)
        if t0 > t1:
            return None
    return (x0 + t0 * dx, y0 + t0 * dy, x0 + t1 * dx, y0 + t1 * dy)


def _pieces(x0, y0, x1, y1, dx, dy, nx, ny, min_len):
    """Split a segment at grid lines: list of (ta, tb, ix, iy)."""
    ts = [0.0, 1.0]
    ddx, ddy = x1 - x0, y1 - y0
    if ddx != 0.0:
        lo, hi = sorted((x0, x1))
        for i in range(int(np.floor(lo / dx)) + 1, int(np.ceil(hi / dx))):
            ts.append((i * dx - x0) / ddx)
    if ddy != 0.0:
        lo, hi = sorted((y0, y1))
        for j in range(int(np.floor(lo / dy)) + 1, int(np.ceil(hi / dy))):
            ts.append((j * dy - y0) / ddy)
    ts = np.unique(np.clip(np.array(ts), 0.0, 1.0))
    seglen = float(np.hypot(ddx, ddy))
    out = []
    for a, b in zip(ts[:-1], ts[1:]):
        if b - a <= 1e-14:
            continue
        tm = 0.5 * (a + b)
        ix = min(max(int(np.floor((x0 + tm * ddx) / dx)), 0), nx - 1)
        iy = min(max(int(np.floor((y0 + tm * ddy) / dy)), 0), ny - 1)
        out.append([a, b, ix, iy])
    # absorb slivers (corner cuts) into a neighbouring piece
    merged = []
    for p in out:
        if merged and (p[1] - p[0]) * seglen < min_len:
            merged[-1][1] = p[1]
        else:
            merged.append(p)
    if len(merged) > 1 and (merged[0][1] - merged[0][0]) * seglen < min_len:
        merged[1][0] = merged[0][0]
        merged.pop(0)
    return merged, seglen


def _mean_distance(ix, iy, dx, dy, px, py, nxv, nyv, q=16):
    """Mean distance from the matrix cell (map view) to the line through
    (px,py) with unit normal (nxv,nyv): midpoint rule on a q x q sub-grid."""
    s = (np.arange(q) + 0.5) / q
    xs = ix * dx + s * dx
    ys = iy * dy + s * dy
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    return float(np.mean(np.abs((X - px) * nxv + (Y - py) * nyv)))


def embed(fracs, nx, ny, nz, dx, dy, dz, layer_depth, perm_m, n_matrix,
          min_piece=None):
    """Build fracture cells and their connections.

    Returns a dict with fracture-cell arrays (pv, depth, host matrix cell,
    fracture id, piece index, layer) and connection arrays (ci, cj, T), plus
    ``cell_of[(frac, piece, layer)]`` for perforations.
    """
    lx, ly = nx * dx, ny * dy
    if min_piece is None:
        min_piece = 0.05 * min(dx, dy)
    pv, dep, host, fid, pid, lay = [], [], [], [], [], []
    ci, cj, tt = [], [], []
    cell_of = {}
    geo = []   # per fracture: (clipped seg, pieces, seglen) or None
    nxt = n_matrix
    for f_i, fr in enumerate(fracs):
        c = _clip(fr.x0, fr.y0, fr.x1, fr.y1, lx, ly)
        if c is None:
            geo.append(None)
            continue
        x0, y0, x1, y1 = c
        if np.hypot(x1 - x0, y1 - y0) < min_piece:
            geo.append(None)
            continue
        pieces, seglen = _pieces(x0, y0, x1, y1, dx, dy, nx, ny, min_piece)
        geo.append(((x0, y0, x1, y1), pieces, seglen))
        ux, uy = (x1 - x0) / seglen, (y1 - y0) / seglen
        nxv, nyv = -uy, ux
        for p_i, (ta, tb, ix, iy) in enumerate(pieces):
            L = (tb - ta) * seglen
            dmean = _mean_distance(ix, iy, dx, dy, x0, y0, nxv, nyv)
            for k in range(fr.k0, fr.k1 + 1):
                cid = nxt
                nxt += 1
                cell_of[(f_i, p_i, k)] = cid
                pv.append(L * dz * fr.w * fr.phi)
                dep.append(layer_depth[k])
                m = ix + nx * (iy + ny * k)
                host.append(m)
                fid.append(f_i)
                pid.append(p_i)
                lay.append(k)
                # matrix-fracture
                ci.append(m)
                cj.append(cid)
                tt.append(2.0 * L * dz * perm_m[m] / dmean)
                # vertical within the fracture (to the layer above)
                if k > fr.k0:
                    up = cell_of[(f_i, p_i, k - 1)]
                    ci.append(up)
                    cj.append(cid)
                    tt.append(fr.kf * fr.w * L / dz)
                # in-plane to the previous piece, same layer
                if p_i > 0:
                    prev = cell_of[(f_i, p_i - 1, k)]
                    Lp = (pieces[p_i - 1][1] - pieces[p_i - 1][0]) * seglen
                    ta_ = fr.kf * fr.w * dz / (0.5 * Lp)
                    tb_ = fr.kf * fr.w * dz / (0.5 * L)
                    ci.append(prev)
                    cj.append(cid)
                    tt.append(ta_ * tb_ / (ta_ + tb_))
    # fracture-fracture intersections
    live = [i for i, g in enumerate(geo) if g is not None]
    if len(live) > 1:
        seg = np.array([geo[i][0] for i in live])
        k0 = np.array([fracs[i].k0 for i in live])
        k1 = np.array([fracs[i].k1 for i in live])
        ax0, ay0, ax1, ay1 = seg.T
        bxmin, bxmax = np.minimum(ax0, ax1), np.maximum(ax0, ax1)
        bymin, bymax = np.minimum(ay0, ay1), np.maximum(ay0, ay1)
        m = len(live)
        chunk = max(1, 4_000_000 // m)
        for s in range(0, m, chunk):
            ia = np.arange(s, min(m, s + chunk))[:, None]
            ib = np.arange(m)[None, :]
            ok = ib > ia
            ok &= (bxmin[ia] <= bxmax[ib]) & (bxmin[ib] <= bxmax[ia])
            ok &= (bymin[ia] <= bymax[ib]) & (bymin[ib] <= bymax[ia])
            ok &= (np.maximum(k0[ia], k0[ib]) <= np.minimum(k1[ia], k1[ib]))
            pa, pb = np.nonzero(ok)
            if pa.size == 0:
                continue
            pa = pa + s
            rx, ry = ax1[pa] - ax0[pa], ay1[pa] - ay0[pa]
            sx, sy = ax1[pb] - ax0[pb], ay1[pb] - ay0[pb]
            den = rx * sy - ry * sx
            qx, qy = ax0[pb] - ax0[pa], ay0[pb] - ay0[pa]
            with np.errstate(divide="ignore", invalid="ignore"):
                t = (qx * sy - qy * sx) / den
                u = (qx * ry - qy * rx) / den
            hit = (np.abs(den) > 1e-12) & (t >= 0) & (t <= 1) & (u >= 0) & (u <= 1)
            for a, b, ta_, ub_ in zip(pa[hit], pb[hit], t[hit], u[hit]):
                fa, fb = live[a], live[b]
                _, pcs_a, la = geo[fa]
                _, pcs_b, lb = geo[fb]
                ia_ = next(i for i, p in enumerate(pcs_a) if p[0] <= ta_ <= p[1])
                ib_ = next(i for i, p in enumerate(pcs_b) if p[0] <= ub_ <= p[1])
                La = (pcs_a[ia_][1] - pcs_a[ia_][0]) * la
                Lb = (pcs_b[ib_][1] - pcs_b[ib_][0]) * lb
                aa = (ta_ - pcs_a[ia_][0]) * la
                bb = (ub_ - pcs_b[ib_][0]) * lb
                da = (aa * aa + (La - aa) ** 2) / (2.0 * La)
                db = (bb * bb + (Lb - bb) ** 2) / (2.0 * Lb)
                for k in range(max(fracs[fa].k0, fracs[fb].k0),
                               min(fracs[fa].k1, fracs[fb].k1) + 1):
                    Ta = fracs[fa].kf * fracs[fa].w * dz / da
                    Tb = fracs[fb].kf * fracs[fb].w * dz / db
                    x, y = cell_of[(fa, ia_, k)], cell_of[(fb, ib_, k)]
                    ci.append(min(x, y))
                    cj.append(max(x, y))
                    tt.append(Ta * Tb / (Ta + Tb))
    return dict(
        pv=np.array(pv, np.float64), depth=np.array(dep, np.float64),
        host=np.array(host, np.int32), fid=np.array(fid, np.int32),
        pid=np.array(pid, np.int32), layer=np.array(lay, np.int32),
        ci=np.array(ci, np.int32), cj=np.array(cj, np.int32),
        T=np.array(tt, np.float64), cell_of=cell_of, geo=geo,
        n_frac_cells=nxt - n_matrix)
