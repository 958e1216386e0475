"""Properties and the discrete residual (oracle; test infrastructure only).

The residual follows the finite-volume, two-point-flux, fully implicit
form of Appendix A (discrete conservation equation and phase flux with
phase-potential upwinding):

    R_{i,c} = (M_{i,c}(u) - M^n_{i,c}) / dt - sum_j F_{c,ij} - Q_{i,c}

with F_{c,ij} the mass of component c flowing from j into i.  Readings
where the paper is silent:

* flux sign: F_{l,ij} = T_ij mob_l,up (Phi_j - Phi_i), inflow into i is
  positive; Phi_l = p - rho_l g z with z the depth (positive down), the only
  sign for which a hydrostatic column carries no flow (Section 2 calls the
  coordinate "height");
* interface density rho_{l,ij}: arithmetic mean of the two cell densities
  (every phase density used here is defined in every cell);
* upwinding: for a connection stored as (a, b) with a < b the upstream cell
  is b iff Phi_b - Phi_a > 0, else a (ties go to the lower index);
* wells: bottom-hole-pressure perforations, q_c = WI sum_l mob_{c,l}
  (p_bhp - p) with cell-side mobilities and no backflow switch;
* rock: pore volume linear in pressure, pv_ref (1 + c_r (p - p_ref)).

Every function accepts complex state so that the Jacobian can be taken by
complex-step differentiation; decisions (upwinding, clamps) use real parts.
"""
from __future__ import annotations

import numpy as np


def _clamp01(x):
    """Clamp to [0, 1] on the real part, derivative kept inside."""
    r = np.real(x)
    return np.where(r < 0.0, 0.0 * x, np.where(r > 1.0, 0.0 * x + 1.0, x))


def pore_volume(pv_ref, rock, p):
    return pv_ref * (1.0 + rock["c_r"] * (p - rock["p_ref"]))


def props(model, u, status):
    """Return (M, rho, mob).

    M   : (b, n) component masses in each cell (kg);
    rho : (nph, n) phase mass densities used in the gravity weight;
    mob : (b, nph, n) mass of component c carried per unit phase-l
          potential drop and unit transmissibility, k_rl xi_{c,l} / mu_l.
    """
    fl = model.fluid
    kind = fl["kind"]
    p = u[0]
    pv = pore_volume(model.pv_ref, model.rock, p)
    if kind == 1:
        rho = fl["rho_ref"] * np.exp(fl["c"] * (p - fl["p_ref"]))
        M = (pv * rho)[None, :]
        mob = (rho / fl["mu"])[None, None, :]
        return M, rho[None, :], mob
    if kind == 2:
        sw = u[1]
        rw = fl["rho_w"] * np.exp(fl["c_w"] * (p - fl["p_ref"]))
        ro = fl["rho_o"] * np.exp(fl["c_o"] * (p - fl["p_ref"]))
        swn = _clamp01((sw - fl["swc"]) / (1.0 - fl["swc"] - fl["sor"]))
        krw = swn * swn
        kro = (1.0 - swn) * (1.0 - swn)
        M = np.stack([pv * rw * sw, pv * ro * (1.0 - sw)])
        z = 0.0 * p
        mob = np.stack([np.stack([rw * krw / fl["mu_w"], z]),
                        np.stack([z, ro * kro / fl["mu_o"]])])
        return M, np.stack([rw, ro]), mob
    # black oil: unknowns p, S_w, X with X = S_g (saturated) or R_s
    sw = u[1]
    x = u[2]
    sat = status == 1
    rs_sat = fl["rs_b"] * p / fl["p_b"]
    sg = np.where(sat, x, 0.0 * x)
    rs = np.where(sat, rs_sat, x)
    so = 1.0 - sw - sg
    bo = (1.0 + fl["bo_slope"] * rs) * np.exp(
        -fl["c_o"] * (p - fl["p_b"] * rs / fl["rs_b"]))
    bg = fl["bg_c"] / p
    bw = np.exp(-fl["c_w"] * (p - fl["p_ref"]))
    xw = fl["rho_wsc"] / bw
    xoo = fl["rho_osc"] / bo
    xgo = rs * fl["rho_gsc"] / bo
    xgg = fl["rho_gsc"] / bg
    span = fl["span"]
    krw = _clamp01((sw - fl["swc"]) / span) ** 2
    krg = _clamp01(sg / span) ** 2
    kro = _clamp01(so / span) ** 2
    M = np.stack([pv * sw * xw, pv * so * xoo, pv * (sg * xgg + so * xgo)])
    rho = np.stack([xw, xoo + xgo, xgg])
    z = 0.0 * p
    lw, lo, lg = krw / fl["mu_w"], kro / fl["mu_o"], krg / fl["mu_g"]
    mob = np.stack([np.stack([xw * lw, z, z]),
                    np.stack([z, xoo * lo, z]),
                    np.stack([z, xgo * lo, xgg * lg])])
    return M, rho, mob


def accumulation(model, u, status):
    return props(model, u, status)[0]


def _scatter(idx, w, n):
    if np.iscomplexobj(w):
        return (np.bincount(idx, np.real(w), n)
                + 1j * np.bincount(idx, np.imag(w), n))
    return np.bincount(idx, w, n)


def residual(model, u, status, m_old, dt):
    """R (b, n) in kg/s for state u at the new time level, given the
    component masses m_old at the old level and the step dt (App. A)."""
    n = model.n
    M, rho, mob = props(model, u, status)
    R = (M - m_old) / dt
    a, b_ = model.conn_i, model.conn_j
    T = model.conn_T
    p = u[0]
    dz = model.depth[b_] - model.depth[a]
    g = model.gravity
    nph = rho.shape[0]
    out = [R[c] for c in range(R.shape[0])]
    for l in range(nph):
        dphi = (p[b_] - p[a]) - 0.5 * (rho[l][a] + rho[l][b_]) * g * dz
        up = np.where(np.real(dphi) > 0.0, b_, a)
        for c in range(R.shape[0]):
            if np.all(mob[c, l] == 0):
                continue     # component c is not carried by phase l
            f = T * mob[c, l][up] * dphi
            out[c] = out[c] - _scatter(a, f, n) + _scatter(b_, f, n)
    pc = model.perf_cell
    if pc.size:
        for c in range(R.shape[0]):
            q = model.perf_wi * mob[c][:, pc].sum(axis=0) * (model.perf_bhp - p[pc])
            out[c] = out[c] - _scatter(pc, q, n)
    return np.stack(out)


def well_rates(model, u, status):
    """Component mass rates into the reservoir at each perforation (b, np)."""
    _, _, mob = props(model, u, status)
    pc = model.perf_cell
    p = u[0]
    return np.stack([model.perf_wi * mob[c][:, pc].sum(axis=0)
                     * (model.perf_bhp - p[pc]) for c in range(mob.shape[0])])
