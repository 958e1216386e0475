"""Pins of the oracle's fluid laws against results that do not come from
the oracle: the Buckley-Leverett solution of 1D immiscible displacement
(relative permeability and phase-potential upwinding of Appendix A), the
reduction of the black-oil model to a dead-oil one above the bubble point,
and linear diffusion with fluid as well as rock compressibility (the
exponential liquid density).  CPU only."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq
from scipy.special import erfc

from fimgen import DAY, FLUID_DEADOIL, PSI, make_small_c3
from fimgen.configs import fluid_deadoil, fluid_single
from fimgen.model import Model
from oracle.newton import Options, Solver, State
from oracle.physics import accumulation, well_rates


def _state(m):
    return State(m.u0.copy(), m.status0.copy())


# Buckley-Leverett ----------------------------------------------------------
# Water (mu 0.5 cP) displacing oil (mu 1 cP) at connate water 0.2 with
# Corey exponent 2, S_or = 0 (the two-phase fluid of the workloads), in a
# rigid 1D chain with incompressible phases and no gravity.  Fractional-flow
# theory gives a shock at the Welge tangent saturation S_f travelling at
# f_w'(S_f) W / (phi A) (W the injected water volume) and a rarefaction
# x(S) = f_w'(S) W / (phi A) behind it.

_SWC, _MUW, _MUO = 0.2, 0.5, 1.0


def _fw(s_w):
    s = (s_w - _SWC) / (1.0 - _SWC)
    lw, lo = s * s / _MUW, (1.0 - s) ** 2 / _MUO
    return lw / (lw + lo)


def _dfw(s_w):
    s = (s_w - _SWC) / (1.0 - _SWC)
    lw, lo = s * s / _MUW, (1.0 - s) ** 2 / _MUO
    dlw, dlo = 2.0 * s / _MUW, -2.0 * (1.0 - s) / _MUO
    return (dlw * lo - lw * dlo) / (lw + lo) ** 2 / (1.0 - _SWC)


def _welge():
    """Shock saturation: the tangent from (S_wc, 0) to the f_w curve."""
    return brentq(lambda s: _dfw(s) * (s - _SWC) - _fw(s), 0.25, 0.99)


def _bl_chain(ncell, nstep, length=100.0, area=1.0, phi=0.2, perm=1e-13,
              p_inj=5100.0 * PSI, p_prod=5000.0 * PSI, t_end=120.0 * DAY):
    """Cell 0 is a water-filled inlet cell fed by a bottom-hole-pressure
    injector (it only holds water, so it injects water only); cells
    1..ncell span [0, length]; the last cell carries a producer."""
    dx = length / ncell
    n = ncell + 1
    pv = np.full(n, area * dx * phi)
    ci = np.arange(n - 1, dtype=np.int32)
    T = np.full(n - 1, perm * area / dx)
    fl = fluid_deadoil()
    fl.update(c_w=0.0, c_o=0.0, p_ref=p_prod)
    sw = np.full(n, _SWC)
    sw[0] = 1.0
    u0 = np.stack([np.full(n, 0.5 * (p_inj + p_prod)), sw])
    wi = 1e3 * T[0]
    m = Model(name="bl", n_matrix=n, pv_ref=pv, depth=np.full(n, 1000.0),
              kind=np.zeros(n, np.int8), always_active=np.zeros(n, np.uint8),
              conn_i=ci, conn_j=ci + 1, conn_T=T,
              perf_cell=np.array([0, n - 1], np.int32),
              perf_wi=np.array([wi, wi]), perf_bhp=np.array([p_inj, p_prod]),
              fluid=fl, rock={"c_r": 0.0, "p_ref": p_prod}, gravity=0.0,
              u0=u0, status0=np.zeros(n, np.int8),
              schedule=np.full(nstep, t_end / nstep),
              grid=dict(nx=n, ny=1, nz=1, dx=dx, dy=1.0, dz=1.0))
    m.validate()
    return m


def _bl_run(ncell):
    m = _bl_chain(ncell, ncell)          # fixed front CFL as dx shrinks
    s = Solver(m, Options.tight_mode())
    st = _state(m)
    w_inj = 0.0
    rho_w = m.fluid["rho_w"]
    for dt in m.schedule:
        st, its = s.solve_timestep(st, dt)
        assert st is not None
        w_inj += dt * well_rates(m, st.u, st.status)[0, 0] / rho_w
    return m, st, w_inj


def _bl_errors(ncell, length=100.0, phi=0.2, area=1.0):
    m, st, w = _bl_run(ncell)
    dx = length / ncell
    x = (np.arange(ncell) + 0.5) * dx
    s_num = st.u[1][1:]
    sf = _welge()
    xf = _dfw(sf) * w / (phi * area)
    assert 0.3 * length < xf < 0.9 * length
    # exact profile: rarefaction S(x) for x < x_f, connate water beyond;
    # the rarefaction is inverted on a fine saturation grid
    sg = np.linspace(sf, 1.0, 20001)
    xs = _dfw(sg) * w / (phi * area)                 # decreasing in S
    xfine = (np.arange(ncell * 50) + 0.5) * (dx / 50)
    s_ex = np.where(xfine < xf, np.interp(xfine, xs[::-1], sg[::-1]), _SWC)
    s_ex_cell = s_ex.reshape(ncell, 50).mean(axis=1)
    l1 = float(np.abs(s_num - s_ex_cell).sum() * dx / (length * (sf - _SWC)))
    # numerical front: where S crosses half the shock height
    half = 0.5 * (sf + _SWC)
    k = int(np.nonzero(s_num < half)[0][0])
    x_num = x[k - 1] + (s_num[k - 1] - half) / (s_num[k - 1] - s_num[k]) * dx
    return xf, x_num, l1, st


def test_buckley_leverett_front_and_profile():
    """Front position and L1 saturation error against fractional-flow
    theory on three grids: both shrink by at least a fifth per halving of
    dx (first-order upwinding smears the shock over a few cells), and the
    finest front sits within 2.5 % of the chain length of the
    Welge-tangent shock."""
    res = [_bl_errors(nc) for nc in (40, 80, 160)]
    ferr = [abs(xn - xf) for xf, xn, _, _ in res]
    l1 = [e for _, _, e, _ in res]
    for e in (ferr, l1):
        assert e[1] < 0.8 * e[0] and e[2] < 0.8 * e[1]
    assert ferr[2] <= 0.025 * 100.0
    assert l1[2] <= 0.04
    # the upstream inlet cell stays water-filled: pure water enters
    assert np.all(res[2][3].u[1][0] == 1.0)


def test_welge_shock_saturation():
    """The tangent condition the pin relies on, checked independently:
    the chord slope from (S_wc, 0) is maximal at S_f."""
    sf = _welge()
    ss = np.linspace(0.21, 1.0, 4000)
    chord = _fw(ss) / (ss - _SWC)
    assert abs(ss[np.argmax(chord)] - sf) < 1e-3
    assert abs(_dfw(sf) - _fw(sf) / (sf - _SWC)) < 1e-10


# P10: black oil above the bubble point reduces to dead oil ----------------
def _undersaturated_pair():
    """A small black-oil model kept above its bubble point (producer at
    4000 psi, bubble point 3500 psi; every cell starts undersaturated at
    R_s = R_s,b), with a varied initial water saturation so that both
    phases flow, and its dead-oil twin: oil density
    (rho_osc + R_s,b rho_gsc) / B_o(p) with the same B_o law, same water."""
    bo = make_small_c3(schedule=np.array([0.01, 0.1, 1.0, 5.0, 20.0]) * DAY)
    fl = bo.fluid
    rng = np.random.default_rng(10)
    u = bo.u0.copy()
    u[1] = rng.uniform(0.25, 0.6, bo.n)
    bo = bo.copy_with(perf_bhp=np.full(bo.perf_bhp.shape, 4000.0 * PSI), u0=u)
    rho_ob = (fl["rho_osc"] + fl["rs_b"] * fl["rho_gsc"]) / (
        1.0 + fl["bo_slope"] * fl["rs_b"])
    dfl = fluid_deadoil()
    dfl.update(rho_w=fl["rho_wsc"], c_w=fl["c_w"], mu_w=fl["mu_w"],
               rho_o=rho_ob * math.exp(fl["c_o"] * (fl["p_ref"] - fl["p_b"])),
               c_o=fl["c_o"], mu_o=fl["mu_o"], p_ref=fl["p_ref"],
               swc=fl["swc"], sor=1.0 - fl["swc"] - fl["span"])
    do = bo.copy_with(fluid=dfl, u0=u[:2].copy())
    assert do.b == FLUID_DEADOIL
    return bo, do


def test_p10_blackoil_above_bubble_point_is_dead_oil():
    bo, do = _undersaturated_pair()
    fl = bo.fluid
    o = Options.tight_mode()
    sb, sd = Solver(bo, o), Solver(do, o)
    stb, std = _state(bo), _state(do)
    moved = 0.0
    for dt in bo.schedule:
        stb, _ = sb.solve_timestep(stb, dt)
        std, _ = sd.solve_timestep(std, dt)
        assert np.all(stb.status == 0)                      # no free gas
        assert stb.u[0].min() > fl["p_b"]
        pref = np.abs(std.u[0]).max()
        assert np.abs(stb.u[0] - std.u[0]).max() <= 1e-10 * pref
        assert np.abs(stb.u[1] - std.u[1]).max() <= 1e-10
        assert np.abs(stb.u[2] - fl["rs_b"]).max() <= 1e-10 * fl["rs_b"]
        mb = accumulation(bo, stb.u, stb.status)
        md = accumulation(do, std.u, std.status)
        # gas carried in the oil is R_s,b rho_gsc / rho_osc per unit oil mass
        ratio = fl["rs_b"] * fl["rho_gsc"] / fl["rho_osc"]
        assert np.allclose(mb[2], ratio * mb[1], rtol=1e-12, atol=0)
        assert np.allclose(mb[1] + mb[2], md[1], rtol=1e-9, atol=0)
        moved = max(moved, np.abs(stb.u[1] - bo.u0[1]).max())
    assert moved > 1e-4        # water saturation really changed


# compressible linear diffusion -----------------------------------------------
def _compressible_chain_error(nc, ns, length=200.0, c_f=0.5e-5 / PSI,
                              c_r=0.5e-5 / PSI, drop=10.0 * PSI):
    """Chain with an exponential liquid of compressibility c_f and rock
    compressibility c_r; a small pressure drop keeps the equation linear to
    O(c drop), and the erfc solution holds with c_t = c_f + c_r."""
    dxc = length / nc
    phi, perm, mu = 0.2, 1e-15, 1e-3
    p_i = 5000.0 * PSI
    pv = np.full(nc, dxc * phi)
    ci = np.arange(nc - 1, dtype=np.int32)
    T = np.full(nc - 1, perm / dxc)
    fl = fluid_single()
    fl.update(c=c_f, p_ref=p_i, mu=mu)
    m = Model(name="cchain", n_matrix=nc, pv_ref=pv, depth=np.full(nc, 1000.0),
              kind=np.zeros(nc, np.int8), always_active=np.zeros(nc, np.uint8),
              conn_i=ci, conn_j=ci + 1, conn_T=T,
              perf_cell=np.array([0], np.int32), perf_wi=np.array([1e6 * T[0]]),
              perf_bhp=np.array([p_i - drop]), fluid=fl,
              rock={"c_r": c_r, "p_ref": p_i}, gravity=0.0,
              u0=np.full((1, nc), p_i), status0=np.zeros(nc, np.int8),
              schedule=np.full(ns, DAY / ns))
    st, _ = Solver(m, Options.tight_mode()).run(_state(m), m.schedule)
    D = perm / (mu * phi * (c_f + c_r))
    x = np.arange(nc) * dxc
    exact = p_i - drop * erfc(x / (2.0 * math.sqrt(D * DAY)))
    return float(np.abs(st.u[0] - exact).max() / drop)


def test_compressible_liquid_diffusion_erfc():
    """Fluid plus rock compressibility: the erfc solution with the total
    compressibility, second-order convergence under refinement (dropping
    the fluid's share of the storage would double the diffusivity)."""
    e1 = _compressible_chain_error(50, 20)
    e2 = _compressible_chain_error(100, 80)
    e3 = _compressible_chain_error(200, 320)
    assert e3 < 1e-3
    for a, b in ((e1, e2), (e2, e3)):
        assert 3.0 < a / b < 5.0
