"""Pins of the FP64 oracle against facts that do not come from the oracle:
closed forms, an analytic diffusion solution, conservation, symmetry,
finite differences and brute force.  CPU only."""
import math

import numpy as np
import pytest
from scipy.special import erfc

from fimgen import (DAY, FLUID_BLACKOIL, FLUID_DEADOIL, FLUID_SINGLE, GRAV,
                    PSI, make_c1, make_c1_variant, make_chain, make_small_c2,
                    make_small_c3, make_tiny)
from fimgen.configs import fluid_deadoil, fluid_single
from fimgen.model import Model
from oracle.jacobian import JacobianBuilder
from oracle.localized import LocalSolver
from oracle.newton import Options, Solver, State, apply_update
from oracle.physics import accumulation, residual, well_rates


def _state(m):
    return State(m.u0.copy(), m.status0.copy())


# P1 ------------------------------------------------------------------
def test_p1_single_cell_closed_form():
    """One cell, incompressible liquid, linear pore volume, BHP well:
    backward Euler gives p1 = (C p0 + W p_bhp) / (C + W) with
    C = pv_ref c_r / dt and W = WI / mu."""
    m = make_tiny("one")
    m.fluid["c"] = 0.0
    dt = 0.37 * DAY
    s = Solver(m, Options.tight_mode())
    st, its = s.solve_timestep(_state(m), dt)
    C = m.pv_ref[0] * m.rock["c_r"] / dt
    W = m.perf_wi[0] / m.fluid["mu"]
    p0 = m.u0[0, 0]
    exact = (C * p0 + W * m.perf_bhp[0]) / (C + W)
    assert abs(st.u[0, 0] - exact) <= 1e-14 * exact
    assert its <= 3


# P2 ------------------------------------------------------------------
def _chain_error(nc, ns, length=200.0):
    m = make_chain(nc, length, schedule=np.full(ns, DAY / ns))
    st, _ = Solver(m, Options.tight_mode()).run(_state(m), m.schedule)
    D = 1e-15 / (m.fluid["mu"] * 0.2 * m.rock["c_r"])
    x = np.arange(nc) * (length / nc)
    pi, pw = m.u0[0, 0], m.perf_bhp[0]
    exact = pi - (pi - pw) * erfc(x / (2.0 * math.sqrt(D * DAY)))
    return float(np.abs(st.u[0] - exact).max() / (pi - pw))


def test_p2_linear_diffusion_erfc():
    """1D linear pressure diffusion against the analytic erfc solution;
    halving dx and quartering dt cuts the error about 4x (O(dx^2 + dt))."""
    e1 = _chain_error(50, 20)
    e2 = _chain_error(100, 80)
    e3 = _chain_error(200, 320)
    assert e3 < 1e-3
    for a, b in ((e1, e2), (e2, e3)):
        assert 3.5 < a / b < 4.5


# P3 ------------------------------------------------------------------
@pytest.mark.parametrize("maker", [make_c1, make_small_c2, make_small_c3])
def test_p3_mass_balance(maker):
    """Per timestep: sum_i (M_i^{n+1} - M_i^n) = dt * (well inflow)."""
    m = maker()
    s = Solver(m, Options.tight_mode())
    st = _state(m)
    for dt in m.schedule[:4]:
        m0 = accumulation(m, st.u, st.status)
        new, _ = s.solve_timestep(st, dt)
        m1 = accumulation(m, new.u, new.status)
        q = well_rates(m, new.u, new.status).sum(axis=1)
        dm = (m1 - m0).sum(axis=1)       # difference per cell, then sum
        assert np.all(np.abs(dm - dt * q) <= 1e-10 * np.abs(dm).max())
        st = new


# P4 ------------------------------------------------------------------
@pytest.mark.parametrize("kind", [FLUID_SINGLE, FLUID_DEADOIL, FLUID_BLACKOIL])
@pytest.mark.parametrize("status", [0, 1])
def test_p4_finite_difference_jacobian(kind, status):
    """Complex-step Jacobian against central differences (h_p = 1 Pa,
    h_S = 1e-7) at a random state away from upwind switch points."""
    if kind != FLUID_BLACKOIL and status == 1:
        pytest.skip("status only matters for black oil")
    m = make_tiny("grid5", kind)
    u = m.u0.copy()
    stt = np.full(m.n, status, np.int8)
    if kind == FLUID_BLACKOIL and status == 1:
        u[2] = np.random.default_rng(3).uniform(0.05, 0.2, m.n)
    m_old = accumulation(m, u, stt) * 0.999
    dt = 0.5 * DAY
    R, J = JacobianBuilder(m).build(u, stt, m_old, dt)
    J = J.toarray()
    b = m.b
    hs = [1.0, 1e-7, 1e-7 if status == 1 else 1e-6]
    for v in range(b):
        for i in range(m.n):
            up, dn = u.copy(), u.copy()
            up[v, i] += hs[v]
            dn[v, i] -= hs[v]
            col = (residual(m, up, stt, m_old, dt)
                   - residual(m, dn, stt, m_old, dt)).T.reshape(-1) / (2 * hs[v])
            ref = J[:, i * b + v]
            for r in range(b * m.n):
                rowmax = np.abs(J[r]).max()
                if abs(ref[r]) < 1e-8 * rowmax:
                    continue
                # central-difference truncation plus round-off floor
                tol = 1e-6 * abs(ref[r]) + 1e-9 * rowmax
                assert abs(col[r] - ref[r]) <= tol, (v, i, r)


# P5 ------------------------------------------------------------------
def _column_model(fluid_kind):
    nz, dz = 10, 5.0
    depth = 2500.0 + dz * (np.arange(nz) + 0.5)
    ci = np.arange(nz - 1, dtype=np.int32)
    T = np.full(nz - 1, 1e-15 * 100.0 / dz)
    fl = fluid_single() if fluid_kind == FLUID_SINGLE else fluid_deadoil()
    rho_r = fl["rho_ref"] if fluid_kind == FLUID_SINGLE else fl["rho_o"]
    c = fl["c"] if fluid_kind == FLUID_SINGLE else fl["c_o"]
    # discrete hydrostatic column: p_{k+1} - p_k = g dz (rho_k + rho_{k+1})/2
    p = np.zeros(nz)
    p[0] = 5000.0 * PSI
    for k in range(nz - 1):
        q = p[k]
        for _ in range(100):
            q = p[k] + GRAV * dz * 0.5 * (
                rho_r * math.exp(c * (p[k] - fl["p_ref"]))
                + rho_r * math.exp(c * (q - fl["p_ref"])))
        p[k + 1] = q
    u0 = p[None, :] if fluid_kind == FLUID_SINGLE else np.stack([p, np.full(nz, 0.2)])
    return Model(name="column", n_matrix=nz, pv_ref=np.full(nz, 30.0),
                 depth=depth, kind=np.zeros(nz, np.int8),
                 always_active=np.zeros(nz, np.uint8), conn_i=ci,
                 conn_j=ci + 1, conn_T=T, perf_cell=np.zeros(0, np.int32),
                 perf_wi=np.zeros(0), perf_bhp=np.zeros(0), fluid=fl,
                 rock={"c_r": 1e-5 / PSI, "p_ref": 5000.0 * PSI},
                 gravity=GRAV, u0=u0, status0=np.zeros(nz, np.int8),
                 schedule=np.array([DAY]))


@pytest.mark.parametrize("kind", [FLUID_SINGLE, FLUID_DEADOIL])
def test_p5_hydrostatic_equilibrium(kind):
    """A discretely hydrostatic column with no wells has zero residual and
    does not move; pressure increases with depth."""
    m = _column_model(kind)
    assert np.all(np.diff(m.u0[0]) > 0)
    st = _state(m)
    m_old = accumulation(m, st.u, st.status)
    R = residual(m, st.u, st.status, m_old, DAY)
    scale = m_old / DAY
    assert np.all(np.abs(R) <= 1e-12 * scale)
    new, _ = Solver(m, Options.tight_mode()).solve_timestep(st, DAY)
    assert np.abs(new.u[0] - m.u0[0]).max() < 1e-6
    # the opposite gravity sign is not in equilibrium
    m2 = m.copy_with(gravity=-GRAV)
    R2 = residual(m2, st.u, st.status, m_old, DAY)
    assert np.abs(R2).max() > 1e3 * np.abs(R).max() + 1e-12


# P6 ------------------------------------------------------------------
def test_p6_mirror_symmetry():
    """Uniform permeability, fracture in the centre column of an odd-width
    grid: the solution is mirror-symmetric in x and in y."""
    m = make_c1_variant()
    st, _ = Solver(m, Options.tight_mode()).run(_state(m), m.schedule)
    nx, ny = m.grid["nx"], m.grid["ny"]
    p = st.u[0][:m.n_matrix].reshape(ny, nx)
    drop = m.u0[0].max() - p.min()
    assert drop > 1e5
    assert np.abs(p - p[:, ::-1]).max() <= 1e-12 * drop * 1e3
    assert np.abs(p - p[::-1, :]).max() <= 1e-12 * drop * 1e3


# P7 ------------------------------------------------------------------
def test_p7_localization_reduces_to_full_newton():
    """eps_loc = 0 starting from V_A = V: Algorithm 1 takes exactly the
    full-Newton iterates (bitwise); eps_loc = 0 from the small initial set
    reaches the same solution."""
    m = make_c1_variant()
    o = Options.tight_mode(eps_loc=0.0)
    full = Solver(m, o)
    loc = LocalSolver(m, o)
    st = _state(m)
    dt = m.schedule[2]
    ref, its = full.solve_timestep(st, dt)
    allc = set(range(m.n))
    import oracle.sets as S
    orig = S.initial_active
    try:
        S.initial_active = lambda *a, **k: set(allc)
        got, its2, _ = loc.alg1_timestep(st, dt, None)
    finally:
        S.initial_active = orig
    assert its2 == its
    assert np.array_equal(got.u, ref.u)
    got2, _, _ = loc.alg1_timestep(st, dt, None)
    assert np.abs(got2.u - ref.u).max() <= 1e-10 * ref.u.max()


# P8 ------------------------------------------------------------------
@pytest.mark.parametrize("kind", [FLUID_SINGLE, FLUID_DEADOIL, FLUID_BLACKOIL])
def test_p8_dense_brute_force(kind):
    """<= 12 unknown cells: a dense Newton with a column-by-column
    complex-step Jacobian and numpy.linalg.solve equals the sparse oracle."""
    m = make_tiny("grid3", kind)
    o = Options.tight_mode()
    st = _state(m)
    dt = 2.0 * DAY
    ref, its = Solver(m, o).solve_timestep(st, dt)
    b, n = m.b, m.n
    u = st.u.copy()
    stt = st.status.copy()
    m_old = accumulation(m, u, stt)
    for _ in range(its):
        R = residual(m, u, stt, m_old, dt).T.reshape(-1)
        J = np.zeros((b * n, b * n))
        for k in range(b * n):
            uc = u.astype(complex)
            uc[k % b, k // b] += 1e-30j
            J[:, k] = np.imag(residual(m, uc, stt, m_old, dt)).T.reshape(-1) / 1e-30
        du = np.linalg.solve(J, -R).reshape(n, b).T
        s2 = State(u, stt)
        apply_update(m, s2, du, o)
        u, stt = s2.u, s2.status
    assert np.abs(u[0] - ref.u[0]).max() <= 1e-13 * np.abs(ref.u[0]).max()
    if b > 1:
        assert np.abs(u[1:] - ref.u[1:]).max() <= 1e-11


# upwinding ------------------------------------------------------------
def test_upwind_direction_carries_upstream_mobility():
    """Two cells: water-filled high-pressure cell next to an oil cell at
    connate water.  Upstream weighting moves water into the oil cell (its
    own water mobility is zero, so downstream weighting could not)."""
    m = make_tiny("grid3", FLUID_DEADOIL)
    n = m.n
    u = m.u0.copy()
    u[1] = 0.2
    u[1, 0] = 1.0
    u[0] = 5000.0 * PSI
    u[0, 0] = 5100.0 * PSI
    m = m.copy_with(perf_cell=np.zeros(0, np.int32), perf_wi=np.zeros(0),
                    perf_bhp=np.zeros(0), u0=u)
    st = State(u.copy(), np.zeros(n, np.int8))
    new, _ = Solver(m, Options.tight_mode()).solve_timestep(st, 10.0 * DAY)
    nb = [j for i, j in zip(m.conn_i, m.conn_j) if i == 0]
    assert all(new.u[1, j] > 0.2 + 1e-6 for j in nb)


# black oil -------------------------------------------------------------
def test_blackoil_switch_preserves_component_masses():
    """At S_g = 0 and R_s = R_s,sat(p) the saturated and undersaturated
    descriptions of a cell are the same state: identical masses."""
    m = make_small_c3()
    fl = m.fluid
    p = np.linspace(2000, 3400, m.n) * PSI
    sw = np.full(m.n, 0.25)
    rs = fl["rs_b"] * p / fl["p_b"]
    Ms = accumulation(m, np.stack([p, sw, np.zeros(m.n)]), np.ones(m.n, np.int8))
    Mu = accumulation(m, np.stack([p, sw, rs]), np.zeros(m.n, np.int8))
    assert np.allclose(Ms, Mu, rtol=1e-14, atol=0)


def test_blackoil_switching_rules():
    m = make_small_c3()
    fl = m.fluid
    n = m.n
    p = np.full(n, 3000.0 * PSI)
    rs_sat = fl["rs_b"] * 3000.0 / 3500.0
    st = State(np.stack([p, np.full(n, 0.3), np.full(n, 0.05)]),
               np.ones(n, np.int8))
    st.status[1::2] = 0
    st.u[2, 1::2] = rs_sat - 1.0
    du = np.zeros((3, n))
    du[2, 0::2] = -0.1        # saturated: S_g goes negative -> undersaturated
    du[2, 1::2] = 2.0         # undersaturated: R_s above R_s,sat -> saturated
    _, _, nsw = apply_update(m, st, du, Options())
    assert nsw == n
    assert np.all(st.status[0::2] == 0) and np.allclose(st.u[2, 0::2], rs_sat)
    assert np.all(st.status[1::2] == 1) and np.all(st.u[2, 1::2] == 0.0)


def test_blackoil_gas_appears_below_bubble_point():
    """Producing a black-oil model below the bubble point liberates gas
    near the well and conserves every component."""
    m = make_small_c3()
    s = Solver(m, Options.tight_mode())
    st = _state(m)
    for dt in m.schedule:
        m0 = accumulation(m, st.u, st.status)
        new, _ = s.solve_timestep(st, dt)
        m1 = accumulation(m, new.u, new.status)
        q = well_rates(m, new.u, new.status).sum(axis=1)
        dm = (m1 - m0).sum(axis=1)
        assert np.all(np.abs(dm - dt * q) <= 1e-9 * np.abs(dm).max())
        st = new
    assert st.status.sum() > 0
    assert st.u[2][st.status == 1].max() > 0.0


# P9 ------------------------------------------------------------------
def test_p9_localized_and_dd_match_full_newton():
    """The paper's claim that the localized solvers reach the standard
    Newton solution under the same tolerance (tight mode, config-1 model)."""
    m = make_c1()
    o = Options.tight_mode()
    full, _ = Solver(m, o).run(_state(m), m.schedule[:8])
    ls = LocalSolver(m, o)
    log = []
    loc, recs = ls.run_local(_state(m), m.schedule[:8], alg=1, log=log)
    dd, _ = ls.run_local(_state(m), m.schedule[:8], alg=2)
    pmin = full.u[0].min()
    assert np.abs(loc.u[0] - full.u[0]).max() <= 1e-8 * pmin
    assert np.abs(dd.u[0] - full.u[0]).max() <= 1e-8 * pmin
    # localization does real work reduction on this model
    ma = sum(r["n_a"] for r in log) / m.n
    assert ma / len(log) < 0.5


@pytest.mark.parametrize("maker", [make_c1, make_small_c2, make_small_c3])
def test_additive_dd_reaches_full_newton(maker):
    """Algorithm 2 with the additive phase 2 (every pending subdomain from
    the same state, restricted combination) reaches the full-Newton
    solution in tight mode, like the multiplicative form (Section 4.4 and
    the claim of Section 5.3)."""
    m = maker()
    sched = m.schedule[:6]
    o = Options.tight_mode()
    full, _ = Solver(m, o).run(_state(m), sched)
    log = []
    add, _ = LocalSolver(m, o).run_local(_state(m), sched, alg=4, log=log)
    pmin = full.u[0].min()
    assert np.abs(add.u[0] - full.u[0]).max() <= 1e-8 * pmin
    if m.b > 1:
        assert np.abs(add.u[1] - full.u[1]).max() <= 1e-8
    if m.b == 3:
        assert np.array_equal(add.status, full.status)
    assert any(r.get("phase") == 2 for r in log)


def test_additive_dd_leaves_cells_outside_total_set_unchanged():
    """The additive form keeps Section 5.3.1's property: cells outside the
    union of the subdomains keep their old state bitwise over the step."""
    m = make_c1()
    st = _state(m)
    log = []
    new, _, _ = LocalSolver(m, Options()).alg2_timestep(st, m.schedule[5], None, log,
                                                        additive=True)
    vt = log[-1]["vt"]
    outside = np.setdiff1d(np.arange(m.n), np.fromiter(vt, np.int64))
    assert outside.size > m.n // 2
    assert np.array_equal(new.u[:, outside], st.u[:, outside])


def _localized_fracture_model():
    """Config-2 recipe (small, hydrostatic initial state) with only the
    perforated cells always active: fracture cells are localized too.  (An
    initial state out of equilibrium, such as water-filled fractures in an
    oil column, starts transients in every fracture at once, which no
    estimate seeded at the wells can follow.)"""
    m = make_small_c2()
    aa = np.zeros_like(m.always_active)
    aa[m.perf_cell] = 1
    return m.copy_with(always_active=aa)


def test_localized_fractures_reach_full_newton():
    """Localized fracture cells (closure under fracture components): tight
    mode Algorithm 1 reaches the full-Newton solution, and some fracture
    cells are left out of the active sets (unlike the default, which keeps
    every fracture cell active)."""
    m = _localized_fracture_model()
    o = Options.tight_mode()
    full, _ = Solver(m, o).run(_state(m), m.schedule)
    ls = LocalSolver(m, o)
    assert ls.fcomp is not None and len(ls.fcomp[1]) > 1
    log = []
    loc, _ = ls.run_local(_state(m), m.schedule, alg=1, log=log)
    pmin = full.u[0].min()
    assert np.abs(loc.u[0] - full.u[0]).max() <= 1e-8 * pmin
    assert np.abs(loc.u[1] - full.u[1]).max() <= 1e-8
    nfrac = int((m.kind == 1).sum())
    assert min(r["n_a"] for r in log) < m.n - (m.kind == 0).sum() + nfrac
    # paper settings: within the 0.3 psi cutoff of full Newton (without the
    # closure the same run ends about 3 psi away)
    o = Options()
    full, _ = Solver(m, o).run(_state(m), m.schedule)
    loc, _ = LocalSolver(m, o).run_local(_state(m), m.schedule, alg=1)
    assert np.abs(loc.u[0] - full.u[0]).max() <= 0.3 * PSI


def test_dd_leaves_cells_outside_total_set_unchanged():
    """Algorithm 2: cells outside the union of the subdomains keep their
    old state bitwise over the step."""
    m = make_c1()
    o = Options()
    ls = LocalSolver(m, o)
    st = _state(m)
    log = []
    new, _, _ = ls.alg2_timestep(st, m.schedule[3], None, log)
    changed = np.nonzero(new.u[0] != st.u[0])[0]
    assert changed.size > 0
    assert changed.size < m.n // 2
    vt = log[-1]["vt"]
    assert set(changed.tolist()) <= vt
    outside = np.setdiff1d(np.arange(m.n), np.fromiter(vt, np.int64))
    assert outside.size > m.n // 2
    assert np.array_equal(new.u[:, outside], st.u[:, outside])
    # the subdomains are the phase-1 solves, numbered in build order
    p1 = [r for r in log if r.get("phase") == 1]
    assert [r["sub"] for r in p1] == list(range(log[-1]["n_sub"]))
