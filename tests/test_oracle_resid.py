"""Pins of the oracle's residual-based localization (the estimator of Lu
and Beckner that Sections 1 and 4.2 describe) against facts that do not
come from the oracle: closed forms of the error measure on one and two
cells, brute-force neighbourhoods on a chain and a grid, the residual
vanishing at the standard Newton solution, and the method reaching that
solution; and the empty active set of Algorithms 1 and 2.  CPU only."""
import numpy as np

from fimgen import DAY, FLUID_DEADOIL, PSI, make_c1, make_chain, make_tiny
from oracle.jacobian import adjacency
from oracle.localized import LocalSolver, resid_error
from oracle.newton import Options, Solver, State
from oracle.physics import accumulation
from oracle import sets


def _state(m):
    return State(m.u0.copy(), m.status0.copy())


def test_error_single_cell_is_relative_pore_volume_change():
    """One cell without connections or well, incompressible liquid: the
    step's mass imbalance is the pore-volume change, so e = c_r |p - p^n|
    whatever dt is."""
    m = make_tiny("one")
    m.fluid["c"] = 0.0
    m.perf_wi[:] = 0.0
    u_old = m.u0.copy()
    dp = 37.0 * PSI
    u = u_old + dp
    for dt in (0.1 * DAY, 3.0 * DAY):
        m_old = accumulation(m, u_old, m.status0)
        e = resid_error(m, u, m.status0, m_old, dt)
        assert abs(e[0] - m.rock["c_r"] * dp) <= 1e-12 * m.rock["c_r"] * dp


def test_error_dead_oil_is_saturation_change():
    """Dead oil in one cell, incompressible phases and rock: moving water
    saturation by ds changes the water mass by V rho_w ds and the oil mass
    by -V rho_o ds, so both components give e = |ds| (a swapped density
    order would give rho_w/rho_o |ds| for one of them)."""
    m = make_tiny("one", fluid_kind=FLUID_DEADOIL)
    m.fluid["c_w"] = m.fluid["c_o"] = 0.0
    m.rock["c_r"] = 0.0
    m.perf_wi[:] = 0.0
    u_old = m.u0.copy()
    ds = 0.0731
    u = u_old.copy()
    u[1] += ds
    m_old = accumulation(m, u_old, m.status0)
    e = resid_error(m, u, m.status0, m_old, 2.0 * DAY)
    assert abs(e[0] - ds) <= 1e-12
    assert m.fluid["rho_w"] != m.fluid["rho_o"]


def test_error_two_cells_is_darcy_volume_over_pore_volume():
    """Two cells of an incompressible chain at rest in time (u = u^n) with
    a pressure difference and no gravity head: each cell's imbalance is the
    Darcy flow T (p_1 - p_0) / mu, so e_i = dt T |p_1 - p_0| / (mu V_i)."""
    m = make_chain(2, 10.0)
    m.perf_wi[:] = 0.0
    m.rock["c_r"] = 0.0
    m.gravity = 0.0
    u = m.u0.copy()
    u[0, 1] += 120.0 * PSI
    dt = 0.4 * DAY
    m_old = accumulation(m, u, m.status0)
    e = resid_error(m, u, m.status0, m_old, dt)
    q = m.conn_T[0] * 120.0 * PSI / m.fluid["mu"]
    exact = dt * q / m.pv_ref
    assert np.all(np.abs(e - exact) <= 1e-12 * exact)


def test_error_vanishes_at_the_newton_solution():
    """At the converged standard Newton state of a step the residual, and
    so the error measure, is at rounding level on every cell."""
    m = make_c1()
    o = Options.tight_mode()
    st = _state(m)
    dt = m.schedule[2]
    new, _ = Solver(m, o).solve_timestep(st, dt)
    m_old = accumulation(m, st.u, st.status)
    e0 = resid_error(m, st.u, st.status, m_old, dt)
    e1 = resid_error(m, new.u, new.status, m_old, dt)
    assert e0.max() > 1e-6
    assert e1.max() < 1e-12


def test_resid_active_chain_and_grid_brute_force():
    """Unconverged cells plus one layer on a chain (intervals) and on a
    5x5 grid (the 5-point star); a value equal to the tolerance counts."""
    m = make_chain(10, 100.0)
    rp, nb = adjacency(m)
    err = np.zeros(10)
    err[3] = 1e-6
    err[8] = 5e-6
    assert sets.resid_active(rp, nb, err, 1e-6, 1) == {2, 3, 4, 7, 8, 9}
    assert sets.resid_active(rp, nb, err, 2e-6, 1) == {7, 8, 9}
    assert sets.resid_active(rp, nb, err, 1e-6, 0) == {3, 8}
    assert sets.resid_active(rp, nb, err, 1e-5, 1) == set()
    g = make_tiny("grid5")
    rp, nb = adjacency(g)
    err = np.zeros(25)
    err[12] = 1.0                     # centre (2, 2); the NNC joins 0 and 24
    assert sets.resid_active(rp, nb, err, 0.5, 1) == {7, 11, 12, 13, 17}
    err[12] = 0.0
    err[0] = 1.0
    assert sets.resid_active(rp, nb, err, 0.5, 1) == {0, 1, 5, 24}


def test_resid_localization_reaches_full_newton():
    """With a vanishing residual tolerance the residual-based localization
    reaches the standard Newton solution (tight mode, config-1 model), and
    every step's first iteration covers the whole domain."""
    m = make_c1()
    o = Options.tight_mode(eps_res=1e-14)
    sched = m.schedule[:5]
    full, _ = Solver(m, o).run(_state(m), sched)
    log = []
    loc, recs = LocalSolver(m, o).run_local(_state(m), sched, alg=3, log=log)
    assert np.abs(loc.u[0] - full.u[0]).max() <= 1e-8 * full.u[0].min()
    k = 0
    for r in recs:
        assert log[k]["n_a"] == m.n
        k += r["iters"]
    assert any(e["n_a"] < m.n for e in log)


def test_resid_localization_costs_more_than_algorithm_1():
    """The paper's argument against the residual-based estimate: starting
    every step from the whole domain makes it do more work than Algorithm 1
    at paper settings, at similar accuracy."""
    m = make_c1()
    o = Options()
    sched = m.schedule[:6]
    full, _ = Solver(m, o).run(_state(m), sched)
    ls = LocalSolver(m, o)
    l1, l3 = [], []
    s1, _ = ls.run_local(_state(m), sched, alg=1, log=l1)
    s3, _ = ls.run_local(_state(m), sched, alg=3, log=l3)
    w1 = sum(e["n_a"] for e in l1)
    w3 = sum(e["n_a"] for e in l3)
    assert w3 > 5 * w1
    assert np.abs(s3.u[0] - full.u[0]).max() < 1.0 * PSI


def test_empty_active_set_leaves_the_state_unchanged():
    """A model with no always-active cells and no history: Algorithms 1 and
    2 start from an empty set, whose restricted Newton step is empty, so
    the step ends after one iteration with u^n unchanged."""
    m = make_tiny("grid3")
    m.always_active[:] = 0
    ls = LocalSolver(m, Options())
    st = _state(m)
    for alg in (ls.alg1_timestep, ls.alg2_timestep):
        log = []
        new, its, sup = alg(st, m.schedule[0], None, log)
        assert its == 1 and log[0]["n_a"] == 0
        assert np.array_equal(new.u, st.u) and not sup
