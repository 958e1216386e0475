"""Parity at the full config-2 size (258,096 cells; config 3's 784,166 for
the sampled rows), in the launch configuration the benchmark times: sampled residual and Jacobian rows
against the oracle evaluated row by row on the sampled cells'
neighbourhoods, the set logic bit for bit, and the converged timestep
checked with the oracle's own residual and mass balance."""
import numpy as np
import pytest

from fimgen import PSI, make_c2
from fimgen.model import Model
from oracle import sets as S
from oracle.jacobian import JacobianBuilder, adjacency
from oracle.physics import accumulation, residual, well_rates

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2():
    return make_c2()


@pytest.fixture(scope="module")
def c2_jb(c2):
    return JacobianBuilder(c2)


def _submodel(m, rows):
    """Cells `rows`, their neighbours, and every connection touching a row:
    the oracle's residual and Jacobian rows of `rows` on this model equal
    the full model's."""
    rp, nb = adjacency(m)
    keep = set(rows.tolist())
    for i in rows:
        keep.update(nb[rp[i]:rp[i + 1]].tolist())
    cells = np.array(sorted(keep))
    idx = -np.ones(m.n, np.int64)
    idx[cells] = np.arange(cells.size)
    isrow = np.zeros(m.n, bool)
    isrow[rows] = True
    sel = isrow[m.conn_i] | isrow[m.conn_j]
    pk = np.isin(m.perf_cell, cells)
    sub = Model(name="sub", n_matrix=0, pv_ref=m.pv_ref[cells], depth=m.depth[cells],
                kind=m.kind[cells], always_active=m.always_active[cells],
                conn_i=idx[m.conn_i[sel]].astype(np.int32),
                conn_j=idx[m.conn_j[sel]].astype(np.int32), conn_T=m.conn_T[sel],
                perf_cell=idx[m.perf_cell[pk]].astype(np.int32), perf_wi=m.perf_wi[pk],
                perf_bhp=m.perf_bhp[pk], fluid=m.fluid, rock=m.rock, gravity=m.gravity,
                u0=m.u0[:, cells], status0=m.status0[cells], schedule=m.schedule)
    return sub, cells, idx


def test_sampled_rows_full_size(c2):
    import paper_2008_01539_amd as P
    rng = np.random.default_rng(21)
    fm = P.FimModel(c2, P.Options(precision=P.MIXED))
    uo = c2.u0.copy()
    ui = c2.u0.copy()
    ui[0] += rng.normal(0, 20 * PSI, c2.n)
    ui[1] = np.clip(ui[1] + rng.uniform(0, 0.3, c2.n), 0, 1)
    dt = c2.schedule[10]
    g = fm.inspect_assemble(uo, ui, c2.status0, dt, cap_blocks=14 * c2.n)
    fm.close()
    assert g["n_active"] == c2.n
    b = c2.b
    # include all fracture/perforated kinds: sample matrix, fracture, perforated
    rows = np.unique(np.concatenate([rng.choice(c2.n_matrix, 300, replace=False),
                                     rng.choice(np.arange(c2.n_matrix, c2.n), 300, replace=False),
                                     c2.perf_cell]))
    sub, cells, idx = _submodel(c2, rows)
    m_old = accumulation(sub, uo[:, cells], c2.status0[cells])
    R, J = JacobianBuilder(sub).build(ui[:, cells], c2.status0[cells], m_old, dt)
    J = J.tocsr()
    for i in rows:
        li = idx[i]
        Fo = R[:, li]
        assert np.allclose(g["F"][i], Fo, rtol=1e-11, atol=1e-12 * np.abs(J[li * b:(li + 1) * b]).sum())
        ro = J[li * b:(li + 1) * b].toarray()
        scale = np.abs(ro).max()
        for q in range(g["row_ptr"][i], g["row_ptr"][i + 1]):
            j = g["col"][q]
            ref = ro[:, idx[j] * b:(idx[j] + 1) * b]
            assert np.abs(g["val"][q] - ref).max() <= 1e-12 * scale


def test_sets_full_size_bitwise(c2):
    import paper_2008_01539_amd as P
    rp, nb = adjacency(c2)
    rng = np.random.default_rng(8)
    aa = np.nonzero(c2.always_active)[0]
    act0 = S.initial_active(rp, nb, aa, 2)
    bnd0 = S.boundary(rp, nb, act0)
    dp = np.zeros(c2.n)
    idx = np.fromiter(act0, np.int64)
    dp[idx] = rng.exponential(0.3 * PSI, idx.size)
    ref_act, ref_bnd, ref_ex = S.alg1_update(rp, nb, act0, bnd0, dp, 0.3 * PSI, 2, aa)
    a = np.zeros(c2.n, np.uint8)
    a[idx] = 1
    fm = P.FimModel(c2, P.Options())
    out = fm.inspect_sets(a, dp, 0.3 * PSI, 2)
    fm.close()
    assert out["is_expand"] == ref_ex
    assert np.array_equal(np.nonzero(out["act"])[0], np.array(sorted(ref_act)))
    assert np.array_equal(np.nonzero(out["bnd"])[0], np.array(sorted(ref_bnd)))


@pytest.mark.parametrize("layers", [4, 2])
def test_dd_expand_full_size_bitwise(c2, layers):
    """Algorithm 2's phase-1 partitions at full size against the oracle's
    set logic, bit for bit (two chained expansions, then a stop)."""
    import paper_2008_01539_amd as P
    from gpu_util import check_dd_expand
    fm = P.FimModel(c2, P.Options(precision=P.MIXED))
    check_dd_expand(fm, c2, np.random.default_rng(90 + layers), layers, 0.3 * PSI, rounds=2)
    fm.close()


@pytest.mark.parametrize("mode_name", ["FULL", "LOCAL", "RESID"])
def test_converged_steps_satisfy_oracle_equations(c2, c2_jb, mode_name):
    """Tight mode, mixed precision, the first three steps at full size: the
    oracle's residual at the GPU state is at the level of a sub-1e-3 Pa
    pressure error per row, and the step mass balance closes (the
    residual-based mode with a vanishing residual cutoff)."""
    import paper_2008_01539_amd as P
    fm = P.FimModel(c2, P.Options.tight_mode(precision=P.MIXED, eps_res=1e-14))
    fm.set_state(c2.u0, c2.status0)
    prev, prev_st = c2.u0.copy(), c2.status0.copy()
    for k, dt in enumerate(c2.schedule[:3]):
        fm.solve_timestep(dt, getattr(P, mode_name))
        u, st = fm.get_state()
        m_old = accumulation(c2, prev, prev_st)
        dm = (accumulation(c2, u, st) - m_old).sum(axis=1)
        q = well_rates(c2, u, st).sum(axis=1)
        assert np.all(np.abs(dm - dt * q) <= 1e-8 * np.abs(dm).max())
        if k == 2:
            R, J = c2_jb.build(u, st, m_old, dt)
            # residual equivalent of a 1e-3 Pa pressure error, per row
            pcols = J[:, 0::2]
            scale = np.asarray(abs(pcols).sum(axis=1)).ravel().reshape(c2.n, 2).T
            assert np.all(np.abs(R) <= 1e-3 * scale + 1e-30)
        prev, prev_st = u, st
    fm.close()


def test_residual_error_measure_full_size(c2):
    """The residual-based mode's error measure on every one of the 258,096
    cells against the oracle's (vectorised over the whole model) at an
    iterate away from convergence: FP64 on both sides, ≤ 1e-11 of the
    largest value; and the unconverged set at the default cutoff with its
    neighbour layer, bit for bit."""
    import paper_2008_01539_amd as P
    from oracle.localized import resid_error
    rng = np.random.default_rng(31)
    u_old = c2.u0.copy()
    u = u_old.copy()
    u[0] += rng.uniform(-5, 5, c2.n) * PSI
    u[1] = np.clip(u[1] + rng.uniform(-0.01, 0.01, c2.n), 0.0, 1.0)
    dt = c2.schedule[4]
    eo = resid_error(c2, u, c2.status0, accumulation(c2, u_old, c2.status0), dt)
    fm = P.FimModel(c2, P.Options(precision=P.MIXED))
    try:
        eg = fm.inspect_resid_error(u_old, u, c2.status0, dt)
        assert np.abs(eg - eo).max() <= 1e-11 * eo.max()
        tol = float(np.quantile(eo, 0.97))
        g = fm.inspect_resid_sets(eo, tol, 1)
    finally:
        fm.close()
    rp, nb = adjacency(c2)
    ref = S.resid_active(rp, nb, eo, tol, 1)
    assert g["n_unconverged"] == int((eo >= tol).sum())
    assert np.array_equal(g["l2g"], np.array(sorted(ref)))


# three steps of the config-3 schedule taken from the initial state (0.03,
# 0.11 and 0.35 days): enough drawdown to take the wells' neighbourhoods
# below the bubble point
C3_STEPS = (12, 16, 20)


@pytest.fixture(scope="module")
def c3():
    from fimgen import make_c3
    return make_c3()


@pytest.fixture(scope="module")
def c3_pscale(c3):
    """Per row and component: the residual change of a 1 Pa error in every
    pressure of the row's stencil, sum_j |dR_i/dp_j| (oracle, pressure
    columns only), at the initial state for the middle step."""
    m_old = accumulation(c3, c3.u0, c3.status0)
    _, J = JacobianBuilder(c3).build(c3.u0, c3.status0, m_old, c3.schedule[C3_STEPS[1]],
                                     variables=(0,))
    return np.asarray(abs(J).sum(axis=1)).ravel().reshape(c3.n, 3).T


@pytest.mark.parametrize("mode_name", ["FULL", "LOCAL"])
def test_converged_steps_full_size_blackoil(c3, c3_pscale, mode_name):
    """Config 3 at full size (784,166 cells, 3x3 blocks), tight mode, mixed
    precision: after each of three steps the step mass balance closes for
    water, oil and gas; the phase status is consistent (saturated cells
    with 0 <= S_g <= 1 - S_w, undersaturated ones at or below R_s,sat(p),
    so the oracle's switching rule changes nothing); after the last step
    the oracle's residual at the GPU state is below a 1e-3 Pa pressure
    error in every row, and gas has come out of solution somewhere."""
    import paper_2008_01539_amd as P
    from oracle.newton import Options as OOptions
    from oracle.newton import State, apply_update
    fl = c3.fluid
    fm = P.FimModel(c3, P.Options.tight_mode(precision=P.MIXED))
    fm.set_state(c3.u0, c3.status0)
    prev, prev_st = c3.u0.copy(), c3.status0.copy()
    try:
        for k, dt in enumerate(c3.schedule[list(C3_STEPS)]):
            fm.solve_timestep(dt, getattr(P, mode_name))
            u, st = fm.get_state()
            m_old = accumulation(c3, prev, prev_st)
            dm = (accumulation(c3, u, st) - m_old).sum(axis=1)
            q = well_rates(c3, u, st).sum(axis=1)
            # water barely moves (connate saturation): its imbalance is
            # measured against the largest component change, as for config 2
            for c in range(3):
                assert abs(dm[c] - dt * q[c]) <= 1e-8 * np.abs(dm).max(), (k, c)
            sat = st == 1
            assert np.all(u[2][sat] >= 0.0) and np.all(u[2][sat] <= 1.0 - u[1][sat])
            rs_sat = fl["rs_b"] * u[0] / fl["p_b"]
            assert np.all(u[2][~sat] <= rs_sat[~sat])
            chk = State(u.copy(), st.copy())
            _, _, nsw = apply_update(c3, chk, np.zeros_like(u), OOptions())
            assert nsw == 0
            prev, prev_st = u, st
        assert sat.sum() > 0
        R = residual(c3, u, st, m_old, dt)
        assert np.all(np.abs(R) <= 1e-3 * c3_pscale + 1e-30)
    finally:
        fm.close()


def test_sampled_rows_full_size_blackoil(c3):
    """Config 3 at full size (784,166 cells, 3x3 blocks, the largest
    system the benchmark assembles): sampled residual and Jacobian rows
    against the oracle on the sampled cells' neighbourhoods, with a random
    third of the cells in the saturated state so that both black-oil
    variable sets and gas-liberating cells are covered."""
    import paper_2008_01539_amd as P
    rng = np.random.default_rng(33)
    status = c3.status0.copy()
    sat = rng.random(c3.n) < 0.33
    status[sat] = 1
    uo = c3.u0.copy()
    uo[2, sat] = 0.03
    ui = uo.copy()
    ui[0] += rng.normal(0, 20 * PSI, c3.n)
    ui[1] = np.clip(ui[1] + rng.uniform(0, 0.05, c3.n), 0, 1)
    ui[2, sat] += rng.uniform(0.0, 0.02, int(sat.sum()))
    dt = c3.schedule[12]
    fm = P.FimModel(c3, P.Options(precision=P.MIXED))
    try:
        g = fm.inspect_assemble(uo, ui, status, dt, cap_blocks=12 * c3.n)
    finally:
        fm.close()
    assert g["n_active"] == c3.n
    b = c3.b
    rows = np.unique(np.concatenate([rng.choice(c3.n_matrix, 300, replace=False),
                                     rng.choice(np.arange(c3.n_matrix, c3.n), 300, replace=False),
                                     c3.perf_cell]))
    sub, cells, idx = _submodel(c3, rows)
    m_old = accumulation(sub, uo[:, cells], status[cells])
    R, J = JacobianBuilder(sub).build(ui[:, cells], status[cells], m_old, dt)
    J = J.tocsr()
    for i in rows:
        li = idx[i]
        assert np.allclose(g["F"][i], R[:, li], rtol=1e-11,
                           atol=1e-12 * np.abs(J[li * b:(li + 1) * b]).sum())
        ro = J[li * b:(li + 1) * b].toarray()
        scale = np.abs(ro).max()
        for q in range(g["row_ptr"][i], g["row_ptr"][i + 1]):
            j = g["col"][q]
            ref = ro[:, idx[j] * b:(idx[j] + 1) * b]
            assert np.abs(g["val"][q] - ref).max() <= 1e-12 * scale
