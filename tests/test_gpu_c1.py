"""GPU parity on the single-phase 2D model (config 1): assembly, sets,
linear solve and whole timesteps against the FP64 oracle."""
import numpy as np
import pytest

from fimgen import PSI, make_c1, make_c1_variant
from oracle import sets as S
from oracle.jacobian import adjacency
from oracle.localized import LocalSolver
from oracle.newton import Options as OOptions
from oracle.newton import Solver, State

from gpu_util import compare_system, oracle_system, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1():
    return make_c1()


@pytest.fixture(scope="module")
def fm_c1(c1):
    from paper_2008_01539_amd import FimModel, Options
    fm = FimModel(c1, Options.tight_mode())
    yield fm
    fm.close()


@pytest.fixture(scope="module")
def oracle_c1(c1):
    return run_oracle(Solver(c1, OOptions.tight_mode()), c1, c1.schedule)


def test_assembly_full_initial_state(c1, fm_c1):
    u = c1.u0
    compare_system(c1, fm_c1, u, u, c1.status0, c1.schedule[0])


def test_assembly_iterate_states(c1, fm_c1, oracle_c1):
    rng = np.random.default_rng(11)
    for k in (0, 5, 12):
        uo = oracle_c1[k].u
        ui = oracle_c1[k + 1].u + rng.normal(0, 5 * PSI, uo.shape)
        compare_system(c1, fm_c1, uo, ui, c1.status0, c1.schedule[k + 1])


def test_assembly_partial_active_set_dirichlet(c1, fm_c1, oracle_c1):
    """Rows of active cells carry the frozen inactive neighbours; columns of
    inactive cells are dropped (J_A = R_A J R_A^T)."""
    rng = np.random.default_rng(12)
    act = (rng.random(c1.n) < 0.3).astype(np.uint8)
    act[c1.n - 3:] = 1
    uo = oracle_c1[3].u
    ui = oracle_c1[4].u
    compare_system(c1, fm_c1, uo, ui, c1.status0, c1.schedule[4], act)
    one = np.zeros(c1.n, np.uint8)
    one[100] = 1
    compare_system(c1, fm_c1, uo, ui, c1.status0, c1.schedule[4], one)


def test_linear_solve_matches_direct_solve(c1, fm_c1, oracle_c1):
    import scipy.sparse.linalg as spla
    uo = oracle_c1[2].u
    ui = oracle_c1[3].u + 7 * PSI
    dt = c1.schedule[3]
    fm_c1.inspect_assemble(uo, ui, c1.status0, dt)
    x, iters, relres = fm_c1.inspect_solve()
    Fo, Jo, _ = oracle_system(c1, uo, ui, c1.status0, dt)
    ref = spla.spsolve(Jo.tocsc(), -Fo.reshape(-1))
    assert relres <= 1e-12
    assert np.abs(x - ref).max() <= 1e-8 * np.abs(ref).max()


@pytest.mark.parametrize("layers", [1, 2, 4])
def test_sets_match_reference_bitwise(c1, fm_c1, layers):
    """m = 2 is Algorithm 1's neighbourhood, m = 4 Algorithm 2's."""
    rp, nb = adjacency(c1)
    rng = np.random.default_rng(5)
    aa = np.nonzero(c1.always_active)[0]
    for trial in range(6):
        act0 = S.initial_active(rp, nb, aa, 2)
        if trial >= 3:
            extra = set(rng.choice(c1.n, 200, replace=False).tolist())
            act0 |= extra
        bnd0 = S.boundary(rp, nb, act0)
        dp = np.zeros(c1.n)
        idx = np.fromiter(act0, np.int64)
        dp[idx] = rng.exponential(1.0, idx.size) * (0.3 * PSI) * (0.5 if trial % 2 else 2.0)
        eps = 0.3 * PSI
        ref_act, ref_bnd, ref_ex = S.alg1_update(rp, nb, act0, bnd0, dp, eps, layers, aa)
        a = np.zeros(c1.n, np.uint8)
        a[idx] = 1
        g = fm_c1.inspect_sets(a, dp, eps, layers)
        assert g["is_expand"] == ref_ex
        assert set(np.nonzero(g["act"])[0].tolist()) == ref_act
        assert set(np.nonzero(g["bnd"])[0].tolist()) == ref_bnd
        assert np.array_equal(g["l2g"], np.array(sorted(ref_act)))


def _run_gpu(model, opts, mode, schedule):
    from paper_2008_01539_amd import FimModel
    fm = FimModel(model, opts)
    fm.set_state(model.u0, model.status0)
    stats = [fm.solve_timestep(dt, mode).as_dict() for dt in schedule]
    u, st = fm.get_state()
    fm.close()
    return u, st, stats


@pytest.mark.parametrize("mode_name", ["FULL", "LOCAL", "DD"])
def test_timesteps_match_oracle_tight(c1, oracle_c1, mode_name):
    import paper_2008_01539_amd as P
    mode = getattr(P, mode_name)
    nsteps = 20 if mode_name != "DD" else 8
    u, _, stats = _run_gpu(c1, P.Options.tight_mode(), mode, c1.schedule[:nsteps])
    ref = oracle_c1[nsteps - 1].u
    err = np.abs(u[0] - ref[0]).max() / ref[0].min()
    assert err <= 1e-8, err
    assert all(s["converged"] for s in stats)
    if mode_name == "LOCAL":
        ma = sum(s["sum_active"] for s in stats) / c1.n
        its = sum(s["iterations"] for s in stats)
        assert ma / its < 0.6


def test_paper_mode_local_vs_full_and_work_ratio(c1):
    """Paper settings (eps = 0.3 psi, m = 2): localized and full Newton agree
    to within the Newton tolerance and localization cuts the work."""
    import paper_2008_01539_amd as P
    uf, _, sf = _run_gpu(c1, P.Options(), P.FULL, c1.schedule)
    ul, _, sl = _run_gpu(c1, P.Options(), P.LOCAL, c1.schedule)
    assert np.abs(uf[0] - ul[0]).max() < 5 * 0.3 * PSI
    ma_l = sum(s["sum_active"] for s in sl) / c1.n
    ma_f = sum(s["sum_active"] for s in sf) / c1.n
    assert ma_f / ma_l > 5


def test_symmetry_on_gpu():
    import paper_2008_01539_amd as P
    m = make_c1_variant()
    u, _, _ = _run_gpu(m, P.Options.tight_mode(), P.FULL, m.schedule)
    nx, ny = m.grid["nx"], m.grid["ny"]
    p = u[0][:m.n_matrix].reshape(ny, nx)
    drop = m.u0[0].max() - p.min()
    assert np.abs(p - p[:, ::-1]).max() <= 1e-9 * drop
    assert np.abs(p - p[::-1, :]).max() <= 1e-9 * drop


def test_run_twice_bitwise(c1):
    import paper_2008_01539_amd as P
    a, _, _ = _run_gpu(c1, P.Options(), P.LOCAL, c1.schedule[:6])
    b, _, _ = _run_gpu(c1, P.Options(), P.LOCAL, c1.schedule[:6])
    assert np.array_equal(a, b)


def test_cell_classes_single_50_day_step(c1):
    """One 50-day step with localized Newton (the paper's flag-profile
    protocol): per iteration the recorded classes match the iteration's
    statistics: boundary and support cells are active, the active count is
    n_A, and the mode is 'expand' exactly when a boundary cell carries a
    non-negligible update."""
    import paper_2008_01539_amd as P
    from fimgen import DAY
    fm = P.FimModel(c1, P.Options())
    fm.set_state(c1.u0, c1.status0)
    fm.record_flags(True)
    seen_expand = seen_shrink = False
    for _ in range(25):
        it = fm.newton_step(50 * DAY, P.LOCAL)
        f = fm.flags()
        act, bnd, sup = (f & 1) > 0, (f & 2) > 0, (f & 4) > 0
        assert act.sum() == it.n_active
        assert not np.any(bnd & ~act) and not np.any(sup & ~act)
        assert bnd.sum() == it.n_boundary
        assert bool(np.any(bnd & sup)) == bool(it.is_expand)
        seen_expand |= bool(it.is_expand)
        seen_shrink |= not it.is_expand
        if it.converged:
            break
    assert it.converged and seen_expand and seen_shrink
    fm.close()
