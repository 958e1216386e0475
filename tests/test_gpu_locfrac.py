"""Localized fracture cells (fracture cells not always active; the active
sets of Algorithm 1 closed under fracture components, the reading of
Section 5.2.3 the oracle states): the set update bit for bit against the
oracle on the small config-2 model and on config 2 at full size, and
timesteps against the oracle's full Newton in tight mode and at the
paper's settings."""
import numpy as np
import pytest

from fimgen import PSI, make_c2, make_small_c2
from oracle import sets as S
from oracle.jacobian import adjacency
from oracle.localized import LocalSolver
from oracle.newton import Options as OOptions
from oracle.newton import Solver, State

from gpu_util import flags_of, run_oracle

pytestmark = pytest.mark.gpu


def _localize(m):
    aa = np.zeros_like(m.always_active)
    aa[m.perf_cell] = 1
    return m.copy_with(always_active=aa)


@pytest.fixture(scope="module")
def c2s_loc():
    return _localize(make_small_c2())


def _check_sets(model, fm, rng, layers, rounds):
    rp, nb = adjacency(model)
    fc = S.fracture_components(rp, nb, model.kind == 1)
    aa = np.nonzero(model.always_active)[0]
    act = S.initial_active(rp, nb, aa, layers, None, fc)
    n = model.n
    saw = set()
    for _ in range(rounds):
        bnd = S.boundary(rp, nb, act)
        dp = np.zeros(n)
        idx = np.fromiter(act, np.int64)
        dp[idx] = rng.exponential(0.2 * PSI, idx.size) * rng.choice([0.0, 1.0], idx.size)
        ref_act, ref_bnd, ref_ex = S.alg1_update(rp, nb, act, bnd, dp, 0.3 * PSI, layers, aa, fc)
        got = fm.inspect_sets(flags_of(act, n), dp, 0.3 * PSI, layers)
        assert got["is_expand"] == ref_ex
        assert np.array_equal(got["act"], flags_of(ref_act, n))
        assert np.array_equal(got["bnd"], flags_of(ref_bnd, n))
        saw.add(ref_ex)
        act = ref_act
    return saw


def test_sets_localized_fractures_bitwise(c2s_loc):
    import paper_2008_01539_amd as P
    fm = P.FimModel(c2s_loc, P.Options())
    saw = _check_sets(c2s_loc, fm, np.random.default_rng(5), 2, 6)
    fm.close()
    assert saw == {True, False} or saw == {True}


def test_sets_localized_fractures_full_size_bitwise():
    import paper_2008_01539_amd as P
    m = _localize(make_c2())
    fm = P.FimModel(m, P.Options(precision=P.MIXED))
    _check_sets(m, fm, np.random.default_rng(6), 2, 2)
    fm.close()


@pytest.mark.parametrize("prec", ["FP64", "MIXED"])
def test_localized_fracture_timesteps_match_oracle(c2s_loc, prec):
    """Tight mode: Algorithm 1 with localized fracture cells reaches the
    oracle's full-Newton solution (1e-8 relative p, 1e-8 S); and it leaves
    some fracture cells out of its active sets."""
    import paper_2008_01539_amd as P
    m = c2s_loc
    ref = run_oracle(Solver(m, OOptions.tight_mode()), m, m.schedule)[-1]
    fm = P.FimModel(m, P.Options.tight_mode(precision=getattr(P, prec)))
    fm.set_state(m.u0, m.status0)
    min_active = m.n
    for dt in m.schedule:
        while True:
            it = fm.newton_step(dt, P.LOCAL)
            min_active = min(min_active, it.n_active)
            if it.converged:
                break
    u, _ = fm.get_state()
    fm.close()
    assert np.abs(u[0] - ref.u[0]).max() <= 1e-8 * ref.u[0].min()
    assert np.abs(u[1] - ref.u[1]).max() <= 1e-8
    assert min_active < int((m.kind == 1).sum())


def test_localized_fractures_paper_mode_within_cutoff(c2s_loc):
    """Paper settings: within the 0.3 psi cutoff of the oracle's full
    Newton, like the oracle's own localized run."""
    import paper_2008_01539_amd as P
    m = c2s_loc
    ref = run_oracle(Solver(m, OOptions()), m, m.schedule)[-1]
    fm = P.FimModel(m, P.Options(lin_rtol=1e-10, forcing_max=0.0))
    fm.set_state(m.u0, m.status0)
    for dt in m.schedule:
        fm.solve_timestep(dt, P.LOCAL)
    u, _ = fm.get_state()
    fm.close()
    assert np.abs(u[0] - ref.u[0]).max() <= 0.3 * PSI
