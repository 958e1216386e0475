"""GPU parity on the smallest models: one cell, 3x3 and 5x5 grids with a
long-range non-neighbour connection (a single ragged slice of 64 rows),
for all three fluid families and every solver mode, against the oracle's
standard Newton solution in tight mode."""
import numpy as np
import pytest

from fimgen import FLUID_BLACKOIL, FLUID_DEADOIL, FLUID_SINGLE, make_tiny
from oracle.newton import Options as OOptions
from oracle.newton import Solver

from gpu_util import run_oracle

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("which", ["one", "grid3", "grid5"])
@pytest.mark.parametrize("kind", [FLUID_SINGLE, FLUID_DEADOIL, FLUID_BLACKOIL])
def test_tiny_models_all_modes_match_oracle(which, kind):
    import paper_2008_01539_amd as P
    m = make_tiny(which, kind)
    ref = run_oracle(Solver(m, OOptions.tight_mode()), m, m.schedule)[-1]
    for mode in (P.FULL, P.LOCAL, P.DD, P.RESID):
        for prec in (P.FP64, P.MIXED):
            o = P.Options.tight_mode(precision=prec, eps_res=1e-14)
            fm = P.FimModel(m, o)
            try:
                fm.set_state(m.u0, m.status0)
                for dt in m.schedule:
                    st = fm.solve_timestep(dt, mode)
                    assert st.converged
                u, s = fm.get_state()
            finally:
                fm.close()
            tag = (which, kind, mode, prec)
            assert np.abs(u[0] - ref.u[0]).max() <= 1e-8 * ref.u[0].min(), tag
            if m.b >= 2:
                assert np.abs(u[1] - ref.u[1]).max() <= 1e-8, tag
            if m.b == 3:
                assert np.array_equal(s, ref.status), tag
                assert np.abs(u[2] - ref.u[2]).max() <= 1e-8 * max(1.0, np.abs(ref.u[2]).max()), tag
