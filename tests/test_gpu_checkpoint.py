"""Checkpoints between timesteps (fim_get_checkpoint / fim_set_checkpoint):
a run resumed from a checkpoint in a fresh model continues bit for bit as
the uninterrupted run, with Algorithm 1's and Algorithm 2's first active
set seeded from the previous step's support (Sections 4.3, 4.4)."""
import numpy as np
import pytest

from fimgen import make_c1, make_small_c2, make_small_c3

pytestmark = pytest.mark.gpu


def _run(fm, dts, mode):
    for dt in dts:
        fm.solve_timestep(dt, mode)


@pytest.mark.parametrize("maker,mode_name", [(make_small_c3, "LOCAL"), (make_small_c2, "LOCAL"),
                                             (make_c1, "DD"), (make_small_c2, "RESID")])
def test_resume_from_checkpoint_is_bitwise(maker, mode_name):
    import paper_2008_01539_amd as P
    m = maker()
    mode = getattr(P, mode_name)
    opts = P.Options(precision=P.MIXED)
    k, n = 3, 6
    ref = P.FimModel(m, opts)
    ref.set_state(m.u0, m.status0)
    _run(ref, m.schedule[:n], mode)
    u_ref, st_ref = ref.get_state()
    ref.close()

    a = P.FimModel(m, opts)
    a.set_state(m.u0, m.status0)
    _run(a, m.schedule[:k], mode)
    blob = a.get_checkpoint()
    a.close()
    b = P.FimModel(m, opts)
    b.set_checkpoint(blob)
    _run(b, m.schedule[k:n], mode)
    u, st = b.get_state()
    b.close()
    assert np.array_equal(u, u_ref)
    assert np.array_equal(st, st_ref)


def test_checkpoint_errors():
    import paper_2008_01539_amd as P
    from paper_2008_01539_amd.fim import FimError
    m = make_small_c2()
    fm = P.FimModel(m, P.Options(precision=P.MIXED))
    fm.set_state(m.u0, m.status0)
    fm.solve_timestep(m.schedule[0], P.LOCAL)
    blob = fm.get_checkpoint()
    u0, st0 = fm.get_state()
    # inside a timestep: refused
    it = fm.newton_step(m.schedule[1], P.LOCAL)
    if not it.converged:
        with pytest.raises(FimError):
            fm.get_checkpoint()
    # truncated or foreign blobs: refused, state kept
    u1, st1 = fm.get_state()
    with pytest.raises(FimError):
        fm.set_checkpoint(blob[:-1])
    with pytest.raises(FimError):
        fm.set_checkpoint(b"x" * len(blob))
    other = P.FimModel(make_c1(), P.Options(precision=P.MIXED))
    other.set_state(make_c1().u0)
    with pytest.raises(FimError):
        fm.set_checkpoint(other.get_checkpoint())
    other.close()
    u2, _ = fm.get_state()
    assert np.array_equal(u1, u2)
    # a valid blob restores the state it was taken at
    fm.set_checkpoint(blob)
    u3, st3 = fm.get_state()
    assert np.array_equal(u3, u0) and np.array_equal(st3, st0)
    fm.close()
