"""The allocation-free Newton iteration (fim_newton_step_noalloc) against
fim_newton_step on identical models: the same state and statistics after
every iteration, on a larger model and then on a smaller one (the shared
scratch array then holds the larger call's contents), and the refusals of
what it does not cover (oversized models, Algorithm 2)."""
import numpy as np
import pytest

FIM_E_ARG, FIM_E_STATE = -1, -4

pytestmark = pytest.mark.gpu


def _pair_run(model, opts, mode, steps, tag):
    """Runs `steps` timesteps twice, Newton iteration by Newton iteration:
    through fim_newton_step and through fim_newton_step_noalloc; asserts
    identical iterates and statistics.  Returns the iteration count."""
    import paper_2008_01539_amd as P
    ref = P.FimModel(model, opts)
    na = P.FimModel(model, opts)
    its = 0
    try:
        ref.set_state(model.u0, model.status0)
        na.set_state(model.u0, model.status0)
        for dt in model.schedule[:steps]:
            while True:
                a = ref.newton_step(dt, mode)
                b = na.newton_step_noalloc(dt, mode)
                its += 1
                ua, sa = ref.get_state()
                ub, sb = na.get_state()
                where = (tag, mode, its)
                # same kernels, launch shapes and reduction order: same bits
                assert np.array_equal(ua, ub), where
                assert np.array_equal(sa, sb), where
                for f in ("n_active", "krylov_iters", "converged", "is_expand",
                          "refine_passes", "n_switch"):
                    assert getattr(a, f) == getattr(b, f), (where, f)
                assert a.dp_max == b.dp_max, where
                # and within the parity bar on pressure in any case
                assert np.abs(ua[0] - ub[0]).max() <= 1e-8 * np.abs(ua[0]).min(), where
                if a.converged:
                    break
                assert its < 400, where
    finally:
        ref.close()
        na.close()
    return its


def test_noalloc_matches_newton_step_larger_then_smaller():
    import paper_2008_01539_amd as P
    from fimgen import make_c1, make_small_c2
    print("noalloc: config 1 (4128 cells), Algorithm 1, FP64", flush=True)
    big = make_c1()
    n1 = _pair_run(big, P.Options(), P.LOCAL, 6, "c1")
    assert n1 >= 6
    print("noalloc: small config 2 (1448 cells), full / Algorithm 1 / residual, mixed",
          flush=True)
    small = make_small_c2()
    assert small.n < big.n
    for mode in (P.LOCAL, P.FULL, P.RESID):
        n2 = _pair_run(small, P.Options(precision=P.MIXED), mode, 3, "c2-small")
        assert n2 >= 3


def test_noalloc_refuses_what_it_does_not_cover():
    import paper_2008_01539_amd as P
    from fimgen import make_c1, make_chain
    m = make_c1()
    fm = P.FimModel(m, P.Options())
    try:
        fm.set_state(m.u0, m.status0)
        with pytest.raises(P.FimError) as e:
            fm.newton_step_noalloc(m.schedule[0], P.DD)
        assert e.value.code == FIM_E_ARG
        fm.profile(True)
        with pytest.raises(P.FimError) as e:
            fm.newton_step_noalloc(m.schedule[0], P.LOCAL)
        assert e.value.code == FIM_E_STATE
        fm.profile(False)
        fm.newton_step_noalloc(m.schedule[0], P.LOCAL)   # usable again
    finally:
        fm.close()
    # one cell more than the scratch array is sized for: refused on the host
    big = make_chain((1 << 22) + 1, 1000.0)
    fb = P.FimModel(big, P.Options())
    try:
        fb.set_state(big.u0, big.status0)
        with pytest.raises(P.FimError) as e:
            fb.newton_step_noalloc(big.schedule[0], P.FULL)
        assert e.value.code == FIM_E_ARG
        assert "4194304" in str(e.value)
    finally:
        fb.close()
