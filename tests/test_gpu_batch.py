"""Batched Newton iterations over several models and the serving loop on
the GPU: every member's result equals its result alone (bitwise, since
each member keeps its own block partition and reduction order)."""
import numpy as np
import pytest

from fimgen import make_c1, make_c1_variant, make_small_c2, make_small_c3

pytestmark = pytest.mark.gpu


def _solo(model, opts, mode, dts):
    import paper_2008_01539_amd as P
    fm = P.FimModel(model, opts)
    fm.set_state(model.u0, model.status0)
    for dt in dts:
        fm.solve_timestep(dt, mode)
    u, st = fm.get_state()
    fm.close()
    return u, st


def _batched(models, opts, mode, nsteps):
    """Continuous batching: members leave the batch when they finished
    their steps; each member advances through its own schedule.  opts may
    be one Options for all members or one per member."""
    import paper_2008_01539_amd as P
    fms = []
    per = opts if isinstance(opts, (list, tuple)) else [opts] * len(models)
    for m, o in zip(models, per):
        fm = P.FimModel(m, o)
        fm.set_state(m.u0, m.status0)
        fms.append(fm)
    step = [0] * len(models)
    live = list(range(len(models)))
    bat = P.FimBatch([fms[i] for i in live])
    sizes = []
    mq = mode if isinstance(mode, (list, tuple)) else [mode] * len(models)
    while live:
        dts = [models[i].schedule[step[i]] for i in live]
        stats, codes = bat.newton_step(dts, [mq[i] for i in live])
        assert np.all(codes == 0)
        sizes.append(len(live))
        nxt = []
        for i, st in zip(live, stats):
            if st["converged"]:
                step[i] += 1
            if step[i] < nsteps:
                nxt.append(i)
        if nxt != live and nxt:
            bat.set_models([fms[i] for i in nxt])
        live = nxt
    out = [fm.get_state() for fm in fms]
    bat.close()
    for fm in fms:
        fm.close()
    return out, sizes


@pytest.mark.parametrize("prec", ["FP64", "MIXED"])
def test_batch_equals_solo_single_phase(prec):
    import paper_2008_01539_amd as P
    models = [make_c1(), make_c1_variant(), make_c1(seed=9, nx=40, ny=30, frac_rows=(5, 25))]
    opts = P.Options(precision=getattr(P, prec))
    n = 6
    got, sizes = _batched(models, opts, P.LOCAL, n)
    for m, (u, st) in zip(models, got):
        ref, _ = _solo(m, opts, P.LOCAL, m.schedule[:n])
        assert np.array_equal(u, ref)
    assert max(sizes) == 3


def test_batch_equals_solo_two_phase_mixed():
    import paper_2008_01539_amd as P
    models = [make_small_c2(), make_small_c2(seed=23, nx=30, ny=14, nfrac=20),
              make_small_c2(seed=24, nx=16, ny=10, nz=3, nfrac=6, nstage=2)]
    opts = P.Options(precision=P.MIXED)
    n = 5
    for mode in (P.LOCAL, P.FULL, P.RESID):
        got, _ = _batched(models, opts, mode, n)
        for m, (u, st) in zip(models, got):
            ref, _ = _solo(m, opts, mode, m.schedule[:n])
            assert np.array_equal(u, ref)


def test_serving_results_same_alone_and_in_the_mix():
    """Poisson requests over sessions of two block sizes, batched
    continuously; each session's state after its requests equals the same
    steps run alone."""
    import paper_2008_01539_amd as P
    from paper_2008_01539_amd.serve import GpuExecutor, Server, SessionSpec
    specs = []
    for k, m in enumerate([make_c1(), make_c1_variant(), make_small_c2(),
                           make_small_c2(seed=23, nx=30, ny=14, nfrac=20)]):
        specs.append(SessionSpec(name=f"s{k}", model=m, options=P.Options(precision=P.MIXED),
                                 schedule=m.schedule))
    ex = GpuExecutor()
    srv = Server(specs, ex, budget_bytes=8 << 30, max_inflight=16,
                 footprint=lambda s: P.estimate_bytes(s.model, s.options))
    summ = srv.run_poisson(rate=40.0, duration=1.5, mix=np.array([0.3, 0.3, 0.2, 0.2]), seed=5)
    assert summ["completed"] == len(srv.done) and summ["failed"] == 0
    assert max(srv.stats.latencies) > 0
    for s in srv.sessions:
        if s.next_step == 0:
            continue
        u, _ = s.handle.get_state()
        sched = s.spec.schedule
        dts = [sched[k % len(sched)] for k in range(s.next_step)]
        ref, _ = _solo(s.spec.model, s.spec.options, s.spec.mode, dts)
        assert np.array_equal(u, ref), s.spec.name
    ex.close()


def test_serving_tight_sessions_match_oracle():
    """Tight-mode sessions served by the continuously batching loop (Poisson
    requests, members joining and leaving the batch) reach the oracle's
    full-Newton solution of the steps each session received (1e-8 relative
    p, 1e-8 S)."""
    import paper_2008_01539_amd as P
    from paper_2008_01539_amd.serve import GpuExecutor, Server, SessionSpec
    from oracle.newton import Options as OOptions
    from oracle.newton import Solver, State
    models = [make_c1_variant(seed=13, nx=20, ny=16), make_small_c2(),
              make_small_c2(seed=26, nx=18, ny=10, nfrac=8)]
    specs = [SessionSpec(name=f"t{k}", model=m, options=P.Options.tight_mode(precision=P.MIXED),
                         schedule=m.schedule) for k, m in enumerate(models)]
    ex = GpuExecutor()
    srv = Server(specs, ex, budget_bytes=8 << 30, max_inflight=8,
                 footprint=lambda s: P.estimate_bytes(s.model, s.options))
    summ = srv.run_poisson(rate=20.0, duration=1.0, mix=np.array([0.4, 0.3, 0.3]), seed=7)
    assert summ["failed"] == 0
    checked = 0
    for s in srv.sessions:
        if s.next_step == 0:
            continue
        u, _ = s.handle.get_state()
        sched = s.spec.schedule
        m = s.spec.model
        st = State(m.u0.copy(), m.status0.copy())
        sol = Solver(m, OOptions.tight_mode())
        for k in range(s.next_step):
            st, _ = sol.solve_timestep(st, sched[k % len(sched)])
        assert np.abs(u[0] - st.u[0]).max() <= 1e-8 * st.u[0].min(), s.spec.name
        if m.b > 1:
            assert np.abs(u[1] - st.u[1]).max() <= 1e-8, s.spec.name
        checked += 1
    assert checked >= 2
    ex.close()


def test_batch_black_oil_mixed_modes_equals_solo():
    """Black-oil members (3x3 blocks, fracture blocks) in one batch, each in
    its own mode (Algorithm 1, full Newton, residual-based): every member
    keeps its solo bits, states and phase status."""
    import paper_2008_01539_amd as P
    models = [make_small_c3(), make_small_c3(seed=43, nx=24, ny=12, nz=4, nfrac=16, nstage=2),
              make_small_c3(seed=44, nx=16, ny=12, nz=3, nfrac=8, nstage=2),
              make_small_c3(seed=45, nx=22, ny=8, nz=4, nfrac=12, nstage=2)]
    modes = [P.LOCAL, P.FULL, P.RESID, P.LOCAL]
    opts = P.Options(precision=P.MIXED)
    n = 4
    got, sizes = _batched(models, opts, modes, n)
    for m, md, (u, st) in zip(models, modes, got):
        ref, ref_st = _solo(m, opts, md, m.schedule[:n])
        assert np.array_equal(u, ref)
        assert np.array_equal(st, ref_st)
    assert max(sizes) == 4


def test_batch_algorithm2_members_equal_solo():
    """Algorithm 2 members (multiplicative and additive) in a batch with
    Algorithm 1 and full-Newton members: each runs its own inner
    iterations inside the batched call and keeps its solo bits."""
    import paper_2008_01539_amd as P
    models = [make_small_c2(), make_small_c2(seed=23, nx=30, ny=14, nfrac=20),
              make_small_c2(seed=24, nx=16, ny=10, nz=3, nfrac=6, nstage=2),
              make_small_c2(seed=25, nx=20, ny=12, nfrac=10)]
    modes = [P.DD, P.LOCAL, P.DD_ADD, P.FULL]
    opts = P.Options(precision=P.MIXED)
    n = 4
    got, sizes = _batched(models, opts, modes, n)
    for m, md, (u, st) in zip(models, modes, got):
        ref, _ = _solo(m, opts, md, m.schedule[:n])
        assert np.array_equal(u, ref)
    assert max(sizes) == 4


def test_batch_two_phase_fp64_equals_solo():
    """FP64 Krylov members with fracture blocks (the batched inversion reads
    FP64 scaled blocks): every member keeps its solo bits."""
    import paper_2008_01539_amd as P
    models = [make_small_c2(seed=31, nx=24, ny=12, nfrac=14),
              make_small_c2(seed=32, nx=20, ny=16, nfrac=18),
              make_small_c2(seed=33, nx=18, ny=10, nz=3, nfrac=8, nstage=2)]
    opts = P.Options(precision=P.FP64)
    n = 4
    got, sizes = _batched(models, opts, P.LOCAL, n)
    for m, (u, st) in zip(models, got):
        ref, ref_st = _solo(m, opts, P.LOCAL, m.schedule[:n])
        assert np.array_equal(u, ref)
        assert np.array_equal(st, ref_st)
    assert max(sizes) == 3


def test_batch_rejects_mixed_precisions():
    import paper_2008_01539_amd as P
    from paper_2008_01539_amd.fim import FimError
    a = P.FimModel(make_small_c2(seed=34), P.Options(precision=P.FP64))
    b = P.FimModel(make_small_c2(seed=35), P.Options(precision=P.MIXED))
    with pytest.raises(FimError):
        P.FimBatch([a, b])
    a.close()
    b.close()


@pytest.mark.parametrize("mode_name", ["LOCAL", "FULL"])
def test_batch_members_match_oracle_tight(mode_name):
    """Tight mode, mixed precision: every member of an uneven batch (two
    config-4-recipe members of different sizes, the small config-2 model
    and a config-1 variant with another seed) advanced by batched Newton
    iterations reaches the oracle's full-Newton solution of its own model
    (1e-8 relative p, 1e-8 S)."""
    import paper_2008_01539_amd as P
    from fimgen.configs import _two_phase_model, c1_schedule
    from fimgen.model import FLUID_DEADOIL
    from oracle.newton import Options as OOptions
    from oracle.newton import Solver, State
    nsteps = 4
    two = [_two_phase_model(f"c4s_{k}", 4000 + k, nx, ny, 4, nf, FLUID_DEADOIL,
                            c1_schedule(8, 1e-3, 10.0), nstage=2)
           for k, (nx, ny, nf) in enumerate(((20, 10, 8), (30, 14, 14)))]
    two.append(make_small_c2())
    outs, sizes = _batched(two, P.Options.tight_mode(precision=P.MIXED),
                           getattr(P, mode_name), nsteps)
    assert max(sizes) == len(two)
    for m, (u, _) in zip(two, outs):
        st = State(m.u0.copy(), m.status0.copy())
        s = Solver(m, OOptions.tight_mode())
        for dt in m.schedule[:nsteps]:
            st, _ = s.solve_timestep(st, dt)
        assert np.abs(u[0] - st.u[0]).max() <= 1e-8 * st.u[0].min()
        assert np.abs(u[1] - st.u[1]).max() <= 1e-8
    one = [make_c1_variant(seed=11, uniform_perm=False), make_c1_variant(seed=12, nx=15, ny=14)]
    outs, _ = _batched(one, P.Options.tight_mode(precision=P.MIXED), getattr(P, mode_name), 3)
    for m, (u, _) in zip(one, outs):
        st = State(m.u0.copy(), m.status0.copy())
        s = Solver(m, OOptions.tight_mode())
        for dt in m.schedule[:3]:
            st, _ = s.solve_timestep(st, dt)
        assert np.abs(u[0] - st.u[0]).max() <= 1e-8 * st.u[0].min()
