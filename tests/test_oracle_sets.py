"""Set logic of Algorithms 1 and 2 (oracle) on hand-made graphs with the
expected sets written out by hand.  CPU only."""
import json
import os

import numpy as np

from oracle import sets as S


def _csr(n, edges):
    nb = [[] for _ in range(n)]
    for a, b in edges:
        nb[a].append(b)
        nb[b].append(a)
    rp = np.zeros(n + 1, np.int64)
    flat = []
    for i in range(n):
        s = sorted(nb[i])
        flat += s
        rp[i + 1] = rp[i] + len(s)
    return rp, np.array(flat, np.int64)


def chain(n=10):
    return _csr(n, [(i, i + 1) for i in range(n - 1)])


def grid(nx=5, ny=5, extra=()):
    e = []
    for r in range(ny):
        for c in range(nx):
            i = r * nx + c
            if c + 1 < nx:
                e.append((i, i + 1))
            if r + 1 < ny:
                e.append((i, i + nx))
    return _csr(nx * ny, list(e) + list(extra))


def test_ball_chain_and_grid():
    rp, nb = chain()
    assert S.ball(rp, nb, 4, 2) == {2, 3, 4, 5, 6}
    assert S.ball(rp, nb, 0, 2) == {0, 1, 2}
    assert S.ball(rp, nb, 4, 0) == {4}
    rp, nb = grid()
    # graph-distance diamond, not a (2m+1)^2 box
    assert S.ball(rp, nb, 12, 2) == {2, 6, 7, 8, 10, 11, 12, 13, 14, 16, 17, 18, 22}
    assert S.ball(rp, nb, 0, 1) == {0, 1, 5}


def test_ball_follows_nonneighbour_connection():
    rp, nb = grid(3, 3, extra=[(0, 8)])
    assert S.ball(rp, nb, 0, 1) == {0, 1, 3, 8}
    assert S.ball(rp, nb, 0, 2) == {0, 1, 2, 3, 4, 6, 5, 7, 8}


def test_boundary_and_outer_layer():
    rp, nb = grid()
    block = {6, 7, 8, 11, 12, 13, 16, 17, 18}
    assert S.boundary(rp, nb, block) == {6, 7, 8, 11, 13, 16, 17, 18}
    assert S.outer_layer(rp, nb, block) == {1, 2, 3, 5, 9, 10, 14, 15, 19, 21, 22, 23}
    assert S.boundary(rp, nb, set(range(25))) == set()


def test_alg1_expand_and_shrink():
    rp, nb = chain()
    act = {3, 4, 5}
    bnd = S.boundary(rp, nb, act)
    assert bnd == {3, 5}
    dp = np.zeros(10)
    dp[3], dp[4] = 1.0, 5.0
    new, nbnd, ex = S.alg1_update(rp, nb, act, bnd, dp, 1.0, 2, [])
    assert ex and new == {1, 2, 3, 4, 5} and nbnd == {1, 5}
    dp[:] = 0.0
    dp[4] = 1.0
    new, nbnd, ex = S.alg1_update(rp, nb, act, bnd, dp, 1.0, 2, [])
    assert not ex and new == {4} and nbnd == {4}
    # always-active cells stay in the shrunk set
    new, _, ex = S.alg1_update(rp, nb, act, bnd, dp, 1.0, 2, [9])
    assert not ex and new == {4, 9}
    # an update just below the cutoff is negligible
    dp[3] = np.nextafter(1.0, 0.0)
    new, _, ex = S.alg1_update(rp, nb, act, bnd, dp, 1.0, 2, [])
    assert not ex and new == {4}


def test_initial_active_set():
    rp, nb = chain()
    assert S.initial_active(rp, nb, [5], 2) == {3, 4, 5, 6, 7}
    assert S.initial_active(rp, nb, [5], 2, prev_support={0, 1}) == {0, 1, 5}


def test_alg2_expand():
    rp, nb = chain()
    vt = {3, 4, 5}
    bnd = {3, 5}
    dp = np.zeros(10)
    dp[5] = 1.0
    nxt, vt2, vb, db, ex = S.alg2_expand(rp, nb, vt, bnd, dp, 1.0, 2)
    assert ex
    assert nxt == {3, 4, 5, 6, 7}
    assert vt2 == {3, 4, 5, 6, 7}
    assert vb == {3, 7}
    assert db == {2, 8}
    dp[:] = 0.0
    nxt, vt3, vb, db, ex = S.alg2_expand(rp, nb, vt2, vb, dp, 1.0, 2)
    assert not ex and nxt == set() and vt3 == vt2


def test_alg2_boundary_only_where_total_set_ends():
    """V_B^{k+1} = boundary(V_T) intersected with V_A^{k+1}: cells of the new
    subdomain that border the old total set are not boundary cells."""
    rp, nb = chain()
    vt = {2, 3, 4, 5, 6}
    dp = np.zeros(10)
    dp[6] = 2.0
    nxt, vt2, vb, db, ex = S.alg2_expand(rp, nb, vt, {2, 6}, dp, 1.0, 1)
    assert nxt == {5, 6, 7}
    assert vt2 == {2, 3, 4, 5, 6, 7}
    assert vb == {7}
    assert db == {4, 8}


def test_alg2_sub_max_and_skip_test():
    """Skip test of Algorithm 2, Step 2: the largest latest update over the
    subdomain and its outer layer, by hand."""
    last = np.array([0.0, 0.1, 0.5, 2.0, 0.2, 0.0, 3.0])
    assert S.alg2_sub_max([0, 1, 2], [3], last) == 2.0    # outer layer counts
    assert S.alg2_sub_max([4, 5], [], last) == 0.2
    assert S.alg2_sub_max([], [], last) == 0.0
    assert S.alg2_sub_max([6], [0], last) == 3.0


def test_alg2_sweep_cap():
    """A step that needs a second sweep fails with max_sweeps = 1 and
    succeeds with the default cap; the sweep count of the log is the
    number of outer passes."""
    from fimgen import make_c1
    from oracle.localized import LocalSolver
    from oracle.newton import Options, State
    m = make_c1()
    st = State(m.u0.copy(), m.status0.copy())
    log = []
    new, _, _ = LocalSolver(m, Options()).alg2_timestep(st, m.schedule[5], None, log)
    assert new is not None
    sweeps = log[-1]["sweeps"]
    assert sweeps == max(r.get("sweep", 0) for r in log)
    assert sweeps >= 2
    bad, _, _ = LocalSolver(m, Options(max_sweeps=sweeps - 1)).alg2_timestep(
        st, m.schedule[5], None)
    assert bad is None


def _fractured_chain():
    """Matrix chain 0..7; fracture A = cells 8-9-10 (8-9, 9-10), hosted by
    matrix cells 2, 3, 4; fracture B = cells 11-12, intersecting A at 10
    (10-11) and hosted by 5, 6; fracture C = cell 13 alone, hosted by 7."""
    edges = [(i, i + 1) for i in range(7)]
    edges += [(8, 9), (9, 10), (10, 11), (11, 12)]
    edges += [(2, 8), (3, 9), (4, 10), (5, 11), (6, 12), (7, 13)]
    rp, nb = _csr(14, edges)
    is_frac = np.array([0] * 8 + [1] * 6, bool)
    return rp, nb, is_frac


def test_fracture_components_and_closure_by_hand():
    """Localized fracture cells: components through fracture-fracture
    connections (the intersection 10-11 joins A and B), and the closure of
    a set under them."""
    rp, nb, is_frac = _fractured_chain()
    comp, members = S.fracture_components(rp, nb, is_frac)
    assert comp[:8] == [-1] * 8
    assert members == [{8, 9, 10, 11, 12}, {13}]
    assert comp[12] == 0 and comp[13] == 1
    assert S.frac_closure({1, 9}, comp, members) == {1, 8, 9, 10, 11, 12}
    assert S.frac_closure({1, 2, 3}, comp, members) == {1, 2, 3}
    assert S.frac_closure({13, 0}, comp, members) == {0, 13}


def test_alg1_update_with_localized_fractures():
    """An expansion whose ball reaches one fracture cell takes the whole
    component; a shrink keeps whole components; the initial set is closed
    too."""
    rp, nb, is_frac = _fractured_chain()
    fc = S.fracture_components(rp, nb, is_frac)
    act = {0, 1}
    bnd = S.boundary(rp, nb, act)
    dp = np.zeros(14)
    dp[1] = 5.0
    new, vb, ex = S.alg1_update(rp, nb, act, bnd, dp, 1.0, 1, [0], fc)
    assert ex and new == {0, 1, 2}                  # 2 hosts fracture cell 8 ...
    new, vb, ex = S.alg1_update(rp, nb, act, bnd, dp, 1.0, 2, [0], fc)
    assert ex and new == {0, 1, 2, 3} | {8, 9, 10, 11, 12}   # ... reached at m = 2
    assert vb == {3, 10, 11, 12}   # 10, 11, 12 border their inactive hosts 4..6
    dp[:] = 0.0
    dp[9] = 2.0
    new, vb, ex = S.alg1_update(rp, nb, {0, 1, 8, 9}, set(), dp, 1.0, 1, [0], fc)
    assert not ex and new == {0, 8, 9, 10, 11, 12}  # shrink, then closure
    assert S.initial_active(rp, nb, [13], 1, None, fc) == {7, 13}
    assert S.initial_active(rp, nb, [0], 1, {10}, fc) == {0, 8, 9, 10, 11, 12}


def test_alg2_owner_by_hand():
    """Additive phase 2: each cell's update comes from the first subdomain
    containing it."""
    subs = [[2, 3, 4], [4, 5, 6, 7], [1, 2, 7, 8]]
    assert S.alg2_owner(subs, 10) == [-1, 2, 0, 0, 0, 1, 1, 1, 2, -1]
    assert S.alg2_owner([], 3) == [-1, -1, -1]


def test_work_ratio_definition_matches_paper_tables():
    """M_A per iteration is n_A / n; the tables' average column equals the
    total divided by the iteration count (to the printed rounding)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")
    with open(path) as f:
        rows = json.load(f)["rows"]
    for r in rows:
        avg = r["total_ma"] / r["iterations"]
        assert abs(avg - r["average_ma"]) <= 0.5 * 10 ** (-r["avg_decimals"]) + 1e-12, r
