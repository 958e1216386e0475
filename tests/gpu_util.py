"""Helpers shared by the GPU parity tests (comparison against the oracle)."""
import numpy as np
import scipy.sparse as sp

from oracle.jacobian import JacobianBuilder
from oracle.newton import State
from oracle.physics import accumulation


def oracle_system(model, u_old, u_iter, status, dt, act=None):
    """Oracle F_A, J_A (dense blocks per active row) on the active set."""
    b = model.b
    m_old = accumulation(model, u_old, status)
    R, J = JacobianBuilder(model).build(u_iter, status, m_old, dt)
    cells = np.arange(model.n) if act is None else np.nonzero(act)[0]
    rows = (cells[:, None] * b + np.arange(b)[None, :]).reshape(-1)
    return R[:, cells].T.copy(), J[rows][:, rows].tocsr(), cells


def gpu_matrix(sysd, b):
    """Block CSR from fim_inspect_assemble as a scipy matrix."""
    na = sysd["n_active"]
    rp, col, val = sysd["row_ptr"], sysd["col"], sysd["val"]
    rows, cols, vals = [], [], []
    for r in range(na):
        for q in range(rp[r], rp[r + 1]):
            c = col[q]
            for e in range(b):
                for v in range(b):
                    rows.append(r * b + e)
                    cols.append(c * b + v)
                    vals.append(val[q, e, v])
    return sp.csr_matrix((vals, (rows, cols)), shape=(na * b, na * b))


def compare_system(model, fm, u_old, u_iter, status, dt, act=None, rtol=1e-12):
    """Assemble on the GPU and in the oracle; assert agreement.  Returns the
    worst relative deviations (J per row max, F per row scale)."""
    b = model.b
    g = fm.inspect_assemble(u_old, u_iter, status, dt, act)
    Fo, Jo, cells = oracle_system(model, u_old, u_iter, status, dt, act)
    assert g["n_active"] == cells.size
    assert np.array_equal(g["l2g"], cells)
    Jg = gpu_matrix(g, b)
    D = (Jg - Jo).tocsr()
    absJ = abs(Jo).tocsr()
    rowmax = np.maximum(absJ.max(axis=1).toarray().ravel(), 1e-300)
    dmax = abs(D).max(axis=1).toarray().ravel()
    jerr = float((dmax / rowmax).max()) if dmax.size else 0.0
    uu = np.abs(u_iter[:, cells].T.reshape(-1))
    scale = abs(Jo) @ uu
    m_new = accumulation(model, u_iter, status)[:, cells].T.reshape(-1)
    scale = scale + np.abs(m_new) / dt
    ferr = float((np.abs(g["F"].reshape(-1) - Fo.reshape(-1)) / scale).max())
    assert jerr <= rtol, jerr
    assert ferr <= rtol, ferr
    return jerr, ferr


def run_oracle(solver, model, schedule):
    st = State(model.u0.copy(), model.status0.copy())
    out = []
    for dt in schedule:
        st, its = solver.solve_timestep(st, dt)
        assert st is not None
        out.append(st.copy())
    return out


def flags_of(cells, n):
    f = np.zeros(n, np.uint8)
    idx = np.fromiter((int(i) for i in cells), np.int64)
    f[idx] = 1
    return f


def check_dd_expand(fm, model, rng, layers, eps, rounds=3):
    """Algorithm 2's phase-1 set logic on the GPU against the oracle's
    alg2_expand, bit for bit, over a few chained rounds on synthetic but
    consistent inputs: V_A^0 = the always-active cells and their
    neighbourhood, V_T = V_A^0 plus some distant balls, V_B^0 =
    boundary(V_T) ^ V_A^0; |dp| drawn around eps on the boundary (ties at
    eps included), large values inside (which must not seed)."""
    from oracle import sets as S
    from oracle.jacobian import adjacency
    rp, nb = adjacency(model)
    n = model.n
    aa = np.nonzero(model.always_active)[0]
    va = S.initial_active(rp, nb, aa, 1)
    vt = set(va)
    for c in rng.choice(n, 6, replace=False):
        vt |= S.ball(rp, nb, int(c), 3)
    vb = S.boundary(rp, nb, vt) & va
    seen_expand = seen_stop = False
    for rnd in range(rounds + 1):
        dp = np.zeros(n)
        inner = np.fromiter(va, np.int64)
        dp[inner] = rng.exponential(4 * eps, inner.size)   # not on V_B: no seed
        bl = np.fromiter(sorted(vb), np.int64)
        if rnd == rounds:
            dp[bl] = rng.uniform(0, 0.999 * eps, bl.size)   # nothing qualifies
        elif bl.size:
            dp[bl] = eps * rng.choice([0.0, 0.3, 0.999999, 1.0, 1.5, 7.0], bl.size,
                                      p=[0.4, 0.3, 0.1, 0.05, 0.1, 0.05])
        ref = S.alg2_expand(rp, nb, vt, vb, dp, eps, layers)
        got = fm.inspect_dd_expand(flags_of(vt, n), flags_of(va, n), flags_of(vb, n), dp,
                                   eps, layers)
        nxt, vt2, vb2, db2, ex = ref
        assert got["is_expand"] == ex
        assert np.array_equal(got["vt"], flags_of(vt2, n))
        assert np.array_equal(got["act"], flags_of(nxt, n))
        assert np.array_equal(got["bnd"], flags_of(vb2, n))
        assert np.array_equal(got["outer"], flags_of(db2, n))
        assert got["n_active"] == len(nxt)
        seen_expand |= ex
        seen_stop |= not ex
        if not ex:
            break
        va, vt, vb = nxt, vt2, vb2
    assert seen_expand and seen_stop
