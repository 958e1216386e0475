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
