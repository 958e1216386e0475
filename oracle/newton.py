"""Newton's method with a direct solve (oracle; test infrastructure only).

Section 4.1: at each timestep, given u^n and dt, solve F(u^{n+1}) = 0 by
Newton iterates J(u^nu) du^nu = -F(u^nu), u^{nu+1} = u^nu + du^nu.  The
linear systems are solved by SuperLU (scipy.sparse.linalg.splu, COLAMD column
ordering, partial pivoting) in FP64.
Section 5 states the convergence test ||dp||_inf < eps_p.

Readings where the paper is silent (shared with the HIP library):

* saturation chop: a cell's saturation updates are scaled so that none
  exceeds ``ds_max`` (0.2) in magnitude; S_w is clamped to [0, 1] and S_g to
  at most 1 - S_w; pressure is never chopped;
* black-oil variable switching after each update (the black-oil analogue
  of the substitution rules of Section 3.1): a saturated cell whose S_g
  turns negative becomes undersaturated with R_s = R_s,sat(p); an
  undersaturated cell whose R_s exceeds R_s,sat(p) becomes saturated with
  S_g = 0;
* "tight" convergence additionally requires ||dS||_inf < eps_s and no
  switch in the iteration;
* failure (iteration cap, non-finite values or a singular Jacobian) rolls
  the state back to u^n and the driver halves dt, at most ``max_cuts``
  times;
* an iteration restricted to an empty active set (a model with no
  always-active cells and nothing in the previous step's support) updates
  nothing: du = 0, which meets the convergence test at once.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse.linalg as spla

from fimgen.units import PSI
from .jacobian import JacobianBuilder
from .physics import accumulation


@dataclass
class Options:
    eps_conv: float = 0.3 * PSI      # ||dp||_inf convergence (Pa)
    eps_loc: float = 0.3 * PSI       # active / boundary cutoff (Pa)
    eps_s: float = 1e-10             # saturation change (tight mode)
    tight: bool = False
    m_layers: int = 2                # neighbour layers (Alg. 1)
    m_layers_dd: int = 4             # neighbour layers (Alg. 2)
    max_newton: int = 25
    ds_max: float = 0.2
    max_cuts: int = 8
    max_sweeps: int = 40             # Alg. 2 outer iterations cap
    eps_res: float = 1e-6            # residual-based localization cutoff
    res_layers: int = 1              # its neighbour inflation

    @staticmethod
    def tight_mode(**kw):
        o = Options(eps_conv=1e-7 * PSI, eps_loc=1e-7 * PSI, eps_s=1e-10,
                    tight=True, max_newton=40)
        for k, v in kw.items():
            setattr(o, k, v)
        return o


@dataclass
class State:
    u: np.ndarray          # (b, n)
    status: np.ndarray     # (n,) int8

    def copy(self):
        return State(self.u.copy(), self.status.copy())


def apply_update(model, st: State, du: np.ndarray, opts: Options):
    """Apply a Newton update du (b, n) in place: chop, clamp, switch.

    Returns (dp_abs (n,), ds_max_abs, n_switch)."""
    fl = model.fluid
    b = model.b
    du = du.copy()
    if b >= 2:
        sat_like = np.abs(du[1])
        if b == 3:
            sat_like = np.maximum(sat_like, np.where(st.status == 1,
                                                     np.abs(du[2]), 0.0))
        scale = np.where(sat_like > opts.ds_max, opts.ds_max / np.maximum(sat_like, 1e-300), 1.0)
        du[1] *= scale
        if b == 3:
            du[2] = np.where(st.status == 1, du[2] * scale, du[2])
    st.u += du
    dp_abs = np.abs(du[0])
    ds = np.abs(du[1]) if b >= 2 else np.zeros_like(dp_abs)
    nsw = 0
    if b >= 2:
        st.u[1] = np.clip(st.u[1], 0.0, 1.0)
    if b == 3:
        sat = st.status == 1
        ds = np.maximum(ds, np.where(sat, np.abs(du[2]), 0.0))
        st.u[2] = np.where(sat, np.minimum(st.u[2], 1.0 - st.u[1]), st.u[2])
        rs_sat = fl["rs_b"] * st.u[0] / fl["p_b"]
        to_under = sat & (st.u[2] < 0.0)
        to_sat = (~sat) & (st.u[2] > rs_sat)
        st.u[2] = np.where(to_under, rs_sat, np.where(to_sat, 0.0, st.u[2]))
        st.status = np.where(to_under, 0, np.where(to_sat, 1, st.status)).astype(np.int8)
        nsw = int(to_under.sum() + to_sat.sum())
    return dp_abs, float(ds.max()) if ds.size else 0.0, nsw


def converged(opts: Options, dp_max, ds_max, nsw):
    ok = dp_max < opts.eps_conv
    if opts.tight:
        ok = ok and ds_max < opts.eps_s and nsw == 0
    return ok


class Solver:
    """Full (standard) Newton with SuperLU, the plain definition."""

    def __init__(self, model, opts: Options | None = None):
        self.model = model
        self.opts = opts or Options()
        self.jb = JacobianBuilder(model)

    def linear_solve(self, J, R, rows=None):
        """Solve J du = -R, optionally restricted to unknown indices rows
        (J_A = R_A J R_A^T, F_A = R_A F of Section 4.3)."""
        rhs = -R.T.reshape(-1)        # cell-major
        if rows is not None:
            J = J[rows][:, rows]
            rhs = rhs[rows]
        try:
            lu = spla.splu(J.tocsc(), permc_spec="COLAMD")
        except RuntimeError:
            # a singular (or non-finite) Jacobian: the iteration fails like
            # one that produced non-finite values
            return np.full(rhs.shape, np.nan)
        return lu.solve(rhs)

    def newton_iteration(self, st: State, m_old, dt, active=None):
        """One Newton iteration on all cells (active=None) or on the cells
        listed in ``active`` with the others frozen (Dirichlet).
        Returns (dp_abs, ds_max, n_switch)."""
        b = self.model.b
        R, J = self.jb.build(st.u, st.status, m_old, dt)
        if active is None:
            x = self.linear_solve(J, R)
            du = x.reshape(self.model.n, b).T
        else:
            act = np.asarray(sorted(active), np.int64)
            du = np.zeros((b, self.model.n))
            if act.size:   # an empty restriction leaves nothing to solve
                rows = (act[:, None] * b + np.arange(b)[None, :]).reshape(-1)
                x = self.linear_solve(J, R, rows)
                du[:, act] = x.reshape(act.size, b).T
        return apply_update(self.model, st, du, self.opts)

    def solve_timestep(self, st: State, dt):
        """Full Newton for one step; returns (new state, iterations) or
        (None, iterations) on failure (state untouched)."""
        m_old = accumulation(self.model, st.u, st.status)
        work = st.copy()
        for it in range(1, self.opts.max_newton + 1):
            dp, ds, nsw = self.newton_iteration(work, m_old, dt)
            if not np.all(np.isfinite(work.u)):
                return None, it
            if converged(self.opts, float(dp.max()), ds, nsw):
                return work, it
        return None, self.opts.max_newton

    def run(self, st: State, schedule, record=None):
        """Run a schedule with dt halving on failure.  Returns the final
        state and a list of per-step records."""
        recs = []
        for dt in schedule:
            pending = [dt]
            while pending:
                h = pending.pop(0)
                new, its = self.solve_timestep(st, h)
                if new is None:
                    if h < dt / 2 ** self.opts.max_cuts:
                        raise RuntimeError("timestep cut limit reached")
                    pending = [h / 2, h / 2] + pending
                    continue
                recs.append(dict(dt=h, iters=its))
                st = new
                if record is not None:
                    record(st)
        return st, recs
