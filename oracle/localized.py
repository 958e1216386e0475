"""Algorithm 1 (localized Newton), Algorithm 2 (adaptive nonlinear
domain decomposition) and the residual-based localization the paper
compares against (Sections 1 and 4.2), oracle versions (test
infrastructure only).

Each local solve is the restricted Newton step of Section 4.3,
J_A du_A = -F_A with J_A = R_A J R_A^T: the full residual and Jacobian are
formed (the plain definition) and restricted to the active rows and
columns, so inactive neighbours enter as frozen Dirichlet values.

Readings where the paper is silent (shared with the HIP library):

* the loop of Algorithm 1 starts in 'expand' mode; convergence is
  ||dp||_inf over the active cells below eps_conv, and the loop continues
  while expanding even when converged;
* the initial active set is the fracture/perforated cells and their m-layer
  neighbourhood on the first step, then the previous step's support
  {|p^n - p^{n-1}| >= eps_loc} plus the always-active cells;
* with localized fracture cells (not all fracture cells always active),
  every active set of Algorithm 1 is closed under fracture components
  (sets.frac_closure); Algorithm 2 and the residual-based mode leave the
  fracture cells as the model marks them;
* Algorithm 2: each visit of a subdomain is one Newton iteration on it
  (its additive form: every pending subdomain of a sweep from the same
  state, each cell taking the update of the first subdomain containing it,
  sets.alg2_owner);
  last_dp[i] holds |dp_i| from the latest solve that touched cell i; a
  subdomain is skipped when last_dp < eps on V_A^k and on its outer layer;
  the sweeps stop when no subdomain would be solved; the step fails when
  phase 1 would need more than max_newton solves, when a sweep beyond
  max_sweeps starts, or when the inner iterations would pass
  8 max_newton (the paper states no caps);
* residual-based localization (Lu and Beckner, as Sections 1 and 4.2
  describe it: the first iteration of a timestep takes the whole domain,
  later ones the unconverged cells plus one layer of neighbours): a cell is
  unconverged when its error measure
      e_i = dt max_c |R_{i,c}| / (V_i rho_c)
  is at or above eps_res, with R the residual at the current iterate (kg/s),
  V_i the reference pore volume and rho_c the reference density of
  component c (the mass imbalance over the step as a fraction of the pore
  volume filled with that component); the timestep ends when the update
  meets the usual convergence test or when no cell is unconverged.
"""
from __future__ import annotations

import numpy as np

from .jacobian import adjacency
from .newton import Options, Solver, State, converged
from .physics import accumulation, residual
from . import sets


def reference_densities(fluid):
    """rho_c of the error measure, in component order (single phase;
    water, oil; water, oil, gas)."""
    k = fluid["kind"]
    if k == 1:
        return np.array([fluid["rho_ref"]])
    if k == 2:
        return np.array([fluid["rho_w"], fluid["rho_o"]])
    return np.array([fluid["rho_wsc"], fluid["rho_osc"], fluid["rho_gsc"]])


def resid_error(model, u, status, m_old, dt):
    """e_i = dt max_c |R_{i,c}| / (V_i rho_c) at state u (n,)."""
    R = residual(model, u, status, m_old, dt)
    scale = model.pv_ref[None, :] * reference_densities(model.fluid)[:, None]
    return dt * np.max(np.abs(R) / scale, axis=0)


class LocalSolver(Solver):
    def __init__(self, model, opts: Options | None = None):
        super().__init__(model, opts)
        self.rp, self.nb = adjacency(model)
        self.aa = np.nonzero(model.always_active)[0]
        # localized fracture cells (some fracture cell not always active):
        # Algorithm 1's sets are closed under fracture components
        frac = model.kind == 1
        self.fcomp = None
        if np.any(frac & (model.always_active == 0)):
            self.fcomp = sets.fracture_components(self.rp, self.nb, frac)

    # ------------------------------------------------------ Algorithm 1
    def alg1_timestep(self, st: State, dt, prev_support, log=None):
        o = self.opts
        m_old = accumulation(self.model, st.u, st.status)
        work = st.copy()
        act = sets.initial_active(self.rp, self.nb, self.aa, o.m_layers,
                                  prev_support, self.fcomp)
        bnd = sets.boundary(self.rp, self.nb, act)
        is_expand, conv = True, False
        it = 0
        while is_expand or not conv:
            it += 1
            if it > o.max_newton:
                return None, it, None
            n_a = len(act)
            dp, ds, nsw = self.newton_iteration(work, m_old, dt, active=act)
            if not np.all(np.isfinite(work.u)):
                return None, it, None
            conv = converged(o, float(dp.max()), ds, nsw)
            if log is not None:
                log.append(dict(n_a=n_a, n_b=len(bnd), dp=float(dp.max())))
            act, bnd, is_expand = sets.alg1_update(
                self.rp, self.nb, act, bnd, dp, o.eps_loc, o.m_layers, self.aa, self.fcomp)
        support = set(np.nonzero(np.abs(work.u[0] - st.u[0]) >= o.eps_loc)[0].tolist())
        return work, it, support

    # ------------------------------------------------------ Algorithm 2
    def alg2_timestep(self, st: State, dt, prev_support, log=None, additive=False):
        """Algorithm 2.  additive=True: the additive form of phase 2 (the
        additive Schwarz form Section 4.4 starts from, with the paper's
        adaptive subdomains): each sweep solves every pending subdomain
        from the same state, and each cell takes the update of the first
        subdomain (in build order) that contains it, so the overlapping
        updates combine as in restricted additive Schwarz."""
        o = self.opts
        m = o.m_layers_dd
        m_old = accumulation(self.model, st.u, st.status)
        work = st.copy()
        va = sets.initial_active(self.rp, self.nb, self.aa, m, prev_support)
        vt = set(va)
        vb = sets.boundary(self.rp, self.nb, va)
        db = sets.outer_layer(self.rp, self.nb, va)
        last_dp = np.zeros(self.model.n)
        subs = []
        inner = 0
        is_expand = True
        while is_expand:                       # phase 1: build subdomains
            inner += 1
            if inner > o.max_newton:
                return None, inner, None
            dp, _, _ = self.newton_iteration(work, m_old, dt, active=va)
            if not np.all(np.isfinite(work.u)):
                return None, inner, None
            idx = np.fromiter(sorted(va), np.int64)
            last_dp[idx] = dp[idx]
            subs.append((idx, np.fromiter(sorted(db), np.int64)))
            if log is not None:
                log.append(dict(n_a=len(va), phase=1, sub=len(subs) - 1,
                                dp=float(dp.max())))
            va, vt, vb, db, is_expand = sets.alg2_expand(
                self.rp, self.nb, vt, vb, dp, o.eps_loc, m)

        def pending(k):
            a, d = subs[k]
            return sets.alg2_sub_max(a, d, last_dp) >= o.eps_loc

        sweeps = 0
        owner = np.array(sets.alg2_owner([a for a, _ in subs], self.model.n))
        while additive and any(pending(k) for k in range(len(subs))):
            sweeps += 1
            if sweeps > o.max_sweeps:
                return None, inner, None
            todo = [k for k in range(len(subs)) if pending(k)]
            if inner + len(todo) > 8 * o.max_newton:
                return None, inner, None
            base = work.copy()
            trials = []
            for k in todo:                      # all from the same state
                trial = base.copy()
                dp, _, _ = self.newton_iteration(trial, m_old, dt,
                                                 active=set(subs[k][0].tolist()))
                trials.append((k, trial, dp))
            for k, trial, dp in trials:          # restricted combination
                own = np.nonzero(owner == k)[0]
                work.u[:, own] = trial.u[:, own]
                work.status[own] = trial.status[own]
                last_dp[own] = dp[own]
                inner += 1
                if log is not None:
                    log.append(dict(n_a=int(subs[k][0].size), phase=2, sweep=sweeps,
                                    sub=k, dp=float(dp.max())))
            if not np.all(np.isfinite(work.u)):
                return None, inner, None
        while not additive and any(pending(k) for k in range(len(subs))):   # phase 2
            sweeps += 1
            if sweeps > o.max_sweeps:
                return None, inner, None
            for k in range(len(subs)):
                if not pending(k):
                    continue
                a = subs[k][0]
                inner += 1
                if inner > 8 * o.max_newton:
                    return None, inner, None
                dp, _, _ = self.newton_iteration(work, m_old, dt,
                                                 active=set(a.tolist()))
                if not np.all(np.isfinite(work.u)):
                    return None, inner, None
                last_dp[a] = dp[a]
                if log is not None:
                    log.append(dict(n_a=int(a.size), phase=2, sweep=sweeps,
                                    sub=k, dp=float(dp.max())))
        if log is not None:
            log.append(dict(phase=0, n_sub=len(subs), sweeps=sweeps, vt=set(vt)))
        support = set(np.nonzero(np.abs(work.u[0] - st.u[0]) >= o.eps_loc)[0].tolist())
        return work, inner, support

    # ------------------------------------ residual-based (Lu and Beckner)
    def resid_timestep(self, st: State, dt, prev_support=None, log=None):
        o = self.opts
        m_old = accumulation(self.model, st.u, st.status)
        work = st.copy()
        act = None                              # first iteration: all cells
        for it in range(1, o.max_newton + 1):
            n_a = self.model.n if act is None else len(act)
            dp, ds, nsw = self.newton_iteration(work, m_old, dt, active=act)
            if not np.all(np.isfinite(work.u)):
                return None, it, None
            if log is not None:
                log.append(dict(n_a=n_a, dp=float(dp.max())))
            if converged(o, float(dp.max()), ds, nsw):
                return work, it, None
            err = resid_error(self.model, work.u, work.status, m_old, dt)
            act = sets.resid_active(self.rp, self.nb, err, o.eps_res, o.res_layers)
            if not act:
                return work, it, None
        return None, o.max_newton, None

    # ------------------------------------------------------ schedules
    def run_local(self, st: State, schedule, alg=1, log=None):
        """Run a schedule with Algorithm 1 or 2 (alg=3: the residual-based
        localization; alg=4: Algorithm 2 with the additive phase 2),
        halving dt on failure."""
        step = {1: self.alg1_timestep, 2: self.alg2_timestep,
                3: self.resid_timestep,
                4: lambda *a: self.alg2_timestep(*a, additive=True)}[alg]
        prev = None
        recs = []
        for dt in schedule:
            pending = [dt]
            while pending:
                h = pending.pop(0)
                new, its, sup = step(st, h, prev, log)
                if new is None:
                    if h < dt / 2 ** self.opts.max_cuts:
                        raise RuntimeError("timestep cut limit reached")
                    pending = [h / 2, h / 2] + pending
                    continue
                recs.append(dict(dt=h, iters=its))
                st, prev = new, sup
        return st, recs
