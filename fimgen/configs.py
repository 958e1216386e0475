"""The synthetic workloads.

* ``make_c1``: single-phase 2D 64x64 grid, one 32-cell vertical fracture,
  producer at the fracture midpoint (stand-in for the paper's Case 1
  geometry, whose figures are not available);
* ``make_c2``: water/dead-oil 3D 200x100x10 grid with a seeded discrete
  fracture network of 2000 vertical fractures and one horizontal well with
  10 stage fractures;
* ``make_c3``: black oil (gas liberation below a 3500 psi bubble point)
  on a 400x200x8 grid with 5000 fractures;
* ``make_c4_member``: one member of the uneven batched ensemble;
* small and tiny variants with the same recipes for tests.

Fluid parameter dictionaries are SI.  The paper gives no fluid data for its
oil-water cases and uses compositional (not black-oil) physics, so every
fluid below is a stated synthetic choice.
"""
from __future__ import annotations

import math

import numpy as np

from .edfm import Fracture, embed
from .grid import cartesian_connections, layer_depths, lognormal_perm
from .model import FLUID_BLACKOIL, FLUID_DEADOIL, FLUID_SINGLE, Model
from .units import CP, DAY, GRAV, MD, PSI

P_REF = 5000.0 * PSI


def fluid_single():
    return {"kind": FLUID_SINGLE, "rho_ref": 800.0, "c": 1e-5 / PSI,
            "mu": 1.0 * CP, "p_ref": P_REF}


def fluid_deadoil():
    return {"kind": FLUID_DEADOIL, "rho_w": 1000.0, "c_w": 3e-6 / PSI,
            "mu_w": 0.5 * CP, "rho_o": 800.0, "c_o": 1e-5 / PSI,
            "mu_o": 1.0 * CP, "p_ref": P_REF, "swc": 0.2, "sor": 0.0}


def fluid_blackoil():
    return {"kind": FLUID_BLACKOIL, "rs_b": 100.0, "p_b": 3500.0 * PSI,
            "bo_slope": 0.0025, "c_o": 1e-5 / PSI,
            "bg_c": 14.696 * 1.24 * PSI, "c_w": 3e-6 / PSI, "p_ref": P_REF,
            "rho_osc": 800.0, "rho_gsc": 0.9, "rho_wsc": 1000.0,
            "mu_o": 1.0 * CP, "mu_g": 0.02 * CP, "mu_w": 0.5 * CP,
            "swc": 0.2, "span": 0.8}


def rock_default():
    return {"c_r": 1e-5 / PSI, "p_ref": P_REF}


def c1_schedule(n=20, first=1e-3, last=30.0):
    """Timesteps growing geometrically from ``first`` to ``last`` days."""
    k = np.arange(n)
    return first * (last / first) ** (k / (n - 1)) * DAY


def geometric_schedule(n, first_days, total_days):
    """n steps, first step ``first_days``, ratio chosen so they sum to
    ``total_days``."""
    lo, hi = 1.0 + 1e-12, 10.0
    for _ in range(200):
        r = 0.5 * (lo + hi)
        s = first_days * (r ** n - 1.0) / (r - 1.0)
        lo, hi = (r, hi) if s < total_days else (lo, r)
    r = 0.5 * (lo + hi)
    return first_days * r ** np.arange(n) * DAY


def hydrostatic_liquid(depth, z0, p0, rho_r, c, p_r, g=GRAV):
    """Continuous hydrostatic profile of a liquid whose density is
    rho_r exp(c (p - p_r)): the closed-form solution of dp/dz = g rho(p)
    through (z0, p0)."""
    e0 = math.exp(-c * (p0 - p_r))
    return p_r - np.log(e0 - c * g * rho_r * (depth - z0)) / c


def _assemble(name, nx, ny, nz, dx, dy, dz, top, perm, phi, fracs, perfs_fn,
              fluid, rock, schedule, init_fn, always_perf=True):
    n_m = nx * ny * nz
    ld = layer_depths(nz, dz, top)
    depth_m = np.repeat(ld, nx * ny)
    pv_m = np.full(n_m, dx * dy * dz * phi)
    ci, cj, T = cartesian_connections(nx, ny, nz, dx, dy, dz, perm)
    emb = embed(fracs, nx, ny, nz, dx, dy, dz, ld, perm, n_m)
    n = n_m + emb["n_frac_cells"]
    pv = np.concatenate([pv_m, emb["pv"]])
    depth = np.concatenate([depth_m, emb["depth"]])
    kind = np.zeros(n, np.int8)
    kind[n_m:] = 1
    ci = np.concatenate([ci, emb["ci"]]).astype(np.int32)
    cj = np.concatenate([cj, emb["cj"]]).astype(np.int32)
    T = np.concatenate([T, emb["T"]])
    order = np.lexsort((cj, ci))
    ci, cj, T = ci[order], cj[order], T[order]
    pc, wi, bhp = perfs_fn(emb)
    aa = (kind == 1).astype(np.uint8)
    if always_perf:
        aa[pc] = 1
    u0, st0 = init_fn(depth, n)
    m = Model(name=name, n_matrix=n_m, pv_ref=pv, depth=depth, kind=kind,
              always_active=aa, conn_i=ci, conn_j=cj, conn_T=T,
              perf_cell=np.asarray(pc, np.int32),
              perf_wi=np.asarray(wi, np.float64),
              perf_bhp=np.asarray(bhp, np.float64), fluid=fluid, rock=rock,
              gravity=GRAV, u0=u0, status0=st0,
              schedule=np.asarray(schedule, np.float64),
              grid=dict(nx=nx, ny=ny, nz=nz, dx=dx, dy=dy, dz=dz, top=top,
                        n_frac=len(fracs), host=emb["host"], fid=emb["fid"]))
    m.validate()
    return m


# ---------------------------------------------------------------- config 1
def make_c1(seed=1, nx=64, ny=64, perm_median=1e-4 * MD, sigma=0.5,
            uniform_perm=False, frac_rows=(16, 48), frac_col=None,
            schedule=None):
    """Single-phase 2D model: 10 m cells, one 32-segment fracture through
    the centre column, producer at the fracture midpoint (BHP 1000 psi)."""
    rng = np.random.default_rng(seed)
    dx = dy = dz = 10.0
    if uniform_perm:
        perm = np.full(nx * ny, perm_median)
    else:
        perm = lognormal_perm(rng, nx * ny, perm_median, sigma)
    col = nx // 2 if frac_col is None else frac_col
    xf = (col + 0.5) * dx
    r0, r1 = frac_rows
    fr = Fracture(xf, r0 * dy, xf, r1 * dy, 0, 0, 1e-3, 1e4 * MD)

    def perfs(emb):
        npiece = r1 - r0
        mid = [npiece // 2 - 1, npiece // 2] if npiece % 2 == 0 else [npiece // 2]
        cells = [emb["cell_of"][(0, p, 0)] for p in mid]
        wi = [fr.kf * fr.w * dz / (0.5 * dy)] * len(cells)
        return cells, wi, [1000.0 * PSI] * len(cells)

    def init(depth, n):
        u0 = np.full((1, n), P_REF)
        return u0, np.zeros(n, np.int8)

    return _assemble("c1", nx, ny, 1, dx, dy, dz, 2000.0 - 0.5 * dz, perm,
                     0.06, [fr], perfs, fluid_single(), rock_default(),
                     c1_schedule() if schedule is None else schedule, init)


def make_c1_variant(nx=21, ny=20, frac_rows=(5, 15), uniform_perm=True, seed=1,
                    schedule=None):
    """Small single-phase model, symmetric about the fracture (odd nx,
    fracture in the centre column) when ``uniform_perm``."""
    return make_c1(seed=seed, nx=nx, ny=ny, uniform_perm=uniform_perm,
                   frac_rows=frac_rows, frac_col=nx // 2,
                   schedule=c1_schedule(6, 1e-3, 10.0) if schedule is None else schedule)


# ------------------------------------------------------- configs 2, 3, 4
def _dfn(rng, nfrac, lx, ly, nz, lmin=20.0, lmax=200.0, height=2):
    fr = []
    cx = rng.uniform(0.0, lx, nfrac)
    cy = rng.uniform(0.0, ly, nfrac)
    th = rng.uniform(0.0, math.pi, nfrac)
    ln = rng.uniform(lmin, lmax, nfrac)
    k0 = rng.integers(0, max(1, nz - height + 1), nfrac)
    for i in range(nfrac):
        hx, hy = 0.5 * ln[i] * math.cos(th[i]), 0.5 * ln[i] * math.sin(th[i])
        fr.append(Fracture(cx[i] - hx, cy[i] - hy, cx[i] + hx, cy[i] + hy,
                           int(k0[i]), int(min(nz - 1, k0[i] + height - 1)),
                           1e-3, 1e4 * MD))
    return fr


def _stage_well(nx, ny, nz, dx, dy, dz, nstage, x_first, spacing, y_well,
                half_len, well_layer, bhp):
    """Stage fractures striking along y through the well line; returns the
    fracture list and a perforation builder (one perforation per stage, the
    fracture cell crossed by the well, radial in-plane well index)."""
    fr = []
    for s in range(nstage):
        xs = x_first + spacing * s
        fr.append(Fracture(xs, y_well - half_len + 0.5 * dy, xs,
                           y_well + half_len + 0.5 * dy, 0, nz - 1, 1e-3,
                           1e4 * MD))

    def perfs(emb):
        cells, wi = [], []
        for s in range(nstage):
            g = emb["geo"][s]
            (x0, y0, x1, y1), pieces, seglen = g
            t = (y_well - y0) / (y1 - y0)
            p_i = next(i for i, p in enumerate(pieces) if p[0] <= t <= p[1])
            L = (pieces[p_i][1] - pieces[p_i][0]) * seglen
            cells.append(emb["cell_of"][(s, p_i, well_layer)])
            re = 0.14 * math.hypot(L, dz)
            wi.append(2.0 * math.pi * fr[s].kf * fr[s].w / math.log(re / 0.1))
        return cells, wi, [bhp] * nstage

    return fr, perfs


def _two_phase_model(name, seed, nx, ny, nz, nfrac, fluid_kind, schedule,
                     nstage=10, dx=10.0, dy=10.0, dz=5.0, top=2500.0,
                     frac_sw=None):
    rng = np.random.default_rng(seed)
    lx, ly = nx * dx, ny * dy
    perm = lognormal_perm(rng, nx * ny * nz, 1e-4 * MD, 0.5)
    dfn = _dfn(rng, nfrac, lx, ly, nz)
    j_well = ny // 2
    y_well = (j_well + 0.5) * dy
    lat0, lat1 = 0.25 * lx, 0.75 * lx
    spacing = (lat1 - lat0) / nstage
    i_first = int((lat0 + 0.5 * spacing) // dx)
    x_first = (i_first + 0.5) * dx
    spacing = max(dx, round(spacing / dx) * dx)
    half = min(100.0, 0.2 * ly)
    wl = nz // 2
    stages, perfs = _stage_well(nx, ny, nz, dx, dy, dz, nstage, x_first,
                                spacing, y_well, half, wl, 1000.0 * PSI)
    fracs = stages + dfn
    z_top = top + 0.5 * dz
    if fluid_kind == FLUID_DEADOIL:
        fl = fluid_deadoil()

        def init(depth, n):
            p = hydrostatic_liquid(depth, z_top, P_REF, fl["rho_o"], fl["c_o"],
                                   fl["p_ref"])
            sw = np.full(n, fl["swc"])
            if frac_sw is not None:
                sw[kind_of(n)] = frac_sw
            return np.stack([p, sw]), np.zeros(n, np.int8)
    else:
        fl = fluid_blackoil()
        rho_ob = (fl["rho_osc"] + fl["rs_b"] * fl["rho_gsc"]) / (
            1.0 + fl["bo_slope"] * fl["rs_b"])

        def init(depth, n):
            p = hydrostatic_liquid(depth, z_top, P_REF, rho_ob, fl["c_o"],
                                   fl["p_b"])
            sw = np.full(n, fl["swc"])
            rs = np.full(n, fl["rs_b"])
            return np.stack([p, sw, rs]), np.zeros(n, np.int8)

    n_m = nx * ny * nz

    def kind_of(n):
        return np.arange(n) >= n_m

    return _assemble(name, nx, ny, nz, dx, dy, dz, top, perm, 0.06, fracs,
                     perfs, fl, rock_default(), schedule, init)


def make_c2(seed=2):
    """Water/dead-oil, 200x100x10 (10x10x5 m cells) + 2000-fracture DFN,
    horizontal well with 10 stage fractures, 20 steps to 71.6 days."""
    return _two_phase_model("c2", seed, 200, 100, 10, 2000, FLUID_DEADOIL,
                            c1_schedule())


def make_small_c2(seed=22, nx=24, ny=12, nz=4, nfrac=12, nstage=3,
                  schedule=None, frac_sw=None):
    """Same recipe as config 2 at a size the oracle solves in seconds."""
    return _two_phase_model("c2s", seed, nx, ny, nz, nfrac, FLUID_DEADOIL,
                            c1_schedule(6, 1e-3, 10.0) if schedule is None else schedule,
                            nstage=nstage, frac_sw=frac_sw)


def make_c3(seed=3):
    """Black oil, 400x200x8 + 5000-fracture DFN, 40 steps to 365 days."""
    return _two_phase_model("c3", seed, 400, 200, 8, 5000, FLUID_BLACKOIL,
                            geometric_schedule(40, 1e-3, 365.0))


def make_small_c3(seed=33, nx=20, ny=10, nz=4, nfrac=10, nstage=2,
                  schedule=None):
    return _two_phase_model("c3s", seed, nx, ny, nz, nfrac, FLUID_BLACKOIL,
                            geometric_schedule(8, 1e-3, 60.0) if schedule is None else schedule,
                            nstage=nstage)


def make_c4_member(k, base_seed=4000):
    """Member k of the batched ensemble: cell count uniform in 5k-200k,
    nz = 10, nx = 2 ny, DFN count proportional to the cell count."""
    rng = np.random.default_rng(base_seed + k)
    n_target = rng.uniform(5e3, 2e5)
    nz = 10
    ny = max(5, int(round(math.sqrt(n_target / 20.0))))
    nx = 2 * ny
    nfrac = int(round(2000 * nx * ny * nz / 2e5))
    return _two_phase_model(f"c4_{k}", base_seed + k, nx, ny, nz, nfrac,
                            FLUID_DEADOIL, c1_schedule())


# ------------------------------------------------------------ tiny models
def make_chain(ncell, length, perm=1e-15, phi=0.2, area=1.0, p_init=P_REF,
               p_w=1000.0 * PSI, wi_factor=1e6, schedule=None, c_r=1e-5 / PSI):
    """1D chain for linear pressure diffusion: incompressible liquid, linear
    porosity; cell 0 holds p_w through a very large well index."""
    dxc = length / ncell
    pv = np.full(ncell, area * dxc * phi)
    ci = np.arange(ncell - 1, dtype=np.int32)
    cj = ci + 1
    T = np.full(ncell - 1, perm * area / dxc)
    fl = fluid_single()
    fl["c"] = 0.0
    fl["p_ref"] = p_init
    m = Model(name="chain", n_matrix=ncell, pv_ref=pv,
              depth=np.full(ncell, 1000.0), kind=np.zeros(ncell, np.int8),
              always_active=np.zeros(ncell, np.uint8), conn_i=ci, conn_j=cj,
              conn_T=T, perf_cell=np.array([0], np.int32),
              perf_wi=np.array([wi_factor * T[0]]),
              perf_bhp=np.array([p_w]), fluid=fl,
              rock={"c_r": c_r, "p_ref": p_init}, gravity=GRAV,
              u0=np.full((1, ncell), p_init),
              status0=np.zeros(ncell, np.int8),
              schedule=np.array([DAY]) if schedule is None else np.asarray(schedule),
              grid=dict(nx=ncell, ny=1, nz=1, dx=dxc, dy=1.0, dz=1.0))
    m.always_active[0] = 1
    m.validate()
    return m


def make_tiny(which="grid5", fluid_kind=FLUID_SINGLE, seed=7):
    """Tiny models for brute-force checks: 'one' (a single cell with a well),
    'grid3' / 'grid5' (3x3 / 5x5 2D grids plus one long-range NNC)."""
    rng = np.random.default_rng(seed)
    if which == "one":
        nx = ny = 1
    elif which == "grid3":
        nx = ny = 3
    else:
        nx = ny = 5
    nz = 1
    dx = dy = dz = 10.0
    n = nx * ny
    perm = lognormal_perm(rng, n, 1e-3 * MD, 0.5)
    ci, cj, T = cartesian_connections(nx, ny, nz, dx, dy, dz, perm)
    if n > 2:
        ci = np.append(ci, 0).astype(np.int32)
        cj = np.append(cj, n - 1).astype(np.int32)
        T = np.append(T, 3.0 * T.mean())
    depth = 2000.0 + rng.uniform(-5.0, 5.0, n)
    pv = np.full(n, dx * dy * dz * 0.1)
    if fluid_kind == FLUID_SINGLE:
        fl = fluid_single()
        u0 = np.full((1, n), P_REF) + rng.uniform(-50, 50, (1, n)) * PSI
    elif fluid_kind == FLUID_DEADOIL:
        fl = fluid_deadoil()
        u0 = np.stack([np.full(n, P_REF) + rng.uniform(-50, 50, n) * PSI,
                       rng.uniform(0.25, 0.7, n)])
    else:
        fl = fluid_blackoil()
        u0 = np.stack([np.full(n, P_REF) + rng.uniform(-50, 50, n) * PSI,
                       rng.uniform(0.25, 0.4, n), np.full(n, 80.0)])
    m = Model(name="tiny_" + which, n_matrix=n, pv_ref=pv, depth=depth,
              kind=np.zeros(n, np.int8),
              always_active=np.zeros(n, np.uint8),
              conn_i=ci.astype(np.int32), conn_j=cj.astype(np.int32),
              conn_T=T, perf_cell=np.array([n // 2], np.int32),
              perf_wi=np.array([5.0 * (T.mean() if T.size else 1e-15)]),
              perf_bhp=np.array([3000.0 * PSI]), fluid=fl,
              rock=rock_default(), gravity=GRAV, u0=u0,
              status0=np.zeros(n, np.int8),
              schedule=np.array([0.1, 1.0, 10.0]) * DAY,
              grid=dict(nx=nx, ny=ny, nz=nz, dx=dx, dy=dy, dz=dz))
    m.always_active[n // 2] = 1
    m.validate()
    return m
