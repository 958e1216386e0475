#!/usr/bin/env python3
"""Benchmark: active-cell Newton updates/s of localized vs full Newton on one
MI355X, with p50/p99 Newton-step latency, the roofline of the dominant kernel
and the FP64 oracle timed on the host cores.

Workload (one "step" = one fully implicit timestep solved to convergence):
the black-oil model of 400x200x8 matrix cells plus a seeded 5000-fracture
DFN and a 10-stage horizontal well (784,166 cells, 3x3 blocks), its
40-step schedule to 365 days; the first `warmup` steps run untimed, the
next `steps` are timed (warmup + steps must fit the schedule); localized
Newton (Algorithm 1, eps_p = 0.3 psi, m = 2) with FP64 assembly, flash and
switching and an FP32 BiCGStab inside FP64 refinement.  `--workload c2`
runs the water/dead-oil config-2 model (258,096 cells) the same way.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor peak


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def plan_bytes(kernel, rec, b, kbytes):
    """Algorithmic bytes of the method's work in the launches of one profile
    record, by the per-row figures of the measurement plan (one unit = one
    active row, i.e. one row of the local block system; nnzb = blocks of the
    active rows, diagonal included, so nnzb = rows (1 + f') with f' the
    active-active connections per row):

    * matrix product (BSR SpMV): s b^2 + 4 bytes per block (values,
      column index), 4 per row (row pointer), 2 s b per row (source and
      result vectors);
    * block-Jacobi apply: s b^2 + 2 s b per row;
    * one BiCGStab iteration = 2 products + 2 applies + about 20 vector
      passes of s b bytes per row; each of the library's two kernels per
      iteration carries one product, one apply and 10 passes;
    * assembly: reads 8 (2b + 1) per row plus 20 per connection (neighbour
      index, T, neighbour state counted once; f taken as f'), writes 8b +
      8b^2 (1 + f') + 4 (1 + f') + 4 per row, plus the s b^2 (1 + f')
      Krylov-precision copy.

    s = bytes of the Krylov precision.  These figures count what the
    method must move on the active rows; the library's own kernels fuse
    the apply into the product (the matrix is stored block-Jacobi scaled
    with an implicit identity diagonal) and move less, and its
    fracture-block preconditioner adds the bytes that fracture_bytes
    reports."""
    rows, nnzb = rec["rows"], rec["nnzb"]
    if kernel in ("bicg_spmv_p", "bicg_spmv_s"):
        spmv = nnzb * (kbytes * b * b + 4) + rows * (4 + 2 * kbytes * b)
        apply = rows * (kbytes * b * b + 2 * kbytes * b)
        return spmv + apply + rows * 10 * kbytes * b
    if kernel == "assemble":
        f = max(nnzb - rows, 0.0)
        return (rows * (8 * (2 * b + 1) + 8 * b + 4) + f * 20
                + nnzb * (8 * b * b + 4 + kbytes * b * b))
    raise KeyError(kernel)


def kernel_bytes(kernel, rec, b, kbytes):
    """Bytes the library's fused kernel itself must move for the same work
    (every entry it reads or writes once, neighbour gathers counted once,
    sliced-ELL padding excluded), without its fracture-block preconditioner
    (fracture_bytes)."""
    rows, nnzb = rec["rows"], rec["nnzb"]
    off = max(nnzb - rows, 0.0)
    if kernel == "bicg_spmv_p":
        # col + block per off-diagonal; s, t, p, v, x, rh read; x, r, p, v written
        return off * (4 + kbytes * b * b) + rows * 10 * b * kbytes
    if kernel == "bicg_spmv_s":   # col + block; r, v, rh read; s, t written
        return off * (4 + kbytes * b * b) + rows * 5 * b * kbytes
    if kernel == "assemble":
        # per row: l2g 4, state 8b, status 1, pv 8, depth 8, flags 1, old
        # masses 8b, adjacency pointers 8, residual 8b written; per
        # connection of an active pair: neighbour id 4, T 8, g2l 4; per
        # block: 8 b^2 values + 4 col written
        return rows * (30 + 24 * b) + off * 16 + nnzb * (8 * b * b + 4)
    raise KeyError(kernel)


def fracture_bytes(kernel, rec):
    """Bytes of the fracture-block preconditioner inside a product kernel:
    the FP32 inverse entries it applied (aux) and 8 bytes of block layout
    per row."""
    if kernel not in ("bicg_spmv_p", "bicg_spmv_s") or not rec.get("aux"):
        return 0.0
    return 4.0 * rec["aux"] + 8.0 * rec["rows"]


PROFILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
PROFILE_SUMMARY = {"c3": os.path.join(PROFILES, "c3_local_kernels.md"),
                   "c2": os.path.join(PROFILES, "c2_local_kernels.md")}
KERNEL_SOURCES = ["fim_krylov.hip", "fim_fracpc.hip", "fim_internal.hpp", "fim_device.hpp"]


def measured_traffic_per_row(workload):
    """HBM bytes per row of each kernel from the committed rocprofv3 counter
    summary of the workload, or {} when the kernel sources changed since it
    was taken."""
    import hashlib
    try:
        text = open(PROFILE_SUMMARY[workload]).read()
    except (OSError, KeyError):
        return {}
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2008_01539_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    out, ok = {}, False
    for line in text.splitlines():
        parts = line.split()
        if len(parts) == 2 and parts[0] == "sources_sha256":
            ok = parts[1] == h.hexdigest()
        elif len(parts) == 3 and parts[0] == "traffic_bytes_per_row":
            out[parts[1]] = float(parts[2])
    return out if ok else {}


def roofline_of(prof, b, kbytes=4, names=("assemble", "bicg_spmv_p", "bicg_spmv_s")):
    """The kernel with the most time in an event-profiled run: algorithmic
    bytes per launch (plan_bytes) over its average launch duration; beside
    it the bytes of the fused kernel itself and of the fracture-block
    preconditioner it applies (not part of frac)."""
    cands = {k: v for k, v in prof.items() if k in names and v["launches"]}
    dom = max(cands, key=lambda k: cands[k]["total_ms"])
    rec = cands[dom]
    L = rec["launches"]
    avg_s = rec["total_ms"] / L * 1e-3
    byt = plan_bytes(dom, rec, b, kbytes) / L
    own = kernel_bytes(dom, rec, b, kbytes) / L
    frc = fracture_bytes(dom, rec) / L
    ach = byt / avg_s / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "avg_launch_us": avg_s * 1e6,
            "bytes_per_launch": byt, "rows_per_launch": rec["rows"] / L,
            "blocks_per_launch": rec["nnzb"] / L,
            "kernel_own_bytes_per_launch": own,
            "kernel_own_gbs": own / avg_s / 1e9,
            "fracture_block_bytes_per_launch": frc,
            "fracture_block_gbs": frc / avg_s / 1e9}


def copy_bandwidth(mib=1024, reps=10):
    """Read + write bytes per second of a plain device-to-device copy of
    `mib` MiB (larger than the 256 MiB Infinity Cache), timed with events."""
    import torch
    n_el = mib * 2**20 // 4
    src = torch.ones(n_el, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * n_el * 4 / sec / 1e9


def run_gpu(model, opts, mode, steps, warmup, profile=False):
    """Timesteps warmup .. warmup+steps-1 of the model's schedule with
    `mode`; the first `warmup` steps run untimed from the initial state.
    Returns totals over the timed steps, Newton-step and timestep
    latencies and the final state."""
    import numpy as np
    import torch
    import paper_2008_01539_amd as P
    sched = model.schedule
    assert warmup + steps <= len(sched)
    fm = P.FimModel(model, opts)
    fm.set_state(model.u0, model.status0)

    def one_step(dt, lat):
        act = its = kry = 0
        t0 = time.perf_counter()
        while True:
            t1 = time.perf_counter()
            it = fm.newton_step(dt, mode)
            if lat is not None:
                lat.append(time.perf_counter() - t1)
            if it.converged and mode == P.DD and it.phase == 2 and it.n_active == 0:
                break                 # Algorithm 2 found nothing left to solve
            act += it.n_active
            its += 1
            kry += it.krylov_iters
            if it.converged:
                break
        return act, its, kry, time.perf_counter() - t0

    for dt in sched[:warmup]:
        one_step(dt, None)
    torch.cuda.synchronize()
    if profile:
        fm.profile(True)
    lat, step_lat = [], []
    tot_act = tot_its = tot_kry = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for dt in sched[warmup:warmup + steps]:
        a, i, kr, st = one_step(dt, lat)
        tot_act += a
        tot_its += i
        tot_kry += kr
        step_lat.append(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = fm.profile_read() if profile else None
    u, _ = fm.get_state()
    fm.close()
    lat_ms = np.array(lat) * 1e3
    return dict(wall=wall, active=tot_act, iters=tot_its, krylov=tot_kry,
                p50=float(np.percentile(lat_ms, 50)), p99=float(np.percentile(lat_ms, 99)),
                step_p50=float(np.percentile(np.array(step_lat) * 1e3, 50)),
                step_p99=float(np.percentile(np.array(step_lat) * 1e3, 99)),
                u=u, prof=prof)


def _oracle_schedule(model, schedule, runs):
    """The oracle's full Newton over a schedule from the initial state, the
    median wall of `runs` runs; returns (wall, iterations, steps)."""
    import numpy as np
    from oracle.newton import Options, Solver, State
    walls = []
    its = 0
    for _ in range(runs):
        s = Solver(model, Options())
        st = State(model.u0.copy(), model.status0.copy())
        its = 0
        t0 = time.perf_counter()
        for dt in schedule:
            st, i = s.solve_timestep(st, dt)
            assert st is not None
            its += i
        walls.append(time.perf_counter() - t0)
    return float(np.median(walls)), its, len(schedule)


def cpu_baseline(log_fn, workload, warmup, steps):
    """The FP64 oracle (full Newton, complex-step Jacobian, SuperLU) on one
    host thread: a bounded sample of the benchmark workload (its recipe on
    a reduced grid over the same timestep window) and config 1 over its
    whole 20-step schedule (median of three runs)."""
    os.environ["OMP_NUM_THREADS"] = "1"
    from fimgen import make_c1
    from fimgen.configs import _two_phase_model, c1_schedule, geometric_schedule
    from fimgen.model import FLUID_BLACKOIL, FLUID_DEADOIL
    if workload == "c3":
        m = _two_phase_model("c3_sample", 3, 24, 12, 8, 18, FLUID_BLACKOIL,
                             geometric_schedule(40, 1e-3, 365.0), nstage=2)
        desc = "config-3 recipe (black oil) on a 24x12x8 grid + 18 fractures + 2 stages"
    else:
        m = _two_phase_model("c2_sample", 2, 30, 15, 10, 45, FLUID_DEADOIL, c1_schedule())
        desc = "config-2 recipe (water/dead oil) on a 30x15x10 grid + 45 fractures"
    sched = m.schedule[:min(len(m.schedule), warmup + steps)]
    wall, its, nst = _oracle_schedule(m, sched, 1)
    log_fn(f"oracle sample: n={m.n} steps={nst} iterations={its} wall={wall:.1f}s")
    c1 = make_c1()
    w1, i1, n1 = _oracle_schedule(c1, c1.schedule, 3)
    log_fn(f"oracle config 1: {n1} steps, {i1} iterations, median wall {w1:.1f}s")
    return dict(value=m.n * its / wall, unit="cell-updates/s", cores=1, kind="oracle",
                sample=f"{desc} (n={m.n} cells), timesteps 0..{nst - 1} of its schedule "
                       f"(the benchmark's window from the initial state), full Newton + "
                       f"SuperLU, FP64, 1 thread: {its} iterations in {wall:.1f} s",
                s_per_iteration=wall / its, s_per_timestep=wall / nst,
                config1={"n_cells": c1.n, "timesteps": n1, "iterations": i1,
                         "wall_s_median_of_3": w1, "s_per_iteration": w1 / i1,
                         "s_per_timestep": w1 / n1, "cell_updates_per_s": c1.n * i1 / w1},
                host_cpu=_cpu_name(), host_cores=os.cpu_count())


def _cpu_name():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor()


# ------------------------------------------------------------- other workloads
def _member(k):
    from fimgen import make_c4_member
    return make_c4_member(k)


def _pool_models(fn, ids, procs=16):
    """Builds models in worker processes; called before this process
    initialises the GPU (the workers are forked from it)."""
    import multiprocessing as mp
    log(f"generating {len(ids)} models")
    with mp.get_context("fork").Pool(min(procs, len(ids))) as pool:
        return pool.map(fn, ids)


def run_c4(models, steps):
    """Batched ensemble: the config-4 models advanced together, one Newton
    iteration of every live member per batched call, each member through
    its own schedule; then the same members one after another."""
    import numpy as np
    import torch
    import paper_2008_01539_amd as P
    members = len(models)
    ncell = sum(m.n for m in models)
    log(f"total cells {ncell}")
    opts = P.Options(precision=P.MIXED)
    fms = [P.FimModel(m, opts) for m in models]
    for fm, m in zip(fms, models):
        fm.set_state(m.u0, m.status0)
    log(f"device bytes {sum(fm.device_bytes() for fm in fms) / 2**30:.1f} GiB")
    step = [0] * members
    live = list(range(members))
    bat = P.FimBatch([fms[i] for i in live])
    lat, act = [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while live:
        dts = [models[i].schedule[step[i]] for i in live]
        t1 = time.perf_counter()
        stats, codes = bat.newton_step(dts, [P.LOCAL] * len(live))
        lat.append(time.perf_counter() - t1)
        nxt = []
        for i, st, c in zip(live, stats, codes):
            act += st["n_active"]
            if st["converged"]:
                step[i] += 1
            if c == 0 and step[i] < steps:
                nxt.append(i)
        if nxt != live and nxt:
            bat.set_models([fms[i] for i in nxt])
        live = nxt
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    bat.close()
    u_batch = [fm.get_state()[0] for fm in fms]
    for fm in fms:
        fm.close()
    log(f"batched: {len(lat)} calls, wall {wall:.2f}s")
    # the same members one after another
    t0 = time.perf_counter()
    same = True
    for i, m in enumerate(models):
        fm = P.FimModel(m, opts)
        fm.set_state(m.u0, m.status0)
        for dt in m.schedule[:steps]:
            fm.solve_timestep(dt, P.LOCAL)
        same = same and bool(np.array_equal(fm.get_state()[0], u_batch[i]))
        fm.close()
    torch.cuda.synchronize()
    wall_seq = time.perf_counter() - t0
    log(f"sequential: wall {wall_seq:.2f}s, identical results {same}")
    lat_ms = np.array(lat) * 1e3
    return {
        "metric": "active-cell Newton updates/s, batched ensemble (1 GPU); p50/p99 batched-call latency",
        "value": act / wall, "unit": "active-cell Newton updates/s", "n_gpus": 1,
        "steps": steps, "warmup": 0, "higher_is_better": True, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"config 4: {members} water/dead-oil members (seeds 4000+k, "
                               f"5k-200k cells each, {ncell} cells), first {steps} timesteps of "
                               "each member's schedule, localized Newton, one Newton iteration "
                               "of every live member per batched call", "members": members},
        "batched_wall_s": wall, "sequential_wall_s": wall_seq,
        "batching_speedup": wall_seq / wall, "batch_equals_solo_bitwise": same,
        "call_ms_p50": float(np.percentile(lat_ms, 50)),
        "call_ms_p99": float(np.percentile(lat_ms, 99)), "calls": len(lat),
    }


def _c5_session(args):
    kind, k = args
    from fimgen import make_c1, make_c2, make_c3
    if kind == 1:
        return make_c1(seed=5000 + k)
    if kind == 2:
        return make_c2(seed=6000 + k)
    return make_c3(seed=7000 + k)


def run_c5(models, ids, seconds, pool, budget_gib, rate=50.0):
    """Serving: Poisson timestep requests at `rate`/s over a pool of
    config-1, -2 and -3 sessions (50/40/10 % of requests); sessions are
    admitted up to the HBM budget before the clock starts, the rest on
    demand (evicting idle ones)."""
    import numpy as np
    import paper_2008_01539_amd as P
    from paper_2008_01539_amd.serve import GpuExecutor, Server, SessionSpec
    n1, n2, n3 = pool
    specs = [SessionSpec(name=f"{kind}-{k}", model=m, options=P.Options(precision=P.MIXED),
                         schedule=m.schedule) for (kind, k), m in zip(ids, models)]
    mix = np.array([0.5 / n1] * n1 + [0.4 / n2] * n2 + [0.1 / n3] * n3)
    ex = GpuExecutor()
    srv = Server(specs, ex, budget_bytes=int(budget_gib * 2**30), max_inflight=64,
                 footprint=lambda sp: P.estimate_bytes(sp.model, sp.options))
    t0 = time.perf_counter()
    res = srv.warm()
    log(f"warm: {res} sessions resident ({srv.used / 2**30:.1f} GiB) in "
        f"{time.perf_counter() - t0:.1f}s; serving {seconds}s at {rate}/s")
    summ = srv.run_poisson(
        rate=rate, duration=seconds, mix=mix, seed=5,
        progress=lambda t, st: log(f"t={t:.0f}s completed {st.completed} ticks {st.ticks} "
                                   f"queued {len(srv.queue)} inflight {len(srv.inflight)}"))
    ex.close()
    return {
        "metric": "served timestep requests/s and p50/p99 request latency (1 GPU)",
        "value": summ["throughput_rps"], "unit": "requests/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"config 5: Poisson arrivals at {rate}/s for {seconds}s, "
                               f"50/40/10 % of requests over {n1} config-1, {n2} config-2 and "
                               f"{n3} config-3 sessions (full sizes; seeds 5000+k, 6000+k, "
                               f"7000+k), HBM budget {budget_gib} GiB, continuous batching",
                   "rate": rate, "seconds": seconds, "pool": list(pool),
                   "budget_gib": budget_gib},
        "serving": summ,
    }


WORKLOADS = {
    "c3": "config 3: black oil (bubble point 3500 psi, S_g/R_s switching), 400x200x8 grid "
          "+ seeded 5000-fracture DFN + 10-stage horizontal well ({n} cells, {nc} "
          "connections, 3x3 blocks), 40-step schedule to 365 d",
    "c2": "config 2: water/dead-oil, 200x100x10 grid + seeded 2000-fracture DFN + 10-stage "
          "horizontal well ({n} cells, {nc} connections, 2x2 blocks), 20-step schedule to "
          "71.6 d",
}


def _rel_dp(u, ref):
    import numpy as np
    return float(np.abs(u[0] - ref[0]).max() / ref[0].min())


def _max_dp_psi(u, ref):
    import numpy as np
    return float(np.abs(u[0] - ref[0]).max() / 6894.757293168)


def _leg(r, model, full_wall=None, ref=None):
    out = {"iterations": r["iters"], "sum_active": r["active"],
           "avg_ma": r["active"] / model.n / max(r["iters"], 1),
           "updates_per_s": r["active"] / r["wall"], "krylov_iters": r["krylov"],
           "wall_s": r["wall"], "newton_step_ms_p50": r["p50"],
           "newton_step_ms_p99": r["p99"], "timestep_ms_p50": r["step_p50"],
           "timestep_ms_p99": r["step_p99"]}
    if full_wall is not None:
        out["speedup_vs_full"] = full_wall / r["wall"]
    if ref is not None:
        out["max_rel_dp_vs_tight_ref"] = _rel_dp(r["u"], ref)
        out["max_dp_vs_tight_ref_psi"] = _max_dp_psi(r["u"], ref)
    return out


def run_single(workload, args):
    """One model at full size: localized Newton (Algorithm 1, the headline),
    full Newton, Algorithm 2 and the residual-based localization on the same
    timesteps, each from the initial state with the same untimed warm-up
    steps; a tight FP64 full-Newton reference over the same steps for the
    accuracy of every leg; the roofline of the dominant kernel from an
    event-profiled replay of the localized leg."""
    import numpy as np
    import torch
    import paper_2008_01539_amd as P
    from fimgen import make_c2, make_c3
    log(f"building the {workload} model")
    model = make_c3() if workload == "c3" else make_c2()
    L = len(model.schedule)
    if args.warmup + args.steps > L:
        print(f"bench.py: warmup + steps = {args.warmup + args.steps} exceeds the "
              f"{L}-step schedule of {workload}", file=sys.stderr)
        sys.exit(2)
    # fracture cells localized too: only perforated cells always active
    aa = np.zeros_like(model.always_active)
    aa[np.asarray(model.perf_cell, dtype=np.int64)] = 1
    model_lf = model.copy_with(always_active=aa)
    if args.localize_fractures:
        model = model_lf
    log(f"n={model.n} connections={model.nc}")
    opts = P.Options(precision=P.MIXED)
    W, K = args.warmup, args.steps
    log(f"localized Newton: warm-up steps 0..{W - 1}, timed steps {W}..{W + K - 1}")
    loc = run_gpu(model, opts, P.LOCAL, K, W)
    log(f"local: {loc['iters']} iterations, wall {loc['wall']:.3f}s, krylov {loc['krylov']}")
    prof_run = None
    if args.profile:
        # the same steps again with launch events (they add host work, so the
        # headline comes from the run above)
        prof_run = run_gpu(model, opts, P.LOCAL, K, W, profile=True)
        log(f"local (events): wall {prof_run['wall']:.3f}s")
    legs = {}
    if not args.no_full:
        for name, mode in (("full", P.FULL), ("dd", P.DD), ("dd_add", P.DD_ADD),
                           ("resid", P.RESID)):
            legs[name] = run_gpu(model, opts, mode, K, W)
            log(f"{name}: {legs[name]['iters']} iterations, wall {legs[name]['wall']:.3f}s, "
                f"krylov {legs[name]['krylov']}")
        if not args.localize_fractures:
            legs["local_frac"] = run_gpu(model_lf, opts, P.LOCAL, K, W)
            log(f"local, fracture cells localized: wall {legs['local_frac']['wall']:.3f}s")
        legs["local_fp64"] = run_gpu(model, P.Options(precision=P.FP64), P.LOCAL, K, W)
        log(f"local FP64: wall {legs['local_fp64']['wall']:.3f}s")
        if args.profile:
            # the product kernels over the whole system: full Newton's first
            # three timed steps again with launch events
            legs["full_events"] = run_gpu(model, opts, P.FULL, min(3, K), W, profile=True)
            log(f"full (events, {min(3, K)} steps): wall {legs['full_events']['wall']:.3f}s")
        ref = run_gpu(model, P.Options.tight_mode(precision=P.FP64), P.FULL, K, W)["u"]
        log("tight FP64 full-Newton reference done")
    value = loc["active"] / loc["wall"]
    out = {
        "metric": "active-cell Newton updates/s, local vs full Newton (1 GPU); "
                  "p50/p99 step latency",
        "value": value,
        "unit": "active-cell Newton updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": loc["wall"] / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS[workload].format(n=model.n, nc=model.nc)
                        + f"; timed steps {W}..{W + K - 1} after {W} untimed; localized "
                          "Newton (Algorithm 1, eps_p 0.3 psi, m 2), FP64 assembly/update/"
                          "switching, FP32 BiCGStab (block-Jacobi scaling + fracture-block "
                          "inverses) inside FP64 refinement to the Eisenstat-Walker forcing "
                          "term in [1e-4, 0.1]",
            "n_cells": model.n,
            "fractures_always_active": not args.localize_fractures,
            "krylov_dtype": "f32",
            "parallelism": "1 GPU",
        },
        "local": _leg(loc, model),
    }
    if legs:
        fw = legs["full"]["wall"]
        out["local"].update(speedup_vs_full=fw / loc["wall"],
                            max_rel_dp_vs_tight_ref=_rel_dp(loc["u"], ref),
                            max_dp_vs_tight_ref_psi=_max_dp_psi(loc["u"], ref),
                            max_rel_dp_mixed_vs_fp64=_rel_dp(loc["u"], legs["local_fp64"]["u"]))
        out["full"] = _leg(legs["full"], model, ref=ref)
        out["dd"] = _leg(legs["dd"], model, fw, ref)
        # NEXT-3 of the scope: Algorithm 2 with the additive phase 2 (an
        # iteration here is one sweep over the pending subdomains)
        out["dd_additive"] = _leg(legs["dd_add"], model, fw, ref)
        out["resid"] = _leg(legs["resid"], model, fw, ref)
        out["resid"]["local_speedup_vs_resid"] = legs["resid"]["wall"] / loc["wall"]
        out["local_fp64"] = _leg(legs["local_fp64"], model, fw, ref)
        if "local_frac" in legs:
            # NEXT-1 of the scope: fracture cells localized as well, the
            # active sets closed under fracture components
            out["local_localized_fractures"] = _leg(legs["local_frac"], model, fw, ref)
        out["speedup_local_vs_full"] = fw / loc["wall"]
        out["accuracy_reference"] = ("tight-mode FP64 full Newton (eps 1e-7 psi, linear rtol "
                                     "1e-12) over the same steps from the same initial state")
    prof = prof_run["prof"] if prof_run else None
    if prof:
        copy = copy_bandwidth()
        roof = roofline_of(prof, model.b)
        per_row = measured_traffic_per_row(workload).get(roof["kernel"])
        out["roofline"] = {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac")}
        # counter-measured HBM bytes per launch (FETCH_SIZE + WRITE_SIZE scaled
        # by a plain copy, per row, times this run's rows per launch); None
        # once the kernels changed since the counters were taken
        out["roofline"]["traffic"] = per_row * roof["rows_per_launch"] if per_row else None
        out["roofline"].update({k: v for k, v in roof.items() if k not in out["roofline"]})
        out["roofline"].update(copy_gbps=copy, frac_of_copy=roof["achieved"] / copy,
                               profiled_wall_s=prof_run["wall"])
        out["kernel_profile_local"] = prof
        if "full_events" in legs:
            # the same kernel class over the whole system (every cell a row),
            # the same byte definitions; context beside the headline's kernel
            rf = roofline_of(legs["full_events"]["prof"], model.b, names=(roof["kernel"],))
            out["roofline_full_system"] = {k: rf[k] for k in (
                "kernel", "achieved", "peak", "unit", "frac", "avg_launch_us", "bytes_per_launch",
                "rows_per_launch", "kernel_own_gbs", "fracture_block_gbs")}
            out["roofline_full_system"]["frac_of_copy"] = rf["achieved"] / copy
    if args.calibrate_copy:
        # one plain device-to-device copy of known size (memory-counter scale)
        n_el = args.calibrate_copy * 2**20 // 4
        src = torch.ones(n_el, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = n_el * 4
        del src, dst
    if not args.no_cpu:
        log("oracle CPU baseline")
        out["cpu_baseline"] = cpu_baseline(log, workload, W, K)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=["c2", "c3", "c4", "c5"])
    ap.add_argument("--localize-fractures", action="store_true",
                    help="fracture cells not always active (only perforated cells are); "
                         "the default keeps them active as in the paper's runs")
    ap.add_argument("--members", type=int, default=256)
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--pool", default="256,64,16",
                    help="serving: config-1,2,3 session counts")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-full", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the run, copy MIB MiB device to device once (a plain copy "
                         "kernel of known size for scaling memory counters)")
    ap.add_argument("--profile", type=int, default=1,
                    help="replay the timed localized steps with per-kernel hipEvents")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(the multi-GPU design is documented, not built)", file=sys.stderr)
        sys.exit(2)
    if args.workload in ("c4", "c5"):
        # the ensemble and serving pools are generated in worker processes
        # before this process touches the GPU
        if args.workload == "c4":
            models = _pool_models(_member, list(range(args.members)))
        else:
            pool = tuple(int(v) for v in args.pool.split(","))
            ids = ([(1, k) for k in range(pool[0])] + [(2, k) for k in range(pool[1])]
                   + [(3, k) for k in range(pool[2])])
            models = _pool_models(_c5_session, ids)
    import torch
    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    if args.workload == "c4":
        print(json.dumps(run_c4(models, max(1, args.steps))), flush=True)
        return
    if args.workload == "c5":
        print(json.dumps(run_c5(models, ids, args.serve_seconds, pool, args.budget_gib)),
              flush=True)
        return
    print(json.dumps(run_single(args.workload, args)), flush=True)


if __name__ == "__main__":
    main()
