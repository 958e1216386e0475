#!/usr/bin/env python3
"""Benchmark: active-cell Newton updates/s of localized vs full Newton on one
MI355X, with p50/p99 Newton-step latency, the roofline of the dominant kernel
and the FP64 oracle timed on the host cores.

Workload (one "step" = one fully implicit timestep solved to convergence):
the water/dead-oil model of 200x100x10 matrix cells plus a seeded
2000-fracture DFN and a 10-stage horizontal well (258,096 cells), its 20-step
schedule to 71.6 days, localized Newton (Algorithm 1, eps_p = 0.3 psi,
m = 2) with FP64 assembly and an FP32 BiCGStab inside FP64 refinement.
Steps past the end of the schedule restart it from the initial state.

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


def algorithmic_bytes(kernel, rec, b, kbytes, pc=True):
    """Bytes a kernel must move per the work it did (one active row = one
    unit): every array entry it reads or writes once, neighbour gathers
    counted once (cache reuse), padding of the sliced-ELL matrix excluded.
    rec: profile record with rows, nnzb (blocks incl. diagonal) and aux
    (FP32 fracture-block inverse entries applied by the product kernels)."""
    rows, nnzb = rec["rows"], rec["nnzb"]
    off = max(nnzb - rows, 0.0)
    aux = rec.get("aux", 0.0)
    blk = 8 if (pc and aux > 0) else 0   # block layout words per row
    if kernel == "bicg_spmv_p":
        # col + block per off-diagonal; s, t, p, v, x, rh read; x, r, p, v
        # written; the inverse entries of the fracture blocks
        return off * (4 + kbytes * b * b) + rows * (10 * b * kbytes + blk) + 4 * aux
    if kernel == "bicg_spmv_s":   # col + block; r, v, rh read; s, t written
        return off * (4 + kbytes * b * b) + rows * (5 * b * kbytes + blk) + 4 * aux
    if kernel == "assemble":
        # per row: l2g 4, state 8b, status 1, pv 8, depth 8, flags 1, old
        # masses 8b, adjacency pointers 8, residual 8b written; per
        # connection of an active pair: neighbour id 4, T 8, g2l 4; per
        # block: 8 b^2 values + 4 col written
        return rows * (30 + 24 * b) + off * 16 + nnzb * (8 * b * b + 4)
    raise KeyError(kernel)


PROFILE_SUMMARY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                               "c2_local_kernels.md")
KERNEL_SOURCES = ["fim_krylov.hip", "fim_fracpc.hip", "fim_internal.hpp", "fim_device.hpp"]


def measured_traffic_per_row():
    """HBM bytes per row of each kernel from the committed rocprofv3 counter
    summary, or {} when the kernel sources changed since it was taken."""
    import hashlib
    try:
        text = open(PROFILE_SUMMARY).read()
    except OSError:
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
    """Achieved algorithmic bandwidth of the kernel with the most time in an
    event-profiled run: bytes per launch / average launch duration."""
    cands = {k: v for k, v in prof.items() if k in names and v["launches"]}
    dom = max(cands, key=lambda k: cands[k]["total_ms"])
    rec = cands[dom]
    avg_s = rec["total_ms"] / rec["launches"] * 1e-3
    byt = algorithmic_bytes(dom, rec, b, kbytes) / rec["launches"]
    ach = byt / avg_s / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "avg_launch_us": avg_s * 1e6,
            "bytes_per_launch": byt, "rows_per_launch": rec["rows"] / rec["launches"]}


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
    import numpy as np
    import torch
    import paper_2008_01539_amd as P
    fm = P.FimModel(model, opts)
    fm.set_state(model.u0, model.status0)
    sched = model.schedule
    L = len(sched)
    k = 0

    def one_step(lat):
        nonlocal k
        if k > 0 and k % L == 0:
            fm.set_state(model.u0, model.status0)
        dt = sched[k % L]
        k += 1
        act = its = kry = 0
        t0 = time.perf_counter()
        while True:
            t1 = time.perf_counter()
            it = fm.newton_step(dt, mode)
            if lat is not None:
                lat.append(time.perf_counter() - t1)
            act += it.n_active
            its += 1
            kry += it.krylov_iters
            if it.converged:
                break
        return act, its, kry, time.perf_counter() - t0

    for _ in range(warmup):
        one_step(None)
    torch.cuda.synchronize()
    if profile:
        fm.profile(True)
    lat, step_lat = [], []
    tot_act = tot_its = tot_kry = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        a, i, kr, st = one_step(lat)
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
                u=u, prof=prof, k_end=k)


def cpu_baseline(log_fn):
    """The FP64 oracle (full Newton, SuperLU) on a bounded sample of the
    same workload: the config-2 recipe (same physics, DFN density and well
    layout) on a 30x15x10 grid, its first 8 timesteps, single thread."""
    os.environ["OMP_NUM_THREADS"] = "1"
    from fimgen.configs import _two_phase_model, c1_schedule
    from fimgen.model import FLUID_DEADOIL
    from oracle.newton import Options, Solver, State
    m = _two_phase_model("c2_sample", 2, 30, 15, 10, 45, FLUID_DEADOIL, c1_schedule())
    s = Solver(m, Options())
    st = State(m.u0.copy(), m.status0.copy())
    t0 = time.perf_counter()
    its = 0
    for dt in m.schedule[:8]:
        st, i = s.solve_timestep(st, dt)
        its += i
    wall = time.perf_counter() - t0
    log_fn(f"oracle sample: n={m.n} iterations={its} wall={wall:.1f}s")
    return dict(value=m.n * its / wall, unit="cell-updates/s", cores=1, kind="oracle",
                sample=f"config-2 recipe on a 30x15x10 grid + 45 fractures (n={m.n} cells), "
                       f"first 8 timesteps, full Newton + SuperLU, FP64, 1 thread: "
                       f"{its} iterations in {wall:.1f} s",
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
    import multiprocessing as mp
    with mp.get_context("fork").Pool(min(procs, len(ids))) as pool:
        return pool.map(fn, ids)


def run_c4(members, steps):
    """Batched ensemble: `members` config-4 models advanced together, one
    Newton iteration of every live member per batched call, each member
    through its own schedule; then the same members one after another."""
    import numpy as np
    import torch
    import paper_2008_01539_amd as P
    log(f"generating {members} ensemble members")
    models = _pool_models(_member, list(range(members)))
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


def run_c5(seconds, pool, budget_gib, rate=50.0):
    """Serving: Poisson timestep requests at `rate`/s over a pool of
    config-1, -2 and -3 sessions (50/40/10 % of requests); sessions are
    admitted up to the HBM budget before the clock starts, the rest on
    demand (evicting idle ones)."""
    import numpy as np
    import paper_2008_01539_amd as P
    from paper_2008_01539_amd.serve import GpuExecutor, Server, SessionSpec
    n1, n2, n3 = pool
    log(f"generating sessions {n1}/{n2}/{n3}")
    ids = [(1, k) for k in range(n1)] + [(2, k) for k in range(n2)] + [(3, k) for k in range(n3)]
    models = _pool_models(_c5_session, ids)
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


def run_c3(steps, warmup):
    import numpy as np
    import paper_2008_01539_amd as P
    from fimgen import make_c3
    log("building config 3")
    model = make_c3()
    log(f"n={model.n}")
    opts = P.Options(precision=P.MIXED)
    loc = run_gpu(model, opts, P.LOCAL, steps, warmup)
    full = run_gpu(model, opts, P.FULL, steps, warmup)
    res = run_gpu(model, opts, P.RESID, steps, warmup)
    # the whole 784k-cell system: full Newton again with launch events
    full_prof = run_gpu(model, opts, P.FULL, steps, warmup, profile=True)
    roof = roofline_of(full_prof["prof"], model.b)
    copy = copy_bandwidth()
    roof.update(copy_gbps=copy, frac_of_copy=roof["achieved"] / copy)
    return {
        "metric": "active-cell Newton updates/s, local vs full Newton (1 GPU); p50/p99 step latency",
        "value": loc["active"] / loc["wall"], "unit": "active-cell Newton updates/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "higher_is_better": True,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"config 3: black oil (bubble point 3500 psi, Sg/Rs switching), "
                               f"400x200x8 + 5000-fracture DFN ({model.n} cells), 3x3 blocks, "
                               f"timesteps {warmup}..{warmup + steps - 1} of 40, localized Newton, "
                               "FP32 Krylov in FP64 refinement"},
        "local": {k: loc[k] for k in ("iters", "krylov", "wall", "p50", "p99")},
        "full": {"updates_per_s": full["active"] / full["wall"], "wall": full["wall"]},
        "speedup_local_vs_full": full["wall"] / loc["wall"],
        "max_dp_local_vs_full_psi": float(np.abs(full["u"][0] - loc["u"][0]).max() / 6894.757293168),
        "resid": {"iters": res["iters"], "krylov": res["krylov"], "wall": res["wall"],
                  "sum_active": res["active"],
                  "max_dp_vs_full_psi":
                      float(np.abs(full["u"][0] - res["u"][0]).max() / 6894.757293168)},
        "roofline_full_system": roof,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5"])
    ap.add_argument("--localize-fractures", action="store_true",
                    help="fracture cells not always active (only perforated cells are); "
                         "the default keeps them active as in the paper's runs")
    ap.add_argument("--members", type=int, default=256)
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--pool", default="256,64,16",
                    help="serving: config-1,2,3 session counts")
    ap.add_argument("--steps", type=int, default=18)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-full", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the run, copy MIB MiB device to device once (a plain copy "
                         "kernel of known size for scaling memory counters)")
    ap.add_argument("--profile", type=int, default=1,
                    help="record per-kernel hipEvents during the timed local run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(the multi-GPU design is documented, not built)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    from fimgen import PSI, make_c2
    import paper_2008_01539_amd as P
    if args.workload == "c4":
        print(json.dumps(run_c4(args.members, max(1, args.steps))), flush=True)
        return
    if args.workload == "c5":
        pool = tuple(int(v) for v in args.pool.split(","))
        print(json.dumps(run_c5(args.serve_seconds, pool, args.budget_gib)), flush=True)
        return
    if args.workload == "c3":
        print(json.dumps(run_c3(args.steps, args.warmup)), flush=True)
        return

    log("building the config-2 model")
    model = make_c2()
    if args.localize_fractures:
        aa = np.zeros_like(model.always_active)
        aa[np.asarray(model.perf_cell, dtype=np.int64)] = 1
        model.always_active = aa
    log(f"n={model.n} connections={model.nc}")
    opts = P.Options(precision=P.MIXED)
    if args.localize_fractures:
        # the active set has to grow along whole fractures, m layers per
        # expanding iteration
        opts.max_newton = 400
    log(f"localized Newton: warmup {args.warmup}, timed {args.steps} steps")
    loc = run_gpu(model, opts, P.LOCAL, args.steps, args.warmup)
    log(f"local: {loc['iters']} iterations, wall {loc['wall']:.3f}s, "
        f"krylov {loc['krylov']}")
    prof_run = None
    if args.profile:
        # the same timed region again with hipEvents around every launch
        # (the events add host work, so the headline value comes from the
        # run above)
        prof_run = run_gpu(model, opts, P.LOCAL, args.steps, args.warmup, profile=True)
        log(f"local (events): wall {prof_run['wall']:.3f}s")
    full = None
    full_prof = None
    dd = None
    res = None
    if not args.no_full:
        log("full Newton on the same steps")
        full = run_gpu(model, opts, P.FULL, args.steps, args.warmup)
        log(f"full: {full['iters']} iterations, wall {full['wall']:.3f}s, "
            f"krylov {full['krylov']}")
        if args.profile:
            full_prof = run_gpu(model, opts, P.FULL, args.steps, args.warmup, profile=True)
        log("Algorithm 2 (adaptive localized DD) on the same steps")
        dd = run_gpu(model, opts, P.DD, args.steps, args.warmup)
        log(f"dd: {dd['iters']} inner iterations, wall {dd['wall']:.3f}s, "
            f"krylov {dd['krylov']}")
        log("residual-based localization (the prior method) on the same steps")
        res = run_gpu(model, opts, P.RESID, args.steps, args.warmup)
        log(f"resid: {res['iters']} iterations, wall {res['wall']:.3f}s, "
            f"krylov {res['krylov']}")
    value = loc["active"] / loc["wall"]
    out = {
        "metric": "active-cell Newton updates/s, local vs full Newton (1 GPU); "
                  "p50/p99 step latency",
        "value": value,
        "unit": "active-cell Newton updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": loc["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "config 2: water/dead-oil, 200x100x10 grid + seeded 2000-fracture "
                        "DFN + 10-stage horizontal well (258096 cells, 722225 connections), "
                        "20-step schedule to 71.6 d; localized Newton (Algorithm 1, "
                        "eps_p 0.3 psi, m 2); FP64 assembly/update, FP32 BiCGStab "
                        "(block-Jacobi scaling + fracture-block inverses) inside FP64 "
                        "refinement",
            "n_cells": model.n,
            "fractures_always_active": not args.localize_fractures,
            "krylov_dtype": "f32",
            "parallelism": "1 GPU",
        },
        "local": {"iterations": loc["iters"], "sum_active": loc["active"],
                  "avg_ma": loc["active"] / model.n / loc["iters"],
                  "krylov_iters": loc["krylov"], "wall_s": loc["wall"],
                  "newton_step_ms_p50": loc["p50"], "newton_step_ms_p99": loc["p99"],
                  "timestep_ms_p50": loc["step_p50"], "timestep_ms_p99": loc["step_p99"]},
    }
    if full is not None:
        dp = float(np.abs(full["u"][0] - loc["u"][0]).max())
        out["full"] = {"iterations": full["iters"], "updates_per_s": full["active"] / full["wall"],
                       "krylov_iters": full["krylov"], "wall_s": full["wall"],
                       "newton_step_ms_p50": full["p50"], "newton_step_ms_p99": full["p99"]}
        out["speedup_local_vs_full"] = full["wall"] / loc["wall"]
        out["max_dp_local_vs_full_psi"] = dp / PSI
    if dd is not None:
        out["dd"] = {"inner_iterations": dd["iters"], "sum_active": dd["active"],
                     "updates_per_s": dd["active"] / dd["wall"], "krylov_iters": dd["krylov"],
                     "wall_s": dd["wall"], "newton_step_ms_p50": dd["p50"],
                     "newton_step_ms_p99": dd["p99"],
                     "speedup_vs_full": full["wall"] / dd["wall"],
                     "max_dp_vs_full_psi": float(np.abs(full["u"][0] - dd["u"][0]).max()) / PSI}
    if res is not None:
        out["resid"] = {"iterations": res["iters"], "sum_active": res["active"],
                        "avg_ma": res["active"] / model.n / res["iters"],
                        "updates_per_s": res["active"] / res["wall"],
                        "krylov_iters": res["krylov"], "wall_s": res["wall"],
                        "newton_step_ms_p50": res["p50"], "newton_step_ms_p99": res["p99"],
                        "speedup_vs_full": full["wall"] / res["wall"],
                        "local_speedup_vs_resid": res["wall"] / loc["wall"],
                        "max_dp_vs_full_psi":
                            float(np.abs(full["u"][0] - res["u"][0]).max()) / PSI}
    # roofline of the dominant matrix kernel (local run, events on its stream)
    prof = prof_run["prof"] if prof_run else None
    if prof:
        copy = copy_bandwidth()
        roof = roofline_of(prof, model.b)
        per_row = measured_traffic_per_row().get(roof["kernel"])
        out["roofline"] = {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac")}
        # counter-measured bytes per launch (FETCH_SIZE + WRITE_SIZE scaled by a
        # plain copy, per row, times this run's rows per launch); None once the
        # kernels changed since the counters were taken
        out["roofline"]["traffic"] = per_row * roof["rows_per_launch"] if per_row else None
        out["roofline"].update({k: roof[k] for k in ("kernel", "avg_launch_us",
                                                     "bytes_per_launch", "rows_per_launch")})
        out["roofline"].update(copy_gbps=copy, frac_of_copy=roof["achieved"] / copy,
                               profiled_wall_s=prof_run["wall"])
        out["kernel_profile_local"] = prof
    if full_prof is not None:
        out["roofline_full_newton"] = roofline_of(full_prof["prof"], model.b)
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
        out["cpu_baseline"] = cpu_baseline(log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
