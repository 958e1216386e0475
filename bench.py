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


def algorithmic_bytes(kernel, rec, b, kbytes):
    """Bytes a kernel must move per the work it did (one active row = one
    unit): every array entry it reads or writes once, neighbour gathers
    counted once (cache reuse), padding of the sliced-ELL matrix excluded.
    rec: profile record with rows and nnzb (blocks incl. diagonal)."""
    rows, nnzb = rec["rows"], rec["nnzb"]
    off = max(nnzb - rows, 0.0)
    if kernel == "bicg_spmv_p":
        # col + block per off-diagonal; s, t, p, v, x, rh read; x, r, p, v written
        return off * (4 + kbytes * b * b) + rows * (10 * b * kbytes)
    if kernel == "bicg_spmv_s":   # col + block; r, v, rh read; s, t written
        return off * (4 + kbytes * b * b) + rows * (5 * b * kbytes)
    if kernel == "assemble":
        # per row: l2g 4, state 8b, status 1, pv 8, depth 8, flags 1, old
        # masses 8b, adjacency pointers 8, residual 8b written; per
        # connection of an active pair: neighbour id 4, T 8, g2l 4; per
        # block: 8 b^2 values + 4 col written
        return rows * (30 + 24 * b) + off * 16 + nnzb * (8 * b * b + 4)
    raise KeyError(kernel)


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
    layout) on a 30x15x10 grid, its first 3 timesteps, single thread."""
    os.environ["OMP_NUM_THREADS"] = "1"
    from fimgen.configs import _two_phase_model, c1_schedule
    from fimgen.model import FLUID_DEADOIL
    from oracle.newton import Options, Solver, State
    m = _two_phase_model("c2_sample", 2, 30, 15, 10, 45, FLUID_DEADOIL, c1_schedule())
    s = Solver(m, Options())
    st = State(m.u0.copy(), m.status0.copy())
    t0 = time.perf_counter()
    its = 0
    for dt in m.schedule[:3]:
        st, i = s.solve_timestep(st, dt)
        its += i
    wall = time.perf_counter() - t0
    log_fn(f"oracle sample: n={m.n} iterations={its} wall={wall:.1f}s")
    return dict(value=m.n * its / wall, unit="cell-updates/s", cores=1, kind="oracle",
                sample=f"config-2 recipe on a 30x15x10 grid + 45 fractures (n={m.n} cells), "
                       f"first 3 timesteps, full Newton + SuperLU, FP64, 1 thread: "
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=18)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-full", action="store_true")
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

    log("building the config-2 model")
    model = make_c2()
    log(f"n={model.n} connections={model.nc}")
    opts = P.Options(precision=P.MIXED)
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
    if not args.no_full:
        log("full Newton on the same steps")
        full = run_gpu(model, opts, P.FULL, args.steps, args.warmup)
        log(f"full: {full['iters']} iterations, wall {full['wall']:.3f}s, "
            f"krylov {full['krylov']}")
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
                        "eps_p 0.3 psi, m 2); FP64 assembly/update, FP32 BiCGStab with "
                        "block-Jacobi inside FP64 refinement",
            "n_cells": model.n,
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
    # roofline of the dominant matrix kernel (local run, events on its stream)
    prof = prof_run["prof"] if prof_run else None
    if prof:
        cands = {k: v for k, v in prof.items()
                 if k in ("assemble", "bicg_spmv_p", "bicg_spmv_s") and v["launches"]}
        dom = max(cands, key=lambda k: cands[k]["total_ms"])
        rec = cands[dom]
        avg_s = rec["total_ms"] / rec["launches"] * 1e-3
        byt = algorithmic_bytes(dom, rec, model.b, 4) / rec["launches"]
        ach = byt / avg_s / 1e9
        out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": ach,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                           "traffic": None, "avg_launch_us": avg_s * 1e6,
                           "bytes_per_launch": byt,
                           "rows_per_launch": rec["rows"] / rec["launches"]}
        out["kernel_profile_local"] = prof
        out["roofline"]["profiled_wall_s"] = prof_run["wall"]
    if not args.no_cpu:
        log("oracle CPU baseline")
        out["cpu_baseline"] = cpu_baseline(log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
