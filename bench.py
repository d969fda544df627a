#!/usr/bin/env python3
"""Benchmark: multigrid-preconditioned BiCGSTAB pressure solve on one MI355X.

A step is one whole PPE solve (RHS assembly, pinned MG-BiCGSTAB to the
tolerance, gauge) of the configured workload with its inputs resident in
HBM.  Default workload: 512^3 tanh-stretched grid (ratio 1.05) around a
cambered zero-thickness plate (40k triangles), uniform-noise RHS, mixed
precision (FP32 V-cycle and inner BiCGSTAB with BF16 coarse right-hand
sides inside FP64 iterative refinement) to 1e-8 relative residual; the plain
FP64 solve of the same system is timed beside it.

Prints one JSON line.  Only one GPU is used: --gpus above 1 is refused.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MG-BiCGSTAB pressure solve Mpts/s to 1e-8 resid, % HBM peak; serve p50/p99"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_problem(cfg):
    from paper_2605_04335_amd import workloads as W
    if cfg == "c3":
        p = W.membrane_case(512)
        p.tol = 1e-8
        return p, "membrane plate 512^3 tanh-stretched, 40k triangles, noise RHS, mixed MG-BiCGSTAB to 1e-8"
    if cfg == "c2":
        p = W.sphere_ellipsoid_case(256)
        p.tol = 1e-8
        p.mixed = True
        return p, "sphere+ellipsoid 256^3 tanh-stretched, noise RHS, mixed MG-BiCGSTAB to 1e-8"
    if cfg == "c4":
        p = W.spheres_case(1024)
        p.mixed = True
        return p, "20 spheres 1024^3 uniform, Gaussian-bump RHS, mixed MG-BiCGSTAB to 1e-8"
    if cfg == "c1":
        p = W.sphere_case(32)
        p.tol = 1e-8
        p.mixed = True
        return p, "sphere 32^3 uniform, manufactured RHS, mixed MG-BiCGSTAB to 1e-8"
    raise SystemExit("unknown config " + cfg)


def sweep_source_digest():
    """Digest of the level-0 half-sweep kernel's source (its column helpers
    and the kernel itself): HBM counters taken for another version of the
    kernel do not describe this one."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_2605_04335_amd", "csrc", "kernels.hpp")).read()
    a = src.index("struct Col0 {")
    b = src.index("// First level-0 half-sweep of a V-cycle, from a zero iterate")
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def solver_source_digest():
    """Digest of every kernel and host source of the solve: whole-solve HBM
    counters describe only the version they were taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hpp", "setup.hpp", "solver.hip", "common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2605_04335_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_solve_traffic(workload_key):
    """HBM bytes of one whole mixed solve (FETCH_SIZE + WRITE_SIZE of every
    solve kernel, scaled by a plain copy) from the committed rocprofv3
    summary, or None when missing or taken on other sources."""
    path = os.path.join(ROOT, "profiles", "mg_bicgstab_%s_solve_traffic.md" % workload_key)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_digest") != solver_source_digest():
        return None
    try:
        return float(vals["traffic_bytes_per_solve"])
    except (KeyError, ValueError):
        return None


def measured_traffic(workload_key):
    """HBM bytes per launch of k0_sweep from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy), or None when
    the summary is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "k0_sweep_%s_traffic.md" % workload_key)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_digest") != sweep_source_digest():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def serving_bench(P, rates, nreq, seed=5, slots=16, budget=64 << 30):
    """Poisson arrivals of mixed-precision solve requests (grid edge
    log-uniform in [64, 384], cube or 2:1:1, 1-4 bodies, tol 1e-8) into the
    continuous-batching server; latency = done - submit on the server clock.
    Every rate gets requests of its own (no set-up is reused from the cache),
    and the latency is split into queueing (submit to admission), set-up
    (classification, ghost rows, hierarchy), solve (RHS upload to solution on
    the host) and the rest (release of the request's memory)."""
    from paper_2605_04335_amd import workloads as W

    def make(q0, n):
        rng = np.random.default_rng(seed + q0)
        reqs = []
        for q in range(n):
            p = W.serving_request(rng)
            p.f = W.noise_rhs(p.npts, seed + 1000 + q0 + q)
            reqs.append(p)
        return reqs

    # one warm-up request outside the measurement (first-use costs of the runtime)
    srv = P.Server(hbm_budget=budget, max_slots=slots)
    w = make(10 ** 6, 1)[0]
    t = srv.submit(w.xf, w.yf, w.zf, w.bodies, w.f, precision="mixed", tol=1e-8)
    while srv.poll(t, want_x=False)[0] == P.IBM_EAGAIN:
        time.sleep(0.001)
    out = []
    for rate in rates:
        reqs = make(10000 * int(rate), nreq)  # the same requests for a rate in every run
        arr = np.cumsum(np.random.default_rng(seed + int(rate)).exponential(1.0 / rate, nreq))
        pending, done = {}, []
        t0 = time.perf_counter()
        q = 0
        while q < nreq or pending:
            now = time.perf_counter() - t0
            while q < nreq and arr[q] <= now:
                p = reqs[q]
                pending[srv.submit(p.xf, p.yf, p.zf, p.bodies, p.f, precision="mixed", tol=1e-8)] = p.npts
                q += 1
            for tk in list(pending):
                rc, state, _, st, tm = srv.poll(tk, want_x=False)
                if rc == P.IBM_EAGAIN:
                    continue
                done.append((tm.submit_ms, tm.done_ms, pending.pop(tk), rc, st.rel_residual, tm.admit_ms,
                             tm.setup_ms, tm.solve_ms, tm.cache_hit))
            time.sleep(0.0005)
        del reqs
        lat = np.array([d[1] - d[0] for d in done])
        span_s = (max(d[1] for d in done) - min(d[0] for d in done)) / 1e3
        pts = sum(d[2] for d in done)
        ok = sum(1 for d in done if d[3] == 0 and d[4] <= 1e-8)
        queue = np.array([d[5] - d[0] for d in done])
        setup = np.array([d[6] for d in done])
        solve = np.array([d[7] for d in done])
        rest = lat - queue - setup - solve
        out.append({"rate_req_s": rate, "requests": nreq, "ok": ok, "p50_ms": round(float(np.percentile(lat, 50)), 2),
                    "p99_ms": round(float(np.percentile(lat, 99)), 2), "solves_s": round(nreq / span_s, 2),
                    "Mpts_s": round(pts / span_s / 1e6, 1), "cache_hits": int(sum(d[8] for d in done)),
                    "mean_ms": {"queue": round(float(queue.mean()), 2), "setup": round(float(setup.mean()), 2),
                                "solve": round(float(solve.mean()), 2), "release": round(float(rest.mean()), 2)}})
        log("serve rate %g req/s: p50 %.1f ms p99 %.1f ms, %.1f solves/s, %.0f Mpts/s, %d/%d ok; mean queue %.1f "
            "set-up %.1f solve %.1f release %.1f ms" %
            (rate, out[-1]["p50_ms"], out[-1]["p99_ms"], out[-1]["solves_s"], out[-1]["Mpts_s"], ok, nreq,
             queue.mean(), setup.mean(), solve.mean(), rest.mean()))
    srv.close()
    return {"workload": "Poisson arrivals, edge log-uniform [64, 384], cube or 2:1:1, 1-4 bodies (spheres, "
                        "ellipsoids, plates), noise RHS, mixed MG-BiCGSTAB to 1e-8; distinct requests per rate",
            "max_slots": slots, "hbm_budget_GB": budget >> 30, "sweep": out}


def moving_bench(P, n=512, steps=3):
    """Moving-body time steps (flapping plate + heaving sphere, stretched
    grid, mixed MG-BiCGSTAB to 1e-8): per step re-classification, ghost
    rows, context update, fresh-cell fill, the solve from the previous
    pressure and the nodal pressure forces, each timed with a device
    synchronisation around it."""
    import torch
    from paper_2605_04335_amd import workloads as W

    def now():
        torch.cuda.synchronize()
        return time.perf_counter()

    p = W.flapping_case(n, 0)
    fl, st, sol, _ = P.setup(p.xf, p.yf, p.zf, p.bodies, precision="mixed", tol=1e-8, max_iter=100)
    f = torch.from_numpy(p.f).cuda()
    x, s = sol.solve(f)
    rows = []
    for k in range(1, steps + 1):
        q = W.flapping_case(n, k)
        t0 = now()
        fq, cq = P.classify(q.xf, q.yf, q.zf, q.bodies)
        t1 = now()
        sq = P.build_ghost_stencils(q.xf, q.yf, q.zf, q.bodies, fq)
        t2 = now()
        sol.update(fq, sq)
        t3 = now()
        x0 = x[: q.npts].clone()
        nf = P.fill_fresh(q.xf, q.yf, q.zf, fl, fq, x0)
        t4 = now()
        x, s = sol.solve_from(f, x0)
        t5 = now()
        F, dp, lost = P.surface_forces(q.xf, q.yf, q.zf, q.bodies, fq, x)
        t6 = now()
        rows.append({"classify_ms": (t1 - t0) * 1e3, "stencils_ms": (t2 - t1) * 1e3, "update_ms": (t3 - t2) * 1e3,
                     "fresh_ms": (t4 - t3) * 1e3, "solve_ms": (t5 - t4) * 1e3, "forces_ms": (t6 - t5) * 1e3,
                     "iterations": s.iterations,
                     "fresh_cells": nf, "ghosts": cq["n_ghost"], "membrane_ghosts": cq["n_mghost"],
                     "ok": int(s.status == 0 and s.rel_residual <= 1e-8)})
        fl = fq
        log("moving step %d: classify %.1f stencils %.1f update %.1f fresh %.1f solve %.1f forces %.1f ms (%d its)" %
            (k, *(rows[-1][c] for c in ("classify_ms", "stencils_ms", "update_ms", "fresh_ms", "solve_ms",
                                        "forces_ms")), s.iterations))
    del sol
    torch.cuda.empty_cache()
    mean = {c: round(float(np.mean([r[c] for r in rows])), 2)
            for c in ("classify_ms", "stencils_ms", "update_ms", "fresh_ms", "solve_ms", "forces_ms", "iterations")}
    resetup = mean["classify_ms"] + mean["stencils_ms"] + mean["update_ms"] + mean["fresh_ms"]
    return {"workload": "flapping plate (14.4k triangles) + heaving sphere, %d^3 tanh-stretched, noise RHS, "
                        "mixed MG-BiCGSTAB to 1e-8 from the previous step's pressure" % n,
            "steps": steps, "mean": mean, "resetup_ms": round(resetup, 2),
            "ms_per_step": round(resetup + mean["solve_ms"] + mean["forces_ms"], 2),
            "ok": sum(r["ok"] for r in rows)}


def max_diag(xf, yf, zf):
    """Largest sum of the 7-point coefficients of a cell (zero-flux walls)."""
    tot = 0.0
    for f in (xf, yf, zf):
        c = 0.5 * (f[1:] + f[:-1])
        w = np.diff(f)
        d = np.zeros(len(w))
        d[:-1] += 1.0 / (w[:-1] * np.diff(c))
        d[1:] += 1.0 / (w[1:] * np.diff(c))
        tot += d.max()
    return float(tot)


def ad_bench(P, n=512, components=3):
    """Advection-diffusion step of the momentum equations (SRJ, Dirichlet
    ghost rows) on the moving-body geometry: beta = nu dt / 2 at Re 1000 and
    CFL 0.5 on the finest cell, one solve per velocity component to 1e-10."""
    import torch
    from paper_2605_04335_amd import workloads as W
    p = W.flapping_case(n, 0, rhs=False)
    flags, _ = P.classify(p.xf, p.yf, p.zf, p.bodies)
    st = P.build_ghost_stencils(p.xf, p.yf, p.zf, p.bodies, flags, bc="dirichlet")
    h = min(np.diff(p.xf).min(), np.diff(p.yf).min(), np.diff(p.zf).min())
    beta = 0.5 * 1e-3 * 0.5 * h
    sol = P.AdSolver(p.xf, p.yf, p.zf, flags, st, beta, tol=1e-10, sweeps=8)
    ng, nm, _ = st.info()
    rows = []
    for c in range(components + 1):
        f = torch.from_numpy(W.noise_rhs(p.npts, 70 + c)).cuda()
        g = torch.from_numpy(np.random.default_rng(80 + c).uniform(-0.5, 0.5, ng + nm)).cuda()
        u, s = sol.solve(f, g)
        if c:  # the first solve is a warm-up
            rows.append((s.solve_ms, s.cycles, s.sweeps, s.status, s.rel_residual))
    del sol
    torch.cuda.empty_cache()
    ms = float(np.mean([r[0] for r in rows]))
    sweeps = float(np.mean([r[2] for r in rows]))
    cycles = float(np.mean([r[1] for r in rows]))
    # a sweep reads the iterate, the right-hand side and the flags and writes
    # the new iterate (FP64): 25 bytes per cell; the residual before the first
    # and after every cycle reads the same without writing: 17 bytes per cell
    log("ad: %.1f ms per component, %.0f cycles, %.0f sweeps" % (ms, cycles, sweeps))
    return {"workload": "u - beta L u = f per velocity component, flapping plate + heaving sphere, %d^3 "
                        "tanh-stretched, Dirichlet ghost rows, beta = nu dt / 2 (Re 1000, CFL 0.5), SRJ to 1e-10" % n,
            "ms_per_component": round(ms, 2), "cycles": cycles, "sweeps": sweeps,
            "beta": beta, "beta_times_max_diag": round(beta * max_diag(p.xf, p.yf, p.zf), 3),
            "GB_s": round(p.npts * (25.0 * sweeps + 17.0 * (cycles + 1)) / (ms * 1e-3) / 1e9, 1),
            "ok": sum(1 for r in rows if r[3] == 0 and r[4] <= 1e-10), "components": components}


def cpu_baseline(cfg, budget_s):
    """The FP64 oracle on a bounded sample of the same workload recipe."""
    import oracle
    from paper_2605_04335_amd import workloads as W
    n = {"c3": 256, "c2": 128, "c4": 256, "c1": 32}[cfg]
    if cfg == "c3":
        p = W.membrane_case(n)
    elif cfg == "c2":
        p = W.sphere_ellipsoid_case(n)
    elif cfg == "c4":
        p = W.spheres_case(n)
    else:
        p = W.sphere_case(n)
    t0 = time.time()
    S = oracle.setup(p.xf, p.yf, p.zf, p.bodies)
    t_setup = time.time() - t0
    b = oracle.assemble_rhs(S.xf, S.yf, S.zf, S.flags, S.st, p.f)
    t0 = time.time()
    x, info = oracle.solve(S.xf, S.yf, S.zf, S.flags, S.st, b, tol=1e-8, maxit=200)
    t = time.time() - t0
    N = p.npts
    return {"value": N / t / 1e6, "unit": "Mpts/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": "same recipe at %d^3 (%d points): FP64 oracle MG-BiCGSTAB to 1e-8, %d iterations, %.1f s solve"
                      " (+%.1f s setup)" % (n, N, info.iters, t, t_setup)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison solve")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-loop measurement")
    ap.add_argument("--no-moving", action="store_true", help="skip the moving-body time-step measurement")
    ap.add_argument("--no-ad", action="store_true", help="skip the advection-diffusion step measurement")
    ap.add_argument("--serve-rates", default="5,20,80,200", help="request arrival rates (req/s) of the serving sweep")
    ap.add_argument("--serve-requests", type=int, default=48, help="requests per arrival rate")
    ap.add_argument("--serve-slots", type=int, default=16, help="concurrently active solves in the server")
    ap.add_argument("--serve-small-budget-gb", type=int, default=8,
                    help="HBM budget (GB) of a second run at the highest rate, where admission binds; 0: skip")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="finish with 3 plain device copies of 1 GiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the PPE solve runs on a single MI355X; "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import torch
    import paper_2605_04335_amd as P

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    p, desc = make_problem(args.config)
    nx, ny, nz = p.shape
    N = p.npts
    log("workload", desc)
    t0 = time.time()
    flags, cst = P.classify(p.xf, p.yf, p.zf, p.bodies)
    st = P.build_ghost_stencils(p.xf, p.yf, p.zf, p.bodies, flags)
    ng, nm, nfb = st.info()
    solm = P.Solver(p.xf, p.yf, p.zf, flags, st, precision=P.PREC_MIXED, tol=p.tol, max_iter=60)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    log("setup %.2f s: ghosts %d, membrane ghosts %d, fallback %d" % (setup_s, ng, nm, nfb))
    f = torch.from_numpy(p.f).to(dev)

    for _ in range(args.warmup):
        x, stm = solm.solve(f)
        log("warmup mixed: its %d outer %d rel %.2e %.1f ms" % (stm.iterations, stm.outer_steps, stm.rel_residual,
                                                                stm.solve_ms))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev_ms = []
    for k in range(args.steps):
        x, stm = solm.solve(f)
        dev_ms.append(stm.solve_ms)
        log("step %d: its %d outer %d rel %.2e %.1f ms" % (k, stm.iterations, stm.outer_steps, stm.rel_residual,
                                                           stm.solve_ms))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    value = N / (ms_per_step / 1e3) / 1e6

    # dominant kernel, timed per launch with HIP events on the library's stream
    roof = None
    kern_ms = {}
    for kid, name in ((0, "k0_sweep"), (1, "k0_apply"), (2, "k_xr_update")):
        P.lib().poisson_kernel_timing(solm.h, kid, 1, None, None)
        solm.solve(f)
        tot = P.ctypes.c_double()
        cnt = P.ctypes.c_int64()
        P.lib().poisson_kernel_timing(solm.h, -1, 1, P.ctypes.byref(tot), P.ctypes.byref(cnt))
        kern_ms[name] = (tot.value, cnt.value)
    tot, cnt = kern_ms["k0_sweep"]
    if cnt:
        avg_ms = tot / cnt
        T = 4  # FP32 inner vectors
        # red/black half-sweep over half of the cells: read the other colour's values, this colour's RHS and
        # flag byte, write this colour's values
        bytes_launch = (1.5 * T + 0.5) * N
        ach = bytes_launch / (avg_ms * 1e-3) / 1e9
        tr = measured_traffic({"c3": "membrane512", "c2": "spheroids256", "c4": "spheres1024",
                               "c1": "sphere32"}[args.config])
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": (int(tr) if tr else None), "kernel": "k0_sweep<float>",
                "avg_launch_ms": round(avg_ms, 4), "launches_per_solve": cnt,
                "algorithmic_bytes_per_launch": int(bytes_launch)}

    out = {"metric": METRIC, "value": round(value, 2), "unit": "Mpts/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32+bf16", "data": "synthetic",
           "config": {"workload": desc, "grid": [nx, ny, nz], "points": N, "tol": p.tol,
                      "precision": "mixed (FP32/BF16 V-cycle and inner BiCGSTAB, FP64 refinement)",
                      "iterations": stm.iterations, "outer_steps": stm.outer_steps,
                      "rel_residual": stm.rel_residual, "device_ms_per_solve": round(float(np.median(dev_ms)), 3),
                      "setup_s": round(setup_s, 2), "ghosts": ng, "membrane_ghosts": nm, "fallback_rows": nfb},
           "roofline": roof,
           "kernel_ms": {k: {"total_ms": round(v[0], 3), "launches": v[1]} for k, v in kern_ms.items()}}
    # whole solve: measured HBM bytes of every solve kernel over the solve time
    ts = measured_solve_traffic({"c3": "membrane512", "c2": "spheroids256", "c4": "spheres1024",
                                 "c1": "sphere32"}[args.config])
    if ts:
        gbs = ts / (ms_per_step * 1e-3) / 1e9
        out["solve_hbm"] = {"bytes_per_solve": int(ts), "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}
    # whole solve against the compulsory-traffic model of the mixed form: per
    # inner iteration 86 B/pt of FP32 Krylov kernels and two FP32/BF16
    # V-cycles of 75 B/pt; per refinement step an FP64 residual and update of
    # 41 B/pt
    model = (236.0 * stm.iterations + 41.0 * stm.outer_steps) * N
    gbm = model / (ms_per_step * 1e-3) / 1e9
    out["solve_model"] = {"bytes_per_solve": int(model), "achieved": round(gbm, 1), "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": round(gbm / HBM_PEAK_GBS, 4)}

    if not args.no_fp64:
        del solm
        torch.cuda.empty_cache()
        sol64 = P.Solver(p.xf, p.yf, p.zf, flags, st, precision=P.PREC_FP64, tol=p.tol, max_iter=100)
        x64, s64 = sol64.solve(f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = max(1, min(3, args.steps))
        for _ in range(reps):
            x64, s64 = sol64.solve(f)
        torch.cuda.synchronize()
        ms64 = (time.perf_counter() - t0) / reps * 1e3
        err = float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))
        out["config"]["fp64"] = {"ms_per_solve": round(ms64, 3), "Mpts_s": round(N / ms64 * 1e3 / 1e6, 2),
                                 "iterations": s64.iterations, "rel_residual": s64.rel_residual}
        out["config"]["mixed_speedup_vs_fp64"] = round(ms64 / ms_per_step, 3)
        out["config"]["mixed_rel_error_vs_fp64"] = err
        log("fp64: %.1f ms/solve, %d its; mixed speed-up %.2fx, rel error %.2e" % (ms64, s64.iterations,
                                                                                   ms64 / ms_per_step, err))
    if not args.no_serve:
        out["serving"] = serving_bench(P, [float(r) for r in args.serve_rates.split(",")], args.serve_requests,
                                       slots=args.serve_slots)
        if args.serve_small_budget_gb > 0:
            # the highest rate's requests again under a budget small enough
            # that admission waits for memory
            rate = max(float(r) for r in args.serve_rates.split(","))
            out["serving_small_budget"] = serving_bench(P, [rate], args.serve_requests, slots=args.serve_slots,
                                                        budget=args.serve_small_budget_gb << 30)
    if not args.no_moving:
        out["moving"] = moving_bench(P)
    if not args.no_ad:
        out["advection_diffusion"] = ad_bench(P)
    if args.copy_calibration:
        import torch as _t
        nbytes = 1 << 30
        src = _t.ones(nbytes, dtype=_t.uint8, device=dev)
        dst = _t.empty_like(src)
        _t.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        _t.cuda.synchronize()
        log("copy calibration: 3 device-to-device copies of %d bytes" % nbytes)
        del src, dst
    if rank == 0 and not args.no_cpu:
        try:
            out["cpu_baseline"] = cpu_baseline(args.config, 30)
        except Exception as e:  # reported, never fatal
            out["cpu_baseline"] = {"value": None, "error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
