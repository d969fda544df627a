#!/usr/bin/env python3
"""Benchmark: multigrid-preconditioned BiCGSTAB pressure solve on one MI355X.

A step is one whole PPE solve (RHS assembly, pinned MG-BiCGSTAB to a 1e-8
relative residual, gauge) of the configured workload with its inputs
resident in HBM.  The headline is the paper's precision, FP64 throughout
(Sec. 3 states every figure in double precision).  Default workload: 512^3
tanh-stretched grid (ratio 1.05) around a cambered zero-thickness plate (40k
triangles) with ghost unknowns on both sides, uniform-noise RHS.

Beside the headline: the mixed form (FP32 V-cycle and inner BiCGSTAB with
BF16 coarse right-hand sides inside FP64 iterative refinement) on the same
system, the error of both against a stored sample of the FP64 oracle's
solution and the speed-up at equal accuracy; the 1024^3, 20-sphere case in
both forms; the device's streaming ceiling; the serving sweep; the
moving-body and advection-diffusion steps; and the oracle timed on the host.

Prints one JSON line.  Only one GPU is used: --gpus above 1 is refused.
"""
from __future__ import annotations

import argparse
import faulthandler
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
KEYS = {"c3": "membrane512", "c2": "spheroids256", "c4": "spheres1024", "c1": "sphere32"}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_problem(cfg):
    from paper_2605_04335_amd import workloads as W
    if cfg == "c3":
        p = W.membrane_case(512)
        desc = "membrane plate 512^3 tanh-stretched, 40k triangles, noise RHS, MG-BiCGSTAB to 1e-8"
    elif cfg == "c2":
        p = W.sphere_ellipsoid_case(256)
        desc = "sphere+ellipsoid 256^3 tanh-stretched, noise RHS, MG-BiCGSTAB to 1e-8"
    elif cfg == "c4":
        p = W.spheres_case(1024)
        desc = "20 spheres 1024^3 uniform, Gaussian-bump RHS, MG-BiCGSTAB to 1e-8"
    elif cfg == "c1":
        p = W.sphere_case(32)
        desc = "sphere 32^3 uniform, manufactured RHS, MG-BiCGSTAB to 1e-8"
    else:
        raise SystemExit("unknown config " + cfg)
    p.tol = 1e-8
    return p, desc


def oracle_sample(cfg):
    """Stored sample of the FP64 oracle's gauged solution of the workload
    (tests/golden, written by a script that runs only the oracle), or None."""
    path = os.path.join(ROOT, "tests", "golden", "c3_membrane512_oracle_sample.npz")
    if cfg != "c3" or not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def sampled_error(x, G):
    """Relative L2 error of a gauged solution (device tensor, N + n_mghost)
    against the oracle's on the stored sample of cells and membrane ghost
    unknowns."""
    import torch
    N = x.numel() - int(G["n_mghost"])
    idx = np.concatenate([G["cells"], N + G["mghost"]])
    ref = np.concatenate([G["cell_values"], G["mghost_values"]])
    got = x[torch.from_numpy(idx).to(x.device)].cpu().numpy()
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def time_solves(sol, f, reps):
    """Wall milliseconds per solve over reps back-to-back solves (device
    synchronised on both sides), the last solution and its stats."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        x, st = sol.solve(f)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps * 1e3, x, st


def sweep_roofline(P, sol, f, T, N, traffic):
    """Roofline of the level-0 red/black half-sweep (k0_sweep): its launches
    in one solve timed with HIP events on the solve stream.  Algorithmic bytes
    per launch: the other colour's values (T bytes each), this colour's RHS
    and flag byte and its new values, over N/2 cells each: (1.5 T + 0.5) N."""
    sol.kernel_timing(P.KERNEL_SWEEP0)
    sol.solve(f)
    tot, cnt = sol.kernel_timing(-1)
    if not cnt:
        return None
    avg_ms = tot / cnt
    bytes_launch = (1.5 * T + 0.5) * N
    ach = bytes_launch / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": (int(traffic) if traffic else None),
            "kernel": "k0_sweep<%s>" % ("double" if T == 8 else "float"), "avg_launch_ms": round(avg_ms, 4),
            "launches_per_solve": cnt, "algorithmic_bytes_per_launch": int(bytes_launch)}


def hbm_ceiling(P, nbytes=4 << 30, reps=10):
    """Streaming bandwidth of the device over buffers of nbytes each (far
    above the 256 MB Infinity Cache), 16-byte accesses."""
    out = {"buffer_bytes": nbytes}
    for name, kind in (("copy", P.STREAM_COPY), ("read3_write1", P.STREAM_TRIAD), ("read", P.STREAM_READ)):
        gbs, ms, moved = P.hbm_stream(kind, nbytes, reps)
        out[name] = {"GB_s": round(gbs, 1), "ms": round(ms, 4), "bytes_per_pass": int(moved),
                     "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}
        log("stream %s: %.1f GB/s (%.3f ms per pass of %d bytes)" % (name, gbs, ms, moved))
    return out


def sweep_source_digest():
    """Digest of the level-0 half-sweep kernel's source (its column helpers
    and the kernel itself): HBM counters taken for another version of the
    kernel do not describe this one."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_2605_04335_amd", "csrc", "kernels.hpp")).read()
    a = src.index("struct Col0 {")
    b = src.index("// sum of coefficient * other-colour neighbour at slot s of plane k")
    c = src.index("// Level-0 Gauss-Seidel half-sweep of colour c (ordinary mode)")
    d = src.index("// First level-0 half-sweep of a V-cycle, from a zero iterate")
    return hashlib.sha256((src[a:b] + src[c:d]).encode()).hexdigest()[:16]


def solver_source_digest():
    """Digest of every kernel and host source of the solve: whole-solve HBM
    counters describe only the version they were taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hpp", "setup.hpp", "solver.hip", "common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2605_04335_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_solve_traffic(workload_key, prec="f64"):
    """HBM bytes of one whole solve in one form ("f64" or "mixed"):
    FETCH_SIZE + WRITE_SIZE of every solve kernel, scaled by a plain copy,
    from the committed rocprofv3 summary, or None when missing or taken on
    other sources."""
    path = os.path.join(ROOT, "profiles", "mg_bicgstab_%s_%s_solve_traffic.md" % (prec, workload_key))
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


def measured_traffic(workload_key, prec="f64"):
    """HBM bytes per launch of k0_sweep in one precision ("f64" or "f32")
    from the committed rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE,
    scaled by a plain copy), or None when the summary is missing or was taken
    on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "k0_sweep_%s_%s_traffic.md" % (prec, workload_key))
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
    try:  # the server's threads end with it, also when a leg fails
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
            # device occupancy: a request holds the device from admission to
            # completion; the share of the span with at least one admitted
            # request, and the mean number admitted at once
            iv = sorted((d[5], d[1]) for d in done)
            busy, cur0, cur1 = 0.0, None, None
            for a0, a1 in iv:
                if cur1 is None or a0 > cur1:
                    if cur1 is not None:
                        busy += cur1 - cur0
                    cur0, cur1 = a0, a1
                else:
                    cur1 = max(cur1, a1)
            if cur1 is not None:
                busy += cur1 - cur0
            span_ms = span_s * 1e3
            out.append({"rate_req_s": rate, "requests": nreq, "ok": ok, "p50_ms": round(float(np.percentile(lat, 50)), 2),
                        "p99_ms": round(float(np.percentile(lat, 99)), 2), "solves_s": round(nreq / span_s, 2),
                        "Mpts_s": round(pts / span_s / 1e6, 1), "cache_hits": int(sum(d[8] for d in done)),
                        "mean_ms": {"queue": round(float(queue.mean()), 2), "setup": round(float(setup.mean()), 2),
                                    "solve": round(float(solve.mean()), 2), "release": round(float(rest.mean()), 2)},
                        "busy_frac": round(busy / span_ms, 3),
                        "mean_active": round(float(sum(d[1] - d[5] for d in done)) / span_ms, 2),
                        "mean_Mpts_per_request": round(pts / nreq / 1e6, 2)})
            log("serve rate %g req/s: p50 %.1f ms p99 %.1f ms, %.1f solves/s, %.0f Mpts/s, %d/%d ok; mean queue %.1f "
                "set-up %.1f solve %.1f release %.1f ms; busy %.2f, %.2f active" %
                (rate, out[-1]["p50_ms"], out[-1]["p99_ms"], out[-1]["solves_s"], out[-1]["Mpts_s"], ok, nreq,
                 queue.mean(), setup.mean(), solve.mean(), rest.mean(), out[-1]["busy_frac"], out[-1]["mean_active"]))
    finally:
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


def host_cpu():
    """Model name and logical CPU count of the host."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(cfg, p, G, iters=2):
    """The FP64 oracle on the benchmarked system itself, bounded: its set-up
    (classification and ghost rows) and `iters` MG-BiCGSTAB iterations are
    timed, and the solve time to 1e-8 is the time per iteration times the
    oracle's own iteration count to 1e-8 (from the residual history of its
    full solve, stored with the oracle sample).  Without that history (no
    sample for this workload) the whole solve to 1e-8 is run."""
    import oracle
    t0 = time.time()
    S = oracle.setup(p.xf, p.yf, p.zf, p.bodies)
    t_setup = time.time() - t0
    b = oracle.assemble_rhs(S.xf, S.yf, S.zf, S.flags, S.st, p.f)
    model, ncpu = host_cpu()
    N = p.npts
    if G is not None and "hist" in G:
        its = int(np.argmax(G["hist"] <= 1e-8)) + 1
        t0 = time.time()
        x, info = oracle.solve(S.xf, S.yf, S.zf, S.flags, S.st, b, tol=1e-30, maxit=iters)
        per = (time.time() - t0) / iters
        t = per * its
        sample = ("the %s system itself (%d points): oracle set-up %.1f s, then %d FP64 MG-BiCGSTAB iterations "
                  "timed (%.2f s each) and scaled to the oracle's %d iterations to 1e-8" %
                  (cfg, N, t_setup, iters, per, its))
    else:
        t0 = time.time()
        x, info = oracle.solve(S.xf, S.yf, S.zf, S.flags, S.st, b, tol=1e-8, maxit=200)
        t = time.time() - t0
        its = info.iters
        sample = "the %s system itself (%d points): FP64 oracle MG-BiCGSTAB to 1e-8, %d iterations, %.1f s solve " \
                 "(+%.1f s set-up)" % (cfg, N, its, t, t_setup)
    return {"value": round(N / t / 1e6, 3), "unit": "Mpts/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": sample, "host_cpu": model, "nproc": ncpu, "seconds_per_solve": round(t, 2),
            "setup_s": round(t_setup, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision solve and the accuracy ladder")
    ap.add_argument("--no-ladder", action="store_true", help="skip the equal-accuracy tolerance ladder")
    ap.add_argument("--no-c4", action="store_true", help="skip the 1024^3 twenty-sphere leg")
    ap.add_argument("--no-stream", action="store_true", help="skip the streaming-bandwidth ceiling")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-loop measurement")
    ap.add_argument("--no-moving", action="store_true", help="skip the moving-body time-step measurement")
    ap.add_argument("--no-ad", action="store_true", help="skip the advection-diffusion step measurement")
    ap.add_argument("--serve-rates", default="5,10,20,50",
                    help="request arrival rates (req/s) of the serving sweep; 100 and 200 are opt-in: a host "
                         "segmentation fault seen once at 100 req/s is unresolved")
    ap.add_argument("--serve-requests", type=int, default=150, help="requests per arrival rate")
    ap.add_argument("--serve-slots", type=int, default=16, help="concurrently active solves in the server")
    ap.add_argument("--serve-small-budget-gb", type=int, default=0,
                    help="HBM budget (GB) of a second run at the highest rate, where admission binds (8 with "
                         "--serve-rates ...,200 gives the admission-bound case); 0: skip")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="finish with three plain 1 GiB stream copies (reference for HBM byte counters)")
    ap.add_argument("--profile", default="none", choices=["none", "mixed", "stream", "moving"],
                    help="profiler runs: 'mixed' times only the mixed form (--warmup and --steps solves and one "
                         "with per-launch sweep timing), 'stream' only the streaming ceiling, 'moving' only the "
                         "moving-body steps and the advection-diffusion step")
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
    if args.profile == "stream":
        out = {"hbm_ceiling": hbm_ceiling(P)}
        if args.copy_calibration:
            P.hbm_stream(P.STREAM_COPY, 1 << 30, 3)
        print(json.dumps(out), flush=True)
        return
    if args.profile == "moving":
        print(json.dumps({"moving": moving_bench(P), "advection_diffusion": ad_bench(P)}), flush=True)
        return
    p, desc = make_problem(args.config)
    nx, ny, nz = p.shape
    N = p.npts
    key = KEYS[args.config]
    G = oracle_sample(args.config)
    log("workload", desc)
    t0 = time.time()
    flags, cst = P.classify(p.xf, p.yf, p.zf, p.bodies)
    st = P.build_ghost_stencils(p.xf, p.yf, p.zf, p.bodies, flags)
    ng, nm, nfb = st.info()
    f = torch.from_numpy(p.f).to(dev)
    if args.profile == "mixed":
        solm = P.Solver(p.xf, p.yf, p.zf, flags, st, precision=P.PREC_MIXED, tol=p.tol, max_iter=60)
        for _ in range(args.warmup):
            solm.solve(f)
        msm, xm, sm = time_solves(solm, f, args.steps)
        roofm = sweep_roofline(P, solm, f, 4, N, measured_traffic(key, "f32"))
        if args.copy_calibration:
            P.hbm_stream(P.STREAM_COPY, 1 << 30, 3)
        print(json.dumps({"mixed": {"ms_per_solve": round(msm, 3), "iterations": sm.iterations,
                                    "outer_steps": sm.outer_steps, "roofline": roofm}}), flush=True)
        return
    sol = P.Solver(p.xf, p.yf, p.zf, flags, st, precision=P.PREC_FP64, tol=p.tol, max_iter=200)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    log("setup %.2f s: ghosts %d, membrane ghosts %d, fallback %d" % (setup_s, ng, nm, nfb))

    # ---- headline: the FP64 solve
    for _ in range(args.warmup):
        x, s64 = sol.solve(f)
        log("warmup fp64: its %d rel %.2e %.1f ms" % (s64.iterations, s64.rel_residual, s64.solve_ms))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev_ms = []
    for k in range(args.steps):
        x, s64 = sol.solve(f)
        dev_ms.append(s64.solve_ms)
        log("step %d: its %d rel %.2e %.1f ms" % (k, s64.iterations, s64.rel_residual, s64.solve_ms))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    value = N / (ms_per_step / 1e3) / 1e6
    err64 = sampled_error(x, G) if G is not None else None
    roof = sweep_roofline(P, sol, f, 8, N, measured_traffic(key, "f64"))
    out = {"metric": METRIC, "value": round(value, 2), "unit": "Mpts/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": desc, "grid": [nx, ny, nz], "points": N, "tol": p.tol,
                      "precision": "FP64 throughout (vectors, V-cycle, dots, ghost weights)",
                      "iterations": s64.iterations, "rel_residual": s64.rel_residual,
                      "device_ms_per_solve": round(float(np.median(dev_ms)), 3), "setup_s": round(setup_s, 2),
                      "ghosts": ng, "membrane_ghosts": nm, "fallback_rows": nfb,
                      "rel_error_vs_oracle_sample": err64},
           "roofline": roof}
    # whole FP64 solve against the compulsory-traffic model (463 B/pt/iteration)
    model = 463.0 * s64.iterations * N
    out["solve_model"] = {"bytes_per_solve": int(model), "GB_s": round(model / (ms_per_step * 1e-3) / 1e9, 1),
                          "frac": round(model / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    # and its measured HBM traffic (every solve kernel's counters)
    ts64 = measured_solve_traffic(key, "f64")
    if ts64:
        out["solve_hbm"] = {"bytes_per_solve": int(ts64), "GB_s": round(ts64 / (ms_per_step * 1e-3) / 1e9, 1),
                            "frac": round(ts64 / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                            "vs_model": round(ts64 / model, 3)}
    if roof:
        log("fp64 %.1f ms/solve (%.1f Mpts/s, %d its); k0_sweep<double> %.1f GB/s (%.3f of peak); error vs oracle "
            "sample %s" % (ms_per_step, value, s64.iterations, roof["achieved"], roof["frac"], err64))
    x = None

    # ---- the mixed form on the same system
    if not args.no_mixed:
        solm = P.Solver(p.xf, p.yf, p.zf, flags, st, precision=P.PREC_MIXED, tol=p.tol, max_iter=60)
        solm.solve(f)
        reps = max(2, min(5, args.steps))
        msm, xm, sm = time_solves(solm, f, reps)
        errm = sampled_error(xm, G) if G is not None else None
        roofm = sweep_roofline(P, solm, f, 4, N, measured_traffic(key, "f32"))
        ts = measured_solve_traffic(key, "mixed")
        out["mixed"] = {"ms_per_solve": round(msm, 3), "Mpts_s": round(N / msm * 1e3 / 1e6, 2),
                        "dtype": "f64+f32+bf16", "tol": p.tol, "iterations": sm.iterations,
                        "outer_steps": sm.outer_steps, "rel_residual": sm.rel_residual,
                        "speedup_vs_fp64": round(ms_per_step / msm, 3), "rel_error_vs_oracle_sample": errm,
                        "roofline": roofm}
        if ts:
            out["mixed"]["solve_hbm"] = {"bytes_per_solve": int(ts), "GB_s": round(ts / (msm * 1e-3) / 1e9, 1),
                                         "frac": round(ts / (msm * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        log("mixed %.1f ms/solve (%d its, %d outer): %.2fx; error vs oracle sample %s" %
            (msm, sm.iterations, sm.outer_steps, ms_per_step / msm, errm))
        xm = None
        del solm
        torch.cuda.empty_cache()
        # equal accuracy: for each form the loosest tolerance whose solution is
        # within 1e-8 of the oracle's (on the stored sample), and the times there
        if G is not None and not args.no_ladder:
            ladder = [1e-8, 5e-9, 2e-9, 1e-9, 5e-10, 2e-10, 1e-10]
            eq = {}
            for name, prec in (("fp64", P.PREC_FP64), ("mixed", P.PREC_MIXED)):
                rows = []
                for tol in ladder:
                    sl = P.Solver(p.xf, p.yf, p.zf, flags, st, precision=prec, tol=tol, max_iter=200)
                    sl.solve(f)
                    ms, xl, sx = time_solves(sl, f, 2)
                    e = sampled_error(xl, G)
                    rows.append({"tol": tol, "ms": round(ms, 3), "iterations": sx.iterations, "error": e})
                    xl = None
                    del sl
                    log("ladder %s tol %.0e: %.1f ms, %d its, error %.2e" % (name, tol, ms, sx.iterations, e))
                    if e <= 1e-8:
                        break
                torch.cuda.empty_cache()
                eq[name] = rows
            f64ok = [r for r in eq["fp64"] if r["error"] <= 1e-8]
            mok = [r for r in eq["mixed"] if r["error"] <= 1e-8]
            out["mixed"]["equal_accuracy"] = {
                "target": "rel L2 error <= 1e-8 against the oracle sample", "fp64": eq["fp64"], "mixed": eq["mixed"],
                "speedup": (round(f64ok[0]["ms"] / mok[0]["ms"], 3) if f64ok and mok else None)}
    del sol
    torch.cuda.empty_cache()

    # ---- the 1024^3, twenty-sphere case in both forms
    if not args.no_c4 and args.config != "c4":
        from paper_2605_04335_amd import workloads as W
        q = W.spheres_case(1024)
        fl4, _ = P.classify(q.xf, q.yf, q.zf, q.bodies)
        st4 = P.build_ghost_stencils(q.xf, q.yf, q.zf, q.bodies, fl4)
        f4 = torch.from_numpy(q.f).to(dev)
        leg = {"workload": "20 spheres 1024^3 uniform, Gaussian-bump RHS, MG-BiCGSTAB to 1e-8",
               "points": q.npts, "ghosts": st4.info()[0]}
        keep = None
        for name, prec in (("fp64", P.PREC_FP64), ("mixed", P.PREC_MIXED)):
            s4 = P.Solver(q.xf, q.yf, q.zf, fl4, st4, precision=prec, tol=1e-8, max_iter=200)
            s4.solve(f4)
            ms, x4, t4 = time_solves(s4, f4, 2)
            leg[name] = {"ms_per_solve": round(ms, 2), "Mpts_s": round(q.npts / ms * 1e3 / 1e6, 1),
                         "iterations": t4.iterations, "outer_steps": t4.outer_steps,
                         "rel_residual": t4.rel_residual}
            if keep is None:
                keep = x4
            else:
                d = x4 - keep
                leg["mixed_rel_diff_vs_fp64"] = float(torch.linalg.norm(d) / torch.linalg.norm(keep))
            x4 = None
            del s4
            torch.cuda.empty_cache()
            log("c4 %s: %.1f ms/solve, %d its" % (name, ms, t4.iterations))
        leg["speedup"] = round(leg["fp64"]["ms_per_solve"] / leg["mixed"]["ms_per_solve"], 3)
        leg["oracle"] = "not run: the 1024^3 oracle solve needs ~90 GB of host memory and hours of CPU time"
        out["c4"] = leg
        keep = f4 = None
        del st4, fl4
        torch.cuda.empty_cache()

    # ---- the device's streaming ceiling
    if not args.no_stream:
        ceil = hbm_ceiling(P)
        out["hbm_ceiling"] = ceil
        cgb = ceil["read3_write1"]["GB_s"]
        for r in (out.get("roofline"), out.get("mixed", {}).get("roofline")):
            if r:
                r["ceiling_GB_s"] = cgb
                r["frac_of_ceiling"] = round(r["achieved"] / cgb, 4)

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
        P.hbm_stream(P.STREAM_COPY, 1 << 30, 3)
        log("copy calibration: 3 stream copies of 1 GiB (k_st_copy)")
    if rank == 0 and not args.no_cpu:
        try:
            out["cpu_baseline"] = cpu_baseline(args.config, p, G)
            log("cpu baseline: %s Mpts/s (%s)" % (out["cpu_baseline"]["value"], out["cpu_baseline"]["sample"]))
        except Exception as e:  # reported, never fatal
            out["cpu_baseline"] = {"value": None, "error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    # on a fatal signal: every Python thread's position (faulthandler) and,
    # from the solve server, the faulting native thread's stack
    faulthandler.enable()
    os.environ.setdefault("IBM_CRASH_TRACE", "1")
    main()
