"""Serving loop through the C ABI (needs an MI355X).

Every request solved in the mix must equal the same request solved alone
(the solve is deterministic, so the target is bitwise; the hard bound is the
1e-8 tolerance), admission must follow the memory budget and the slot limit,
and requests that arrive while others run must overlap with them.
"""
import time

import numpy as np
import pytest

import oracle
from paper_2605_04335_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_04335_amd as P
    return P


def requests(n, seed, emin=32, emax=64):
    rng = np.random.default_rng(seed)
    out = []
    for q in range(n):
        p = W.serving_request(rng, emin, emax)
        p.f = W.noise_rhs(p.npts, 1000 + seed * 100 + q)
        out.append(p)
    return out


def solve_alone(P, p, **opts):
    import torch
    flags, _ = P.classify(p.xf, p.yf, p.zf, p.bodies)
    st = P.build_ghost_stencils(p.xf, p.yf, p.zf, p.bodies, flags)
    sol = P.Solver(p.xf, p.yf, p.zf, flags, st, **opts)
    x, stats = sol.solve(torch.from_numpy(p.f).cuda())
    return x.cpu().numpy(), stats


def wait_all(P, srv, tickets, timeout_s=120):
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        assert time.time() - t0 < timeout_s, "serving timed out"
        for t in tickets:
            if t in res:
                continue
            rc, state, x, st, tm = srv.poll(t)
            if rc != P.IBM_EAGAIN:
                res[t] = (rc, state, x, st, (tm.submit_ms, tm.admit_ms, tm.done_ms))
        time.sleep(0.002)
    return res


def test_mix_equals_alone(P):
    reqs = requests(5, 11)
    reqs.append(W.membrane_case(64, nc=40, ns=120))
    opts = dict(precision="mixed", tol=1e-8, max_iter=60)
    alone = []
    for q, p in enumerate(reqs):
        say("alone", q, p.shape, len(p.bodies))
        alone.append(solve_alone(P, p, **opts))
    srv = P.Server(hbm_budget=16 << 30, max_slots=3)
    try:
        tickets = [srv.submit(p.xf, p.yf, p.zf, p.bodies, p.f, **opts) for p in reqs]
        res = wait_all(P, srv, tickets)
    finally:
        srv.close()
    identical = 0
    for q, t in enumerate(tickets):
        rc, state, x, st, times = res[t]
        xa, sa = alone[q]
        assert rc == P.IBM_OK and state == P.IBM_REQ_DONE
        assert st.rel_residual <= 1e-8
        assert x.shape == xa.shape
        d = float(np.linalg.norm(x - xa) / np.linalg.norm(xa))
        say("request", q, "rel diff %.3e" % d, "iterations", st.iterations, sa.iterations)
        assert d <= 1e-8
        identical += int(np.array_equal(x, xa))
    say("bitwise identical:", identical, "of", len(tickets))
    assert identical == len(tickets)
    # with 3 slots, some requests ran at the same time
    iv = sorted(r[4][1:] for r in res.values())
    assert any(iv[q + 1][0] < iv[q][1] for q in range(len(iv) - 1))


def test_served_results_match_oracle(P):
    """Requests served together (three slots, arrivals while others run),
    one of them at the serving workload's sizes (edge >= 128), mixed
    precision with the tolerance tightened to 1e-10 for the parity check:
    each result matches the FP64 oracle's 1e-13 solution of the same request
    to 1e-8 relative L2 after the gauge."""
    reqs = requests(4, 17) + requests(1, 18, 128, 160)
    assert max(max(q.shape) for q in reqs) >= 128
    opts = dict(precision="mixed", tol=1e-10, max_iter=60, max_outer=20)
    srv = P.Server(hbm_budget=16 << 30, max_slots=3)
    try:
        tickets = [srv.submit(p.xf, p.yf, p.zf, p.bodies, p.f, **opts) for p in reqs]
        res = wait_all(P, srv, tickets)
    finally:
        srv.close()
    for q, (p, t) in enumerate(zip(reqs, tickets)):
        rc, state, x, st, _ = res[t]
        assert rc == P.IBM_OK and st.rel_residual <= 1e-10
        O = oracle.setup(p.xf, p.yf, p.zf, p.bodies)
        xo, _, _, info = oracle.solve_problem(O, p.f, tol=1e-13, maxit=200)
        assert info.rc == 0
        e = float(np.linalg.norm(x - xo) / np.linalg.norm(xo))
        say("request", q, p.shape, len(p.bodies), "bodies: %d iterations, error vs oracle %.2e" % (st.iterations, e))
        assert e < 1e-8


def test_slot_limit_serialises(P):
    reqs = requests(3, 12)
    srv = P.Server(hbm_budget=16 << 30, max_slots=1)
    try:
        tickets = [srv.submit(p.xf, p.yf, p.zf, p.bodies, p.f, precision="mixed", tol=1e-8) for p in reqs]
        res = wait_all(P, srv, tickets)
    finally:
        srv.close()
    iv = sorted(r[4][1:] for r in res.values())
    for q in range(len(iv) - 1):
        assert iv[q + 1][0] >= iv[q][1]
    assert all(r[0] == P.IBM_OK for r in res.values())


def test_admission_by_footprint(P):
    p = requests(1, 13)[0]
    bytes_needed = P.workspace_estimate(*p.shape, 0, "mixed")
    srv = P.Server(hbm_budget=max(1, bytes_needed // 4), max_slots=4)
    try:
        t = srv.submit(p.xf, p.yf, p.zf, p.bodies, p.f, precision="mixed", tol=1e-8)
        res = wait_all(P, srv, [t])
        rc, state = res[t][0], res[t][1]
        assert rc == P.IBM_ENOMEM and state == P.IBM_REQ_FAILED
        rc, *_ = srv.poll(t)
        assert rc == P.IBM_ENOTFOUND
    finally:
        srv.close()


def test_poll_states(P):
    p = W.sphere_ellipsoid_case(96)
    srv = P.Server(hbm_budget=16 << 30, max_slots=2)
    try:
        t = srv.submit(p.xf, p.yf, p.zf, p.bodies, p.f, precision="mixed", tol=1e-8)
        rc, state, x, st, tm = srv.poll(t)
        assert rc in (P.IBM_EAGAIN, P.IBM_OK)
        if rc == P.IBM_EAGAIN:
            assert state in (P.IBM_REQ_QUEUED, P.IBM_REQ_RUNNING)
            res = wait_all(P, srv, [t])
            assert res[t][0] == P.IBM_OK
        rc, *_ = srv.poll(123456789)
        assert rc == P.IBM_ENOTFOUND
        srv.drain()
    finally:
        srv.close()


def test_setup_cache(P):
    """A repeated (grid, bodies, options) request reuses the cached set-up and
    returns bitwise the same solution; an admission that needs the memory
    evicts the idle set-up."""
    a, b = requests(2, 14, 48, 64)
    opts = dict(precision="mixed", tol=1e-8)

    srv = P.Server(hbm_budget=16 << 30, max_slots=2, cache_entries=4)
    try:
        ta = srv.submit(a.xf, a.yf, a.zf, a.bodies, a.f, **opts)
        r1 = wait_all(P, srv, [ta])[ta]
        tb = srv.submit(a.xf, a.yf, a.zf, a.bodies, a.f, **opts)
        # poll by hand to read the cache flag
        while True:
            rc, state, x2, st2, tm2 = srv.poll(tb)
            if rc != P.IBM_EAGAIN:
                break
            time.sleep(0.002)
        assert r1[0] == P.IBM_OK and rc == P.IBM_OK
        assert tm2.cache_hit == 1
        assert np.array_equal(r1[2], x2)
    finally:
        srv.close()
    # a budget that holds one set-up (the server's footprint: workspace plus
    # classification temporaries): b evicts a's cached set-up and vice versa
    fa, fb = (P.workspace_estimate(*q.shape, q.npts // 8, "mixed") + int(17.5 * q.npts) for q in (a, b))
    assert min(fa, fb) > 0.1 * max(fa, fb)
    srv = P.Server(hbm_budget=int(1.1 * max(fa, fb)), max_slots=1, cache_entries=4)
    try:
        hits = []
        for p in (a, b, a):
            t = srv.submit(p.xf, p.yf, p.zf, p.bodies, p.f, **opts)
            while True:
                rc, state, x, st, tm = srv.poll(t)
                if rc != P.IBM_EAGAIN:
                    break
                time.sleep(0.002)
            assert rc == P.IBM_OK
            hits.append(tm.cache_hit)
        say("cache hits", hits)
        assert hits == [0, 0, 0]
    finally:
        srv.close()


def _poll_done(P, srv, t, timeout_s=120):
    t0 = time.time()
    while True:
        rc, state, x, st, tm = srv.poll(t)
        if rc != P.IBM_EAGAIN:
            return rc, x, st, tm
        assert time.time() - t0 < timeout_s, "serving timed out"
        time.sleep(0.002)


def test_cache_key_holds_every_option(P):
    """Requests that differ only in the preconditioner, or only in the SRJ
    sweep count, get set-ups of their own: no cache hit, and each result and
    iteration count equals a solo solve with the same options."""
    (a,) = requests(1, 16, 40, 48)
    variants = [dict(precision="fp64", tol=1e-8, precond="mg"),
                dict(precision="fp64", tol=1e-8, precond="srj", srj_sweeps=8),
                dict(precision="fp64", tol=1e-8, precond="srj", srj_sweeps=12),
                dict(precision="fp64", tol=1e-8, precond="mg")]
    srv = P.Server(hbm_budget=16 << 30, max_slots=1, cache_entries=8)
    try:
        got = []
        for v in variants:
            rc, x, st, tm = _poll_done(P, srv, srv.submit(a.xf, a.yf, a.zf, a.bodies, a.f, max_iter=1000, **v))
            assert rc == P.IBM_OK
            got.append((x, st.iterations, tm.cache_hit))
    finally:
        srv.close()
    say("iterations", [g[1] for g in got], "cache hits", [g[2] for g in got])
    assert [g[2] for g in got] == [0, 0, 0, 1]
    for v, (x, its, _) in zip(variants, got):
        xa, sa = solve_alone(P, a, max_iter=1000, **v)
        assert its == sa.iterations
        assert np.array_equal(x, xa)


def test_burst_with_cache_all_succeed(P):
    """Requests arriving together, with new set-ups (and their first graph
    captures) overlapping cached ones and evictions: every one succeeds.
    Guards against runtime calls that a graph capture in another worker
    thread does not allow (synchronous legacy-stream copies, frees)."""
    reqs = requests(12, 15, 32, 96)
    srv = P.Server(hbm_budget=16 << 30, max_slots=4, cache_entries=3)
    try:
        for rnd in range(2):
            tickets = [srv.submit(p.xf, p.yf, p.zf, p.bodies, p.f, precision="mixed", tol=1e-8) for p in reqs]
            res = wait_all(P, srv, tickets)
            bad = [(q, r[0], r[3].rel_residual) for q, r in enumerate(res[t] for t in tickets)
                   if r[0] != P.IBM_OK or r[3].rel_residual > 1e-8]
            say("round", rnd, "failures", bad)
            assert not bad
    finally:
        srv.close()
