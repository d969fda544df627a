"""Device memory reuse through the C ABI (needs an MI355X).

The library keeps released device blocks and hands them to later
allocations of the same size class, with whatever the previous owner left in
them.  A solve must therefore not depend on the initial contents of any
buffer it allocates: the same problem solved before and after other
problems (of other sizes, so that blocks change roles) must give the same
bits.  The server's per-request phase times are checked for consistency.
"""
import time

import numpy as np
import pytest

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


def request(seed, emin, emax):
    p = W.serving_request(np.random.default_rng(seed), emin, emax)
    p.f = W.noise_rhs(p.npts, 5000 + seed)
    return p


def solve(P, p, precision):
    import torch
    flags, _ = P.classify(p.xf, p.yf, p.zf, p.bodies)
    st = P.build_ghost_stencils(p.xf, p.yf, p.zf, p.bodies, flags)
    sol = P.Solver(p.xf, p.yf, p.zf, flags, st, precision=precision, tol=1e-8)
    x, stats = sol.solve(torch.from_numpy(p.f).cuda())
    out = x.cpu().numpy()
    del sol, st, flags, x
    return out, stats


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solution_independent_of_reused_blocks(P, precision):
    a = request(11, 48, 64)
    say("reuse", precision, "grid", a.npts)
    xa, sa = solve(P, a, precision)
    assert sa.status == 0
    for seed, lo, hi in [(12, 64, 96), (13, 32, 48), (14, 96, 128)]:
        b = request(seed, lo, hi)
        say("reuse", precision, "other grid", b.npts)
        _, sb = solve(P, b, precision)
        assert sb.status == 0
        time.sleep(0.05)  # let released blocks become reusable
    xa2, sa2 = solve(P, a, precision)
    assert sa2.iterations == sa.iterations
    assert np.array_equal(xa, xa2)


def test_server_phase_times(P):
    srv = P.Server(hbm_budget=8 << 30, max_slots=4, cache_entries=0)
    reqs = [request(20 + q, 32, 64) for q in range(6)]
    tickets = [srv.submit(p.xf, p.yf, p.zf, p.bodies, p.f, precision="mixed", tol=1e-8) for p in reqs]
    done = {}
    t0 = time.time()
    while len(done) < len(tickets):
        assert time.time() - t0 < 120, "serving timed out"
        for t in tickets:
            if t in done:
                continue
            rc, state, _, st, tm = srv.poll(t, want_x=False)
            if rc != P.IBM_EAGAIN:
                done[t] = (rc, tm)
        time.sleep(0.001)
    srv.close()
    for rc, tm in done.values():
        assert rc == 0
        assert tm.cache_hit == 0
        assert tm.setup_ms > 0.0 and tm.solve_ms > 0.0
        assert tm.submit_ms <= tm.admit_ms <= tm.done_ms
        assert tm.setup_ms + tm.solve_ms <= tm.done_ms - tm.admit_ms + 1e-6
