"""Moving bodies through the C ABI (needs an MI355X): re-set-up of a context
for a new classification, fresh-cell initial values, and solves from an
initial guess.

poisson_update must give bit for bit the same solves as a fresh set-up of the
same geometry (including updates that add or drop every membrane ghost
unknown); ibm_fill_fresh must equal the oracle's fresh-cell fill bit for bit;
a solve from a guess must reach the same solution as the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2605_04335_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_04335_amd as P
    return P


def sequence(n=64):
    """the sphere alone (no membrane ghost unknowns), then flapping steps:
    the first update grows the unknown count past the set-up's vectors, the
    later ones shrink and regrow it within the headroom"""
    a = W.flapping_case(n, 450)
    a.bodies = a.bodies[:1]
    return [a, W.flapping_case(n, 0), W.flapping_case(n, 300), W.flapping_case(n, 600)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_update_equals_fresh_setup(P, precision):
    import torch
    seq = sequence()
    opts = dict(precision=precision, tol=1e-10, max_iter=100)
    flags, st, sol, _ = P.setup(seq[0].xf, seq[0].yf, seq[0].zf, seq[0].bodies, **opts)
    f = torch.from_numpy(seq[0].f).cuda()
    for q, p in enumerate(seq):
        fl, stq, fresh, _ = P.setup(p.xf, p.yf, p.zf, p.bodies, **opts)
        if q:
            sol.update(fl, stq)
        say(precision, "step", q, "membrane ghosts", sol.nm)
        xu, su = sol.solve(f)
        xf_, sf = fresh.solve(f)
        assert su.status == 0 and su.iterations == sf.iterations
        assert torch.equal(xu, xf_)
        del fresh
    # the last geometry against the oracle
    O = oracle.setup(p.xf, p.yf, p.zf, p.bodies)
    xo, _, _, _ = oracle.solve_problem(O, p.f, tol=1e-13, maxit=100)
    assert rel(xu.cpu().numpy(), xo) < (1e-9 if precision == "fp64" else 1e-8)


def test_fill_fresh_matches_oracle(P):
    import torch
    a, b = W.flapping_case(64, 0), W.flapping_case(64, 150)
    fa, _ = P.classify(a.xf, a.yf, a.zf, a.bodies)
    fb, _ = P.classify(b.xf, b.yf, b.zf, b.bodies)
    x = np.random.default_rng(51).uniform(-1, 1, a.npts)
    xd = torch.from_numpy(x).cuda()
    n = P.fill_fresh(a.xf, a.yf, a.zf, fa, fb, xd)
    xo, no = oracle.fill_fresh(len(a.xf) - 1, len(a.yf) - 1, len(a.zf) - 1, fa.cpu().numpy(), fb.cpu().numpy(), x)
    say("fresh cells", n)
    assert n == no and n > 0
    assert np.array_equal(xd.cpu().numpy(), xo)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_from_previous_step(P, precision):
    """Step b from step a's pressure (fresh cells filled): the oracle's
    solution, and no more iterations than from zero."""
    import torch
    a, b = W.flapping_case(64, 0), W.flapping_case(64, 40)
    tol = 1e-12
    opts = dict(precision=precision, tol=tol, max_iter=100, max_outer=20)
    fa, sta, sol, _ = P.setup(a.xf, a.yf, a.zf, a.bodies, **opts)
    xa, _ = sol.solve(torch.from_numpy(a.f).cuda())
    fb, _ = P.classify(b.xf, b.yf, b.zf, b.bodies)
    stb = P.build_ghost_stencils(b.xf, b.yf, b.zf, b.bodies, fb)
    sol.update(fb, stb)
    x0 = xa[: a.npts].clone()
    P.fill_fresh(a.xf, a.yf, a.zf, fa, fb, x0)
    fbd = torch.from_numpy(b.f).cuda()
    xw, sw = sol.solve_from(fbd, x0)
    xc, sc = sol.solve(fbd)
    say(precision, "warm its %d (outer %d), cold its %d (outer %d)" % (sw.iterations, sw.outer_steps,
                                                                       sc.iterations, sc.outer_steps))
    assert sw.status == 0 and sw.rel_residual <= tol
    assert sw.iterations <= sc.iterations
    O = oracle.setup(b.xf, b.yf, b.zf, b.bodies)
    xo, _, _, _ = oracle.solve_problem(O, b.f, tol=1e-13, maxit=100)
    assert rel(xw.cpu().numpy(), xo) < 1e-9
    # from the solution itself (with its membrane ghost values): no
    # iteration is needed
    xs, ss = sol.solve_from(fbd, xc)
    say(precision, "from the solution: its %d" % ss.iterations)
    assert ss.status == 0 and ss.iterations <= 1
    assert rel(xs.cpu().numpy(), xo) < 1e-9
    with pytest.raises(P.IbmError) as e:
        sol.solve_from(fbd, xc[: b.npts - 1].contiguous())
    assert e.value.code == P.IBM_EINVAL


def test_solve_from_zero_rhs(P):
    """f = 0: the solution is zero whatever the guess."""
    import torch
    p = W.flapping_case(32, 0)
    flags, st, sol, _ = P.setup(p.xf, p.yf, p.zf, p.bodies, tol=1e-10)
    x0 = torch.from_numpy(np.random.default_rng(3).uniform(-1, 1, p.npts)).cuda()
    x, s = sol.solve_from(torch.zeros(p.npts, dtype=torch.float64, device="cuda"), x0)
    assert s.status == 0 and float(x.abs().max()) == 0.0
