"""Full-size checks on the benchmark configurations (needs an MI355X): the
512^3 membrane case the benchmark times, the 1024^3 spheres case and the
256^3 plain FP64 case.

At this size the oracle still classifies, builds the ghost rows, applies the
operator and runs one V-cycle in seconds, so those are compared element by
element.  The benchmarked 512^3 system's solution is compared with the
oracle's (solved to 1e-13 once, off line, by tests/golden/
make_c3_oracle_sample.py, which runs only the oracle) on a stored seeded
sample of cells and membrane ghost unknowns.  Manufactured systems
(b = A x_true) add checks that hold at any size: the oracle's own operator
applied to the GPU solution leaves a residual within the tolerance, the
error stays within kappa * tol, and the mixed and FP64 solutions agree.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2605_04335_amd import workloads as W
from tests import refpy

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_mod_const(x, xt, flags):
    """Relative error modulo a constant.  The pressure is defined up to a
    constant; the pinned system fixes it only through a single cell, so its
    near-null vector (a constant minus the pin's point-source response) is
    not resolved by the residual and a solve that meets the tolerance may
    carry a near-constant error of any size below kappa * tol.  The error is
    therefore measured after removing its mean over the fluid cells from
    every active unknown."""
    N = len(flags)
    fluid = (flags & 1) == 0
    act = refpy.active_mask(flags, len(x) - N)
    e = x - xt
    e = np.where(act, e - e[:N][fluid].mean(), 0.0)
    t = np.where(act, xt - xt[:N][fluid].mean(), 0.0)
    return float(np.linalg.norm(e) / np.linalg.norm(t))


@pytest.fixture(scope="module")
def c3():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_04335_amd as P
    p = W.membrane_case(512)
    say("c3 oracle classification + ghost rows")
    O = oracle.setup(p.xf, p.yf, p.zf, p.bodies)
    flags, cst = P.classify(p.xf, p.yf, p.zf, p.bodies)
    st = P.build_ghost_stencils(p.xf, p.yf, p.zf, p.bodies, flags)
    return P, p, O, flags, st


def test_c3_classification_and_ghost_rows(c3):
    P, p, O, flags, st = c3
    say("c3 flags")
    g = flags.cpu().numpy()
    assert np.array_equal(g, O.flags), "mismatching cells: %d" % int(np.sum(g != O.flags))
    e = st.export()
    assert e["ng"] == O.st.ng and e["nm"] == O.st.nm
    assert np.array_equal(e["cell"], O.st.row_cell)
    assert np.array_equal(e["col"], O.st.col)
    assert np.array_equal(e["rfl"], O.st.rfl)
    assert np.abs(e["w"] - O.st.w).max(initial=0) < 1e-13
    assert np.allclose(e["sG"], O.st.sG, rtol=1e-14, atol=0)
    assert np.abs(e["dlb"] - O.st.dlb).max(initial=0) < 1e-13


def test_c3_operator_and_vcycle(c3):
    import torch
    P, p, O, flags, st = c3
    sol = P.Solver(p.xf, p.yf, p.zf, flags, st, precision="fp64")
    n = sol.n_unknowns
    x = np.random.default_rng(31).uniform(-1, 1, n)
    x[~refpy.active_mask(O.flags, O.st.nm)] = 0.0
    say("c3 operator")
    y = sol.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    assert rel(y, oracle.apply(p.xf, p.yf, p.zf, O.flags, O.st, x)) < 1e-14
    say("c3 rhs")
    b = sol.assemble_rhs(torch.from_numpy(p.f).cuda()).cpu().numpy()
    bo = oracle.assemble_rhs(p.xf, p.yf, p.zf, O.flags, O.st, p.f)
    assert rel(b, bo) < 1e-14
    say("c3 V-cycle")
    z = sol.precond(torch.from_numpy(bo).cuda()).cpu().numpy()
    # one linear map, but its global sums (the pin sink over 1.3e8 terms with
    # heavy cancellation, divided by the pin volume ~1e-9, and one mean per
    # coarse level) are reduced in a different order than the oracle's:
    # measured 6.9e-11 here (1.5e-12 at 64^3)
    assert rel(z, oracle.vcycle(p.xf, p.yf, p.zf, O.flags, O.st, bo)) < 1e-9


def test_c3_manufactured_mixed_and_fp64(c3):
    import torch
    P, p, O, flags, st = c3
    s64 = P.Solver(p.xf, p.yf, p.zf, flags, st, precision="fp64", tol=1e-12, max_iter=200)
    n = s64.n_unknowns
    xt = np.random.default_rng(32).uniform(-1, 1, n)
    xt[~refpy.active_mask(O.flags, O.st.nm)] = 0.0
    xt[int(np.nonzero(O.flags & 8)[0][0])] = 0.0
    b = oracle.apply(p.xf, p.yf, p.zf, O.flags, O.st, xt)
    bd = torch.from_numpy(b).cuda()
    nb = np.linalg.norm(b)
    say("c3 fp64 solve")
    x64, st64 = s64.solve_assembled(bd)
    x64 = x64.cpu().numpy()
    r64 = np.linalg.norm(b - oracle.apply(p.xf, p.yf, p.zf, O.flags, O.st, x64)) / nb
    say("fp64: its %d, own residual %.2e, oracle residual %.2e, error %.2e (modulo a constant %.2e)" %
        (st64.iterations, st64.rel_residual, r64, rel(x64, xt), rel_mod_const(x64, xt, O.flags)))
    assert st64.status == 0 and r64 <= 1.01e-12
    del s64
    torch.cuda.empty_cache()
    smx = P.Solver(p.xf, p.yf, p.zf, flags, st, precision="mixed", tol=1e-12, max_iter=60, max_outer=20)
    say("c3 mixed solve")
    xm, stm = smx.solve_assembled(bd)
    xm = xm.cpu().numpy()
    rm = np.linalg.norm(b - oracle.apply(p.xf, p.yf, p.zf, O.flags, O.st, xm)) / nb
    say("mixed: its %d outer %d, own residual %.2e, oracle residual %.2e, error %.2e, vs fp64 %.2e" %
        (stm.iterations, stm.outer_steps, stm.rel_residual, rm, rel(xm, xt), rel(xm, x64)))
    assert stm.status == 0 and rm <= 1.01e-12
    # kappa ~ (12 / h_min^2) / (3 pi^2) ~ 3e5 of the Laplacian bounds each
    # error modulo a constant by kappa * residual (a 1e-8 solution match is
    # not implied by any attainable residual here); iterative refinement must
    # reach the FP64 residual, so the mixed solution is held to the same bound
    kappa = 3e5
    assert rel_mod_const(x64, xt, O.flags) < kappa * 1e-12
    assert rel_mod_const(xm, xt, O.flags) < kappa * 1e-12
    assert rel_mod_const(xm, x64, O.flags) < kappa * 2e-12


def c3_oracle_sample():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_membrane512_oracle_sample.npz")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def sampled_rel(x, G):
    """Relative L2 difference from the oracle on the stored sample."""
    N = len(x) - int(G["n_mghost"])
    got = np.concatenate([x[G["cells"]], x[N + G["mghost"]]])
    ref = np.concatenate([G["cell_values"], G["mghost_values"]])
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def test_c3_solution_matches_oracle():
    """The benchmarked system itself (512^3 tanh-stretched grid, the seeded
    40k-triangle cambered plate with ghost unknowns on both sides, the seeded
    noise RHS): the GPU FP64 solve to 1e-12 matches the oracle's 1e-13
    solution to 1e-10 and the mixed solve to 1e-10 matches it to 1e-8,
    relative L2 after the gauge on 65,536 sampled cells and 4,096 sampled
    membrane ghost unknowns (two independent oracle runs agree to 7e-13 on
    this sample); the whole fluid field's norm matches the oracle's to 1e-10."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_04335_amd as P
    G = c3_oracle_sample()
    p = W.membrane_case(512)
    say("c3 classification, ghost rows")
    flags, cst = P.classify(p.xf, p.yf, p.zf, p.bodies)
    assert int(flags.to(torch.int64).sum()) == int(G["flags_sum"])
    assert cst["n_mghost"] == int(G["n_mghost"])
    st = P.build_ghost_stencils(p.xf, p.yf, p.zf, p.bodies, flags)
    f = torch.from_numpy(p.f).cuda()
    say("c3 fp64 solve to 1e-12")
    s64 = P.Solver(p.xf, p.yf, p.zf, flags, st, precision="fp64", tol=1e-12, max_iter=200)
    x64, st64 = s64.solve(f)
    x64 = x64.cpu().numpy()
    del s64
    torch.cuda.empty_cache()
    N = p.npts
    e64 = sampled_rel(x64, G)
    en = abs(np.linalg.norm(x64[:N]) - float(G["norm_fluid"])) / float(G["norm_fluid"])
    say("c3 mixed solve to 1e-10")
    smx = P.Solver(p.xf, p.yf, p.zf, flags, st, precision="mixed", tol=1e-10, max_iter=60, max_outer=20)
    xm, stm = smx.solve(f)
    em = sampled_rel(xm.cpu().numpy(), G)
    say("c3 vs oracle: fp64 %d its, error %.2e (norm %.2e); mixed %d its (%d outer), error %.2e" %
        (st64.iterations, e64, en, stm.iterations, stm.outer_steps, em))
    assert st64.status == 0 and st64.rel_residual <= 1e-12
    assert e64 < 1e-10 and en < 1e-10
    assert stm.status == 0 and stm.rel_residual <= 1e-10
    assert em < 1e-8


# ---------------------------------------------------------------- 1024^3, 20 spheres
@pytest.fixture(scope="module")
def c4():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_04335_amd as P
    p = W.spheres_case(1024, rhs=False)
    return P, p


def test_c4_classification(c4):
    """Largest configuration (1.07e9 cells): flags bit-exact against the oracle."""
    P, p = c4
    say("c4 classification")
    flags, cst = P.classify(p.xf, p.yf, p.zf, p.bodies)
    o = oracle.classify(p.xf, p.yf, p.zf, p.bodies)
    g = flags.cpu().numpy()
    assert np.array_equal(g, o), "mismatching cells: %d" % int(np.sum(g != o))
    assert cst["n_ghost"] == int(np.sum((o & 2) > 0))


def test_c4_manufactured_fp64_and_mixed(c4):
    """b = A x_true on 1024^3: the FP64 and the mixed solve meet 1e-11 and their errors
    modulo a constant stay within kappa * tol with the Laplacian's
    kappa = (12/h^2)/(3 pi^2) ~ 4e5 (the near-constant part of the error
    reached 1.7e-4 in one run: the single-cell pin does not resolve it)."""
    import torch
    P, p = c4
    flags, cst = P.classify(p.xf, p.yf, p.zf, p.bodies)
    st = P.build_ghost_stencils(p.xf, p.yf, p.zf, p.bodies, flags)
    sol = P.Solver(p.xf, p.yf, p.zf, flags, st, precision="fp64", tol=1e-11, max_iter=300)
    fl = flags.cpu().numpy()
    n = sol.n_unknowns
    xt = np.random.default_rng(41).uniform(-1, 1, n)
    xt[~refpy.active_mask(fl, sol.nm)] = 0.0
    xt[int(np.nonzero(fl & 8)[0][0])] = 0.0
    xd = torch.from_numpy(xt).cuda()
    b = sol.apply(xd)
    del xd
    say("c4 fp64 solve")
    x, stats = sol.solve_assembled(b)
    xn = x.cpu().numpy()
    err = rel_mod_const(xn, xt, fl)
    say("c4 fp64: its %d residual %.2e error %.2e, modulo a constant %.2e" % (stats.iterations, stats.rel_residual,
                                                                            rel(xn, xt), err))
    assert stats.status == 0 and stats.rel_residual <= 1e-11
    assert err < 4e5 * 1e-11
    # the mixed form on the same system: refinement reaches the same FP64
    # residual, so the same bound holds, and the two solutions agree modulo a
    # constant within twice that bound
    del sol, x
    torch.cuda.empty_cache()
    smx = P.Solver(p.xf, p.yf, p.zf, flags, st, precision="mixed", tol=1e-11, max_iter=60, max_outer=20)
    say("c4 mixed solve")
    xm, sm = smx.solve_assembled(b)
    xmn = xm.cpu().numpy()
    errm = rel_mod_const(xmn, xt, fl)
    dmx = rel_mod_const(xmn, xn, fl)
    say("c4 mixed: its %d outer %d residual %.2e error modulo a constant %.2e, vs fp64 %.2e" %
        (sm.iterations, sm.outer_steps, sm.rel_residual, errm, dmx))
    assert sm.status == 0 and sm.rel_residual <= 1e-11
    assert errm < 4e5 * 1e-11
    assert dmx < 4e5 * 2e-11


# ---------------------------------------------------------------- 256^3 plain FP64 configuration
def test_c2_full_size_matches_oracle():
    """256^3 tanh-stretched grid, sphere + rotated ellipsoid, noise RHS (the
    plain FP64 configuration): classification bit-exact, and with the oracle
    solving the same system to 1e-13 the GPU FP64 solve (to 1e-12) matches it
    to 1e-10 and the mixed solve (to 1e-10) to 1e-8, relative L2."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_04335_amd as P
    p = W.sphere_ellipsoid_case(256)
    say("c2 oracle set-up and solve")
    O = oracle.setup(p.xf, p.yf, p.zf, p.bodies)
    xo, _, _, info = oracle.solve_problem(O, p.f, tol=1e-13, maxit=100)
    assert info.rc == 0
    flags, _ = P.classify(p.xf, p.yf, p.zf, p.bodies)
    assert np.array_equal(flags.cpu().numpy(), O.flags)
    st = P.build_ghost_stencils(p.xf, p.yf, p.zf, p.bodies, flags)
    f = torch.from_numpy(p.f).cuda()
    s64 = P.Solver(p.xf, p.yf, p.zf, flags, st, precision="fp64", tol=1e-12, max_iter=100)
    x64, st64 = s64.solve(f)
    e64 = rel(x64.cpu().numpy(), xo)
    del s64
    smx = P.Solver(p.xf, p.yf, p.zf, flags, st, precision="mixed", tol=1e-10, max_iter=60, max_outer=20)
    xm, stm = smx.solve(f)
    em = rel(xm.cpu().numpy(), xo)
    say("c2: fp64 %d its, error vs oracle %.2e; mixed %d its (%d outer), error %.2e" %
        (st64.iterations, e64, stm.iterations, stm.outer_steps, em))
    assert st64.status == 0 and e64 < 1e-10
    assert stm.status == 0 and em < 1e-8
