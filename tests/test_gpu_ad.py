"""Advection-diffusion step through the C ABI (needs an MI355X): Dirichlet
ghost rows, the operator H and the SRJ solve against the oracle; closed form
without bodies; a 512^3 solve checked by the oracle's own operator."""
import math

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


def beta_for(xf, yf, zf, re=1000.0, cfl=0.5):
    """nu dt / 2 (Crank-Nicolson) at the paper's Re = 1000 with dt from CFL
    0.5 on the finest cell at unit velocity."""
    h = min(np.diff(xf).min(), np.diff(yf).min(), np.diff(zf).min())
    return 0.5 * (1.0 / re) * cfl * h


CASES = {
    "sphere_plate_32": lambda: W.Problem("sp32", W.uniform_faces(32), W.uniform_faces(32), W.uniform_faces(32),
                                         [W.sphere((0.33, 0.5, 0.5), 0.17, freq=8),
                                          W.plate((0.72, 0.5, 0.5), 0.2, 0.4, 10, 20, 0.04, 0.3)]),
    "flapping_48": lambda: W.flapping_case(48, 200, rhs=False),
    # a sphere cut by the x = 0 wall, an ellipsoid under half a cell thick and
    # a membrane through both y walls
    "walls_thin_40": lambda: W.Problem(
        "walls_thin_40", W.uniform_faces(40), W.uniform_faces(40), W.uniform_faces(40),
        [W.sphere((0.08, 0.5, 0.45), 0.2, freq=8),
         W.ellipsoid((0.6, 0.5, 0.5123), (0.2, 0.15, 0.011), W.rotation_zyx(0.3, 0.0, 0.0), freq=8),
         W.plate((0.65, 0.5, 0.27), 0.3, 1.3, 12, 52, 0.03, 0.4)]),
}


@pytest.mark.parametrize("name", list(CASES))
def test_dirichlet_stencils_match(P, name):
    p = CASES[name]()
    flags, _ = P.classify(p.xf, p.yf, p.zf, p.bodies)
    st = P.build_ghost_stencils(p.xf, p.yf, p.zf, p.bodies, flags, bc="dirichlet")
    O = oracle.stencils(p.xf, p.yf, p.zf, p.bodies, flags.cpu().numpy(), bc="dirichlet")
    e = st.export()
    say(name, "rows", e["ng"], e["nm"])
    assert e["ng"] == O.ng and e["nm"] == O.nm
    assert np.array_equal(e["col"], O.col)
    assert np.array_equal(e["rfl"], O.rfl)
    assert np.abs(e["w"] - O.w).max(initial=0) < 1e-13
    assert np.abs(e["dlb"] - O.dlb).max(initial=0) < 1e-13
    assert np.allclose(e["sG"], O.sG, rtol=1e-14, atol=0)


@pytest.mark.parametrize("name", list(CASES))
def test_ad_apply_and_solve_match_oracle(P, name):
    import torch
    p = CASES[name]()
    flags, _ = P.classify(p.xf, p.yf, p.zf, p.bodies)
    st = P.build_ghost_stencils(p.xf, p.yf, p.zf, p.bodies, flags, bc="dirichlet")
    fl = flags.cpu().numpy()
    O = oracle.stencils(p.xf, p.yf, p.zf, p.bodies, fl, bc="dirichlet")
    beta = 4.0 / oracle.max_cell_scale(p.xf, p.yf, p.zf)
    sol = P.AdSolver(p.xf, p.yf, p.zf, flags, st, beta, tol=1e-12, sweeps=8)
    N = len(fl)
    rng = np.random.default_rng(61)
    x = rng.uniform(-1, 1, N + O.nm)
    x[:N][((fl & 1) != 0) & ((fl & 2) == 0)] = 0.0
    y = sol.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    yo = oracle.ad_apply(p.xf, p.yf, p.zf, fl, O, beta, x)
    say(name, "apply rel %.2e, bitwise equal %d/%d" % (rel(y, yo), int(np.sum(y == yo)), len(y)))
    assert rel(y, yo) < 1e-14
    f = rng.uniform(-1, 1, N)
    g = rng.uniform(-0.5, 0.5, O.ng + O.nm)
    u, s = sol.solve(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda())
    rhs = oracle.ad_rhs(p.xf, p.yf, p.zf, fl, O, f, g)
    om = oracle.ad_schedule(8, beta, oracle.max_cell_scale(p.xf, p.yf, p.zf))
    uo, cyc, relo, rc = oracle.ad_solve(p.xf, p.yf, p.zf, fl, O, beta, rhs, om, tol=1e-12)
    say(name, "solve: %d cycles (oracle %d), residual %.2e, vs oracle %.2e" % (s.cycles, cyc, s.rel_residual,
                                                                            rel(u.cpu().numpy(), uo)))
    assert s.status == 0 and rc == 0 and abs(s.cycles - cyc) <= 1
    assert rel(u.cpu().numpy(), uo) < 1e-10


def test_ad_neumann_eigenvector_closed_form(P):
    """No bodies: H v = (1 + beta lam) v for products of cos(pi k (i+1/2)/n)."""
    import torch
    nx, ny, nz = 40, 24, 20
    xf, yf, zf = W.uniform_faces(nx), W.uniform_faces(ny, ny / nx), W.uniform_faces(nz, nz / nx)
    flags, _ = P.classify(xf, yf, zf, [])
    st = P.build_ghost_stencils(xf, yf, zf, [], flags, bc="dirichlet")
    h = 1.0 / nx
    k = (5, 3, 7)
    vx = np.cos(np.pi * k[0] * (np.arange(nx) + 0.5) / nx)
    vy = np.cos(np.pi * k[1] * (np.arange(ny) + 0.5) / ny)
    vz = np.cos(np.pi * k[2] * (np.arange(nz) + 0.5) / nz)
    v = (vz[:, None, None] * vy[None, :, None] * vx[None, None, :]).ravel()
    lam = sum(4 * math.sin(math.pi * kd / (2 * nd)) ** 2 / h ** 2 for kd, nd in zip(k, (nx, ny, nz)))
    beta = 2.0 / oracle.max_cell_scale(xf, yf, zf)
    sol = P.AdSolver(xf, yf, zf, flags, st, beta, tol=1e-13, sweeps=8)
    u, s = sol.solve(torch.from_numpy(v).cuda())
    assert s.status == 0
    assert np.abs(u.cpu().numpy() - v / (1 + beta * lam)).max() < 1e-12


def test_ad_full_size_512(P):
    """Flapping plate and heaving sphere on the 512^3 stretched grid at
    Re 1000, CFL 0.5: the SRJ solve meets 1e-10, checked with the oracle's
    own operator and rows, and the GPU Dirichlet rows equal the oracle's."""
    import torch
    p = W.flapping_case(512, 11)
    flags, _ = P.classify(p.xf, p.yf, p.zf, p.bodies)
    fl = flags.cpu().numpy()
    say("512 oracle Dirichlet rows")
    O = oracle.stencils(p.xf, p.yf, p.zf, p.bodies, fl, bc="dirichlet")
    st = P.build_ghost_stencils(p.xf, p.yf, p.zf, p.bodies, flags, bc="dirichlet")
    e = st.export()
    assert np.array_equal(e["col"], O.col)
    assert np.abs(e["w"] - O.w).max(initial=0) < 1e-13
    beta = beta_for(p.xf, p.yf, p.zf)
    say("beta %.3e, beta * max diag %.2f" % (beta, beta * oracle.max_cell_scale(p.xf, p.yf, p.zf)))
    sol = P.AdSolver(p.xf, p.yf, p.zf, flags, st, beta, tol=1e-10, sweeps=8)
    N = len(fl)
    rng = np.random.default_rng(62)
    f = W.noise_rhs(N, 63)
    g = rng.uniform(-0.5, 0.5, O.ng + O.nm)
    u, s = sol.solve(torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda())
    say("512: %d cycles, residual %.2e, %.1f ms" % (s.cycles, s.rel_residual, s.solve_ms))
    assert s.status == 0
    un = u.cpu().numpy()
    del u, sol
    rhs = oracle.ad_rhs(p.xf, p.yf, p.zf, fl, O, f, g)
    r = rhs - oracle.ad_apply(p.xf, p.yf, p.zf, fl, O, beta, un)
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(rhs)
