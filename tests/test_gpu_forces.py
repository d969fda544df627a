"""Surface pressure loads through the C ABI (needs an MI355X): nodal forces
and pressure jumps of the GPU against the oracle's plain definition, on the
pressure the GPU solve produced, at a small size and at 512^3."""
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


def check(P, p, x, flags):
    F, dp, lost = P.surface_forces(p.xf, p.yf, p.zf, p.bodies, flags, x)
    Fo, dpo, losto = oracle.surface_forces(p.xf, p.yf, p.zf, p.bodies, flags.cpu().numpy(), x.cpu().numpy())
    Fo = np.concatenate(Fo)
    dpo = np.concatenate(dpo)
    F = F.cpu().numpy()
    dp = dp.cpu().numpy()
    # same operations in the same order, no contraction on either side
    exact = int(np.sum(np.all(F == Fo, axis=1)))
    say("%s: %d nodes (%d bitwise equal), %d triangles, lost %d/%d" % (p.name, len(F), exact, len(dp), lost, losto))
    assert lost == losto
    assert np.abs(dp - dpo).max() <= 1e-13 * np.abs(dpo).max()
    assert np.abs(F - Fo).max() <= 1e-13 * np.abs(Fo).max()
    return F, Fo


@pytest.mark.parametrize("n", [48, 64])
def test_forces_match_oracle(P, n):
    import torch
    p = W.flapping_case(n, 100)
    flags, st, sol, _ = P.setup(p.xf, p.yf, p.zf, p.bodies, tol=1e-10)
    x, s = sol.solve(torch.from_numpy(p.f).cuda())
    F, Fo = check(P, p, x, flags)
    # the area rule partitions each triangle's load: per-body totals agree
    nv0 = len(p.bodies[0].verts)
    assert np.allclose(F[:nv0].sum(0), Fo[:nv0].sum(0), rtol=1e-12, atol=1e-18)


def test_forces_walls_and_thin_body(P):
    """Probes near the domain walls and on a body under half a cell thick:
    a sphere cut by the x = 0 wall, a thin ellipsoid, a membrane through both
    y walls."""
    import torch
    p = W.Problem("walls_thin_40", W.uniform_faces(40), W.uniform_faces(40), W.uniform_faces(40),
                  [W.sphere((0.08, 0.5, 0.45), 0.2, freq=8),
                   W.ellipsoid((0.6, 0.5, 0.5123), (0.2, 0.15, 0.011), W.rotation_zyx(0.3, 0.0, 0.0), freq=8),
                   W.plate((0.65, 0.5, 0.27), 0.3, 1.3, 12, 52, 0.03, 0.4)])
    p.f = W.noise_rhs(40 ** 3, 12)
    flags, st, sol, _ = P.setup(p.xf, p.yf, p.zf, p.bodies, tol=1e-10)
    x, s = sol.solve(torch.from_numpy(p.f).cuda())
    assert s.status == 0
    check(P, p, x, flags)


def test_forces_linear_field_closed_form(P):
    """The closed-form case of the oracle's pins, on the GPU: a cube in
    p = a.x on a uniform grid gets -(a L^3 + 2 d L^2 a)."""
    import torch
    n = 40
    f = W.uniform_faces(n)
    lo, hi = np.array([0.3137, 0.2911, 0.3323]), np.array([0.6589, 0.6402, 0.6871])
    L = hi - lo
    body = W.box(lo, hi)
    flags, _ = P.classify(f, f, f, [body])
    c = W.centres(f)
    a = np.array([0.7, -1.3, 2.1])
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    p = torch.from_numpy((a[0] * X + a[1] * Y + a[2] * Z).ravel().copy()).cuda()
    F, dp, lost = P.surface_forces(f, f, f, [body], flags, p)
    side = np.array([L[1] * L[2], L[0] * L[2], L[0] * L[1]])
    want = -(a * np.prod(L) + 2 * (2.0 / n) * a * side)
    assert lost == 0
    assert np.allclose(F.cpu().numpy().sum(0), want, rtol=1e-12, atol=1e-14)


def test_forces_full_size_512(P):
    """Flapping plate and heaving sphere on the 512^3 stretched grid: every
    node and triangle against the oracle on the GPU pressure."""
    import torch
    p = W.flapping_case(512, 7)
    flags, st, sol, _ = P.setup(p.xf, p.yf, p.zf, p.bodies, precision="mixed", tol=1e-8)
    x, s = sol.solve(torch.from_numpy(p.f).cuda())
    assert s.status == 0
    del sol
    check(P, p, x, flags)
