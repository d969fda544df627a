"""FP64 CPU oracle for the ghost-cell pressure-Poisson solve.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark; never by the product library.  It
shares no code with the HIP path (its arithmetic lives in ``ibm_oracle.c``
and in the plain numpy below).

Pins (tests/test_oracle_*.py) tie it to the paper and to mathematics:
closed-form eigenvector solutions, direct sparse solves of an independently
assembled matrix, exact rational ray parity, the closest point against an
independent construction, trilinear reproduction by the ghost rows of closed
bodies and of a cambered membrane (whose columns include other membrane
ghost unknowns) with the mirror geometry of their image points, flat-wall
and flat-membrane equivalence.  The degenerate-stencil fallback is pinned
by its invariants only: it reproduces constants, reads face neighbours on
the ghost's own side, and misses a linear field by at most its gradient
times the farthest neighbour.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ibm_oracle.c")
# IBM_ORACLE_LIB selects another build of the same source (the sanitizer
# test loads an ASan/UBSan build through it)
_LIB = os.environ.get("IBM_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

F_SOLID, F_GHOST, F_MGHOST, F_PIN = 1, 2, 4, 8
F_CUTX, F_CUTY, F_CUTZ = 16, 32, 64


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _grid_args(xf, yf, zf):
    return [ctypes.c_int(len(xf) - 1), ctypes.c_int(len(yf) - 1), ctypes.c_int(len(zf) - 1), _p(xf), _p(yf), _p(zf)]


def _bodies_args(bodies):
    kind = np.array([b.kind for b in bodies], dtype=np.int32)
    nv = np.array([len(b.verts) for b in bodies], dtype=np.int32)
    nt = np.array([len(b.tris) for b in bodies], dtype=np.int32)
    V = np.ascontiguousarray(np.concatenate([b.verts.ravel() for b in bodies]) if bodies else np.zeros(3))
    T = np.ascontiguousarray(np.concatenate([b.tris.ravel() for b in bodies]).astype(np.int32) if bodies
                             else np.zeros(3, np.int32))
    keep = (kind, nv, nt, V, T)
    return keep, [ctypes.c_int(len(bodies)), _p(kind), _p(nv), _p(nt), _p(V), _p(T)]


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
def classify(xf, yf, zf, bodies) -> np.ndarray:
    """uint8 flags[N] (x fastest): bit0 solid, bit1 closed ghost, bit2
    membrane ghost, bit3 pin, bits 4-6 cut +x/+y/+z links."""
    xf, yf, zf = _f64(xf), _f64(yf), _f64(zf)
    N = (len(xf) - 1) * (len(yf) - 1) * (len(zf) - 1)
    flags = np.zeros(N, dtype=np.uint8)
    keep, bargs = _bodies_args(bodies)
    rc = lib().orc_classify(*_grid_args(xf, yf, zf), *bargs, _p(flags))
    if rc != 0:
        raise ValueError("orc_classify failed: %d" % rc)
    return flags


@dataclass
class Stencils:
    gcell: np.ndarray     # closed ghost cells, idx order
    mcell: np.ndarray     # membrane ghost cells, idx order
    mg_of: np.ndarray     # int32[N], membrane ghost index or -1
    col: np.ndarray       # int32[(ng+nm), 8]
    w: np.ndarray         # float64[(ng+nm), 8]
    sG: np.ndarray
    dlb: np.ndarray       # dl - beta_BI
    rfl: np.ndarray       # bit0 fallback, bit1 derivative row, bit2 degenerate distance
    geo: np.ndarray       # [(ng+nm), 12]: BI, IP, n, dl, beta_BI, dist
    box: np.ndarray       # [(ng+nm), 3]

    @property
    def ng(self):
        return len(self.gcell)

    @property
    def nm(self):
        return len(self.mcell)

    @property
    def row_cell(self):
        return np.ascontiguousarray(np.concatenate([self.gcell, self.mcell]).astype(np.int32))


def ghost_lists(flags: np.ndarray):
    gcell = np.nonzero(flags & F_GHOST)[0].astype(np.int32)
    mcell = np.nonzero(flags & F_MGHOST)[0].astype(np.int32)
    mg_of = np.full(len(flags), -1, dtype=np.int32)
    mg_of[mcell] = np.arange(len(mcell), dtype=np.int32)
    return gcell, mcell, mg_of


def stencils(xf, yf, zf, bodies, flags, bc: str = "neumann") -> Stencils:
    """Ghost rows: Neumann rows of the pressure system (bc "neumann") or
    Dirichlet rows of the advection-diffusion step (bc "dirichlet")."""
    assert bc in ("neumann", "dirichlet")
    xf, yf, zf = _f64(xf), _f64(yf), _f64(zf)
    gcell, mcell, mg_of = ghost_lists(flags)
    rows = np.ascontiguousarray(np.concatenate([gcell, mcell]).astype(np.int32))
    mem = np.ascontiguousarray(np.concatenate([np.zeros(len(gcell), np.int32), np.ones(len(mcell), np.int32)]))
    nr = len(rows)
    col = np.full((max(nr, 1), 8), -1, dtype=np.int32)
    w = np.zeros((max(nr, 1), 8))
    sG = np.zeros(max(nr, 1))
    dlb = np.zeros(max(nr, 1))
    rfl = np.zeros(max(nr, 1), dtype=np.uint8)
    geo = np.zeros((max(nr, 1), 12))
    box = np.zeros((max(nr, 1), 3), dtype=np.int32)
    keep, bargs = _bodies_args(bodies)
    rc = lib().orc_ghost_stencils(*_grid_args(xf, yf, zf), *bargs, _p(flags), _p(mg_of), ctypes.c_int32(nr),
                                  _p(rows), _p(mem), ctypes.c_int(1 if bc == "dirichlet" else 0), _p(col), _p(w),
                                  _p(sG), _p(dlb), _p(rfl), _p(geo), _p(box))
    if rc != 0:
        raise ValueError("orc_ghost_stencils failed: %d" % rc)
    return Stencils(gcell, mcell, mg_of, col[:nr], w[:nr], sG[:nr], dlb[:nr], rfl[:nr], geo[:nr], box[:nr])


def closest_point(p, a, b, c) -> np.ndarray:
    """Closest point of triangle abc to p: the routine that picks each ghost
    row's boundary intercept (Sec. 2.5, module 2)."""
    q = np.zeros(3)
    args = [_f64(v) for v in (p, a, b, c)]
    lib().orc_closest_point(*[_p(v) for v in args], _p(q))
    return q


def _sys_args(xf, yf, zf, flags, st: Stencils):
    rows = st.row_cell
    col = np.ascontiguousarray(st.col, dtype=np.int32)
    w = np.ascontiguousarray(st.w)
    sG = np.ascontiguousarray(st.sG)
    keep = (rows, col, w, sG)
    return keep, [*_grid_args(xf, yf, zf), _p(flags), _p(st.mg_of), ctypes.c_int32(st.ng), ctypes.c_int32(st.nm),
                  _p(rows), _p(col), _p(w), _p(sG)]


def apply(xf, yf, zf, flags, st: Stencils, x) -> np.ndarray:
    """y = A x for the pinned operator (length N + nm)."""
    xf, yf, zf = _f64(xf), _f64(yf), _f64(zf)
    x = _f64(x)
    y = np.zeros_like(x)
    keep, a = _sys_args(xf, yf, zf, flags, st)
    lib().orc_apply(*a, _p(x), _p(y))
    return y


def assemble_rhs(xf, yf, zf, flags, st: Stencils, f, g=None) -> np.ndarray:
    xf, yf, zf = _f64(xf), _f64(yf), _f64(zf)
    N = len(flags)
    b = np.zeros(N + st.nm)
    f = _f64(f)
    gg = _f64(g) if g is not None else None
    rows = st.row_cell
    lib().orc_assemble_rhs(*_grid_args(xf, yf, zf), _p(flags), ctypes.c_int32(st.ng), ctypes.c_int32(st.nm),
                           _p(rows), _p(_f64(st.sG)), _p(_f64(st.dlb)), _p(f), _p(gg), _p(b))
    return b


def gauge(xf, yf, zf, flags, nm, x) -> np.ndarray:
    xf, yf, zf = _f64(xf), _f64(yf), _f64(zf)
    x = _f64(x).copy()
    lib().orc_gauge(*_grid_args(xf, yf, zf), _p(flags), ctypes.c_int32(nm), _p(x))
    return x


def vcycle(xf, yf, zf, flags, st: Stencils, b, nu1=2, nu2=2, ncs=32) -> np.ndarray:
    xf, yf, zf = _f64(xf), _f64(yf), _f64(zf)
    b = _f64(b)
    x = np.zeros_like(b)
    keep, a = _sys_args(xf, yf, zf, flags, st)
    lib().orc_vcycle(*a, ctypes.c_int(nu1), ctypes.c_int(nu2), ctypes.c_int(ncs), _p(b), _p(x))
    return x


def num_levels(nx, ny, nz) -> int:
    return lib().orc_num_levels(nx, ny, nz)


@dataclass
class SolveInfo:
    rc: int
    iters: int
    relres: float
    restarts: int
    hist: np.ndarray


def solve(xf, yf, zf, flags, st: Stencils, b, tol=1e-10, maxit=200, x0=None, nu1=2, nu2=2, ncs=32,
          precond=True):
    """MG-preconditioned BiCGSTAB on the pinned system; returns (x, info)."""
    xf, yf, zf = _f64(xf), _f64(yf), _f64(zf)
    b = _f64(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    info = np.zeros(3)
    hist = np.zeros(maxit + 1)
    keep, a = _sys_args(xf, yf, zf, flags, st)
    rc = lib().orc_solve(*a, _p(b), _p(x), ctypes.c_double(tol), ctypes.c_int(maxit), ctypes.c_int(nu1),
                         ctypes.c_int(nu2), ctypes.c_int(ncs), ctypes.c_int(1 if precond else 0), _p(info), _p(hist))
    it = int(info[0])
    return x, SolveInfo(rc, it, float(info[1]), int(info[2]), hist[:it].copy())


def srj_schedule(m: int, kmin: float = None) -> np.ndarray:
    """Relaxation factors of an m-sweep scheduled-relaxation Jacobi schedule.

    The amplification of a mode with eigenvalue k of D^-1 A (k in (0, 2] for
    this operator) after the schedule is prod_s (1 - w_s k); the factors that
    minimise its maximum over [kmin, 2] are the reciprocals of the roots of
    the degree-m Chebyshev polynomial mapped onto that interval.  They are
    applied smallest, largest, second smallest, ... so that partial products
    stay bounded.  kmin defaults to 16 / m^2 (smaller values make the largest
    factors grow like 1/kmin and the schedule sensitive to rounding).
    """
    if kmin is None:
        kmin = 16.0 / (m * m)
    j = np.arange(1, m + 1)
    kap = 0.5 * (2.0 + kmin) - 0.5 * (2.0 - kmin) * np.cos(np.pi * (2 * j - 1) / (2.0 * m))
    w = np.sort(1.0 / kap)
    order = []
    lo, hi = 0, m - 1
    while lo <= hi:
        order.append(lo)
        if hi != lo:
            order.append(hi)
        lo += 1
        hi -= 1
    return np.ascontiguousarray(w[order])


def srj(xf, yf, zf, flags, st: Stencils, b, omega, pinned=True, shift=True) -> np.ndarray:
    """len(omega) SRJ sweeps from zero on A x = b (optionally shifted like the V-cycle output)."""
    xf, yf, zf = _f64(xf), _f64(yf), _f64(zf)
    b = _f64(b)
    om = _f64(omega)
    x = np.zeros_like(b)
    keep, a = _sys_args(xf, yf, zf, flags, st)
    lib().orc_srj(*a, ctypes.c_int(1 if pinned else 0), ctypes.c_int(1 if shift else 0), ctypes.c_int(len(om)),
                  _p(om), _p(b), _p(x))
    return x


def solve_srj(xf, yf, zf, flags, st: Stencils, b, omega, tol=1e-10, maxit=500, x0=None):
    """SRJ-preconditioned BiCGSTAB on the pinned system; returns (x, info)."""
    xf, yf, zf = _f64(xf), _f64(yf), _f64(zf)
    b = _f64(b)
    om = _f64(omega)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    info = np.zeros(3)
    hist = np.zeros(maxit + 1)
    keep, a = _sys_args(xf, yf, zf, flags, st)
    rc = lib().orc_solve_srj(*a, _p(b), _p(x), ctypes.c_double(tol), ctypes.c_int(maxit), ctypes.c_int(len(om)),
                             _p(om), _p(info), _p(hist))
    it = int(info[0])
    return x, SolveInfo(rc, it, float(info[1]), int(info[2]), hist[:it].copy())


# --------------------------------------------------------------------------
@dataclass
class Setup:
    xf: np.ndarray
    yf: np.ndarray
    zf: np.ndarray
    flags: np.ndarray
    st: Stencils

    @property
    def N(self):
        return len(self.flags)


def setup(xf, yf, zf, bodies) -> Setup:
    flags = classify(xf, yf, zf, bodies)
    st = stencils(xf, yf, zf, bodies, flags)
    return Setup(_f64(xf), _f64(yf), _f64(zf), flags, st)


def solve_problem(S: Setup, f, tol=1e-13, maxit=300, g=None):
    """Full PPE pipeline: RHS assembly, pinned MG-BiCGSTAB, gauge."""
    b = assemble_rhs(S.xf, S.yf, S.zf, S.flags, S.st, f, g)
    x, info = solve(S.xf, S.yf, S.zf, S.flags, S.st, b, tol=tol, maxit=maxit)
    xg = gauge(S.xf, S.yf, S.zf, S.flags, S.st.nm, x)
    return xg, b, x, info


def threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(lib().orc_threads())


def fill_fresh(nx, ny, nz, flags_old, flags_new, x) -> Tuple[np.ndarray, int]:
    """Initial values of fresh cells for a moving-body step (the time loop of
    Sec. 2.4 re-classifies the grid every step): a cell that is fluid under
    flags_new and was solid under flags_old has no pressure history and takes
    the mean of its face neighbours that are fluid under both, added in the
    order -x, +x, -y, +y, -z, +z; with no such neighbour it keeps its value.
    Returns (new x, fresh-cell count); a plain loop over the fresh cells."""
    fo = np.asarray(flags_old, dtype=np.uint8)
    fn = np.asarray(flags_new, dtype=np.uint8)
    out = np.array(x, dtype=np.float64, copy=True)
    fresh = np.nonzero(((fn & F_SOLID) == 0) & ((fo & F_SOLID) != 0))[0]
    fluid_both = ((fn & F_SOLID) == 0) & ((fo & F_SOLID) == 0)
    for p in fresh:
        p = int(p)
        i, j, k = p % nx, (p // nx) % ny, p // (nx * ny)
        acc, cnt = 0.0, 0
        for (d, n_d, c_d, stride) in ((0, nx, i, 1), (1, ny, j, nx), (2, nz, k, nx * ny)):
            for sg in (-1, 1):
                if 0 <= c_d + sg < n_d:
                    q = p + sg * stride
                    if fluid_both[q]:
                        acc += float(x[q])
                        cnt += 1
        if cnt:
            out[p] = acc / cnt
    return out, len(fresh)


# --------------------------------------------------------------------------
# Surface loads (Sec. 2.3.1, Eq. fext, pressure part)
def _trilinear(centres, field3, flags3, pts):
    """Trilinear interpolation of a cell-centred field at points: the box of
    the eight centres around each point (clamped to the outermost centres),
    nodes in solid non-ghost cells dropped and the remaining weights
    renormalised; (values, number of points with no valid node)."""
    n = [len(c) for c in centres]
    idx, frac = [], []
    for d in range(3):
        c = centres[d]
        i0 = np.clip(np.searchsorted(c, pts[:, d], side="right") - 1, 0, n[d] - 2)
        t = (pts[:, d] - c[i0]) / (c[i0 + 1] - c[i0])
        idx.append(i0)
        frac.append(np.clip(t, 0.0, 1.0))
    num = np.zeros(len(pts))
    den = np.zeros(len(pts))
    for q in range(8):
        o = [(q >> d) & 1 for d in range(3)]
        w = np.ones(len(pts))
        for d in range(3):
            w = w * (frac[d] if o[d] else 1.0 - frac[d])
        ii, jj, kk = idx[0] + o[0], idx[1] + o[1], idx[2] + o[2]
        f = flags3[kk, jj, ii]
        ok = ((f & F_SOLID) == 0) | ((f & F_GHOST) != 0)
        w = np.where(ok, w, 0.0)
        num = num + w * field3[kk, jj, ii]
        den = den + w
    val = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
    return val, int(np.sum(den == 0))


def surface_forces(xf, yf, zf, bodies, flags, p):
    """Nodal pressure forces on every body (plain definition, not tuned).

    Per triangle j (vertices in the body's order): centroid c, area A, unit
    normal n = (v1 - v0) x (v2 - v0) / |.|, and probe distance d = 2 max of
    the widths of the cell that contains c.  p+ is the pressure interpolated
    at c + d n; for a membrane p- at c - d n and dp = p+ - p-, for a closed
    body (outward normals, fluid outside) dp = p+.  Each of the triangle's
    three nodes receives -(1/3) dp n A (the area rule of Eq. fext without
    the shear term).  Returns (list of (n_vert, 3) forces per body, per-body
    dp arrays, number of probes with no valid interpolation node)."""
    xf, yf, zf = _f64(xf), _f64(yf), _f64(zf)
    faces = [xf, yf, zf]
    centres = [0.5 * (f[1:] + f[:-1]) for f in faces]
    widths = [np.diff(f) for f in faces]
    n = [len(c) for c in centres]
    f3 = np.asarray(flags, dtype=np.uint8).reshape(n[2], n[1], n[0])
    p3 = np.asarray(p, dtype=np.float64)[: n[0] * n[1] * n[2]].reshape(n[2], n[1], n[0])
    forces, dps, lost = [], [], 0
    for b in bodies:
        v = np.asarray(b.verts, dtype=np.float64)
        t = np.asarray(b.tris, dtype=np.int64)
        a, bb, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
        cen = (a + bb + c) / 3.0
        cr = np.cross(bb - a, c - a)
        nrm = np.linalg.norm(cr, axis=1)
        un = cr / nrm[:, None]
        area = 0.5 * nrm
        h = np.zeros(len(t))
        for d in range(3):
            k = np.clip(np.searchsorted(faces[d], cen[:, d], side="right") - 1, 0, n[d] - 1)
            h = np.maximum(h, widths[d][k])
        dist = 2.0 * h
        pp, l1 = _trilinear(centres, p3, f3, cen + dist[:, None] * un)
        lost += l1
        if b.kind == 1:
            pm, l2 = _trilinear(centres, p3, f3, cen - dist[:, None] * un)
            lost += l2
            dp = pp - pm
        else:
            dp = pp
        contrib = -(dp * area)[:, None] * un / 3.0
        F = np.zeros((len(v), 3))
        for m in range(3):
            np.add.at(F, t[:, m], contrib)
        forces.append(F)
        dps.append(dp)
    return forces, dps, lost


# --------------------------------------------------------------------------
# Advection-diffusion step (Sec. 2.1: SRJ for the momentum equations)
def ad_schedule(m: int, beta: float, dg_max: float) -> np.ndarray:
    """Relaxation factors of an m-sweep SRJ cycle for H = I - beta L: the
    eigenvalues of D^-1 H lie in [a, 2 - a], a = 1 / (1 + beta dg_max), and
    the factors are the reciprocals of the degree-m Chebyshev roots on that
    interval, applied smallest, largest, second smallest, ..."""
    a = 1.0 / (1.0 + beta * dg_max)
    b = 2.0 - a
    j = np.arange(1, m + 1)
    kap = 0.5 * (a + b) - 0.5 * (b - a) * np.cos(np.pi * (2 * j - 1) / (2.0 * m))
    w = np.sort(1.0 / kap)
    order = []
    lo, hi = 0, m - 1
    while lo <= hi:
        order.append(lo)
        if hi != lo:
            order.append(hi)
        lo += 1
        hi -= 1
    return np.ascontiguousarray(w[order])


def max_cell_scale(xf, yf, zf) -> float:
    """Largest diagonal sum of the 7-point coefficients over the grid."""
    parts = []
    for f in (xf, yf, zf):
        f = _f64(f)
        c = 0.5 * (f[1:] + f[:-1])
        w = np.diff(f)
        n = len(w)
        cp = np.zeros(n)
        cm = np.zeros(n)
        cp[:-1] = 1.0 / (w[:-1] * (c[1:] - c[:-1]))
        cm[1:] = 1.0 / (w[1:] * (c[1:] - c[:-1]))
        parts.append((cp + cm).max())
    return float(sum(parts))


def ad_apply(xf, yf, zf, flags, st: Stencils, beta, x) -> np.ndarray:
    """y = H x for the advection-diffusion step (st: Dirichlet rows)."""
    xf, yf, zf = _f64(xf), _f64(yf), _f64(zf)
    x = _f64(x)
    y = np.zeros_like(x)
    keep, a = _sys_args(xf, yf, zf, flags, st)
    lib().orc_ad_apply(*a, ctypes.c_double(beta), _p(x), _p(y))
    return y


def ad_rhs(xf, yf, zf, flags, st: Stencils, f, g=None) -> np.ndarray:
    """Right-hand side of the step: f on fluid cells, sG dlb g on ghost rows
    (g: wall velocity at each row's BI; None for a wall at rest), 0 on solid cells."""
    N = len(flags)
    b = np.zeros(N + st.nm)
    fl = np.asarray(flags)
    b[:N] = np.where((fl & F_SOLID) == 0, _f64(f)[:N], 0.0)
    rows = np.concatenate([st.gcell.astype(np.int64), N + np.arange(st.nm)])
    b[rows] = 0.0 if g is None else st.sG * st.dlb * _f64(g)
    return b


def ad_solve(xf, yf, zf, flags, st: Stencils, beta, rhs, omega, tol=1e-10, maxcyc=1000, x0=None):
    """SRJ cycles on H u = rhs; returns (u, cycles, relative residual, rc)."""
    xf, yf, zf = _f64(xf), _f64(yf), _f64(zf)
    rhs = _f64(rhs)
    om = _f64(omega)
    x = np.zeros_like(rhs) if x0 is None else _f64(x0).copy()
    info = np.zeros(2)
    keep, a = _sys_args(xf, yf, zf, flags, st)
    rc = lib().orc_ad_solve(*a, ctypes.c_double(beta), _p(rhs), _p(x), ctypes.c_double(tol), ctypes.c_int(maxcyc),
                            ctypes.c_int(len(om)), _p(om), _p(info))
    return x, int(info[0]), float(info[1]), int(rc)
