"""Seeded synthetic inputs for the ghost-cell pressure-Poisson solve.

This module only *generates inputs*: grid face coordinates, triangulated
bodies and right-hand-side fields.  It holds none of the solver's arithmetic
(no classification, no stencils, no projection of the RHS, no operator), so
both the FP64 CPU oracle and the HIP path can be fed the identical arrays it
produces.

The paper (Sec. 2.1) solves the pressure Poisson equation of a fractional-step
method with second-order finite differences on a non-conformal Cartesian grid,
stretched away from a uniform core (Sec. 3.2), around triangulated bodies that
are either closed or zero-thickness membranes (Sec. 2.3, 2.5).  It measures on
its own wing and bat setups, which are not available; the workloads below are
synthetic stand-ins with the grid sizes, stretching, body kinds and triangle
counts of the benchmark configurations.

Seeds: geometry draws use ``numpy.random.default_rng(s)``, RHS draws use
``default_rng(s + 1000)`` (repetition r adds 10000*r to both).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

KIND_CLOSED = 0
KIND_MEMBRANE = 1


# --------------------------------------------------------------------------
# grids
# --------------------------------------------------------------------------
def uniform_faces(n: int, length: float = 1.0) -> np.ndarray:
    """Face coordinates of n equal cells on [0, length]."""
    i = np.arange(n + 1, dtype=np.float64)
    return (i / float(n)) * length


def _tanh_faces(n: int, beta: float) -> np.ndarray:
    i = np.arange(n + 1, dtype=np.float64)
    s = (2.0 * i / n - 1.0) * math.tanh(beta)
    f = 0.5 + np.arctanh(s) / (2.0 * beta)
    f[0] = 0.0
    f[-1] = 1.0
    return f


def _max_adjacent_ratio(f: np.ndarray) -> float:
    w = np.diff(f)
    r = w[1:] / w[:-1]
    return float(max(r.max(), (1.0 / r).max()))


def stretched_faces(n: int, ratio: float = 1.05, length: float = 1.0) -> Tuple[np.ndarray, float]:
    """Two-sided tanh stretching that clusters cells at the centre.

    Faces are 0.5 + atanh((2i/n - 1) tanh(beta)) / (2 beta), with beta found by
    200 bisection steps so that the largest ratio of adjacent cell widths
    equals ``ratio``.  Returns (faces scaled to [0, length], beta).
    """
    lo, hi = 1e-6, 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _max_adjacent_ratio(_tanh_faces(n, mid)) > ratio:
            hi = mid
        else:
            lo = mid
    beta = 0.5 * (lo + hi)
    f = _tanh_faces(n, beta) * length
    f[0] = 0.0
    f[-1] = length
    return f, beta


# --------------------------------------------------------------------------
# bodies
# --------------------------------------------------------------------------
@dataclass
class Body:
    verts: np.ndarray          # (nv, 3) float64
    tris: np.ndarray           # (nt, 3) int32
    kind: int = KIND_CLOSED    # 0 closed (outward oriented), 1 membrane

    def __post_init__(self):
        self.verts = np.ascontiguousarray(self.verts, dtype=np.float64)
        self.tris = np.ascontiguousarray(self.tris, dtype=np.int32)


def _icosahedron() -> Tuple[np.ndarray, np.ndarray]:
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    v = []
    for a in (-1.0, 1.0):
        for b in (-phi, phi):
            v.append((0.0, a, b))
            v.append((a, b, 0.0))
            v.append((b, 0.0, a))
    v = np.array(v, dtype=np.float64)
    faces = []
    n = len(v)
    for a in range(n):
        for b in range(a + 1, n):
            if abs(np.sum((v[a] - v[b]) ** 2) - 4.0) > 1e-9:
                continue
            for c in range(b + 1, n):
                if abs(np.sum((v[a] - v[c]) ** 2) - 4.0) > 1e-9:
                    continue
                if abs(np.sum((v[b] - v[c]) ** 2) - 4.0) > 1e-9:
                    continue
                nrm = np.cross(v[b] - v[a], v[c] - v[a])
                if np.dot(nrm, v[a] + v[b] + v[c]) < 0:
                    faces.append((a, c, b))
                else:
                    faces.append((a, b, c))
    assert len(faces) == 20
    return v, np.array(faces, dtype=np.int64)


def geodesic_sphere(freq: int = 10) -> Tuple[np.ndarray, np.ndarray]:
    """Class-I geodesic icosahedron on the unit sphere: 20 f^2 triangles.

    Every icosahedron face is split into f x f sub-triangles; shared points
    are merged through exact integer barycentric keys, then projected to the
    unit sphere.  Orientation is outward.  freq=10 gives 2000 triangles and
    1002 vertices.
    """
    base, faces = _icosahedron()
    keys = {}
    verts = []
    tris = []

    def vid(weights):
        key = tuple(sorted((int(c), int(w)) for c, w in weights if w != 0))
        if key not in keys:
            p = np.zeros(3)
            for c, w in key:
                p = p + w * base[c]
            p = p / np.linalg.norm(p)
            keys[key] = len(verts)
            verts.append(p)
        return keys[key]

    f = freq
    for (a, b, c) in faces:
        def P(i, j):
            return vid(((a, f - i - j), (b, i), (c, j)))
        for i in range(f):
            for j in range(f - i):
                tris.append((P(i, j), P(i + 1, j), P(i, j + 1)))
                if i + j < f - 1:
                    tris.append((P(i + 1, j), P(i + 1, j + 1), P(i, j + 1)))
    return np.array(verts), np.array(tris, dtype=np.int32)


def sphere(center, radius: float, freq: int = 10) -> Body:
    v, t = geodesic_sphere(freq)
    return Body(v * radius + np.asarray(center, dtype=np.float64), t, KIND_CLOSED)


def rotation_zyx(alpha: float, beta: float, gamma: float) -> np.ndarray:
    """R = Rz(gamma) Ry(beta) Rx(alpha)."""
    ca, sa = math.cos(alpha), math.sin(alpha)
    cb, sb = math.cos(beta), math.sin(beta)
    cg, sg = math.cos(gamma), math.sin(gamma)
    rx = np.array([[1, 0, 0], [0, ca, -sa], [0, sa, ca]])
    ry = np.array([[cb, 0, sb], [0, 1, 0], [-sb, 0, cb]])
    rz = np.array([[cg, -sg, 0], [sg, cg, 0], [0, 0, 1]])
    return rz @ ry @ rx


def ellipsoid(center, semi_axes, rot: np.ndarray, freq: int = 10) -> Body:
    v, t = geodesic_sphere(freq)
    v = (v * np.asarray(semi_axes, dtype=np.float64)) @ rot.T
    return Body(v + np.asarray(center, dtype=np.float64), t, KIND_CLOSED)


def box(lo, hi) -> Body:
    """Axis-aligned closed box, 12 outward-oriented triangles."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    v = np.array([[lo[0] if (c & 1) == 0 else hi[0],
                   lo[1] if (c & 2) == 0 else hi[1],
                   lo[2] if (c & 4) == 0 else hi[2]] for c in range(8)])
    quads = [(0, 2, 6, 4), (1, 5, 7, 3),   # -x, +x
             (0, 4, 5, 1), (2, 3, 7, 6),   # -y, +y
             (0, 1, 3, 2), (4, 6, 7, 5)]   # -z, +z
    tris = []
    for a, b, c, d in quads:
        tris.append((a, b, c))
        tris.append((a, c, d))
    t = np.array(tris, dtype=np.int32)
    ctr = 0.5 * (lo + hi)
    for k in range(len(t)):
        p = v[t[k]]
        nrm = np.cross(p[1] - p[0], p[2] - p[0])
        if np.dot(nrm, p.mean(0) - ctr) < 0:
            t[k] = t[k][[0, 2, 1]]
    return Body(v, t, KIND_CLOSED)


def plate(center, chord: float, span: float, nc: int, ns: int,
          camber: float = 0.0, phase: float = 0.0) -> Body:
    """Zero-thickness rectangular membrane, chord along x and span along y.

    (nc x ns) quads, each split along its (i,j)-(i+1,j+1) diagonal, so
    2 nc ns triangles; camber w = camber * sin(pi * xi + phase) with xi in
    [0, 1] the chordwise coordinate.
    """
    cx, cy, cz = center
    xi = np.arange(nc + 1) / nc
    eta = np.arange(ns + 1) / ns
    X, Y = np.meshgrid(cx - 0.5 * chord + chord * xi, cy - 0.5 * span + span * eta, indexing="ij")
    Z = cz + camber * np.sin(math.pi * xi + phase)[:, None] * np.ones_like(eta)[None, :]
    v = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    tris = []
    for i in range(nc):
        for j in range(ns):
            a = i * (ns + 1) + j
            b = (i + 1) * (ns + 1) + j
            c = (i + 1) * (ns + 1) + j + 1
            d = i * (ns + 1) + j + 1
            tris.append((a, b, c))
            tris.append((a, c, d))
    return Body(v, np.array(tris, dtype=np.int32), KIND_MEMBRANE)


def random_spheres(rng: np.random.Generator, count: int, rmin: float, rmax: float,
                   gap: float = 0.02, freq: int = 10) -> List[Body]:
    out = []
    placed = []
    while len(placed) < count:
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(r + gap, 1.0 - r - gap, size=3)
        if all(np.linalg.norm(c - c2) >= r + r2 + gap for c2, r2 in placed):
            placed.append((c, r))
    for c, r in placed:
        out.append(sphere(c, r, freq))
    return out


# --------------------------------------------------------------------------
# right-hand sides (inputs; each side projects them itself)
# --------------------------------------------------------------------------
def centres(f: np.ndarray) -> np.ndarray:
    return 0.5 * (f[:-1] + f[1:])


def manufactured_rhs(xf, yf, zf) -> np.ndarray:
    """f = -3 pi^2 cos(pi x) cos(pi y) cos(pi z) at cell centres, x fastest."""
    x, y, z = centres(xf), centres(yf), centres(zf)
    p = np.cos(math.pi * z)[:, None, None] * np.cos(math.pi * y)[None, :, None] * np.cos(math.pi * x)[None, None, :]
    return np.ascontiguousarray((-3.0 * math.pi ** 2 * p).ravel())


def manufactured_p(xf, yf, zf) -> np.ndarray:
    x, y, z = centres(xf), centres(yf), centres(zf)
    p = np.cos(math.pi * z)[:, None, None] * np.cos(math.pi * y)[None, :, None] * np.cos(math.pi * x)[None, None, :]
    return np.ascontiguousarray(p.ravel())


def noise_rhs(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def bumps_rhs(xf, yf, zf, seed: int, k: int = 16) -> np.ndarray:
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1, 1, k)
    c = rng.uniform(0.1, 0.9, (k, 3))
    s = rng.uniform(0.03, 0.1, k)
    x, y, z = centres(xf), centres(yf), centres(zf)
    out = np.zeros((len(z), len(y), len(x)))
    for m in range(k):
        gx = np.exp(-(x - c[m, 0]) ** 2 / (2 * s[m] ** 2))
        gy = np.exp(-(y - c[m, 1]) ** 2 / (2 * s[m] ** 2))
        gz = np.exp(-(z - c[m, 2]) ** 2 / (2 * s[m] ** 2))
        out += a[m] * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    return np.ascontiguousarray(out.ravel())


# --------------------------------------------------------------------------
# benchmark configurations
# --------------------------------------------------------------------------
@dataclass
class Problem:
    name: str
    xf: np.ndarray
    yf: np.ndarray
    zf: np.ndarray
    bodies: List[Body]
    f: np.ndarray = None          # RHS input, length nx*ny*nz, x fastest
    tol: float = 1e-10
    mixed: bool = False
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return (len(self.xf) - 1, len(self.yf) - 1, len(self.zf) - 1)

    @property
    def npts(self):
        nx, ny, nz = self.shape
        return nx * ny * nz


def sphere_case(n: int = 32, rhs: bool = True) -> Problem:
    """32^3 uniform unit cube, sphere r=0.25 centred, 2000-triangle mesh,
    manufactured RHS, tolerance 1e-10, FP64."""
    f = uniform_faces(n)
    p = Problem("sphere%d" % n, f, f.copy(), f.copy(), [sphere((0.5, 0.5, 0.5), 0.25)], tol=1e-10)
    if rhs:
        p.f = manufactured_rhs(p.xf, p.yf, p.zf)
    return p


def sphere_ellipsoid_case(n: int = 256, seed: int = 2, rhs: bool = True) -> Problem:
    """Tanh-stretched grid (ratio 1.05), sphere r=0.2 at (0.35,.5,.5) and an
    ellipsoid of full axes 0.3/0.1/0.1 at (0.72,.5,.5) rotated by seeded
    random angles; uniform noise RHS; tolerance 1e-10."""
    f, beta = stretched_faces(n)
    rng = np.random.default_rng(seed)
    al, be, ga = rng.uniform(0, 2 * math.pi, 3)
    bodies = [sphere((0.35, 0.5, 0.5), 0.2),
              ellipsoid((0.72, 0.5, 0.5), (0.15, 0.05, 0.05), rotation_zyx(al, be, ga))]
    p = Problem("sphere_ellipsoid%d" % n, f, f.copy(), f.copy(), bodies, tol=1e-10,
                meta={"beta": beta, "angles": (al, be, ga)})
    if rhs:
        p.f = noise_rhs(p.npts, seed + 1000)
    return p


def membrane_case(n: int = 512, seed: int = 3, rhs: bool = True, nc: int = 80, ns: int = 250) -> Problem:
    """Tanh-stretched grid, cambered zero-thickness plate (chord 0.2, span
    0.6, camber 0.05 sin(pi xi + phase), 2 nc ns triangles), noise RHS,
    tolerance 1e-8, mixed precision."""
    f, beta = stretched_faces(n)
    rng = np.random.default_rng(seed)
    phase = rng.uniform(0, 2 * math.pi)
    bodies = [plate((0.5, 0.5, 0.5), 0.2, 0.6, nc, ns, 0.05, phase)]
    p = Problem("membrane%d" % n, f, f.copy(), f.copy(), bodies, tol=1e-8, mixed=True,
                meta={"beta": beta, "phase": phase})
    if rhs:
        p.f = noise_rhs(p.npts, seed + 1000)
    return p


def spheres_case(n: int = 1024, seed: int = 4, count: int = 20, rhs: bool = True) -> Problem:
    """Uniform grid, ``count`` seeded spheres r in [0.02, 0.08], sum of 16
    Gaussian bumps as RHS, tolerance 1e-8."""
    f = uniform_faces(n)
    rng = np.random.default_rng(seed)
    bodies = random_spheres(rng, count, 0.02, 0.08)
    p = Problem("spheres%d" % n, f, f.copy(), f.copy(), bodies, tol=1e-8)
    if rhs:
        p.f = bumps_rhs(p.xf, p.yf, p.zf, seed + 1000)
    return p


def flapping_case(n: int = 512, step: int = 0, period: int = 1600, seed: int = 5, rhs: bool = True,
                  nc: int = 60, ns: int = 120) -> Problem:
    """One time step of a moving-body sequence on the tanh-stretched grid: a
    zero-thickness plate (chord 0.2 along x, span 0.4 along y from its root
    at y = 0.3, mild camber) flapping about the x-parallel line through its
    root with amplitude 0.5 rad, and a sphere (r 0.08, centre x = 0.3)
    heaving in z with amplitude 0.1; both follow sin(2 pi step / period).
    At 512^3 and period 1600 the plate tip moves at most 0.7 of the finest
    cell per step and the sphere 0.4.  Noise RHS seeded by ``seed`` only, so
    consecutive steps share f."""
    f, beta = stretched_faces(n)
    ph = 2 * math.pi * step / period
    th = 0.5 * math.sin(ph)
    root_y, cz = 0.3, 0.5
    body = plate((0.6, root_y + 0.2, cz), 0.2, 0.4, nc, ns, 0.02, 0.0)
    v = body.verts.copy()
    dy, dz = v[:, 1] - root_y, v[:, 2] - cz
    v[:, 1] = root_y + dy * math.cos(th) - dz * math.sin(th)
    v[:, 2] = cz + dy * math.sin(th) + dz * math.cos(th)
    bodies = [sphere((0.3, 0.5, 0.5 + 0.1 * math.sin(ph)), 0.08), Body(v, body.tris, KIND_MEMBRANE)]
    p = Problem("flapping%d_step%d" % (n, step), f, f.copy(), f.copy(), bodies, tol=1e-8, mixed=True,
                meta={"beta": beta, "theta": th, "step": step, "period": period})
    if rhs:
        p.f = noise_rhs(p.npts, seed + 2000)
    return p


def serving_request(rng: np.random.Generator, emin: int = 64, emax: int = 384) -> Problem:
    """One request of the serving stream: edge log-uniform in [emin, emax]
    rounded to a multiple of 32, cube or 2:1:1 box, 1-4 bodies."""
    e = int(32 * round(math.exp(rng.uniform(math.log(emin), math.log(emax))) / 32))
    e = max(e, 32)
    cube = rng.uniform() < 0.5
    if cube:
        xf = uniform_faces(e); yf = uniform_faces(e); zf = uniform_faces(e)
        ext = np.array([1.0, 1.0, 1.0])
    else:
        xf = uniform_faces(e); yf = uniform_faces(e // 2, 0.5); zf = uniform_faces(e // 2, 0.5)
        ext = np.array([1.0, 0.5, 0.5])
    h = 1.0 / e
    nb = int(rng.integers(1, 5))
    bodies: List[Body] = []
    boxes = []
    tries = 0
    while len(bodies) < nb and tries < 200:
        tries += 1
        kind = int(rng.integers(0, 3))
        if kind == 0:
            r = rng.uniform(0.05, 0.15) * min(1.0, ext.min() / 0.5)
            half = np.array([r, r, r])
        elif kind == 1:
            s = rng.uniform(0.5, 1.0)
            half = np.array([0.15, 0.15, 0.15]) * s
        else:
            chord = rng.uniform(0.1, 0.2)
            half = np.array([0.5 * chord, 1.5 * chord, 0.06])
        if np.any(2 * half + 0.04 >= ext):
            continue
        c = np.array([rng.uniform(half[d] + 0.02, ext[d] - half[d] - 0.02) for d in range(3)])
        if any(np.all(np.abs(c - c2) < half + h2 + 0.02) for c2, h2 in boxes):
            continue
        boxes.append((c, half))
        if kind == 0:
            bodies.append(sphere(c, half[0]))
        elif kind == 1:
            al, be, ga = rng.uniform(0, 2 * math.pi, 3)
            bodies.append(ellipsoid(c, (0.15 * s, 0.05 * s, 0.05 * s), rotation_zyx(al, be, ga)))
        else:
            nc = max(2, int(round(chord / h)))
            ns = max(2, int(round(3 * chord / h)))
            while 2 * nc * ns > 40000:
                nc = max(2, nc - 1); ns = max(2, int(round(3 * nc)))
            bodies.append(plate(c, chord, 3 * chord, nc, ns, 0.05 * chord / 0.2, rng.uniform(0, 2 * math.pi)))
    p = Problem("serve%dx%dx%d" % (len(xf) - 1, len(yf) - 1, len(zf) - 1), xf, yf, zf, bodies, tol=1e-8, mixed=True)
    p.f = rng.uniform(-1.0, 1.0, p.npts)
    return p


CONFIGS = {
    "c1": sphere_case,
    "c2": sphere_ellipsoid_case,
    "c3": membrane_case,
    "c4": spheres_case,
}
