"""Independent Python cross-checks used to pin the oracle.

Nothing here shares code with the oracle's C file or with the HIP library:
  * brute-force ray parity with exact integers and Fractions (intercepts
    computed explicitly from the plane equation),
  * a scipy.sparse assembler of the pinned ghost-cell system,
  * closed-form solutions of the discrete Neumann problem,
  * closest points on triangles by plane projection and barycentric
    coordinates, else the nearest clamped edge projection (a construction
    unlike the Voronoi-region walk the oracle and the library use).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import scipy.sparse as sp


def centres(f):
    f = np.asarray(f, dtype=np.float64)
    return 0.5 * (f[:-1] + f[1:])


def lattice(xf, yf, zf):
    """Lattice of the classification: 2^16 units over the longest edge,
    q(v) = floor((v - lo) * S + 0.5) (Python floats: IEEE, no contraction)."""
    L = max(xf[-1] - xf[0], yf[-1] - yf[0], zf[-1] - zf[0])
    S = 65536.0 / L
    lo = (float(xf[0]), float(yf[0]), float(zf[0]))

    def q(v, d):
        return int(math.floor((float(v) - lo[d]) * S + 0.5))
    return q


def _side(U, V, P, u, w):
    """Sign of the edge function at P moved by (+e, +e^2) in (u, w)."""
    e0 = (V[u] - U[u]) * (P[w] - U[w]) - (V[w] - U[w]) * (P[u] - U[u])
    if e0 != 0:
        return e0 > 0
    e1 = -(V[w] - U[w])          # coefficient of e
    if e1 != 0:
        return e1 > 0
    return (V[u] - U[u]) > 0     # coefficient of e^2


def _tri_lattice(body, q):
    return [[tuple(q(body.verts[t[m]][d], d) for d in range(3)) for m in range(3)] for t in body.tris]


def brute_flags(xf, yf, zf, bodies):
    """Solid bits and cut-link bits by explicit exact intercepts.

    Returns (solid[N] bool, cut[3][N] bool) with cut[d][cell] the link
    cell -> cell + e_d (before clearing links that touch solid cells)."""
    q = lattice(xf, yf, zf)
    n = (len(xf) - 1, len(yf) - 1, len(zf) - 1)
    cs = [centres(xf), centres(yf), centres(zf)]
    qc = [[q(c, d) for c in cs[d]] for d in range(3)]
    N = n[0] * n[1] * n[2]
    solid = np.zeros(N, bool)
    cut = [np.zeros(N, bool) for _ in range(3)]

    def idx(c):
        return c[0] + n[0] * (c[1] + n[1] * c[2])

    for body in bodies:
        T = _tri_lattice(body, q)
        dirs = [0] if body.kind == 0 else [0, 1, 2]
        par = np.zeros(N, np.int64)
        for d in dirs:
            u, w = (d + 1) % 3, (d + 2) % 3
            for A, B, C in T:
                # plane normal
                e1 = [B[i] - A[i] for i in range(3)]
                e2 = [C[i] - A[i] for i in range(3)]
                Nn = [e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]]
                if Nn[d] == 0:
                    continue
                P0, P1, P2 = (A, B, C) if Nn[d] > 0 else (A, C, B)
                us = [A[u], B[u], C[u]]
                ws = [A[w], B[w], C[w]]
                for ia in range(n[u]):
                    if not (min(us) <= qc[u][ia] <= max(us)):
                        continue
                    for ib in range(n[w]):
                        if not (min(ws) <= qc[w][ib] <= max(ws)):
                            continue
                        P = [0, 0, 0]
                        P[u] = qc[u][ia]
                        P[w] = qc[w][ib]
                        if not (_side(P0, P1, P, u, w) and _side(P1, P2, P, u, w) and _side(P2, P0, P, u, w)):
                            continue
                        # intercept along d: Nn . (X - A) = 0
                        rest = Nn[u] * (P[u] - A[u]) + Nn[w] * (P[w] - A[w])
                        xs = Fraction(A[d]) - Fraction(rest, Nn[d])
                        beyond = [Fraction(qc[d][i]) > xs for i in range(n[d])]
                        for i in range(n[d]):
                            c = [0, 0, 0]
                            c[d] = i
                            c[u] = ia
                            c[w] = ib
                            if body.kind == 0:
                                if beyond[i]:
                                    par[idx(c)] += 1
                            elif i + 1 < n[d] and beyond[i] != beyond[i + 1]:
                                cut[d][idx(c)] ^= True
        if body.kind == 0:
            solid |= (par % 2) == 1
    return solid, cut


def expected_flags(xf, yf, zf, solid, cut):
    """Flag byte from solid/cut bits, written out directly from the rules."""
    n = (len(xf) - 1, len(yf) - 1, len(zf) - 1)
    S = solid.reshape(n[2], n[1], n[0])
    fl = np.zeros((n[2], n[1], n[0]), np.uint8)
    fl[S] |= 1
    # closed ghosts
    g = np.zeros_like(S)
    for ax in range(3):
        a = 2 - ax
        fluid = ~S
        sh = np.zeros_like(S)
        sl = [slice(None)] * 3
        sl2 = [slice(None)] * 3
        sl[a] = slice(1, None)
        sl2[a] = slice(None, -1)
        sh[tuple(sl)] |= fluid[tuple(sl2)]
        sh[tuple(sl2)] |= fluid[tuple(sl)]
        g |= sh
    fl[S & g] |= 2
    mg = np.zeros_like(S)
    for d in range(3):
        a = 2 - d
        C = cut[d].reshape(n[2], n[1], n[0]).copy()
        last = [slice(None)] * 3
        last[a] = -1
        C[tuple(last)] = False
        nb = np.zeros_like(S)
        sl = [slice(None)] * 3
        sl2 = [slice(None)] * 3
        sl[a] = slice(None, -1)
        sl2[a] = slice(1, None)
        nb[tuple(sl)] = S[tuple(sl2)]
        C &= ~S & ~nb
        fl[C] |= np.uint8(16 << d)
        mg |= C
        up = np.zeros_like(S)
        up[tuple(sl2)] = C[tuple(sl)]
        mg |= up
    fl[mg] |= 4
    flat = fl.ravel()
    cand = np.nonzero((flat & 5) == 0)[0]
    flat[cand[0]] |= 8
    return flat


# --------------------------------------------------------------------------
def assemble(xf, yf, zf, flags, st, pinned=True):
    """scipy.sparse CSR of the pinned operator over N + nm unknowns, written
    row by row from the definitions (fluid FV rows, ghost rows, pin)."""
    nx, ny, nz = len(xf) - 1, len(yf) - 1, len(zf) - 1
    N = nx * ny * nz
    nm = len(st.mcell)
    cs = [centres(xf), centres(yf), centres(zf)]
    ws = [np.diff(np.asarray(xf, float)), np.diff(np.asarray(yf, float)), np.diff(np.asarray(zf, float))]
    mg_of = {int(c): m for m, c in enumerate(st.mcell)}
    rows, cols, vals = [], [], []
    nn = (nx, ny, nz)
    stride = (1, nx, nx * ny)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                p = i + nx * (j + ny * k)
                f = int(flags[p])
                if f & 1:
                    continue
                ci = (i, j, k)
                diag = 0.0
                for d in range(3):
                    for sgn in (-1, 1):
                        c2 = ci[d] + sgn
                        if c2 < 0 or c2 >= nn[d]:
                            continue
                        coef = 1.0 / (ws[d][ci[d]] * abs(cs[d][c2] - cs[d][ci[d]]))
                        diag += coef
                        q = p + sgn * stride[d]
                        lo = p if sgn > 0 else q
                        if flags[lo] & (16 << d):
                            qq = N + mg_of[q]
                        else:
                            qq = q
                        if not ((f & 8) and pinned):
                            rows.append(p); cols.append(qq); vals.append(coef)
                rows.append(p); cols.append(p); vals.append(-diag)
    for r in range(st.ng + st.nm):
        u = int(st.gcell[r]) if r < st.ng else N + (r - st.ng)
        s = st.sG[r]
        for m in range(8):
            c = int(st.col[r, m])
            if c >= 0:
                rows.append(u); cols.append(c); vals.append(s * st.w[r, m])
        rows.append(u); cols.append(u); vals.append(-s)
    A = sp.coo_matrix((vals, (rows, cols)), shape=(N + nm, N + nm)).tocsr()
    return A


def active_mask(flags, nm=0):
    a = ((flags & 1) == 0) | ((flags & 2) != 0)
    return np.concatenate([a, np.ones(nm, bool)])


def solve_direct(A, b, flags, nm):
    """Direct solve on the active rows (solid non-ghost cells are fixed 0)."""
    from scipy.sparse.linalg import spsolve
    act = np.nonzero(active_mask(flags, nm))[0]
    Aa = A[act][:, act].tocsc()
    x = np.zeros(len(b))
    x[act] = spsolve(Aa, b[act])
    return x


def vol(xf, yf, zf):
    w = [np.diff(np.asarray(a, float)) for a in (xf, yf, zf)]
    return (w[2][:, None, None] * w[1][None, :, None] * w[0][None, None, :]).ravel()


def assemble_masked_box(xf, yf, zf, closed_faces, pin=0):
    """Pinned Neumann box operator with selected interior faces closed.
    closed_faces: set of (d, cell) meaning the face cell -> cell + e_d."""
    nx, ny, nz = len(xf) - 1, len(yf) - 1, len(zf) - 1
    N = nx * ny * nz
    cs = [centres(xf), centres(yf), centres(zf)]
    ws = [np.diff(np.asarray(a, float)) for a in (xf, yf, zf)]
    nn = (nx, ny, nz)
    stride = (1, nx, nx * ny)
    rows, cols, vals = [], [], []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                p = i + nx * (j + ny * k)
                ci = (i, j, k)
                diag = 0.0
                for d in range(3):
                    for sgn in (-1, 1):
                        c2 = ci[d] + sgn
                        if c2 < 0 or c2 >= nn[d]:
                            continue
                        coef = 1.0 / (ws[d][ci[d]] * abs(cs[d][c2] - cs[d][ci[d]]))
                        diag += coef
                        q = p + sgn * stride[d]
                        if (d, min(p, q)) in closed_faces:
                            continue
                        if p != pin:
                            rows.append(p); cols.append(q); vals.append(coef)
                if p != pin:
                    # closed faces drop out of the diagonal too
                    dd = 0.0
                    for d in range(3):
                        for sgn in (-1, 1):
                            c2 = ci[d] + sgn
                            if c2 < 0 or c2 >= nn[d]:
                                continue
                            q = p + sgn * stride[d]
                            if (d, min(p, q)) in closed_faces:
                                continue
                            dd += 1.0 / (ws[d][ci[d]] * abs(cs[d][c2] - cs[d][ci[d]]))
                    rows.append(p); cols.append(p); vals.append(-dd)
                else:
                    rows.append(p); cols.append(p); vals.append(-diag)
    return sp.coo_matrix((vals, (rows, cols)), shape=(N, N)).tocsr()


def closest_points_on_triangles(p, A, B, C):
    """Closest point of each triangle (A[t], B[t], C[t]) to the point p, and
    its squared distance.

    The orthogonal projection of p onto the triangle's plane is kept when its
    barycentric coordinates, from the 2x2 Gram system of the edges AB and AC,
    are all non-negative; otherwise the closest point lies on the boundary
    and is the nearest of the three projections of p onto the edge segments,
    clamped to the segment.  Returns (Q[T, 3], d2[T], feature[T]) with
    feature 0 for the face, 1-3 for the edges AB, BC, CA, 4-6 for the
    vertices A, B, C."""
    p = np.asarray(p, dtype=np.float64)
    A, B, C = (np.atleast_2d(np.asarray(v, dtype=np.float64)) for v in (A, B, C))
    e0, e1, v = B - A, C - A, p[None, :] - A
    d00 = np.sum(e0 * e0, 1)
    d01 = np.sum(e0 * e1, 1)
    d11 = np.sum(e1 * e1, 1)
    d20 = np.sum(v * e0, 1)
    d21 = np.sum(v * e1, 1)
    den = d00 * d11 - d01 * d01
    s = (d11 * d20 - d01 * d21) / den
    t = (d00 * d21 - d01 * d20) / den
    inside = (s >= 0) & (t >= 0) & (s + t <= 1)
    proj = A + s[:, None] * e0 + t[:, None] * e1
    best_q = np.empty_like(A)
    best_d = np.full(len(A), np.inf)
    feat = np.zeros(len(A), dtype=np.int64)
    for k, (U, V) in enumerate(((A, B), (B, C), (C, A))):
        e = V - U
        u = np.clip(np.sum((p[None, :] - U) * e, 1) / np.sum(e * e, 1), 0.0, 1.0)
        q = U + u[:, None] * e
        d = np.sum((q - p[None, :]) ** 2, 1)
        better = d < best_d
        best_q[better] = q[better]
        best_d[better] = d[better]
        # a clamped parameter puts the point on a vertex: the segment's start or end
        fk = np.where(u <= 0.0, 4 + k, np.where(u >= 1.0, 4 + (k + 1) % 3, 1 + k))
        feat[better] = fk[better]
    dproj = np.sum((proj - p[None, :]) ** 2, 1)
    Q = np.where(inside[:, None], proj, best_q)
    d2 = np.where(inside, dproj, best_d)
    feat = np.where(inside, 0, feat)
    return Q, d2, feat


def cell_centre_points(xf, yf, zf, cells):
    """Centres of cells given by natural index (x fastest)."""
    cs = [centres(xf), centres(yf), centres(zf)]
    nx, ny = len(cs[0]), len(cs[1])
    cells = np.asarray(cells, dtype=np.int64)
    return np.stack([cs[0][cells % nx], cs[1][(cells // nx) % ny], cs[2][cells // (nx * ny)]], 1)


def nearest_surface_points(G, bodies, kind):
    """For each point of G, the closest point over every triangle of the bodies
    of the given kind (0 closed, 1 membrane), ties broken by the lowest
    triangle index in (body, triangle) order.  Returns (Q[n, 3], d2[n],
    tri[n], ties[n]): ties counts the triangles within a relative 1e-12 of the
    minimum squared distance."""
    tris = [np.asarray(b.verts, dtype=np.float64)[np.asarray(b.tris)] for b in bodies if b.kind == kind]
    T = np.concatenate(tris, 0)
    out_q = np.zeros((len(G), 3))
    out_d = np.zeros(len(G))
    out_t = np.zeros(len(G), dtype=np.int64)
    ties = np.zeros(len(G), dtype=np.int64)
    for n, g in enumerate(np.asarray(G, dtype=np.float64)):
        Q, d2, _ = closest_points_on_triangles(g, T[:, 0], T[:, 1], T[:, 2])
        t = int(np.argmin(d2))  # first index of the minimum
        out_q[n], out_d[n], out_t[n] = Q[t], d2[t], t
        ties[n] = int(np.sum(d2 <= d2[t] * (1 + 1e-12)))
    return out_q, out_d, out_t, ties
