/*
 * FP64 CPU oracle for the sharp-interface (ghost-cell) immersed-boundary
 * pressure-Poisson solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code with the HIP path.
 *
 * What it computes (the paper, Sec. 2.1 and 2.5, names the pieces; the exact
 * definitions are the readings listed in the design notes):
 *   - "iblanking" (Sec. 2.5 item 1): cells are classified solid/fluid against
 *     closed triangulated bodies by exact integer ray parity along x, and
 *     links between face neighbours are marked cut by zero-thickness
 *     membranes (rays along x, y and z);
 *   - the ghost-cell method (Sec. 2.5 item 2): each ghost row becomes an
 *     image-point trilinear stencil enforcing a Neumann condition;
 *   - the PPE of the fractional-step method (Sec. 2.1): a second-order
 *     cell-centred 7-point operator on a stretched Cartesian grid, solved by
 *     right-preconditioned BiCGSTAB (van der Vorst 1992) with a geometric
 *     multigrid V-cycle as preconditioner.
 *
 * Plain loops, FP64 throughout, no blocking or fusion.  Quantisation and the
 * integer predicates must be evaluated without FMA contraction: this file is
 * compiled with -ffp-contract=off.
 *
 * Return codes: 0 ok, -1 invalid argument, -2 bad geometry, -5 no
 * convergence, -6 breakdown.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EINVAL (-1)
#define ORC_EGEOM (-2)
#define ORC_ENOCONV (-5)
#define ORC_EBREAKDOWN (-6)

#define F_SOLID 1u
#define F_GHOST 2u
#define F_MGHOST 4u
#define F_PIN 8u
#define F_CUTX 16u
#define F_CUTY 32u
#define F_CUTZ 64u

/* ------------------------------------------------------------------ grid */
typedef struct {
    int n[3];
    const double *f[3]; /* faces, n+1 */
    double *c[3];       /* centres */
    double *w[3];       /* widths */
    double *cp[3];      /* 1/(w_i (c_{i+1}-c_i)), 0 at the last cell */
    double *cm[3];      /* 1/(w_i (c_i-c_{i-1})), 0 at the first cell */
} Grid;

static int grid_init(Grid *g, int nx, int ny, int nz, const double *xf, const double *yf, const double *zf)
{
    g->n[0] = nx; g->n[1] = ny; g->n[2] = nz;
    g->f[0] = xf; g->f[1] = yf; g->f[2] = zf;
    for (int d = 0; d < 3; ++d) {
        int n = g->n[d];
        if (n < 2) return ORC_EINVAL;
        for (int i = 0; i < n; ++i)
            if (!(g->f[d][i + 1] > g->f[d][i])) return ORC_EINVAL;
        g->c[d] = malloc(sizeof(double) * n);
        g->w[d] = malloc(sizeof(double) * n);
        g->cp[d] = malloc(sizeof(double) * n);
        g->cm[d] = malloc(sizeof(double) * n);
        for (int i = 0; i < n; ++i) {
            g->c[d][i] = 0.5 * (g->f[d][i] + g->f[d][i + 1]);
            g->w[d][i] = g->f[d][i + 1] - g->f[d][i];
        }
        for (int i = 0; i < n; ++i) {
            g->cp[d][i] = (i + 1 < n) ? 1.0 / (g->w[d][i] * (g->c[d][i + 1] - g->c[d][i])) : 0.0;
            g->cm[d][i] = (i > 0) ? 1.0 / (g->w[d][i] * (g->c[d][i] - g->c[d][i - 1])) : 0.0;
        }
    }
    return 0;
}

static void grid_free(Grid *g)
{
    for (int d = 0; d < 3; ++d) {
        free(g->c[d]); free(g->w[d]); free(g->cp[d]); free(g->cm[d]);
    }
}

static inline int64_t IDX(const int *n, int i, int j, int k)
{
    return (int64_t)i + (int64_t)n[0] * ((int64_t)j + (int64_t)n[1] * (int64_t)k);
}

/* ------------------------------------------------------- quantisation */
/* Lattice scale: 2^16 lattice units over the longest domain edge. */
static double lattice_scale(const Grid *g)
{
    double L = 0.0;
    for (int d = 0; d < 3; ++d) {
        double l = g->f[d][g->n[d]] - g->f[d][0];
        if (l > L) L = l;
    }
    return 65536.0 / L;
}

static int64_t quant(double v, double lo, double S)
{
    double t = (v - lo) * S;
    t = t + 0.5;
    return (int64_t)floor(t);
}

/* ------------------------------------------------ exact predicates */
/* Orientation of P against the directed edge U->V, in the plane (u,w) of
 * two coordinate axes. */
static int64_t o2(const int64_t *U, const int64_t *V, const int64_t *P, int u, int w)
{
    return (V[u] - U[u]) * (P[w] - U[w]) - (V[w] - U[w]) * (P[u] - U[u]);
}

/* Edge U->V of a counter-clockwise projected triangle owns points lying
 * exactly on it iff its direction d satisfies d_w < 0, or d_w == 0 and
 * d_u > 0 (the same as moving the ray by (+eps, +eps^2) in (u,w)). */
static int top_left(const int64_t *U, const int64_t *V, int u, int w)
{
    int64_t du = V[u] - U[u], dw = V[w] - U[w];
    return dw < 0 || (dw == 0 && du > 0);
}

static int edge_ok(const int64_t *U, const int64_t *V, const int64_t *P, int u, int w)
{
    int64_t e = o2(U, V, P, u, w);
    if (e > 0) return 1;
    if (e < 0) return 0;
    return top_left(U, V, u, w);
}

/* F(A,B,C,X) = (X-A) . ((B-A) x (C-A)) */
static int64_t Fdet(const int64_t *A, const int64_t *N, const int64_t *X)
{
    return (X[0] - A[0]) * N[0] + (X[1] - A[1]) * N[1] + (X[2] - A[2]) * N[2];
}

static int lower_bound64(const int64_t *a, int n, int64_t v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int m = (lo + hi) / 2;
        if (a[m] < v) lo = m + 1; else hi = m;
    }
    return lo;
}

/* Walk every ray along axis d that the projection of triangle (A,B,C)
 * covers (top-left rule), and call back with the per-cell intercept bits.
 * mode 0: toggle par[cell] for every cell whose centre lies strictly beyond
 * the intercept (closed-body ray parity).  mode 1: toggle cut[cell] of the
 * link cell->cell+e_d when the intercept bit changes between the two
 * centres (membrane cut links). */
static void rays_through_triangle(const Grid *g, int64_t *const qc[3], const int64_t *A, const int64_t *B,
                                  const int64_t *C, int d, int mode, uint8_t *arr)
{
    int u = (d + 1) % 3, w = (d + 2) % 3;
    int64_t N[3];
    int64_t e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    int64_t e2[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
    N[0] = e1[1] * e2[2] - e1[2] * e2[1];
    N[1] = e1[2] * e2[0] - e1[0] * e2[2];
    N[2] = e1[0] * e2[1] - e1[1] * e2[0];
    int64_t a = o2(A, B, C, u, w); /* equals N[d] */
    if (a == 0) return;
    const int64_t *P0 = A, *P1 = B, *P2 = C;
    if (a < 0) { P1 = C; P2 = B; }
    int64_t umin = A[u], umax = A[u], wmin = A[w], wmax = A[w];
    if (B[u] < umin) umin = B[u];
    if (C[u] < umin) umin = C[u];
    if (B[u] > umax) umax = B[u];
    if (C[u] > umax) umax = C[u];
    if (B[w] < wmin) wmin = B[w];
    if (C[w] < wmin) wmin = C[w];
    if (B[w] > wmax) wmax = B[w];
    if (C[w] > wmax) wmax = C[w];
    int nu = g->n[u], nw = g->n[w], nr = g->n[d];
    int a0 = lower_bound64(qc[u], nu, umin);
    int b0 = lower_bound64(qc[w], nw, wmin);
    int64_t X[3];
    for (int ia = a0; ia < nu && qc[u][ia] <= umax; ++ia) {
        for (int ib = b0; ib < nw && qc[w][ib] <= wmax; ++ib) {
            X[u] = qc[u][ia];
            X[w] = qc[w][ib];
            if (!edge_ok(P0, P1, X, u, w) || !edge_ok(P1, P2, X, u, w) || !edge_ok(P2, P0, X, u, w))
                continue;
            int prev = -1;
            for (int i = 0; i < nr; ++i) {
                X[d] = qc[d][i];
                int64_t F = Fdet(A, N, X);
                int sig = (a > 0) ? (F > 0) : (F < 0);
                int cc[3];
                cc[d] = i; cc[u] = ia; cc[w] = ib;
                int64_t id = IDX(g->n, cc[0], cc[1], cc[2]);
                if (mode == 0) {
                    if (sig) arr[id] ^= 1;
                } else if (prev >= 0 && sig != prev) {
                    cc[d] = i - 1;
                    arr[IDX(g->n, cc[0], cc[1], cc[2])] ^= 1;
                }
                prev = sig;
            }
        }
    }
}

/*
 * Cell classification ("iblanking", Sec. 2.5 item 1).
 * Bodies: concatenated vertices (3 doubles each) and triangles (3 local
 * vertex indices each); kind 0 closed (outward), 1 membrane.
 * flags[N] receives: bit0 solid, bit1 closed ghost, bit2 membrane ghost,
 * bit3 pin, bits4-6 cut +x/+y/+z links.
 */
int orc_classify(int nx, int ny, int nz, const double *xf, const double *yf, const double *zf, int nbody,
                 const int32_t *kind, const int32_t *nvert, const int32_t *ntri, const double *verts,
                 const int32_t *tris, uint8_t *flags)
{
    Grid g;
    if (grid_init(&g, nx, ny, nz, xf, yf, zf)) return ORC_EINVAL;
    int64_t N = (int64_t)nx * ny * nz;
    double S = lattice_scale(&g);
    double lo[3] = {xf[0], yf[0], zf[0]};
    int64_t *qc[3];
    for (int d = 0; d < 3; ++d) {
        qc[d] = malloc(sizeof(int64_t) * g.n[d]);
        for (int i = 0; i < g.n[d]; ++i) qc[d][i] = quant(g.c[d][i], lo[d], S);
    }
    uint8_t *solid = calloc(N, 1), *par = malloc(N), *cut[3];
    for (int d = 0; d < 3; ++d) cut[d] = calloc(N, 1);
    int rc = 0;
    int64_t voff = 0, toff = 0;
    for (int b = 0; b < nbody && rc == 0; ++b) {
        int nv = nvert[b], nt = ntri[b];
        int64_t *qv = malloc(sizeof(int64_t) * 3 * (nv > 0 ? nv : 1));
        for (int v = 0; v < nv; ++v)
            for (int d = 0; d < 3; ++d) {
                double x = verts[3 * (voff + v) + d];
                double L = g.f[d][g.n[d]] - g.f[d][0];
                if (!(x >= lo[d] - L && x <= g.f[d][g.n[d]] + L)) rc = ORC_EINVAL;
                qv[3 * v + d] = quant(x, lo[d], S);
            }
        if (kind[b] == 0) memset(par, 0, N);
        for (int t = 0; t < nt && rc == 0; ++t) {
            const int32_t *T = tris + 3 * (toff + t);
            if (T[0] < 0 || T[1] < 0 || T[2] < 0 || T[0] >= nv || T[1] >= nv || T[2] >= nv) { rc = ORC_EGEOM; break; }
            const int64_t *A = qv + 3 * T[0], *B = qv + 3 * T[1], *C = qv + 3 * T[2];
            if (kind[b] == 0) {
                rays_through_triangle(&g, qc, A, B, C, 0, 0, par);
            } else {
                for (int d = 0; d < 3; ++d) rays_through_triangle(&g, qc, A, B, C, d, 1, cut[d]);
            }
        }
        if (kind[b] == 0)
            for (int64_t p = 0; p < N; ++p) solid[p] |= par[p];
        free(qv);
        voff += nv;
        toff += nt;
    }
    if (rc == 0) {
        int64_t pin = -1;
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    int64_t p = IDX(g.n, i, j, k);
                    int ci[3] = {i, j, k};
                    int64_t st[3] = {1, nx, (int64_t)nx * ny};
                    uint8_t fl = 0;
                    if (solid[p]) {
                        fl |= F_SOLID;
                        for (int d = 0; d < 3; ++d) {
                            if (ci[d] > 0 && !solid[p - st[d]]) fl |= F_GHOST;
                            if (ci[d] + 1 < g.n[d] && !solid[p + st[d]]) fl |= F_GHOST;
                        }
                    } else {
                        for (int d = 0; d < 3; ++d) {
                            if (ci[d] + 1 < g.n[d] && cut[d][p] && !solid[p + st[d]]) fl |= (uint8_t)(F_CUTX << d);
                            if (ci[d] > 0 && cut[d][p - st[d]] && !solid[p - st[d]]) fl |= F_MGHOST;
                        }
                        if (fl & (F_CUTX | F_CUTY | F_CUTZ)) fl |= F_MGHOST;
                    }
                    flags[p] = fl;
                }
        for (int64_t p = 0; p < N; ++p)
            if (!(flags[p] & (F_SOLID | F_MGHOST))) { pin = p; break; }
        if (pin < 0) rc = ORC_EGEOM;
        else flags[pin] |= F_PIN;
    }
    for (int d = 0; d < 3; ++d) { free(qc[d]); free(cut[d]); }
    free(solid); free(par);
    grid_free(&g);
    return rc;
}

/* ------------------------------------------------ ghost-cell stencils */
/* Closest point on triangle abc to p: Voronoi-region walk of Ericson,
 * "Real-Time Collision Detection" (2005), Sec. 5.1.5. */
static void closest_on_tri(const double *p, const double *a, const double *b, const double *c, double *q)
{
    double ab[3], ac[3], ap[3], bp[3], cp[3];
    for (int d = 0; d < 3; ++d) {
        ab[d] = b[d] - a[d]; ac[d] = c[d] - a[d]; ap[d] = p[d] - a[d];
        bp[d] = p[d] - b[d]; cp[d] = p[d] - c[d];
    }
#define DOT(x, y) ((x)[0] * (y)[0] + (x)[1] * (y)[1] + (x)[2] * (y)[2])
    double d1 = DOT(ab, ap), d2 = DOT(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) { memcpy(q, a, 24); return; }
    double d3 = DOT(ab, bp), d4 = DOT(ac, bp);
    if (d3 >= 0.0 && d4 <= d3) { memcpy(q, b, 24); return; }
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        double v = d1 / (d1 - d3);
        for (int d = 0; d < 3; ++d) q[d] = a[d] + v * ab[d];
        return;
    }
    double d5 = DOT(ab, cp), d6 = DOT(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) { memcpy(q, c, 24); return; }
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
        double v = d2 / (d2 - d6);
        for (int d = 0; d < 3; ++d) q[d] = a[d] + v * ac[d];
        return;
    }
    double va = d3 * d6 - d5 * d4;
    if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
        double v = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        for (int d = 0; d < 3; ++d) q[d] = b[d] + v * (c[d] - b[d]);
        return;
    }
    double den = 1.0 / (va + vb + vc);
    double v = vb * den, w = vc * den;
    for (int d = 0; d < 3; ++d) q[d] = a[d] + ab[d] * v + ac[d] * w;
#undef DOT
}

/* The same routine for the tests, which pin it against an independent
 * construction (plane projection with barycentric coordinates, else the
 * nearest clamped edge projection). */
void orc_closest_point(const double *p, const double *a, const double *b, const double *c, double *q)
{
    closest_on_tri(p, a, b, c, q);
}

/* largest i <= n-2 with c[i] <= x, for x already clamped into [c0, c_{n-1}] */
static int box_index(const double *c, int n, double x)
{
    int i = 0;
    while (i + 1 <= n - 2 && c[i + 1] <= x) ++i;
    return i;
}

/* Trilinear basis at (xi, eta, zeta): [1, xi, eta, zeta, xi eta, eta zeta, xi zeta, xi eta zeta] */
static void basis(double x, double y, double z, double *b)
{
    b[0] = 1.0; b[1] = x; b[2] = y; b[3] = z;
    b[4] = x * y; b[5] = y * z; b[6] = x * z; b[7] = x * y * z;
}

/* LU with partial pivoting of the 8x8 matrix M (row-major), solving M y = r.
 * Pivot = largest magnitude in the column (first such row on ties).
 * Returns 1 when a pivot falls below 1e-12 max|M|. */
static int lu8_solve(double M[8][8], double *r)
{
    double amax = 0.0;
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j)
            if (fabs(M[i][j]) > amax) amax = fabs(M[i][j]);
    for (int c = 0; c < 8; ++c) {
        int p = c;
        for (int i = c + 1; i < 8; ++i)
            if (fabs(M[i][c]) > fabs(M[p][c])) p = i;
        if (!(fabs(M[p][c]) >= 1e-12 * amax) || amax == 0.0) return 1;
        if (p != c) {
            for (int j = 0; j < 8; ++j) { double t = M[c][j]; M[c][j] = M[p][j]; M[p][j] = t; }
            double t = r[c]; r[c] = r[p]; r[p] = t;
        }
        for (int i = c + 1; i < 8; ++i) {
            double l = M[i][c] / M[c][c];
            for (int j = c; j < 8; ++j) M[i][j] -= l * M[c][j];
            r[i] -= l * r[c];
        }
    }
    for (int c = 7; c >= 0; --c) {
        double s = r[c];
        for (int j = c + 1; j < 8; ++j) s -= M[c][j] * r[j];
        r[c] = s / M[c][c];
    }
    return 0;
}

static double cell_scale(const Grid *g, int i, int j, int k)
{
    return g->cp[0][i] + g->cm[0][i] + g->cp[1][j] + g->cm[1][j] + g->cp[2][k] + g->cm[2][k];
}

/*
 * Ghost-cell rows (Sec. 2.5 item 2; GCM of Mittal et al. 2008, read as the
 * standard image-point stencil).  bc 0: Neumann rows for the pressure,
 * sG (sum w x - x_G) = sG (dl - beta_BI) g with a derivative row at BI when
 * G is a node of the box.  bc 1: Dirichlet rows for the velocity of the
 * advection-diffusion step (the value at BI is the mean of G and IP),
 * sG (sum w x + x_G) = sG (2 - beta_BI) g with a value row at BI; a ghost on
 * the surface (degenerate distance) gets x_G = g.  Rows: closed ghosts and membrane
 * ghost unknowns, given by row_cell[] and row_mem[] (1 for a membrane ghost
 * unknown).  mg_of[N] maps a cell to its membrane-ghost index or -1.
 * Outputs per row r:
 *   col[8r..] value columns (cell index, or N + membrane index; -1 unused
 *              or the derivative node), w[8r..] their weights;
 *   sG[r] row scale; dlb[r] = dl - beta_BI (so the RHS is sG*dlb*g);
 *   rfl[r] bit0 fallback (degenerate stencil), bit1 derivative row used,
 *          bit2 degenerate distance;
 *   geo[12r..] BI[3], IP[3], n[3], dl, beta_BI, distance;
 *   box[3r..] the stencil box origin.
 */
int orc_ghost_stencils(int nx, int ny, int nz, const double *xf, const double *yf, const double *zf, int nbody,
                       const int32_t *kind, const int32_t *nvert, const int32_t *ntri, const double *verts,
                       const int32_t *tris, const uint8_t *flags, const int32_t *mg_of, int32_t nrows,
                       const int32_t *row_cell, const int32_t *row_mem, int bc, int32_t *col, double *w, double *sG,
                       double *dlb, uint8_t *rfl, double *geo, int32_t *box)
{
    Grid g;
    if (grid_init(&g, nx, ny, nz, xf, yf, zf)) return ORC_EINVAL;
    int64_t N = (int64_t)nx * ny * nz;
    int64_t ntot = 0;
    for (int b = 0; b < nbody; ++b) ntot += ntri[b];
    /* flatten triangles with their kind, in (body, triangle) order */
    double *TV = malloc(sizeof(double) * 9 * (ntot > 0 ? ntot : 1));
    int *TK = malloc(sizeof(int) * (ntot > 0 ? ntot : 1));
    int64_t voff = 0, toff = 0, q = 0;
    for (int b = 0; b < nbody; ++b) {
        for (int t = 0; t < ntri[b]; ++t, ++q) {
            for (int m = 0; m < 3; ++m)
                for (int d = 0; d < 3; ++d) TV[9 * q + 3 * m + d] = verts[3 * (voff + tris[3 * (toff + t) + m]) + d];
            TK[q] = kind[b];
        }
        voff += nvert[b];
        toff += ntri[b];
    }
    double hmin = 1e300;
    for (int d = 0; d < 3; ++d)
        for (int i = 0; i < g.n[d]; ++i)
            if (g.w[d][i] < hmin) hmin = g.w[d][i];
    int rc = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int32_t r = 0; r < nrows; ++r) {
        int64_t cell = row_cell[r];
        int mem = row_mem[r];
        int ci = (int)(cell % nx), cj = (int)((cell / nx) % ny), ck = (int)(cell / ((int64_t)nx * ny));
        double G[3] = {g.c[0][ci], g.c[1][cj], g.c[2][ck]};
        /* body intercept: closest point over the triangles of the row's kind */
        double best = INFINITY, BI[3] = {0, 0, 0};
        int64_t bt = -1;
        for (int64_t t = 0; t < ntot; ++t) {
            if (TK[t] != (mem ? 1 : 0)) continue;
            const double *A = TV + 9 * t, *B = A + 3, *C = A + 6;
            double lb = 0.0;
            for (int d = 0; d < 3; ++d) {
                double mn = fmin(A[d], fmin(B[d], C[d])), mx = fmax(A[d], fmax(B[d], C[d]));
                double e = G[d] < mn ? mn - G[d] : (G[d] > mx ? G[d] - mx : 0.0);
                lb += e * e;
            }
            if (lb > best) continue;
            double Q[3];
            closest_on_tri(G, A, B, C, Q);
            double d2 = (Q[0] - G[0]) * (Q[0] - G[0]) + (Q[1] - G[1]) * (Q[1] - G[1]) + (Q[2] - G[2]) * (Q[2] - G[2]);
            if (d2 < best) { best = d2; bt = t; memcpy(BI, Q, 24); }
        }
        if (bt < 0) { rc = ORC_EGEOM; continue; }
        double dist = sqrt(best), nrm[3], IP[3], dl;
        uint8_t fl = 0;
        if (dist < 1e-9 * hmin) {
            const double *A = TV + 9 * bt, *B = A + 3, *C = A + 6;
            double e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]}, e2[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
            double fn[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
            double L = sqrt(fn[0] * fn[0] + fn[1] * fn[1] + fn[2] * fn[2]);
            double hl = fmin(g.w[0][ci], fmin(g.w[1][cj], g.w[2][ck]));
            for (int d = 0; d < 3; ++d) {
                nrm[d] = fn[d] / L;
                BI[d] = G[d];
                IP[d] = G[d] + hl * nrm[d];
            }
            dl = hl;
            fl |= 4;
        } else {
            for (int d = 0; d < 3; ++d) {
                nrm[d] = (BI[d] - G[d]) / dist;
                IP[d] = 2.0 * BI[d] - G[d];
            }
            dl = 2.0 * dist;
        }
        /* stencil box around the (clamped) image point */
        int b0[3];
        double loc[3], del[3], bil[3];
        for (int d = 0; d < 3; ++d) {
            int n = g.n[d];
            double x = IP[d];
            if (x < g.c[d][0]) x = g.c[d][0];
            if (x > g.c[d][n - 1]) x = g.c[d][n - 1];
            b0[d] = box_index(g.c[d], n, x);
            del[d] = g.c[d][b0[d] + 1] - g.c[d][b0[d]];
            loc[d] = (x - g.c[d][b0[d]]) / del[d];
            bil[d] = (BI[d] - g.c[d][b0[d]]) / del[d];
        }
        double V[8][8];
        int32_t cl[8];
        int degenerate = 0, dnode = -1;
        for (int m = 0; m < 8; ++m) {
            int dx = m & 1, dy = (m >> 1) & 1, dz = (m >> 2) & 1;
            int ii = b0[0] + dx, jj = b0[1] + dy, kk = b0[2] + dz;
            int64_t id = IDX(g.n, ii, jj, kk);
            uint8_t f = flags[id];
            cl[m] = -1;
            if (id == cell && bc == 1) {
                basis(bil[0], bil[1], bil[2], V[m]);  /* value row at BI */
                dnode = m;
                continue;
            }
            if (id == cell) {
                double x = bil[0], y = bil[1], z = bil[2];
                double gx[8] = {0, 1, 0, 0, y, 0, z, y * z};
                double gy[8] = {0, 0, 1, 0, x, z, 0, x * z};
                double gz[8] = {0, 0, 0, 1, 0, y, x, x * y};
                for (int c = 0; c < 8; ++c)
                    V[m][c] = nrm[0] / del[0] * gx[c] + nrm[1] / del[1] * gy[c] + nrm[2] / del[2] * gz[c];
                dnode = m;
                continue;
            }
            basis((double)dx, (double)dy, (double)dz, V[m]);
            if (!mem) {
                if (!(f & F_SOLID) || (f & F_GHOST)) cl[m] = (int32_t)id;
                else degenerate = 1;
            } else {
                double side = nrm[0] * (g.c[0][ii] - BI[0]) + nrm[1] * (g.c[1][jj] - BI[1]) + nrm[2] * (g.c[2][kk] - BI[2]);
                if (side > 0.0) {
                    if (!(f & F_SOLID)) cl[m] = (int32_t)id;
                    else degenerate = 1;
                } else {
                    if (mg_of[id] >= 0) cl[m] = (int32_t)(N + mg_of[id]);
                    else degenerate = 1;
                }
            }
        }
        double beta[8];
        if (!degenerate) {
            double M[8][8];
            for (int i = 0; i < 8; ++i)
                for (int j = 0; j < 8; ++j) M[i][j] = V[j][i];
            basis(loc[0], loc[1], loc[2], beta);
            degenerate = lu8_solve(M, beta);
        }
        double s = cell_scale(&g, ci, cj, ck);
        double bbi = 0.0;
        if (!degenerate) {
            for (int m = 0; m < 8; ++m) {
                col[8 * r + m] = cl[m];
                w[8 * r + m] = (cl[m] >= 0) ? beta[m] : 0.0;
            }
            if (dnode >= 0) { bbi = beta[dnode]; fl |= 2; }
            dlb[r] = bc == 1 ? 2.0 - bbi : dl - bbi;
            if (bc == 1 && (fl & 4)) {
                /* G on the surface: x_G = g */
                for (int m = 0; m < 8; ++m) { col[8 * r + m] = -1; w[8 * r + m] = 0.0; }
                dlb[r] = 1.0;
            }
        } else {
            /* first-order fallback: mean of the face neighbours on the relevant side */
            fl |= 1;
            int cnt = 0;
            int32_t nb[6];
            int cc[3] = {ci, cj, ck};
            for (int d = 0; d < 3; ++d)
                for (int sgn = -1; sgn <= 1; sgn += 2) {
                    int c2[3] = {cc[0], cc[1], cc[2]};
                    c2[d] += sgn;
                    if (c2[d] < 0 || c2[d] >= g.n[d]) continue;
                    int64_t id = IDX(g.n, c2[0], c2[1], c2[2]);
                    int use;
                    if (!mem) use = !(flags[id] & F_SOLID);
                    else {
                        int64_t lo_ = sgn > 0 ? cell : id;
                        use = (flags[lo_] & (F_CUTX << d)) != 0;
                    }
                    if (use) nb[cnt++] = (int32_t)id;
                }
            for (int m = 0; m < 8; ++m) { col[8 * r + m] = -1; w[8 * r + m] = 0.0; }
            for (int m = 0; m < cnt; ++m) { col[8 * r + m] = nb[m]; w[8 * r + m] = 1.0 / cnt; }
            dlb[r] = bc == 1 ? 2.0 : 0.0;
            if (cnt == 0) rc = ORC_EGEOM;
        }
        sG[r] = s;
        rfl[r] = fl;
        for (int d = 0; d < 3; ++d) {
            geo[12 * r + d] = BI[d];
            geo[12 * r + 3 + d] = IP[d];
            geo[12 * r + 6 + d] = nrm[d];
            box[3 * r + d] = b0[d];
        }
        geo[12 * r + 9] = dl;
        geo[12 * r + 10] = bbi;
        geo[12 * r + 11] = dist;
    }
    free(TV); free(TK);
    grid_free(&g);
    return rc;
}

/* -------------------------------------------------------- the system */
/* Unknowns: the N cell values (x fastest) followed by n_m membrane ghost
 * unknowns.  Ghost rows: n_g closed ghosts (unknown = their cell) then the
 * n_m membrane ghosts (unknown = N + m). */
typedef struct {
    Grid g;
    int64_t N;
    const uint8_t *flags;
    const int32_t *mg_of;
    int32_t ng, nm;
    const int32_t *row_cell;
    const int32_t *col;
    const double *w;
    const double *sG;
    int64_t pin;
} Sys;

static inline int64_t row_unknown(const Sys *S, int32_t r)
{
    return r < S->ng ? (int64_t)S->row_cell[r] : S->N + (r - S->ng);
}

/* the neighbour value seen by a fluid cell across link (p, q) in axis d */
static inline double nbval(const Sys *S, const double *x, int64_t p, int64_t q, int d, int plus)
{
    int64_t lo = plus ? p : q;
    if (S->flags[lo] & (F_CUTX << d)) return x[S->N + S->mg_of[q]];
    return x[q];
}

/* Inside the smoother a cell next to a cut link sees its neighbour's ghost
 * unknown eliminated: the current value of that ghost row's stencil,
 * sum w x - b/sG, instead of the stored unknown (Gauss-Seidel on the system
 * with the membrane ghost unknowns substituted). */
static inline double nbval_elim(const Sys *S, const double *x, const double *b, int64_t p, int64_t q, int d, int plus)
{
    int64_t lo = plus ? p : q;
    if (S->flags[lo] & (F_CUTX << d)) {
        int32_t r = S->ng + S->mg_of[q];
        double acc = 0.0;
        for (int m = 0; m < 8; ++m) {
            int32_t c = S->col[8 * r + m];
            if (c >= 0) acc += S->w[8 * r + m] * x[c];
        }
        return acc - b[S->N + S->mg_of[q]] / S->sG[r];
    }
    return x[q];
}

/* sum c * neighbour over the faces of a fluid cell, with eliminated ghosts */
static double fluid_offsum_elim(const Sys *S, const double *x, const double *b, int i, int j, int k, int64_t p)
{
    const Grid *g = &S->g;
    int ci[3] = {i, j, k};
    int64_t st[3] = {1, g->n[0], (int64_t)g->n[0] * g->n[1]};
    double acc = 0.0;
    for (int d = 0; d < 3; ++d) {
        if (ci[d] + 1 < g->n[d]) acc += g->cp[d][ci[d]] * nbval_elim(S, x, b, p, p + st[d], d, 1);
        if (ci[d] > 0) acc += g->cm[d][ci[d]] * nbval_elim(S, x, b, p, p - st[d], d, 0);
    }
    return acc;
}

/* (A x) for one fluid (non-pin) cell */
static double fluid_row(const Sys *S, const double *x, int i, int j, int k, int64_t p)
{
    const Grid *g = &S->g;
    int ci[3] = {i, j, k};
    int64_t st[3] = {1, g->n[0], (int64_t)g->n[0] * g->n[1]};
    double xp = x[p], acc = 0.0;
    for (int d = 0; d < 3; ++d) {
        if (ci[d] + 1 < g->n[d]) acc += g->cp[d][ci[d]] * (nbval(S, x, p, p + st[d], d, 1) - xp);
        if (ci[d] > 0) acc += g->cm[d][ci[d]] * (nbval(S, x, p, p - st[d], d, 0) - xp);
    }
    return acc;
}

static double ghost_row(const Sys *S, const double *x, int32_t r)
{
    double acc = 0.0;
    for (int m = 0; m < 8; ++m) {
        int32_t c = S->col[8 * r + m];
        if (c >= 0) acc += S->w[8 * r + m] * x[c];
    }
    return S->sG[r] * (acc - x[row_unknown(S, r)]);
}

/* y = A x; pinned = 0 gives the singular operator whose pin row is an
 * ordinary fluid row (used inside the V-cycle). */
static void sys_apply_m(const Sys *S, const double *x, double *y, int pinned)
{
    const Grid *g = &S->g;
    int nx = g->n[0], ny = g->n[1], nz = g->n[2];
#pragma omp parallel for
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t p = IDX(g->n, i, j, k);
                uint8_t f = S->flags[p];
                if (f & F_SOLID) y[p] = 0.0;
                else if ((f & F_PIN) && pinned) y[p] = -cell_scale(g, i, j, k) * x[p];
                else y[p] = fluid_row(S, x, i, j, k, p);
            }
#pragma omp parallel for
    for (int32_t r = 0; r < S->ng + S->nm; ++r) y[row_unknown(S, r)] = ghost_row(S, x, r);
}

/* y = A x for the pinned operator */
static void sys_apply(const Sys *S, const double *x, double *y) { sys_apply_m(S, x, y, 1); }

static int sys_init(Sys *S, int nx, int ny, int nz, const double *xf, const double *yf, const double *zf,
                    const uint8_t *flags, const int32_t *mg_of, int32_t ng, int32_t nm, const int32_t *row_cell,
                    const int32_t *col, const double *w, const double *sG)
{
    if (grid_init(&S->g, nx, ny, nz, xf, yf, zf)) return ORC_EINVAL;
    S->N = (int64_t)nx * ny * nz;
    S->flags = flags; S->mg_of = mg_of; S->ng = ng; S->nm = nm;
    S->row_cell = row_cell; S->col = col; S->w = w; S->sG = sG;
    S->pin = -1;
    for (int64_t p = 0; p < S->N; ++p)
        if (flags[p] & F_PIN) { S->pin = p; break; }
    return S->pin < 0 ? ORC_EINVAL : 0;
}

void orc_apply(int nx, int ny, int nz, const double *xf, const double *yf, const double *zf, const uint8_t *flags,
               const int32_t *mg_of, int32_t ng, int32_t nm, const int32_t *row_cell, const int32_t *col,
               const double *w, const double *sG, const double *x, double *y)
{
    Sys S;
    if (sys_init(&S, nx, ny, nz, xf, yf, zf, flags, mg_of, ng, nm, row_cell, col, w, sG)) return;
    sys_apply(&S, x, y);
    grid_free(&S.g);
}

/*
 * RHS of the pinned system (Sec. 2.1 PPE; compatibility and gauge are
 * readings): fluid f minus its volume-weighted fluid mean, 0 on the pin and
 * on solid cells, sG*dlb*g on ghost rows (g may be NULL for g = 0).
 */
void orc_assemble_rhs(int nx, int ny, int nz, const double *xf, const double *yf, const double *zf,
                      const uint8_t *flags, int32_t ng, int32_t nm, const int32_t *row_cell, const double *sG,
                      const double *dlb, const double *f, const double *gval, double *b)
{
    Grid g;
    if (grid_init(&g, nx, ny, nz, xf, yf, zf)) return;
    int64_t N = (int64_t)nx * ny * nz;
    double sv = 0.0, svf = 0.0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t p = IDX(g.n, i, j, k);
                if (flags[p] & F_SOLID) continue;
                double V = g.w[0][i] * g.w[1][j] * g.w[2][k];
                sv += V;
                svf += V * f[p];
            }
    double mean = svf / sv;
    for (int64_t p = 0; p < N; ++p) {
        uint8_t fl = flags[p];
        b[p] = (fl & (F_SOLID | F_PIN)) ? 0.0 : f[p] - mean;
    }
    for (int32_t r = 0; r < ng + nm; ++r) {
        int64_t u = r < ng ? row_cell[r] : N + (r - ng);
        b[u] = gval ? sG[r] * dlb[r] * gval[r] : 0.0;
    }
    grid_free(&g);
}

/* Gauge: subtract the volume-weighted fluid mean from fluid, ghost and
 * membrane-ghost values. */
void orc_gauge(int nx, int ny, int nz, const double *xf, const double *yf, const double *zf, const uint8_t *flags,
               int32_t nm, double *x)
{
    Grid g;
    if (grid_init(&g, nx, ny, nz, xf, yf, zf)) return;
    int64_t N = (int64_t)nx * ny * nz;
    double sv = 0.0, svx = 0.0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t p = IDX(g.n, i, j, k);
                if (flags[p] & F_SOLID) continue;
                double V = g.w[0][i] * g.w[1][j] * g.w[2][k];
                sv += V;
                svx += V * x[p];
            }
    double mean = svx / sv;
    for (int64_t p = 0; p < N; ++p)
        if (!(flags[p] & F_SOLID) || (flags[p] & F_GHOST)) x[p] -= mean;
    for (int32_t m = 0; m < nm; ++m) x[N + m] -= mean;
    grid_free(&g);
}

/* ------------------------------------------------------ multigrid */
typedef struct {
    int n[3];
    double *f[3], *c[3], *w[3], *cp[3], *cm[3];
    uint8_t *m;          /* bit0 active, bits1-3 open +x/+y/+z, bits4-6 cut +x/+y/+z */
    double *x, *b, *r;
    /* prolongation from the next coarser level: per fine index, I0 and t */
    int *pi[3];
    double *pt[3];
} Level;

typedef struct {
    int nl;
    Level L[16];
    Sys *S;
    int nu1, nu2, ncs;
    double *tmp; /* ghost Jacobi staging */
    double *bc;  /* level-0 right-hand side with the compensating sink */
} MG;

static int mg_active0(const Sys *S, int64_t p)
{
    uint8_t f = S->flags[p];
    return !(f & F_SOLID) || (f & F_GHOST);
}

static void level_geom(Level *L)
{
    for (int d = 0; d < 3; ++d) {
        int n = L->n[d];
        L->c[d] = malloc(sizeof(double) * n);
        L->w[d] = malloc(sizeof(double) * n);
        L->cp[d] = malloc(sizeof(double) * n);
        L->cm[d] = malloc(sizeof(double) * n);
        for (int i = 0; i < n; ++i) {
            L->c[d][i] = 0.5 * (L->f[d][i] + L->f[d][i + 1]);
            L->w[d][i] = L->f[d][i + 1] - L->f[d][i];
        }
        for (int i = 0; i < n; ++i) {
            L->cp[d][i] = (i + 1 < n) ? 1.0 / (L->w[d][i] * (L->c[d][i + 1] - L->c[d][i])) : 0.0;
            L->cm[d][i] = (i > 0) ? 1.0 / (L->w[d][i] * (L->c[d][i] - L->c[d][i - 1])) : 0.0;
        }
    }
}

static void mg_build(MG *M, Sys *S, int nu1, int nu2, int ncs)
{
    M->S = S; M->nu1 = nu1; M->nu2 = nu2; M->ncs = ncs;
    const Grid *g = &S->g;
    Level *L0 = &M->L[0];
    int64_t N = S->N;
    for (int d = 0; d < 3; ++d) {
        L0->n[d] = g->n[d];
        L0->f[d] = malloc(sizeof(double) * (g->n[d] + 1));
        memcpy(L0->f[d], g->f[d], sizeof(double) * (g->n[d] + 1));
    }
    level_geom(L0);
    L0->m = malloc(N);
    for (int64_t p = 0; p < N; ++p) {
        uint8_t f = S->flags[p];
        L0->m[p] = (uint8_t)(mg_active0(S, p) | (((f >> 4) & 7) << 4));
    }
    L0->x = L0->b = NULL;
    L0->r = malloc(sizeof(double) * (N + S->nm));
    M->tmp = malloc(sizeof(double) * ((S->ng + S->nm) > 0 ? (S->ng + S->nm) : 1));
    M->bc = malloc(sizeof(double) * (N + S->nm));
    int nl = 1;
    while (nl < 16) {
        Level *F = &M->L[nl - 1];
        int ok = 1, mn = F->n[0];
        for (int d = 0; d < 3; ++d) {
            if (F->n[d] % 2) ok = 0;
            if (F->n[d] < mn) mn = F->n[d];
        }
        if (!ok || mn <= 4) break;
        Level *C = &M->L[nl];
        for (int d = 0; d < 3; ++d) {
            C->n[d] = F->n[d] / 2;
            C->f[d] = malloc(sizeof(double) * (C->n[d] + 1));
            for (int i = 0; i <= C->n[d]; ++i) C->f[d][i] = F->f[d][2 * i];
        }
        level_geom(C);
        int64_t Nc = (int64_t)C->n[0] * C->n[1] * C->n[2];
        C->m = calloc(Nc, 1);
        C->x = calloc(Nc, sizeof(double));
        C->b = calloc(Nc, sizeof(double));
        C->r = calloc(Nc, sizeof(double));
        /* active = any active child; cut = any cut child link across the face */
        for (int K = 0; K < C->n[2]; ++K)
            for (int J = 0; J < C->n[1]; ++J)
                for (int I = 0; I < C->n[0]; ++I) {
                    uint8_t act = 0, cut = 0;
                    for (int c = 0; c < 8; ++c) {
                        int i = 2 * I + (c & 1), j = 2 * J + ((c >> 1) & 1), k = 2 * K + ((c >> 2) & 1);
                        uint8_t fm = F->m[IDX(F->n, i, j, k)];
                        act |= fm & 1;
                        if ((c & 1) && (fm & 16)) cut |= 16;
                        if (((c >> 1) & 1) && (fm & 32)) cut |= 32;
                        if (((c >> 2) & 1) && (fm & 64)) cut |= 64;
                    }
                    C->m[IDX(C->n, I, J, K)] = act | cut;
                }
        /* open faces */
        for (int K = 0; K < C->n[2]; ++K)
            for (int J = 0; J < C->n[1]; ++J)
                for (int I = 0; I < C->n[0]; ++I) {
                    int64_t p = IDX(C->n, I, J, K);
                    int ci[3] = {I, J, K};
                    int64_t st[3] = {1, C->n[0], (int64_t)C->n[0] * C->n[1]};
                    if (!(C->m[p] & 1)) continue;
                    for (int d = 0; d < 3; ++d)
                        if (ci[d] + 1 < C->n[d] && (C->m[p + st[d]] & 1) && !(C->m[p] & (16 << d)))
                            C->m[p] |= (uint8_t)(2 << d);
                }
        /* prolongation maps onto the finer level */
        for (int d = 0; d < 3; ++d) {
            int nf = F->n[d], nc = C->n[d];
            F->pi[d] = malloc(sizeof(int) * nf);
            F->pt[d] = malloc(sizeof(double) * nf);
            for (int i = 0; i < nf; ++i) {
                double x = F->c[d][i];
                if (x < C->c[d][0]) x = C->c[d][0];
                if (x > C->c[d][nc - 1]) x = C->c[d][nc - 1];
                int I0 = box_index(C->c[d], nc, x);
                F->pi[d][i] = I0;
                F->pt[d][i] = (x - C->c[d][I0]) / (C->c[d][I0 + 1] - C->c[d][I0]);
            }
        }
        ++nl;
    }
    M->nl = nl;
}

static void mg_free(MG *M)
{
    for (int l = 0; l < M->nl; ++l) {
        Level *L = &M->L[l];
        for (int d = 0; d < 3; ++d) {
            free(L->f[d]); free(L->c[d]); free(L->w[d]); free(L->cp[d]); free(L->cm[d]);
            if (l + 1 < M->nl) { free(L->pi[d]); free(L->pt[d]); }
        }
        free(L->m);
        if (l > 0) { free(L->x); free(L->b); }
        free(L->r);
    }
    free(M->tmp);
    free(M->bc);
}

/* coarse-level operator row: (A x)_p over open faces; returns diag via *dg */
static double coarse_row(const Level *L, const double *x, int i, int j, int k, int64_t p, double *offsum, double *dg)
{
    int ci[3] = {i, j, k};
    int64_t st[3] = {1, L->n[0], (int64_t)L->n[0] * L->n[1]};
    double acc = 0.0, diag = 0.0;
    for (int d = 0; d < 3; ++d) {
        if (L->m[p] & (2 << d)) { acc += L->cp[d][ci[d]] * x[p + st[d]]; diag += L->cp[d][ci[d]]; }
        if (ci[d] > 0 && (L->m[p - st[d]] & (2 << d))) { acc += L->cm[d][ci[d]] * x[p - st[d]]; diag += L->cm[d][ci[d]]; }
    }
    *offsum = acc;
    *dg = diag;
    return acc - diag * x[p];
}

static void coarse_sweep(const Level *L, double *x, const double *b, int color)
{
    int nx = L->n[0], ny = L->n[1], nz = L->n[2];
#pragma omp parallel for
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                if (((i + j + k) & 1) != color) continue;
                int64_t p = IDX(L->n, i, j, k);
                if (!(L->m[p] & 1)) continue;
                double off, dg;
                coarse_row(L, x, i, j, k, p, &off, &dg);
                x[p] = dg > 0.0 ? (off - b[p]) / dg : 0.0;
            }
}

/* Jacobi on every ghost unknown (closed ghosts and membrane ghost
 * unknowns), all rows reading the same iterate */
static void ghost_jacobi(MG *M, double *x, const double *b);

/* level-0 smoothing step: for each colour (red = (i+j+k) even, then black) a
 * Gauss-Seidel half-sweep over the fluid cells, then Jacobi on all ghost
 * unknowns */
static void fine_smooth(MG *M, double *x, const double *b)
{
    const Sys *S = M->S;
    const Grid *g = &S->g;
    int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    for (int color = 0; color < 2; ++color) {
        /* regular fluid cells of this colour: their neighbours all have the other colour */
#pragma omp parallel for
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    if (((i + j + k) & 1) != color) continue;
                    int64_t p = IDX(g->n, i, j, k);
                    uint8_t f = S->flags[p];
                    if (f & (F_SOLID | F_MGHOST)) continue;
                    double s = cell_scale(g, i, j, k);
                    /* fluid row: sum c (nb - xp) = b  =>  xp = (sum c nb - b) / s */
                    x[p] = (fluid_offsum_elim(S, x, b, i, j, k, p) - b[p]) / s;
                }
        /* then the membrane-adjacent cells of this colour, all from the same
         * iterate (their eliminated ghost stencils may reach each other) */
#pragma omp parallel for
        for (int32_t m = 0; m < S->nm; ++m) {
            int64_t p = S->row_cell[S->ng + m];
            int i = (int)(p % nx), j = (int)((p / nx) % ny), k = (int)(p / ((int64_t)nx * ny));
            if (((i + j + k) & 1) != color) continue;
            M->tmp[m] = (fluid_offsum_elim(S, x, b, i, j, k, p) - b[p]) / cell_scale(g, i, j, k);
        }
        for (int32_t m = 0; m < S->nm; ++m) {
            int64_t p = S->row_cell[S->ng + m];
            int i = (int)(p % nx), j = (int)((p / nx) % ny), k = (int)(p / ((int64_t)nx * ny));
            if (((i + j + k) & 1) == color) x[p] = M->tmp[m];
        }
        ghost_jacobi(M, x, b);
    }
}

static void ghost_jacobi(MG *M, double *x, const double *b)
{
    const Sys *S = M->S;
    int32_t nr = S->ng + S->nm;
#pragma omp parallel for
    for (int32_t r = 0; r < nr; ++r) {
        double acc = 0.0;
        for (int m = 0; m < 8; ++m) {
            int32_t c = S->col[8 * r + m];
            if (c >= 0) acc += S->w[8 * r + m] * x[c];
        }
        M->tmp[r] = acc - b[row_unknown(S, r)] / S->sG[r];
    }
    for (int32_t r = 0; r < nr; ++r) x[row_unknown(S, r)] = M->tmp[r];
}

static void project_mean(const Level *L, double *b)
{
    double sv = 0.0, svb = 0.0;
    for (int k = 0; k < L->n[2]; ++k)
        for (int j = 0; j < L->n[1]; ++j)
            for (int i = 0; i < L->n[0]; ++i) {
                int64_t p = IDX(L->n, i, j, k);
                if (!(L->m[p] & 1)) continue;
                double V = L->w[0][i] * L->w[1][j] * L->w[2][k];
                sv += V;
                svb += V * b[p];
            }
    if (sv <= 0.0) return;
    double mean = svb / sv;
    int64_t Nl = (int64_t)L->n[0] * L->n[1] * L->n[2];
    for (int64_t p = 0; p < Nl; ++p)
        if (L->m[p] & 1) b[p] -= mean;
}

/* restriction (finite-volume): coarse RHS = the volume integral of the
 * active children's residuals over the coarse cell, sum V r / V_coarse; the
 * coarse operator is per full coarse volume, so a coarse cell cut by a body
 * receives the residual of its fluid part only */
static void restrict_res(const Level *F, const double *r, Level *C)
{
#pragma omp parallel for
    for (int K = 0; K < C->n[2]; ++K)
        for (int J = 0; J < C->n[1]; ++J)
            for (int I = 0; I < C->n[0]; ++I) {
                int64_t P = IDX(C->n, I, J, K);
                double sv = 0.0, svr = 0.0;
                for (int c = 0; c < 8; ++c) {
                    int i = 2 * I + (c & 1), j = 2 * J + ((c >> 1) & 1), k = 2 * K + ((c >> 2) & 1);
                    int64_t p = IDX(F->n, i, j, k);
                    if (!(F->m[p] & 1)) continue;
                    double V = F->w[0][i] * F->w[1][j] * F->w[2][k];
                    sv += V;
                    svr += V * r[p];
                }
                C->b[P] = sv > 0.0 ? svr / (C->w[0][I] * C->w[1][J] * C->w[2][K]) : 0.0;
            }
}

/* prolongation: trilinear in physical coordinates over the active coarse
 * nodes (weights renormalised: a node inside a body carries no correction),
 * added to active cells */
static void prolong_add(const Level *F, const Level *C, const double *xc, double *xf)
{
#pragma omp parallel for
    for (int k = 0; k < F->n[2]; ++k)
        for (int j = 0; j < F->n[1]; ++j)
            for (int i = 0; i < F->n[0]; ++i) {
                int64_t p = IDX(F->n, i, j, k);
                if (!(F->m[p] & 1)) continue;
                int I = F->pi[0][i], J = F->pi[1][j], K = F->pi[2][k];
                double tx = F->pt[0][i], ty = F->pt[1][j], tz = F->pt[2][k];
                double v = 0.0, sw = 0.0;
                for (int c = 0; c < 8; ++c) {
                    int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
                    int64_t q = IDX(C->n, I + dx, J + dy, K + dz);
                    if (!(C->m[q] & 1)) continue;
                    double wgt = (dx ? tx : 1.0 - tx) * (dy ? ty : 1.0 - ty) * (dz ? tz : 1.0 - tz);
                    v += wgt * xc[q];
                    sw += wgt;
                }
                if (sw > 0.0) xf[p] += v / sw;
            }
}

static void coarse_residual(const Level *L, const double *x, const double *b, double *r)
{
#pragma omp parallel for
    for (int k = 0; k < L->n[2]; ++k)
        for (int j = 0; j < L->n[1]; ++j)
            for (int i = 0; i < L->n[0]; ++i) {
                int64_t p = IDX(L->n, i, j, k);
                double off, dg;
                r[p] = (L->m[p] & 1) ? b[p] - coarse_row(L, x, i, j, k, p, &off, &dg) : 0.0;
            }
}

static void vcycle_level(MG *M, int l)
{
    Level *L = &M->L[l];
    int64_t Nl = (int64_t)L->n[0] * L->n[1] * L->n[2];
    memset(L->x, 0, sizeof(double) * Nl);
    if (l == M->nl - 1) {
        project_mean(L, L->b);
        for (int s = 0; s < M->ncs; ++s) { coarse_sweep(L, L->x, L->b, 0); coarse_sweep(L, L->x, L->b, 1); }
        return;
    }
    project_mean(L, L->b);
    for (int s = 0; s < M->nu1; ++s) { coarse_sweep(L, L->x, L->b, 0); coarse_sweep(L, L->x, L->b, 1); }
    coarse_residual(L, L->x, L->b, L->r);
    restrict_res(L, L->r, &M->L[l + 1]);
    vcycle_level(M, l + 1);
    prolong_add(L, &M->L[l + 1], M->L[l + 1].x, L->x);
    for (int s = 0; s < M->nu2; ++s) { coarse_sweep(L, L->x, L->b, 0); coarse_sweep(L, L->x, L->b, 1); }
}

/* x = M^{-1} b (one V-cycle from a zero guess) */
static void vcycle(MG *M, const double *b, double *x)
{
    const Sys *S = M->S;
    Level *L0 = &M->L[0];
    int64_t Nt = S->N + S->nm;
    memset(x, 0, sizeof(double) * Nt);
    /* compensating sink: move the volume-weighted net of b into the pin row */
    double *bb = M->bc;
    memcpy(bb, b, sizeof(double) * Nt);
    {
        const Grid *g = &S->g;
        double net = 0.0;
        for (int k = 0; k < g->n[2]; ++k)
            for (int j = 0; j < g->n[1]; ++j)
                for (int i = 0; i < g->n[0]; ++i) {
                    int64_t p = IDX(g->n, i, j, k);
                    if (L0->m[p] & 1) net += g->w[0][i] * g->w[1][j] * g->w[2][k] * b[p];
                }
        int pi = (int)(S->pin % g->n[0]), pj = (int)((S->pin / g->n[0]) % g->n[1]), pk = (int)(S->pin / ((int64_t)g->n[0] * g->n[1]));
        bb[S->pin] -= net / (g->w[0][pi] * g->w[1][pj] * g->w[2][pk]);
    }
    b = bb;
    for (int s = 0; s < M->nu1; ++s) fine_smooth(M, x, b);
    if (M->nl > 1) {
        sys_apply_m(S, x, L0->r, 0);
        for (int64_t p = 0; p < Nt; ++p) L0->r[p] = b[p] - L0->r[p];
        restrict_res(L0, L0->r, &M->L[1]);
        vcycle_level(M, 1);
        prolong_add(L0, &M->L[1], M->L[1].x, x);
    }
    for (int s = 0; s < M->nu2; ++s) fine_smooth(M, x, b);
    /* shift into the pinned subspace: active values and ghost unknowns minus the pin value */
    double c = x[S->pin];
    for (int64_t p = 0; p < S->N; ++p)
        if (L0->m[p] & 1) x[p] -= c;
    for (int32_t m = 0; m < S->nm; ++m) x[S->N + m] -= c;
}

static double dotv(const double *a, const double *b, int64_t n)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s)
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

void orc_vcycle(int nx, int ny, int nz, const double *xf, const double *yf, const double *zf, const uint8_t *flags,
                const int32_t *mg_of, int32_t ng, int32_t nm, const int32_t *row_cell, const int32_t *col,
                const double *w, const double *sG, int nu1, int nu2, int ncs, const double *b, double *x)
{
    Sys S;
    if (sys_init(&S, nx, ny, nz, xf, yf, zf, flags, mg_of, ng, nm, row_cell, col, w, sG)) return;
    MG M;
    mg_build(&M, &S, nu1, nu2, ncs);
    vcycle(&M, b, x);
    mg_free(&M);
    grid_free(&S.g);
}

int orc_num_levels(int nx, int ny, int nz)
{
    int n[3] = {nx, ny, nz}, nl = 1;
    while (1) {
        int ok = 1, mn = n[0];
        for (int d = 0; d < 3; ++d) { if (n[d] % 2) ok = 0; if (n[d] < mn) mn = n[d]; }
        if (!ok || mn <= 4) break;
        for (int d = 0; d < 3; ++d) n[d] /= 2;
        ++nl;
    }
    return nl;
}

/*
 * Scheduled relaxation Jacobi (SRJ), the PPE preconditioner of the paper
 * (Sec. 2.1): m weighted-Jacobi sweeps x <- x + omega_s D^{-1} (b - A x)
 * from x = 0, all rows at once, with D the diagonal of the operator (fluid
 * and pin rows: minus the sum of their face coefficients; ghost rows: -sG).
 * pinned = 0 uses the singular operator (the pin row an ordinary fluid row).
 * shift != 0 then moves the result into the pinned subspace exactly as the
 * V-cycle does (active values and ghost unknowns minus the pin value).
 */
typedef struct {
    int m;
    const double *omega;
    double *dinv, *y;
} SRJ;

static void srj_init(SRJ *R, const Sys *S, int m, const double *omega)
{
    const Grid *g = &S->g;
    int64_t n = S->N + S->nm;
    R->m = m;
    R->omega = omega;
    R->dinv = calloc(n, 8);
    R->y = malloc(8 * n);
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                int64_t p = IDX(g->n, i, j, k);
                if (!(S->flags[p] & F_SOLID)) R->dinv[p] = -1.0 / cell_scale(g, i, j, k);
            }
    for (int32_t r = 0; r < S->ng + S->nm; ++r) R->dinv[row_unknown(S, r)] = -1.0 / S->sG[r];
}

static void srj_free(SRJ *R)
{
    free(R->dinv);
    free(R->y);
}

static void srj_apply(const SRJ *R, const Sys *S, int pinned, int shift, const double *b, double *x)
{
    int64_t n = S->N + S->nm;
    memset(x, 0, 8 * n);
    for (int s = 0; s < R->m; ++s) {
        sys_apply_m(S, x, R->y, pinned);
        const double om = R->omega[s];
#pragma omp parallel for
        for (int64_t q = 0; q < n; ++q) x[q] += om * R->dinv[q] * (b[q] - R->y[q]);
    }
    if (shift) {
        double c = x[S->pin];
        for (int64_t p = 0; p < S->N; ++p)
            if (!(S->flags[p] & F_SOLID) || (S->flags[p] & F_GHOST)) x[p] -= c;
        for (int32_t m = 0; m < S->nm; ++m) x[S->N + m] -= c;
    }
}

void orc_srj(int nx, int ny, int nz, const double *xf, const double *yf, const double *zf, const uint8_t *flags,
             const int32_t *mg_of, int32_t ng, int32_t nm, const int32_t *row_cell, const int32_t *col,
             const double *w, const double *sG, int pinned, int shift, int m, const double *omega, const double *b,
             double *x)
{
    Sys S;
    if (sys_init(&S, nx, ny, nz, xf, yf, zf, flags, mg_of, ng, nm, row_cell, col, w, sG)) return;
    SRJ R;
    srj_init(&R, &S, m, omega);
    srj_apply(&R, &S, pinned, shift, b, x);
    srj_free(&R);
    grid_free(&S.g);
}

/*
 * Right-preconditioned BiCGSTAB (van der Vorst 1992) on the pinned system,
 * preconditioned by the V-cycle (precond 1), by SRJ (precond 2) or by the
 * identity (precond 0).  x holds the initial guess on entry and the solution
 * on exit.  Stops when the recursive relative residual is at most tol and the
 * true one confirms it (else the true residual replaces the recursive one).
 * info[0] iterations, info[1] true relative residual, info[2] restarts.
 */
static int solve_impl(int nx, int ny, int nz, const double *xf, const double *yf, const double *zf,
                      const uint8_t *flags, const int32_t *mg_of, int32_t ng, int32_t nm, const int32_t *row_cell,
                      const int32_t *col, const double *w, const double *sG, const double *b, double *x, double tol,
                      int maxit, int nu1, int nu2, int ncs, int precond, int srj_m, const double *srj_omega,
                      double *info, double *hist)
{
    Sys S;
    if (sys_init(&S, nx, ny, nz, xf, yf, zf, flags, mg_of, ng, nm, row_cell, col, w, sG)) return ORC_EINVAL;
    int64_t n = S.N + nm;
    MG M;
    SRJ R;
    if (precond == 1) mg_build(&M, &S, nu1, nu2, ncs);
    if (precond == 2) srj_init(&R, &S, srj_m, srj_omega);
    double *r = malloc(8 * n), *rh = malloc(8 * n), *p = calloc(n, 8), *v = calloc(n, 8), *ph = malloc(8 * n),
           *s = malloc(8 * n), *sh = malloc(8 * n), *t = malloc(8 * n);
    sys_apply(&S, x, r);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    memcpy(rh, r, 8 * n);
    double bn = sqrt(dotv(b, b, n));
    int rc = ORC_ENOCONV, it = 0, restarts = 0;
    double rel = 0.0;
    if (bn == 0.0) {
        memset(x, 0, 8 * n);
        rc = 0;
        goto done;
    }
    rel = sqrt(dotv(r, r, n)) / bn;
    if (rel <= tol) { rc = 0; goto done; }
    double rho_old = 1.0, alpha = 1.0, omega = 1.0;
    for (it = 1; it <= maxit; ++it) {
        double rho = dotv(rh, r, n);
        double beta;
        if (fabs(rho) < 1e-300 * bn * bn) {
            memcpy(rh, r, 8 * n);
            rho = dotv(rh, r, n);
            memset(p, 0, 8 * n);
            memset(v, 0, 8 * n);
            beta = 0.0;
            ++restarts;
        } else {
            beta = (rho / rho_old) * (alpha / omega);
        }
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        if (precond == 1) vcycle(&M, p, ph);
        else if (precond == 2) srj_apply(&R, &S, 1, 1, p, ph);
        else memcpy(ph, p, 8 * n);
        sys_apply(&S, ph, v);
        double rv = dotv(rh, v, n);
        if (rv == 0.0 || !isfinite(rv)) { rc = ORC_EBREAKDOWN; break; }
        alpha = rho / rv;
        for (int64_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        if (precond == 1) vcycle(&M, s, sh);
        else if (precond == 2) srj_apply(&R, &S, 1, 1, s, sh);
        else memcpy(sh, s, 8 * n);
        sys_apply(&S, sh, t);
        double tt = dotv(t, t, n), ts = dotv(t, s, n);
        omega = tt > 0.0 ? ts / tt : 0.0;
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * ph[i] + omega * sh[i];
            r[i] = s[i] - omega * t[i];
        }
        rho_old = rho;
        rel = sqrt(dotv(r, r, n)) / bn;
        if (hist) hist[it - 1] = rel;
        if (!isfinite(rel)) { rc = ORC_EBREAKDOWN; break; }
        if (rel <= tol) {
            sys_apply(&S, x, t);
            for (int64_t i = 0; i < n; ++i) t[i] = b[i] - t[i];
            double tr = sqrt(dotv(t, t, n)) / bn;
            if (tr <= tol) { rel = tr; rc = 0; break; }
            memcpy(r, t, 8 * n);
            rel = tr;
        }
        if (omega == 0.0) { rc = ORC_EBREAKDOWN; break; }
    }
    if (it > maxit) it = maxit;
done:
    {
        sys_apply(&S, x, t);
        for (int64_t i = 0; i < n; ++i) t[i] = b[i] - t[i];
        info[0] = it;
        info[1] = bn > 0.0 ? sqrt(dotv(t, t, n)) / bn : 0.0;
        info[2] = restarts;
    }
    free(r); free(rh); free(p); free(v); free(ph); free(s); free(sh); free(t);
    if (precond == 1) mg_free(&M);
    if (precond == 2) srj_free(&R);
    grid_free(&S.g);
    return rc;
}

int orc_solve(int nx, int ny, int nz, const double *xf, const double *yf, const double *zf, const uint8_t *flags,
              const int32_t *mg_of, int32_t ng, int32_t nm, const int32_t *row_cell, const int32_t *col,
              const double *w, const double *sG, const double *b, double *x, double tol, int maxit, int nu1, int nu2,
              int ncs, int precond, double *info, double *hist)
{
    return solve_impl(nx, ny, nz, xf, yf, zf, flags, mg_of, ng, nm, row_cell, col, w, sG, b, x, tol, maxit, nu1, nu2,
                      ncs, precond ? 1 : 0, 0, NULL, info, hist);
}

/* BiCGSTAB preconditioned by SRJ (m sweeps with the given schedule). */
int orc_solve_srj(int nx, int ny, int nz, const double *xf, const double *yf, const double *zf,
                  const uint8_t *flags, const int32_t *mg_of, int32_t ng, int32_t nm, const int32_t *row_cell,
                  const int32_t *col, const double *w, const double *sG, const double *b, double *x, double tol,
                  int maxit, int m, const double *omega, double *info, double *hist)
{
    return solve_impl(nx, ny, nz, xf, yf, zf, flags, mg_of, ng, nm, row_cell, col, w, sG, b, x, tol, maxit, 0, 0, 0,
                      2, m, omega, info, hist);
}

#ifdef _OPENMP
#include <omp.h>
int orc_threads(void) { return omp_get_max_threads(); }
#else
int orc_threads(void) { return 1; }
#endif

/* ------------------------------------------------ advection-diffusion step */
/*
 * Implicit diffusion of one velocity component in the fractional step
 * (Sec. 2.1: the advection-diffusion equations are solved with scheduled
 * relaxed Jacobi).  H u = u - beta (L u) on fluid cells, L the 7-point
 * operator of the pressure system (zero-flux walls, the neighbour across a
 * cut membrane link is that neighbour's ghost unknown), beta = nu dt (times
 * 1/2 for Crank-Nicolson); Dirichlet ghost rows sG (sum w u + u_G) from
 * orc_ghost_stencils with bc 1; solid non-ghost rows 0.  No pin.
 */
static void ad_apply(const Sys *S, double beta, const double *x, double *y)
{
    const Grid *g = &S->g;
    int nx = g->n[0], ny = g->n[1], nz = g->n[2];
#pragma omp parallel for
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t p = IDX(g->n, i, j, k);
                if (S->flags[p] & F_SOLID) y[p] = 0.0;
                else y[p] = x[p] - beta * fluid_row(S, x, i, j, k, p);
            }
#pragma omp parallel for
    for (int32_t r = 0; r < S->ng + S->nm; ++r) {
        double acc = 0.0;
        for (int m = 0; m < 8; ++m) {
            int32_t c = S->col[8 * r + m];
            if (c >= 0) acc += S->w[8 * r + m] * x[c];
        }
        int64_t u = row_unknown(S, r);
        y[u] = S->sG[r] * (acc + x[u]);
    }
}

void orc_ad_apply(int nx, int ny, int nz, const double *xf, const double *yf, const double *zf, const uint8_t *flags,
                  const int32_t *mg_of, int32_t ng, int32_t nm, const int32_t *row_cell, const int32_t *col,
                  const double *w, const double *sG, double beta, const double *x, double *y)
{
    Sys S;
    if (sys_init(&S, nx, ny, nz, xf, yf, zf, flags, mg_of, ng, nm, row_cell, col, w, sG)) return;
    ad_apply(&S, beta, x, y);
    grid_free(&S.g);
}

/*
 * SRJ solve of H u = rhs: cycles of m weighted Jacobi sweeps
 * u <- u + omega_s D^-1 (rhs - H u), D the diagonal of H (1 + beta * sum c
 * on fluid rows, sG on ghost rows), from the u given on entry, until the
 * relative residual ||rhs - H u|| / ||rhs|| (checked after every cycle) is
 * at most tol.  Solid non-ghost unknowns are left at 0.
 * info[0] cycles, info[1] final relative residual.  Returns 0, or
 * ORC_ENOCONV after maxcyc cycles.
 */
int orc_ad_solve(int nx, int ny, int nz, const double *xf, const double *yf, const double *zf, const uint8_t *flags,
                 const int32_t *mg_of, int32_t ng, int32_t nm, const int32_t *row_cell, const int32_t *col,
                 const double *w, const double *sG, double beta, const double *rhs, double *x, double tol,
                 int maxcyc, int m, const double *omega, double *info)
{
    Sys S;
    if (sys_init(&S, nx, ny, nz, xf, yf, zf, flags, mg_of, ng, nm, row_cell, col, w, sG)) return ORC_EINVAL;
    const Grid *g = &S.g;
    int64_t n = S.N + nm;
    double *dinv = calloc(n, 8), *y = malloc(8 * n);
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                int64_t p = IDX(g->n, i, j, k);
                if (!(flags[p] & F_SOLID)) dinv[p] = 1.0 / (1.0 + beta * cell_scale(g, i, j, k));
            }
    for (int32_t r = 0; r < ng + nm; ++r) dinv[row_unknown(&S, r)] = 1.0 / sG[r];
    for (int64_t q = 0; q < n; ++q)
        if (dinv[q] == 0.0) x[q] = 0.0;
    double rn = 0.0;
    for (int64_t q = 0; q < n; ++q) rn += rhs[q] * rhs[q];
    rn = sqrt(rn);
    int cyc = 0, rc = ORC_ENOCONV;
    double rel = 0.0;
    ad_apply(&S, beta, x, y);
    {
        double s2 = 0.0;
        for (int64_t q = 0; q < n; ++q) s2 += (rhs[q] - y[q]) * (rhs[q] - y[q]);
        rel = rn > 0.0 ? sqrt(s2) / rn : 0.0;
    }
    if (rel <= tol) rc = 0;
    while (rc != 0 && cyc < maxcyc) {
        for (int s = 0; s < m; ++s) {
            if (s > 0) ad_apply(&S, beta, x, y);
            const double om = omega[s];
#pragma omp parallel for
            for (int64_t q = 0; q < n; ++q) x[q] += om * dinv[q] * (rhs[q] - y[q]);
        }
        ++cyc;
        ad_apply(&S, beta, x, y);
        double s2 = 0.0;
        for (int64_t q = 0; q < n; ++q) s2 += (rhs[q] - y[q]) * (rhs[q] - y[q]);
        rel = rn > 0.0 ? sqrt(s2) / rn : 0.0;
        if (rel <= tol) rc = 0;
    }
    info[0] = cyc;
    info[1] = rel;
    free(dinv);
    free(y);
    grid_free(&S.g);
    return rc;
}
