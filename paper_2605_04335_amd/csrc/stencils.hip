// Ghost-cell boundary rows (Sec. 2.5 module 2) on gfx950.
//
// For every closed ghost cell G (solid with a fluid face neighbour) and every
// membrane ghost cell Q (fluid cell next to a cut link, which carries one
// extra unknown: the field of the far side of the sheet extended to Q):
//   BI  = closest point on the triangles of the same body kind (first
//         triangle on ties), Ericson's Voronoi-region walk;
//   IP  = 2 BI - x_G, dl = 2 |BI - x_G| (image point and its distance);
//   the 8 cell centres around IP (clamped to the centre range) give a
//   trilinear fit: value rows for usable nodes, the Neumann derivative row
//   n . grad b at BI for the node G itself, and "degenerate" for nodes on the
//   wrong side; the weights solve V^T beta = b(IP) by LU with partial
//   pivoting (the batched small inversions of Sec. 2.5);
//   the row is sG (sum beta_k x_k - x_G) = sG (dl - beta_BI) g, scaled like
//   a fluid row; a degenerate box falls back to the mean of the face
//   neighbours on the relevant side.
// Ghost lists are compacted in cell order by a block scan (the array
// compaction of Sec. 2.5).  Compiled with -ffp-contract=off so that distance
// ties and side tests round as written.

#include "common.hpp"

#include <algorithm>
#include <cmath>

namespace ibm {
void classify(const ibm_grid *, const ibm_body *, int, uint8_t *, ibm_class_stats *, hipStream_t);

namespace {

constexpr int CH = 4096;  // cells per compaction block

// ---------------------------------------------------------------- compaction
__global__ void k_count(const uint8_t *flags, long long N, uint8_t mask, int *cnt)
{
    __shared__ int s;
    if (threadIdx.x == 0) s = 0;
    __syncthreads();
    long long base = (long long)blockIdx.x * CH;
    int c = 0;
    for (int t = threadIdx.x; t < CH; t += blockDim.x) {
        long long p = base + t;
        if (p < N && (flags[p] & mask)) ++c;
    }
    atomicAdd(&s, c);
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = s;
}

// exclusive scan of n ints in one block (n may be large: sequential per thread)
__global__ void k_scan1(const int *in, int *out, int n, int *total)
{
    __shared__ int part[1024];
    int per = (n + blockDim.x - 1) / blockDim.x;
    int b = threadIdx.x * per, e = min(n, b + per);
    int s = 0;
    for (int i = b; i < e; ++i) s += in[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int t = 0; t < (int)blockDim.x; ++t) { int v = part[t]; part[t] = acc; acc += v; }
        *total = acc;
    }
    __syncthreads();
    int acc = part[threadIdx.x];
    for (int i = b; i < e; ++i) { out[i] = acc; acc += in[i]; }
}

// ordered fill: each block walks its chunk in steps of blockDim cells, with a
// wave ballot prefix plus an LDS prefix across the waves of the block
__global__ void k_fill(const uint8_t *flags, long long N, uint8_t mask, const int *off, int32_t *out)
{
    __shared__ int wsum[16];
    __shared__ int carry;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (threadIdx.x == 0) carry = off[blockIdx.x];
    __syncthreads();
    long long base = (long long)blockIdx.x * CH;
    for (int t0 = 0; t0 < CH; t0 += blockDim.x) {
        long long p = base + t0 + threadIdx.x;
        bool hit = (t0 + (int)threadIdx.x < CH) && p < N && (flags[p] & mask);
        unsigned long long bal = __ballot(hit);
        int before = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[wid] = __popcll(bal);
        __syncthreads();
        int wo = 0, tot = 0;
        for (int q = 0; q < nw; ++q) {
            if (q < wid) wo += wsum[q];
            tot += wsum[q];
        }
        if (hit) out[carry + wo + before] = (int32_t)p;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
}

// ---------------------------------------------------------------- geometry
struct V3 {
    double x, y, z;
};
__device__ __forceinline__ V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 axpy(V3 a, double s, V3 d) { return {a.x + s * d.x, a.y + s * d.y, a.z + s * d.z}; }

// Closest point on triangle (a,b,c) to p: Ericson, Real-Time Collision
// Detection (2005) Sec. 5.1.5, vertex / edge / face Voronoi regions.
__device__ V3 closest_on_triangle(V3 p, V3 a, V3 b, V3 c)
{
    V3 ab = sub(b, a), ac = sub(c, a), ap = sub(p, a);
    double d1 = dot(ab, ap), d2 = dot(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) return a;
    V3 bp = sub(p, b);
    double d3 = dot(ab, bp), d4 = dot(ac, bp);
    if (d3 >= 0.0 && d4 <= d3) return b;
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) return axpy(a, d1 / (d1 - d3), ab);
    V3 cp = sub(p, c);
    double d5 = dot(ab, cp), d6 = dot(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) return c;
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) return axpy(a, d2 / (d2 - d6), ac);
    double va = d3 * d6 - d5 * d4;
    if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
        double s = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        return axpy(b, s, sub(c, b));
    }
    double den = 1.0 / (va + vb + vc);
    double v = vb * den, w = vc * den;
    V3 q;
    q.x = a.x + ab.x * v + ac.x * w;
    q.y = a.y + ab.y * v + ac.y * w;
    q.z = a.z + ab.z * v + ac.z * w;
    return q;
}

// triangles of a body are grouped in runs of TGROUP consecutive triangles
// (mesh order) with one box per run
constexpr int TGROUP = 32;

struct Tris {
    const double *v;    // [nt*9] vertex coordinates
    const double *box;  // [nt*6] min xyz, max xyz
    const int *kind;    // [nt]
    const double *bbox; // [nb*6] per-body boxes
    const int *bfirst;  // [nb+1] first triangle of each body
    const int *bkind;   // [nb]
    const double *gbox; // [ng*6] boxes of the triangle runs
    const int *gfirst;  // [nb+1] first run of each body
    int nb;
};

struct GridD {
    const double *c[3];  // centres
    const double *w[3];  // widths
    const double *cp[3], *cm[3];
    int n[3];
    double hmin;
};

__device__ __forceinline__ double box_lb(const double *bx, V3 p)
{
    double e, s = 0.0;
    e = p.x < bx[0] ? bx[0] - p.x : (p.x > bx[3] ? p.x - bx[3] : 0.0); s += e * e;
    e = p.y < bx[1] ? bx[1] - p.y : (p.y > bx[4] ? p.y - bx[4] : 0.0); s += e * e;
    e = p.z < bx[2] ? bx[2] - p.z : (p.z > bx[5] ? p.z - bx[5] : 0.0); s += e * e;
    return s;
}

// the largest squared distance from p to a point of the box
__device__ __forceinline__ double box_ub(const double *bx, V3 p)
{
    double e, s = 0.0;
    e = fmax(fabs(p.x - bx[0]), fabs(p.x - bx[3])); s += e * e;
    e = fmax(fabs(p.y - bx[1]), fabs(p.y - bx[4])); s += e * e;
    e = fmax(fabs(p.z - bx[2]), fabs(p.z - bx[5])); s += e * e;
    return s;
}

__device__ __forceinline__ int box_index(const double *c, int n, double x)
{
    // largest i <= n-2 with c[i] <= x (x within [c0, c_{n-1}])
    int lo = 0, hi = n - 2;
    while (lo < hi) {
        int m = (lo + hi + 1) >> 1;
        if (c[m] <= x) lo = m; else hi = m - 1;
    }
    return lo;
}

__device__ __forceinline__ int find_sorted(const int32_t *a, int n, int32_t v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int m = (lo + hi) >> 1;
        if (a[m] < v) lo = m + 1; else hi = m;
    }
    return (lo < n && a[lo] == v) ? lo : -1;
}

struct RowOut {
    int32_t *col;
    double *w, *sG, *dlb, *geo;
    uint8_t *rfl;
};

// One thread per ghost row: intercept, image point, box, 8x8 LU, weights.
__global__ void __launch_bounds__(64) k_stencil(Tris T, GridD G, const uint8_t *flags, const int32_t *cells,
                                                int ng, int nrows, const int32_t *mcell, int nm, long long N, int bc,
                                                RowOut O)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const bool mem = r >= ng;
    const int32_t cell = cells[r];
    const int nx = G.n[0], ny = G.n[1];
    const int ci = cell % nx, cj = (cell / nx) % ny, ck = cell / (nx * ny);
    const V3 P = {G.c[0][ci], G.c[1][cj], G.c[2][ck]};
    const int want = mem ? 1 : 0;
    // A bound on the nearest squared distance before the search: the
    // smallest farthest-point distance of any run box (every run holds a
    // triangle at most that far), with a relative margin far above rounding.
    // Runs, and then triangles, whose box lies farther than the bound or the
    // best distance so far are skipped; the rest are visited in triangle
    // order with the same strict comparison as a plain scan, so the chosen
    // triangle (the first of the nearest) is the plain scan's.
    double ub = INFINITY;
    for (int b = 0; b < T.nb; ++b) {
        if (T.bkind[b] != want) continue;
        for (int g = T.gfirst[b]; g < T.gfirst[b + 1]; ++g) ub = fmin(ub, box_ub(T.gbox + 6 * g, P));
    }
    ub *= 1.0 + 1e-9;
    double best = INFINITY;
    V3 BI = {0, 0, 0};
    int bt = -1;
    for (int b = 0; b < T.nb; ++b) {
        if (T.bkind[b] != want) continue;
        if (box_lb(T.bbox + 6 * b, P) > fmin(best, ub)) continue;
        for (int g = T.gfirst[b]; g < T.gfirst[b + 1]; ++g) {
            if (box_lb(T.gbox + 6 * g, P) > fmin(best, ub)) continue;
            const int t0 = T.bfirst[b] + (g - T.gfirst[b]) * TGROUP, t1 = min(t0 + TGROUP, T.bfirst[b + 1]);
            for (int t = t0; t < t1; ++t) {
                if (box_lb(T.box + 6 * t, P) > fmin(best, ub)) continue;
                const double *tv = T.v + 9 * t;
                V3 q = closest_on_triangle(P, {tv[0], tv[1], tv[2]}, {tv[3], tv[4], tv[5]}, {tv[6], tv[7], tv[8]});
                double d2 = (q.x - P.x) * (q.x - P.x) + (q.y - P.y) * (q.y - P.y) + (q.z - P.z) * (q.z - P.z);
                if (d2 < best) { best = d2; bt = t; BI = q; }
            }
        }
    }
    uint8_t fl = 0;
    double dist = sqrt(best);
    V3 nrm, IP;
    double dl;
    if (bt < 0) {  // no body of this kind: cannot happen for a consistent classification
        nrm = {0, 0, 1}; IP = P; dl = 1.0; dist = 0.0; BI = P;
        fl |= 1;
    } else if (dist < 1e-9 * G.hmin) {
        const double *tv = T.v + 9 * bt;
        V3 e1 = {tv[3] - tv[0], tv[4] - tv[1], tv[5] - tv[2]}, e2 = {tv[6] - tv[0], tv[7] - tv[1], tv[8] - tv[2]};
        V3 fn = {e1.y * e2.z - e1.z * e2.y, e1.z * e2.x - e1.x * e2.z, e1.x * e2.y - e1.y * e2.x};
        double L = sqrt(fn.x * fn.x + fn.y * fn.y + fn.z * fn.z);
        double hl = fmin(G.w[0][ci], fmin(G.w[1][cj], G.w[2][ck]));
        nrm = {fn.x / L, fn.y / L, fn.z / L};
        BI = P;
        IP = {P.x + hl * nrm.x, P.y + hl * nrm.y, P.z + hl * nrm.z};
        dl = hl;
        fl |= 4;
    } else {
        nrm = {(BI.x - P.x) / dist, (BI.y - P.y) / dist, (BI.z - P.z) / dist};
        IP = {2.0 * BI.x - P.x, 2.0 * BI.y - P.y, 2.0 * BI.z - P.z};
        dl = 2.0 * dist;
    }
    const double ipa[3] = {IP.x, IP.y, IP.z}, bia[3] = {BI.x, BI.y, BI.z}, na[3] = {nrm.x, nrm.y, nrm.z};
    int b0[3];
    double loc[3], del[3], bil[3];
    for (int d = 0; d < 3; ++d) {
        const int n = G.n[d];
        const double *c = G.c[d];
        double x = ipa[d];
        if (x < c[0]) x = c[0];
        if (x > c[n - 1]) x = c[n - 1];
        b0[d] = box_index(c, n, x);
        del[d] = c[b0[d] + 1] - c[b0[d]];
        loc[d] = (x - c[b0[d]]) / del[d];
        bil[d] = (bia[d] - c[b0[d]]) / del[d];
    }
    // rows of V (node m) become columns of M = V^T
    double M[8][8];
    int32_t cl[8];
    int dnode = -1;
    bool degenerate = (fl & 1) != 0;
    for (int m = 0; m < 8; ++m) {
        const int dx = m & 1, dy = (m >> 1) & 1, dz = (m >> 2) & 1;
        const int ii = b0[0] + dx, jj = b0[1] + dy, kk = b0[2] + dz;
        const long long id = (long long)ii + (long long)nx * (jj + (long long)ny * kk);
        const uint8_t f = flags[id];
        cl[m] = -1;
        double row[8];
        if (id == cell && bc == 1) {
            // Dirichlet: value row at BI
            const double x = bil[0], y = bil[1], z = bil[2];
            row[0] = 1.0; row[1] = x; row[2] = y; row[3] = z;
            row[4] = x * y; row[5] = y * z; row[6] = x * z; row[7] = x * y * z;
            dnode = m;
        } else if (id == cell) {
            const double x = bil[0], y = bil[1], z = bil[2];
            const double gx[8] = {0, 1, 0, 0, y, 0, z, y * z};
            const double gy[8] = {0, 0, 1, 0, x, z, 0, x * z};
            const double gz[8] = {0, 0, 0, 1, 0, y, x, x * y};
            for (int c = 0; c < 8; ++c) row[c] = na[0] / del[0] * gx[c] + na[1] / del[1] * gy[c] + na[2] / del[2] * gz[c];
            dnode = m;
        } else {
            const double x = dx, y = dy, z = dz;
            row[0] = 1.0; row[1] = x; row[2] = y; row[3] = z;
            row[4] = x * y; row[5] = y * z; row[6] = x * z; row[7] = x * y * z;
            if (!mem) {
                if (!(f & F_SOLID) || (f & F_GHOST)) cl[m] = (int32_t)id;
                else degenerate = true;
            } else {
                double side = na[0] * (G.c[0][ii] - bia[0]) + na[1] * (G.c[1][jj] - bia[1]) + na[2] * (G.c[2][kk] - bia[2]);
                if (side > 0.0) {
                    if (!(f & F_SOLID)) cl[m] = (int32_t)id;
                    else degenerate = true;
                } else {
                    int q = find_sorted(mcell, nm, (int32_t)id);
                    if (q >= 0) cl[m] = (int32_t)(N + q);
                    else degenerate = true;
                }
            }
        }
        for (int c = 0; c < 8; ++c) M[c][m] = row[c];
    }
    double beta[8];
    if (!degenerate) {
        const double x = loc[0], y = loc[1], z = loc[2];
        beta[0] = 1.0; beta[1] = x; beta[2] = y; beta[3] = z;
        beta[4] = x * y; beta[5] = y * z; beta[6] = x * z; beta[7] = x * y * z;
        double amax = 0.0;
        for (int i = 0; i < 8; ++i)
            for (int j = 0; j < 8; ++j) amax = fmax(amax, fabs(M[i][j]));
        for (int c = 0; c < 8 && !degenerate; ++c) {
            int p = c;
            for (int i = c + 1; i < 8; ++i)
                if (fabs(M[i][c]) > fabs(M[p][c])) p = i;
            if (!(fabs(M[p][c]) >= 1e-12 * amax) || amax == 0.0) { degenerate = true; break; }
            if (p != c) {
                for (int j = 0; j < 8; ++j) { double t = M[c][j]; M[c][j] = M[p][j]; M[p][j] = t; }
                double t = beta[c]; beta[c] = beta[p]; beta[p] = t;
            }
            for (int i = c + 1; i < 8; ++i) {
                double l = M[i][c] / M[c][c];
                for (int j = c; j < 8; ++j) M[i][j] -= l * M[c][j];
                beta[i] -= l * beta[c];
            }
        }
        if (!degenerate)
            for (int c = 7; c >= 0; --c) {
                double s = beta[c];
                for (int j = c + 1; j < 8; ++j) s -= M[c][j] * beta[j];
                beta[c] = s / M[c][c];
            }
    }
    const double sg = G.cp[0][ci] + G.cm[0][ci] + G.cp[1][cj] + G.cm[1][cj] + G.cp[2][ck] + G.cm[2][ck];
    double bbi = 0.0;
    int32_t *oc = O.col + 8 * (long long)r;
    double *ow = O.w + 8 * (long long)r;
    if (!degenerate) {
        for (int m = 0; m < 8; ++m) {
            oc[m] = cl[m];
            ow[m] = cl[m] >= 0 ? beta[m] : 0.0;
        }
        if (dnode >= 0) { bbi = beta[dnode]; fl |= 2; }
        O.dlb[r] = bc == 1 ? 2.0 - bbi : dl - bbi;
        if (bc == 1 && (fl & 4)) {
            // ghost on the surface: x_G = g
            for (int m = 0; m < 8; ++m) { oc[m] = -1; ow[m] = 0.0; }
            O.dlb[r] = 1.0;
        }
    } else {
        fl |= 1;
        int cnt = 0;
        int32_t nb[6];
        const int cc[3] = {ci, cj, ck};
        const long long st[3] = {1, nx, (long long)nx * ny};
        for (int d = 0; d < 3; ++d)
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                int c2 = cc[d] + sgn;
                if (c2 < 0 || c2 >= G.n[d]) continue;
                long long id = cell + sgn * st[d];
                bool use;
                if (!mem) use = !(flags[id] & F_SOLID);
                else use = (flags[sgn > 0 ? cell : id] & (F_CUTX << d)) != 0;
                if (use) nb[cnt++] = (int32_t)id;
            }
        for (int m = 0; m < 8; ++m) { oc[m] = -1; ow[m] = 0.0; }
        for (int m = 0; m < cnt; ++m) { oc[m] = nb[m]; ow[m] = 1.0 / cnt; }
        O.dlb[r] = bc == 1 ? 2.0 : 0.0;
    }
    O.sG[r] = sg;
    O.rfl[r] = fl;
    double *g = O.geo + 12 * (long long)r;
    g[0] = BI.x; g[1] = BI.y; g[2] = BI.z;
    g[3] = IP.x; g[4] = IP.y; g[5] = IP.z;
    g[6] = nrm.x; g[7] = nrm.y; g[8] = nrm.z;
    g[9] = dl; g[10] = bbi; g[11] = dist;
}

__global__ void k_count_fallback(const uint8_t *rfl, int n, int *cnt)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int c = (i < n && (rfl[i] & 1)) ? 1 : 0;
    unsigned long long b = __ballot(c);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(cnt, __popcll(b));
}

}  // namespace

// Ordered list of the cells whose flag matches mask; returns the count.
int64_t compact_cells(const uint8_t *flags, long long N, uint8_t mask, DBuf<int32_t> &out, hipStream_t s)
{
    int nb = (int)cdiv(N, CH);
    DBuf<int> cnt(nb), off(nb), tot(1);
    k_count<<<nb, 256, 0, s>>>(flags, N, mask, cnt.p);
    k_scan1<<<1, 1024, 0, s>>>(cnt.p, off.p, nb, tot.p);
    IBM_LAUNCH_CHECK();
    int total = 0;
    IBM_HIP(hipMemcpyAsync(&total, tot.p, sizeof(int), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    out.alloc(std::max(total, 1));
    k_fill<<<nb, 256, 0, s>>>(flags, N, mask, off.p, out.p);
    IBM_LAUNCH_CHECK();
    IBM_HIP(hipStreamSynchronize(s));
    return total;
}

void build_stencils(const ibm_grid *grid, const ibm_body *bodies, int n_body, const uint8_t *flags, ibm_stencils **out,
                    hipStream_t s, int bc = 0)
{
    IBM_REQUIRE(bc == IBM_BC_NEUMANN || bc == IBM_BC_DIRICHLET, IBM_EINVAL, "unknown boundary condition");
    HostGrid g = read_grid(grid);
    IBM_REQUIRE(flags && out, IBM_EINVAL, "null argument");
    IBM_REQUIRE(n_body >= 0 && (n_body == 0 || bodies), IBM_EINVAL, "bad body list");
    const long long N = (long long)g.n[0] * g.n[1] * g.n[2];
    auto *S = new ibm_stencils();
    try {
        for (int d = 0; d < 3; ++d) S->n[d] = g.n[d];
        S->N = N;
        S->bc = bc;
        DBuf<int32_t> gl, ml;
        S->ng = compact_cells(flags, N, F_GHOST, gl, s);
        S->nm = compact_cells(flags, N, F_MGHOST, ml, s);
        // stencil columns are int32: grid unknowns, then membrane ghost unknowns
        IBM_REQUIRE(N + S->nm < ((int64_t)1 << 31), IBM_EINVAL, "more than 2^31 unknowns with the membrane ghosts");
        const int64_t rows = S->ng + S->nm;
        S->cell.alloc(std::max<int64_t>(rows, 1));
        if (S->ng) IBM_HIP(hipMemcpyAsync(S->cell.p, gl.p, S->ng * 4, hipMemcpyDeviceToDevice, s));
        if (S->nm) IBM_HIP(hipMemcpyAsync(S->cell.p + S->ng, ml.p, S->nm * 4, hipMemcpyDeviceToDevice, s));
        S->col.alloc(std::max<int64_t>(rows, 1) * 8);
        S->w.alloc(std::max<int64_t>(rows, 1) * 8);
        S->sG.alloc(std::max<int64_t>(rows, 1));
        S->dlb.alloc(std::max<int64_t>(rows, 1));
        S->rfl.alloc(std::max<int64_t>(rows, 1));
        S->geo.alloc(std::max<int64_t>(rows, 1) * 12);
        // pin (kept with the table for the solver)
        {
            DBuf<int32_t> pl;
            int64_t np = compact_cells(flags, N, F_PIN, pl, s);
            IBM_REQUIRE(np == 1, IBM_EGEOM, "flags must hold exactly one pin cell");
            int32_t pin;
            IBM_HIP(hipMemcpyAsync(&pin, pl.p, 4, hipMemcpyDeviceToHost, s));
            IBM_HIP(hipStreamSynchronize(s));
            S->pin = pin;
        }
        if (rows > 0) {
            // grid on device
            std::vector<double> c[3], w[3], cp[3], cm[3];
            double hmin = 1e300;
            for (int d = 0; d < 3; ++d) {
                int n = g.n[d];
                c[d].resize(n); w[d].resize(n); cp[d].resize(n); cm[d].resize(n);
                for (int i = 0; i < n; ++i) {
                    c[d][i] = 0.5 * (g.f[d][i] + g.f[d][i + 1]);
                    w[d][i] = g.f[d][i + 1] - g.f[d][i];
                    hmin = std::min(hmin, w[d][i]);
                }
                for (int i = 0; i < n; ++i) {
                    cp[d][i] = (i + 1 < n) ? 1.0 / (w[d][i] * (c[d][i + 1] - c[d][i])) : 0.0;
                    cm[d][i] = (i > 0) ? 1.0 / (w[d][i] * (c[d][i] - c[d][i - 1])) : 0.0;
                }
            }
            DBuf<double> dc[3], dw[3], dcp[3], dcm[3];
            GridD G;
            for (int d = 0; d < 3; ++d) {
                upload(dc[d], c[d], s); upload(dw[d], w[d], s); upload(dcp[d], cp[d], s); upload(dcm[d], cm[d], s);
                G.c[d] = dc[d].p; G.w[d] = dw[d].p; G.cp[d] = dcp[d].p; G.cm[d] = dcm[d].p; G.n[d] = g.n[d];
            }
            G.hmin = hmin;
            // triangles, flattened in (body, triangle) order
            std::vector<double> tv, tb, bb, gbx;
            std::vector<int> tk, bf, bk, gf;
            bf.push_back(0);
            gf.push_back(0);
            for (int b = 0; b < n_body; ++b) {
                const ibm_body &B = bodies[b];
                IBM_REQUIRE(B.vert && B.tri && B.n_tri > 0, IBM_EINVAL, "empty body");
                double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
                for (int t = 0; t < B.n_tri; ++t) {
                    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
                    for (int m = 0; m < 3; ++m) {
                        int v = B.tri[3 * t + m];
                        IBM_REQUIRE(v >= 0 && v < B.n_vert, IBM_EGEOM, "triangle index out of range");
                        for (int d = 0; d < 3; ++d) {
                            double x = B.vert[3 * v + d];
                            tv.push_back(x);
                            mn[d] = std::min(mn[d], x);
                            mx[d] = std::max(mx[d], x);
                        }
                    }
                    for (int d = 0; d < 3; ++d) { tb.push_back(mn[d]); lo[d] = std::min(lo[d], mn[d]); }
                    for (int d = 0; d < 3; ++d) { tb.push_back(mx[d]); hi[d] = std::max(hi[d], mx[d]); }
                    tk.push_back(B.kind);
                }
                for (int d = 0; d < 3; ++d) bb.push_back(lo[d]);
                for (int d = 0; d < 3; ++d) bb.push_back(hi[d]);
                bk.push_back(B.kind);
                bf.push_back(bf.back() + B.n_tri);
                // boxes of the runs of TGROUP consecutive triangles
                for (int t0 = bf[b]; t0 < bf[b + 1]; t0 += TGROUP) {
                    double glo[3] = {1e300, 1e300, 1e300}, ghi[3] = {-1e300, -1e300, -1e300};
                    for (int t = t0; t < std::min(t0 + TGROUP, bf[b + 1]); ++t)
                        for (int d = 0; d < 3; ++d) {
                            glo[d] = std::min(glo[d], tb[6 * (size_t)t + d]);
                            ghi[d] = std::max(ghi[d], tb[6 * (size_t)t + 3 + d]);
                        }
                    for (int d = 0; d < 3; ++d) gbx.push_back(glo[d]);
                    for (int d = 0; d < 3; ++d) gbx.push_back(ghi[d]);
                }
                gf.push_back((int)(gbx.size() / 6));
            }
            DBuf<double> dtv, dtb, dbb, dgb;
            DBuf<int> dtk, dbf, dbk, dgf;
            upload(dtv, tv, s); upload(dtb, tb, s); upload(dbb, bb, s); upload(dgb, gbx, s);
            upload(dtk, tk, s); upload(dbf, bf, s); upload(dbk, bk, s); upload(dgf, gf, s);
            Tris T{dtv.p, dtb.p, dtk.p, dbb.p, dbf.p, dbk.p, dgb.p, dgf.p, n_body};
            RowOut O{S->col.p, S->w.p, S->sG.p, S->dlb.p, S->geo.p, S->rfl.p};
            k_stencil<<<cdiv(rows, 64), 64, 0, s>>>(T, G, flags, S->cell.p, (int)S->ng, (int)rows, S->cell.p + S->ng,
                                                   (int)S->nm, N, bc, O);
            IBM_LAUNCH_CHECK();
            DBuf<int> nf(1);
            IBM_HIP(hipMemsetAsync(nf.p, 0, 4, s));
            k_count_fallback<<<cdiv(rows, 256), 256, 0, s>>>(S->rfl.p, (int)rows, nf.p);
            IBM_LAUNCH_CHECK();
            int h = 0;
            IBM_HIP(hipMemcpyAsync(&h, nf.p, 4, hipMemcpyDeviceToHost, s));
            IBM_HIP(hipStreamSynchronize(s));
            S->nfallback = h;
        }
    } catch (...) {
        delete S;
        throw;
    }
    *out = S;
}

}  // namespace ibm

extern "C" int32_t ibm_build_ghost_stencils(const ibm_grid *grid, const ibm_body *bodies, int32_t n_body,
                                            const uint8_t *flags_dev, ibm_stencils **out, void *stream)
{
    return ibm::guarded([&] { ibm::build_stencils(grid, bodies, n_body, flags_dev, out, (hipStream_t)stream); });
}

extern "C" int32_t ibm_build_ghost_stencils_bc(const ibm_grid *grid, const ibm_body *bodies, int32_t n_body,
                                               const uint8_t *flags_dev, int32_t bc, ibm_stencils **out, void *stream)
{
    return ibm::guarded(
        [&] { ibm::build_stencils(grid, bodies, n_body, flags_dev, out, (hipStream_t)stream, bc); });
}

extern "C" int32_t ibm_stencils_info(const ibm_stencils *s, int64_t *n_ghost, int64_t *n_mghost, int64_t *n_fallback)
{
    return ibm::guarded([&] {
        IBM_REQUIRE(s, IBM_EINVAL, "null stencils");
        if (n_ghost) *n_ghost = s->ng;
        if (n_mghost) *n_mghost = s->nm;
        if (n_fallback) *n_fallback = s->nfallback;
    });
}

extern "C" int32_t ibm_stencils_export(const ibm_stencils *s, int32_t *cell, int32_t *col, double *w, double *sG,
                                       double *dlb, uint8_t *rflags, double *geo)
{
    return ibm::guarded([&] {
        IBM_REQUIRE(s, IBM_EINVAL, "null stencils");
        size_t rows = (size_t)(s->ng + s->nm);
        if (!rows) return;
        // copies on a private non-blocking stream: nothing here touches the
        // legacy stream, which may not depend on another thread's capture
        hipStream_t st = nullptr;
        IBM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        struct Del {
            hipStream_t q;
            ~Del() { (void)hipStreamDestroy(q); }
        } del{st};
        if (cell) IBM_HIP(hipMemcpyAsync(cell, s->cell.p, rows * 4, hipMemcpyDeviceToHost, st));
        if (col) IBM_HIP(hipMemcpyAsync(col, s->col.p, rows * 32, hipMemcpyDeviceToHost, st));
        if (w) IBM_HIP(hipMemcpyAsync(w, s->w.p, rows * 64, hipMemcpyDeviceToHost, st));
        if (sG) IBM_HIP(hipMemcpyAsync(sG, s->sG.p, rows * 8, hipMemcpyDeviceToHost, st));
        if (dlb) IBM_HIP(hipMemcpyAsync(dlb, s->dlb.p, rows * 8, hipMemcpyDeviceToHost, st));
        if (rflags) IBM_HIP(hipMemcpyAsync(rflags, s->rfl.p, rows, hipMemcpyDeviceToHost, st));
        if (geo) IBM_HIP(hipMemcpyAsync(geo, s->geo.p, rows * 96, hipMemcpyDeviceToHost, st));
        IBM_HIP(hipStreamSynchronize(st));
    });
}

extern "C" void ibm_stencils_free(ibm_stencils *s) { delete s; }
