// Pressure loads on the body surfaces (Sec. 2.3.1, Eq. fext without the
// shear term), the consumer of the pressure in the fluid-structure loop
// (Sec. 2.4).
//
// Per triangle j: centroid c, area A, unit normal n = (v1-v0) x (v2-v0)/|.|,
// probe distance d = 2 max(w_x, w_y, w_z) of the cell containing c.  The
// pressure is interpolated trilinearly from the cell centres at c + d n
// (and at c - d n for a membrane); box nodes in solid non-ghost cells are
// dropped and the remaining weights renormalised.  dp = p+ - p- (membrane)
// or p+ (closed body, fluid outside).  Every node of the triangle receives
// -(1/3) dp n A; a node's sum runs over its triangles in a fixed order (as
// vertex 0 in triangle order, then as vertex 1, then as vertex 2), so the
// result does not depend on scheduling.  Compiled with -ffp-contract=off:
// every product and sum rounds as written.

#include "common.hpp"

#include <algorithm>
#include <cmath>

namespace ibm {
namespace {

struct FGrid {
    const double *c[3];  // cell centres
    const double *f[3];  // faces
    int n[3];
};

// largest i with a[i] <= x among a[0..n), or -1
__device__ int last_le(const double *a, int n, double x)
{
    int lo = 0, hi = n;  // first index with a[i] > x
    while (lo < hi) {
        const int m = (lo + hi) >> 1;
        if (a[m] <= x) lo = m + 1;
        else hi = m;
    }
    return lo - 1;
}

// trilinear interpolation of p at x with solid non-ghost nodes dropped;
// false when no node is usable (value 0)
__device__ bool interp(const FGrid &G, const uint8_t *flags, const double *p, const double x[3], double &out)
{
    int i0[3];
    double t[3];
    for (int d = 0; d < 3; ++d) {
        int i = last_le(G.c[d], G.n[d], x[d]);
        i = min(max(i, 0), G.n[d] - 2);
        double tt = (x[d] - G.c[d][i]) / (G.c[d][i + 1] - G.c[d][i]);
        tt = fmin(fmax(tt, 0.0), 1.0);
        i0[d] = i;
        t[d] = tt;
    }
    double num = 0.0, den = 0.0;
    for (int q = 0; q < 8; ++q) {
        const int o0 = q & 1, o1 = (q >> 1) & 1, o2 = (q >> 2) & 1;
        double w = o0 ? t[0] : 1.0 - t[0];
        w = w * (o1 ? t[1] : 1.0 - t[1]);
        w = w * (o2 ? t[2] : 1.0 - t[2]);
        const long long cell = (long long)(i0[0] + o0) +
                               (long long)G.n[0] * ((i0[1] + o1) + (long long)G.n[1] * (i0[2] + o2));
        const uint8_t f = flags[cell];
        if ((f & F_SOLID) && !(f & F_GHOST)) w = 0.0;
        num = num + w * p[cell];
        den = den + w;
    }
    if (den > 0.0) {
        out = num / den;
        return true;
    }
    out = 0.0;
    return false;
}

// one thread per triangle: dp and the per-node contribution -(1/3) dp n A
__global__ void k_tri_loads(FGrid G, const uint8_t *__restrict__ flags, const double *__restrict__ p,
                            const double *__restrict__ vert, const int32_t *__restrict__ tri,
                            const int32_t *__restrict__ tkind, int nt, double *__restrict__ dp_out,
                            double *__restrict__ contrib, int *lost)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nt) return;
    const double *a = vert + 3 * (long long)tri[3 * j], *b = vert + 3 * (long long)tri[3 * j + 1],
                 *c = vert + 3 * (long long)tri[3 * j + 2];
    double cen[3], u[3], v[3];
    for (int d = 0; d < 3; ++d) {
        cen[d] = (a[d] + b[d] + c[d]) / 3.0;
        u[d] = b[d] - a[d];
        v[d] = c[d] - a[d];
    }
    const double cr[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
    const double nrm = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    const double un[3] = {cr[0] / nrm, cr[1] / nrm, cr[2] / nrm};
    const double area = 0.5 * nrm;
    double h = 0.0;
    for (int d = 0; d < 3; ++d) {
        int k = last_le(G.f[d], G.n[d] + 1, cen[d]);
        k = min(max(k, 0), G.n[d] - 1);
        h = fmax(h, G.f[d][k + 1] - G.f[d][k]);
    }
    const double dist = 2.0 * h;
    double xp[3], xm[3];
    for (int d = 0; d < 3; ++d) {
        const double s = dist * un[d];
        xp[d] = cen[d] + s;
        xm[d] = cen[d] - s;
    }
    double pp, pm = 0.0;
    int bad = interp(G, flags, p, xp, pp) ? 0 : 1;
    if (tkind[j] == IBM_KIND_MEMBRANE) bad += interp(G, flags, p, xm, pm) ? 0 : 1;
    const double dp = tkind[j] == IBM_KIND_MEMBRANE ? pp - pm : pp;
    dp_out[j] = dp;
    const double s = -(dp * area);
    for (int d = 0; d < 3; ++d) contrib[3 * (long long)j + d] = s * un[d] / 3.0;
    if (bad) atomicAdd(lost, bad);
}

// one thread per node: the sum of its triangles' contributions in CSR order
__global__ void k_node_loads(const int64_t *__restrict__ start, const int32_t *__restrict__ list, long long nv,
                             const double *__restrict__ contrib, double *__restrict__ force)
{
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= nv) return;
    double f0 = 0.0, f1 = 0.0, f2 = 0.0;
    for (long long e = start[i]; e < start[i + 1]; ++e) {
        const long long j = list[e];
        f0 = f0 + contrib[3 * j];
        f1 = f1 + contrib[3 * j + 1];
        f2 = f2 + contrib[3 * j + 2];
    }
    force[3 * i] = f0;
    force[3 * i + 1] = f1;
    force[3 * i + 2] = f2;
}

}  // namespace
}  // namespace ibm

using namespace ibm;

extern "C" int32_t ibm_surface_forces(const ibm_grid *grid, const ibm_body *bodies, int32_t n_body,
                                      const uint8_t *flags_dev, const double *p_dev, double *force_dev,
                                      double *dp_dev, int64_t *n_lost, void *stream)
{
    return guarded([&] {
        IBM_REQUIRE(grid && flags_dev && p_dev && force_dev && (n_body == 0 || bodies), IBM_EINVAL,
                    "null argument");
        const HostGrid g = read_grid(grid);
        for (int d = 0; d < 3; ++d) IBM_REQUIRE(g.n[d] >= 2, IBM_EINVAL, "grid needs two cells per axis");
        hipStream_t s = (hipStream_t)stream;
        // flattened mesh: global vertex and triangle numbering, body by body
        std::vector<double> hv;
        std::vector<int32_t> ht, hk;
        long long nv = 0;
        for (int b = 0; b < n_body; ++b) {
            const ibm_body &B = bodies[b];
            IBM_REQUIRE(B.vert && B.tri && B.n_vert > 0 && B.n_tri > 0, IBM_EINVAL, "empty body");
            hv.insert(hv.end(), B.vert, B.vert + 3 * (size_t)B.n_vert);
            for (int t = 0; t < B.n_tri; ++t) {
                for (int m = 0; m < 3; ++m) {
                    const int v = B.tri[3 * t + m];
                    IBM_REQUIRE(v >= 0 && v < B.n_vert, IBM_EGEOM, "triangle index out of range");
                    ht.push_back((int32_t)(nv + v));
                }
                hk.push_back(B.kind);
            }
            nv += B.n_vert;
        }
        const int nt = (int)hk.size();
        if (n_lost) *n_lost = 0;
        if (!nt) return;
        // node -> triangles, ordered by (vertex slot m, triangle j)
        std::vector<int64_t> start(nv + 1, 0);
        for (int m = 0; m < 3; ++m)
            for (int j = 0; j < nt; ++j) ++start[ht[3 * j + m] + 1];
        for (long long i = 0; i < nv; ++i) start[i + 1] += start[i];
        std::vector<int32_t> list(3 * (size_t)nt);
        {
            std::vector<int64_t> pos(start.begin(), start.end() - 1);
            for (int m = 0; m < 3; ++m)
                for (int j = 0; j < nt; ++j) list[pos[ht[3 * j + m]]++] = j;
        }
        std::vector<double> cc[3];
        DBuf<double> dc[3], df[3];
        FGrid G;
        for (int d = 0; d < 3; ++d) {
            cc[d].resize(g.n[d]);
            for (int i = 0; i < g.n[d]; ++i) cc[d][i] = 0.5 * (g.f[d][i] + g.f[d][i + 1]);
            upload(dc[d], cc[d], s);
            upload(df[d], g.f[d], s);
            G.c[d] = dc[d].p;
            G.f[d] = df[d].p;
            G.n[d] = g.n[d];
        }
        DBuf<double> dv, contrib(3 * (size_t)nt), dpb;
        DBuf<int32_t> dt, dk, dl;
        DBuf<int64_t> ds;
        DBuf<int> lost(1);
        upload(dv, hv, s);
        upload(dt, ht, s);
        upload(dk, hk, s);
        upload(ds, start, s);
        upload(dl, list, s);
        double *dpo = dp_dev;
        if (!dpo) {
            dpb.alloc(nt);
            dpo = dpb.p;
        }
        IBM_HIP(hipMemsetAsync(lost.p, 0, sizeof(int), s));
        k_tri_loads<<<(nt + 255) / 256, 256, 0, s>>>(G, flags_dev, p_dev, dv.p, dt.p, dk.p, nt, dpo, contrib.p,
                                                      lost.p);
        k_node_loads<<<(int)((nv + 255) / 256), 256, 0, s>>>(ds.p, dl.p, nv, contrib.p, force_dev);
        IBM_LAUNCH_CHECK();
        int hl = 0;
        IBM_HIP(hipMemcpyAsync(&hl, lost.p, sizeof(int), hipMemcpyDeviceToHost, s));
        IBM_HIP(hipStreamSynchronize(s));
        if (n_lost) *n_lost = hl;
    });
}
