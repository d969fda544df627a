// Implicit advection-diffusion step of one velocity component, solved with
// scheduled relaxed Jacobi (Sec. 2.1: the paper solves the advection-
// diffusion equations with SRJ and the pressure with BiCGStab).
//
// H u = u - beta L u on fluid cells, L the 7-point operator of the pressure
// system (zero-flux walls; across a cut membrane link the neighbour's ghost
// unknown, i.e. the far side's field); Dirichlet ghost rows
// sG (sum w u + u_G) = sG (2 - beta_BI) g from the image-point stencils
// built with IBM_BC_DIRICHLET; solid non-ghost unknowns stay 0.
// An SRJ cycle is m weighted Jacobi sweeps u <- u + omega_s D^-1 (rhs - H u)
// with the Chebyshev factors on the spectrum interval [a, 2 - a] of D^-1 H,
// a = 1 / (1 + beta max sum c); the residual is checked after every cycle.
//
// Unknowns stay in natural order (x fastest; membrane ghost unknowns at
// N + m): Jacobi needs no colouring, and a sweep reads each neighbour plane
// once.  Compiled with -ffp-contract=off: every row is evaluated in the
// order of its definition, so results do not depend on contraction choices.

#include "common.hpp"

#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

namespace ibm {
namespace {

constexpr int ATPB = 256;

struct AdGrid {
    int nx, ny, nz;
    long long N;
    const double *cp[3], *cm[3];  // zero-flux walls: the wall-side coefficient is never used
};

struct AdRows {
    int ng, nm, nrows;
    const int32_t *col;    // [nrows*8] natural unknowns (cell, or N + m), -1 unused
    const double *w, *sG, *dlb;
    const int32_t *rcell;  // [ng] closed ghost cells
    const int32_t *mcell;  // [nm] membrane cells (sorted)
    const int32_t *mcol;   // [nm*6] -x,+x,-y,+y,-z,+z neighbour unknowns (-1 at a wall)
};

__device__ __forceinline__ long long row_unknown(const AdRows &R, const AdGrid &G, int r)
{
    return r < R.ng ? (long long)R.rcell[r] : G.N + (r - R.ng);
}

// membrane cell: neighbours from its six columns (ghost unknowns across cut links)
__device__ __forceinline__ double h_membrane(const AdGrid &G, const AdRows &R, double beta, const double *x, int m,
                                             double &dg)
{
    const long long p = R.mcell[m];
    const int i = (int)(p % G.nx), j = (int)((p / G.nx) % G.ny), k = (int)(p / ((long long)G.nx * G.ny));
    const int ci[3] = {i, j, k};
    const double xp = x[p];
    const int32_t *mc = R.mcol + 6 * (long long)m;
    double acc = 0.0;
    for (int d = 0; d < 3; ++d) {
        if (mc[2 * d + 1] >= 0) acc += G.cp[d][ci[d]] * (x[mc[2 * d + 1]] - xp);
        if (mc[2 * d] >= 0) acc += G.cm[d][ci[d]] * (x[mc[2 * d]] - xp);
    }
    dg = G.cp[0][i] + G.cm[0][i] + G.cp[1][j] + G.cm[1][j] + G.cp[2][k] + G.cm[2][k];
    return xp - beta * acc;
}

__device__ __forceinline__ double h_ghost(const AdGrid &G, const AdRows &R, const double *x, int r, long long u)
{
    double acc = 0.0;
    const int32_t *c = R.col + 8 * (long long)r;
    const double *w = R.w + 8 * (long long)r;
    for (int q = 0; q < 8; ++q)
        if (c[q] >= 0) acc += w[q] * x[c[q]];
    return R.sG[r] * (acc + x[u]);
}

// Jacobi sweep (JAC) or y = H x on the regular cells.  A 64 x 4 block
// covers (i, j) of a tile and each thread walks KZ planes, keeping the
// iterate of planes k-1, k, k+1 in registers (each plane is loaded once).
// Tiles are remapped so that each XCD owns a contiguous range (its own L2).
constexpr int AD_KZ = 16;
enum { AD_APPLY = 0, AD_JACOBI = 1, AD_RESID = 2 };

// block sums of a and b into part[2 blk], part[2 blk + 1] (fixed order)
__device__ __forceinline__ void ad_block_sums(double a, double b, double *part)
{
    __shared__ double s0[ATPB / 64], s1[ATPB / 64];
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_down(a, o, 64);
        b += __shfl_down(b, o, 64);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) { s0[wv] = a; s1[wv] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0;
        for (int q = 0; q < ATPB / 64; ++q) { ta += s0[q]; tb += s1[q]; }
        part[2 * blockIdx.x] = ta;
        part[2 * blockIdx.x + 1] = tb;
    }
}
struct AdTiles {
    int gx, gy, gz, per;
};
// MODE: y = H x (AD_APPLY), a Jacobi sweep into y (AD_JACOBI), or per-block
// sums of (rhs - H x)^2 and rhs^2 into part (AD_RESID, nothing written)
template <int MODE>
__global__ void __launch_bounds__(ATPB) k_ad_dense(AdGrid G, AdTiles T, const uint8_t *__restrict__ flags, double beta,
                                                   double omega, const double *__restrict__ x, double *__restrict__ y,
                                                   const double *__restrict__ rhs, double *part)
{
    const int t = (int)(blockIdx.x & 7) * T.per + (int)(blockIdx.x >> 3);
    const int tx = t % T.gx, ty = (t / T.gx) % T.gy, tz = t / (T.gx * T.gy);
    const int i = tx * 64 + (int)(threadIdx.x & 63), j = ty * 4 + (int)(threadIdx.x >> 6);
    double ra = 0.0, rb = 0.0;
    if (t < T.gx * T.gy * T.gz && i < G.nx && j < G.ny) {
        const int k0 = tz * AD_KZ, k1 = min(k0 + AD_KZ, G.nz);
        const long long pl = (long long)G.nx * G.ny;
        long long p = (long long)i + (long long)G.nx * (j + (long long)G.ny * k0);
        const double cpx = G.cp[0][i], cmx = G.cm[0][i], cpy = G.cp[1][j], cmy = G.cm[1][j];
        const bool hx_p = i + 1 < G.nx, hx_m = i > 0, hy_p = j + 1 < G.ny, hy_m = j > 0;
        double xm = k0 > 0 ? x[p - pl] : 0.0, xc = x[p];
        for (int k = k0; k < k1; ++k, p += pl) {
            const double xn = k + 1 < G.nz ? x[p + pl] : 0.0;
            const uint8_t f = flags[p];
            const double vxp = hx_p ? x[p + 1] : 0.0, vxm = hx_m ? x[p - 1] : 0.0;
            const double vyp = hy_p ? x[p + G.nx] : 0.0, vym = hy_m ? x[p - G.nx] : 0.0;
            const double bv = MODE != AD_APPLY ? rhs[p] : 0.0;
            if (f & F_SOLID) {
                if (!(f & F_GHOST)) {  // ghost rows: the sparse kernel
                    if (MODE == AD_RESID) { ra += bv * bv; rb += bv * bv; }
                    else y[p] = 0.0;
                }
            } else if (!(f & F_MGHOST)) {  // cells with cut links: the sparse kernel
                // the order of the definition: +x, -x, +y, -y, +z, -z
                double acc = 0.0;
                if (hx_p) acc += cpx * (vxp - xc);
                if (hx_m) acc += cmx * (vxm - xc);
                if (hy_p) acc += cpy * (vyp - xc);
                if (hy_m) acc += cmy * (vym - xc);
                if (k + 1 < G.nz) acc += G.cp[2][k] * (xn - xc);
                if (k > 0) acc += G.cm[2][k] * (xm - xc);
                const double hx = xc - beta * acc;
                if (MODE == AD_JACOBI) {
                    const double dg = cpx + cmx + cpy + cmy + G.cp[2][k] + G.cm[2][k];
                    const double dinv = 1.0 / (1.0 + beta * dg);
                    y[p] = xc + omega * dinv * (bv - hx);
                } else if (MODE == AD_RESID) {
                    const double r = bv - hx;
                    ra += r * r;
                    rb += bv * bv;
                } else {
                    y[p] = hx;
                }
            }
            xm = xc;
            xc = xn;
        }
    }
    if (MODE == AD_RESID) ad_block_sums(ra, rb, part);
}

// the same for ghost rows (r < nrows) and membrane cells (nrows + m)
template <int MODE>
__global__ void __launch_bounds__(ATPB) k_ad_sparse(AdGrid G, AdRows R, double beta, double omega,
                                                    const double *__restrict__ x, double *__restrict__ y,
                                                    const double *__restrict__ rhs, double *part)
{
    const int n = R.nrows + R.nm;
    double ra = 0.0, rb = 0.0;
    for (int q = blockIdx.x * ATPB + threadIdx.x; q < n; q += gridDim.x * ATPB) {
        long long u;
        double hx, dinv;
        if (q < R.nrows) {
            u = row_unknown(R, G, q);
            hx = h_ghost(G, R, x, q, u);
            dinv = 1.0 / R.sG[q];
        } else {
            const int m = q - R.nrows;
            u = R.mcell[m];
            double dg;
            hx = h_membrane(G, R, beta, x, m, dg);
            dinv = 1.0 / (1.0 + beta * dg);
        }
        if (MODE == AD_JACOBI) {
            y[u] = x[u] + omega * dinv * (rhs[u] - hx);
        } else if (MODE == AD_RESID) {
            const double r = rhs[u] - hx;
            ra += r * r;
            rb += rhs[u] * rhs[u];
        } else {
            y[u] = hx;
        }
    }
    if (MODE == AD_RESID) ad_block_sums(ra, rb, part);
}

// right-hand side: f on fluid cells, 0 on solid cells, sG dlb g on ghost rows
__global__ void __launch_bounds__(ATPB) k_ad_rhs(AdGrid G, const uint8_t *__restrict__ flags,
                                                 const double *__restrict__ f, double *__restrict__ rhs)
{
    for (long long p = blockIdx.x * (long long)ATPB + threadIdx.x; p < G.N; p += (long long)gridDim.x * ATPB)
        rhs[p] = (flags[p] & F_SOLID) ? 0.0 : f[p];
}
__global__ void __launch_bounds__(ATPB) k_ad_rhs_rows(AdGrid G, AdRows R, const double *__restrict__ g,
                                                      double *__restrict__ rhs)
{
    for (int r = blockIdx.x * ATPB + threadIdx.x; r < R.nrows; r += gridDim.x * ATPB)
        rhs[row_unknown(R, G, r)] = g ? R.sG[r] * R.dlb[r] * g[r] : 0.0;
}

// unknowns of solid non-ghost cells start (and stay) at zero
__global__ void __launch_bounds__(ATPB) k_ad_zero_solid(AdGrid G, const uint8_t *__restrict__ flags, double *x)
{
    for (long long p = blockIdx.x * (long long)ATPB + threadIdx.x; p < G.N; p += (long long)gridDim.x * ATPB)
        if ((flags[p] & F_SOLID) && !(flags[p] & F_GHOST)) x[p] = 0.0;
}

// membrane cells: the unknown behind each face (natural numbering)
__global__ void __launch_bounds__(ATPB) k_ad_membrane(AdGrid G, int nm, const int32_t *__restrict__ mcell,
                                                      const uint8_t *__restrict__ flags, int32_t *__restrict__ mc,
                                                      int *err)
{
    for (int q = blockIdx.x * ATPB + threadIdx.x; q < nm; q += gridDim.x * ATPB) {
        const long long p = mcell[q];
        const int ci[3] = {(int)(p % G.nx), (int)((p / G.nx) % G.ny), (int)(p / ((long long)G.nx * G.ny))};
        const int nd[3] = {G.nx, G.ny, G.nz};
        const long long sd[3] = {1, G.nx, (long long)G.nx * G.ny};
        for (int d = 0; d < 3; ++d)
            for (int sg = 0; sg < 2; ++sg) {
                int32_t out = -1;
                const int c2 = ci[d] + (sg ? 1 : -1);
                if (c2 >= 0 && c2 < nd[d]) {
                    const long long nb = p + (sg ? sd[d] : -sd[d]);
                    if (flags[sg ? p : nb] & (F_CUTX << d)) {
                        int a = 0, b = nm;
                        while (a < b) {
                            const int h = (a + b) >> 1;
                            if (mcell[h] < nb) a = h + 1;
                            else b = h;
                        }
                        if (a < nm && mcell[a] == nb) out = (int32_t)(G.N + a);
                        else *err = 1;
                    } else {
                        out = (int32_t)nb;
                    }
                }
                mc[6 * (long long)q + 2 * d + sg] = out;
            }
    }
}

}  // namespace
}  // namespace ibm

using namespace ibm;

struct ibm_ad_ctx {
    ibm_ad_opts opts;
    AdGrid G;
    AdRows R;
    long long Nt = 0;
    double dg_max = 0.0;
    std::vector<double> omega;
    DBuf<double> cp[3], cm[3];
    DBuf<uint8_t> flags;
    DBuf<int32_t> col, rcell, mcell, mcol;
    DBuf<double> w, sG, dlb;
    DBuf<double> rhs, xa, xb, part;
    DBuf<int> err;
    hipStream_t cs = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr, ej = nullptr;
    ~ibm_ad_ctx()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (ej) (void)hipEventDestroy(ej);
        if (cs) (void)hipStreamDestroy(cs);
    }
};

namespace {


struct AdJoin {
    ibm_ad_ctx &c;
    hipStream_t user;
    AdJoin(ibm_ad_ctx &cc, hipStream_t u) : c(cc), user(u)
    {
        IBM_HIP(hipEventRecord(c.ej, user));
        IBM_HIP(hipStreamWaitEvent(c.cs, c.ej, 0));
    }
    ~AdJoin()
    {
        (void)hipEventRecord(c.ej, c.cs);
        (void)hipStreamWaitEvent(user, c.ej, 0);
    }
};

// SRJ factors: reciprocals of the degree-m Chebyshev roots on [a, 2 - a]
std::vector<double> ad_schedule(int m, double beta, double dg_max)
{
    const double a = 1.0 / (1.0 + beta * dg_max), b = 2.0 - a, pi = 3.14159265358979323846;
    std::vector<double> w(m), out;
    for (int j = 1; j <= m; ++j) w[j - 1] = 1.0 / (0.5 * (a + b) - 0.5 * (b - a) * std::cos(pi * (2 * j - 1) / (2.0 * m)));
    std::sort(w.begin(), w.end());
    for (int lo = 0, hi = m - 1; lo <= hi; ++lo, --hi) {
        out.push_back(w[lo]);
        if (hi != lo) out.push_back(w[hi]);
    }
    return out;
}

int sparse_blocks_ad(long long n) { return (int)std::min<long long>(std::max<long long>((n + ATPB - 1) / ATPB, 1), 4096); }

AdTiles ad_tiles(const AdGrid &G)
{
    AdTiles T;
    T.gx = (G.nx + 63) / 64;
    T.gy = (G.ny + 3) / 4;
    T.gz = (G.nz + AD_KZ - 1) / AD_KZ;
    T.per = (T.gx * T.gy * T.gz + 7) / 8;
    return T;
}

void ad_operator(ibm_ad_ctx &c, bool jac, double omega, const double *x, double *y, hipStream_t s)
{
    const AdTiles T = ad_tiles(c.G);
    const int grid = 8 * T.per, ns = c.R.nrows + c.R.nm;
    if (jac) {
        k_ad_dense<AD_JACOBI><<<grid, ATPB, 0, s>>>(c.G, T, c.flags.p, c.opts.beta, omega, x, y, c.rhs.p, nullptr);
        if (ns)
            k_ad_sparse<AD_JACOBI><<<sparse_blocks_ad(ns), ATPB, 0, s>>>(c.G, c.R, c.opts.beta, omega, x, y, c.rhs.p,
                                                                         nullptr);
    } else {
        k_ad_dense<AD_APPLY><<<grid, ATPB, 0, s>>>(c.G, T, c.flags.p, c.opts.beta, 0.0, x, y, nullptr, nullptr);
        if (ns)
            k_ad_sparse<AD_APPLY><<<sparse_blocks_ad(ns), ATPB, 0, s>>>(c.G, c.R, c.opts.beta, 0.0, x, y, nullptr,
                                                                        nullptr);
    }
    IBM_LAUNCH_CHECK();
}

// relative residual ||rhs - H x|| / ||rhs||: block sums of the dense and the
// sparse rows, added on the host in block order
double ad_residual(ibm_ad_ctx &c, const double *x, hipStream_t s)
{
    const AdTiles T = ad_tiles(c.G);
    const int grid = 8 * T.per, ns = c.R.nrows + c.R.nm, gs = ns ? sparse_blocks_ad(ns) : 0;
    k_ad_dense<AD_RESID><<<grid, ATPB, 0, s>>>(c.G, T, c.flags.p, c.opts.beta, 0.0, x, nullptr, c.rhs.p, c.part.p);
    if (ns)
        k_ad_sparse<AD_RESID><<<gs, ATPB, 0, s>>>(c.G, c.R, c.opts.beta, 0.0, x, nullptr, c.rhs.p,
                                                  c.part.p + 2 * (size_t)grid);
    IBM_LAUNCH_CHECK();
    std::vector<double> h(2 * (size_t)(grid + gs));
    IBM_HIP(hipMemcpyAsync(h.data(), c.part.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    double a = 0.0, b = 0.0;
    for (size_t q = 0; q < h.size() / 2; ++q) { a += h[2 * q]; b += h[2 * q + 1]; }
    return b > 0.0 ? std::sqrt(a / b) : std::sqrt(a);
}

}  // namespace

extern "C" void ibm_ad_default_opts(ibm_ad_opts *o)
{
    if (!o) return;
    o->beta = 0.0;
    o->tol = 1e-10;
    o->sweeps = 8;
    o->max_cycles = 500;
}

extern "C" int32_t ibm_ad_setup(const ibm_grid *grid, const uint8_t *flags_dev, const ibm_stencils *st,
                                const ibm_ad_opts *opts, ibm_ad_ctx **out)
{
    return guarded([&] {
        IBM_REQUIRE(grid && flags_dev && st && opts && out, IBM_EINVAL, "null argument");
        IBM_REQUIRE(st->bc == IBM_BC_DIRICHLET, IBM_EINVAL, "the advection-diffusion step needs Dirichlet ghost rows");
        IBM_REQUIRE(opts->beta >= 0.0 && opts->tol > 0.0 && opts->sweeps >= 1 && opts->sweeps <= 64 &&
                        opts->max_cycles >= 1,
                    IBM_EINVAL, "bad advection-diffusion options");
        const HostGrid g = read_grid(grid);
        for (int d = 0; d < 3; ++d) IBM_REQUIRE(g.n[d] == st->n[d], IBM_EINVAL, "stencil table of another grid");
        std::unique_ptr<ibm_ad_ctx> c(new ibm_ad_ctx());
        c->opts = *opts;
        IBM_HIP(hipStreamCreateWithFlags(&c->cs, hipStreamNonBlocking));
        IBM_HIP(hipEventCreate(&c->e0));
        IBM_HIP(hipEventCreate(&c->e1));
        IBM_HIP(hipEventCreateWithFlags(&c->ej, hipEventDisableTiming));
        hipStream_t s = c->cs;
        AdGrid &G = c->G;
        G.nx = g.n[0]; G.ny = g.n[1]; G.nz = g.n[2];
        G.N = (long long)G.nx * G.ny * G.nz;
        double dgm[3] = {0, 0, 0};
        for (int d = 0; d < 3; ++d) {
            const int n = g.n[d];
            std::vector<double> cc(n), ww(n), cp(n, 0.0), cm(n, 0.0);
            for (int i = 0; i < n; ++i) {
                cc[i] = 0.5 * (g.f[d][i] + g.f[d][i + 1]);
                ww[i] = g.f[d][i + 1] - g.f[d][i];
            }
            for (int i = 0; i < n; ++i) {
                if (i + 1 < n) cp[i] = 1.0 / (ww[i] * (cc[i + 1] - cc[i]));
                if (i > 0) cm[i] = 1.0 / (ww[i] * (cc[i] - cc[i - 1]));
                dgm[d] = std::max(dgm[d], cp[i] + cm[i]);
            }
            upload(c->cp[d], cp, s);
            upload(c->cm[d], cm, s);
            G.cp[d] = c->cp[d].p;
            G.cm[d] = c->cm[d].p;
        }
        c->dg_max = dgm[0] + dgm[1] + dgm[2];
        c->omega = ad_schedule(opts->sweeps, opts->beta, c->dg_max);
        c->flags.alloc(G.N);
        IBM_HIP(hipMemcpyAsync(c->flags.p, flags_dev, G.N, hipMemcpyDeviceToDevice, s));
        AdRows &R = c->R;
        R.ng = (int)st->ng;
        R.nm = (int)st->nm;
        R.nrows = R.ng + R.nm;
        const long long R1 = std::max(R.nrows, 1), M1 = std::max(R.nm, 1), G1 = std::max(R.ng, 1);
        c->col.alloc(8 * R1); c->w.alloc(8 * R1); c->sG.alloc(R1); c->dlb.alloc(R1);
        c->rcell.alloc(G1); c->mcell.alloc(M1); c->mcol.alloc(6 * M1);
        c->err.alloc(1);
        if (R.nrows) {
            IBM_HIP(hipMemcpyAsync(c->col.p, st->col.p, 32 * (size_t)R.nrows, hipMemcpyDeviceToDevice, s));
            IBM_HIP(hipMemcpyAsync(c->w.p, st->w.p, 64 * (size_t)R.nrows, hipMemcpyDeviceToDevice, s));
            IBM_HIP(hipMemcpyAsync(c->sG.p, st->sG.p, 8 * (size_t)R.nrows, hipMemcpyDeviceToDevice, s));
            IBM_HIP(hipMemcpyAsync(c->dlb.p, st->dlb.p, 8 * (size_t)R.nrows, hipMemcpyDeviceToDevice, s));
        }
        if (R.ng) IBM_HIP(hipMemcpyAsync(c->rcell.p, st->cell.p, 4 * (size_t)R.ng, hipMemcpyDeviceToDevice, s));
        if (R.nm) IBM_HIP(hipMemcpyAsync(c->mcell.p, st->cell.p + R.ng, 4 * (size_t)R.nm, hipMemcpyDeviceToDevice, s));
        R.col = c->col.p; R.w = c->w.p; R.sG = c->sG.p; R.dlb = c->dlb.p;
        R.rcell = c->rcell.p; R.mcell = c->mcell.p; R.mcol = c->mcol.p;
        IBM_HIP(hipMemsetAsync(c->err.p, 0, sizeof(int), s));
        if (R.nm)
            k_ad_membrane<<<sparse_blocks_ad(R.nm), ATPB, 0, s>>>(G, R.nm, c->mcell.p, c->flags.p, c->mcol.p, c->err.p);
        IBM_LAUNCH_CHECK();
        int herr = 0;
        IBM_HIP(hipMemcpyAsync(&herr, c->err.p, sizeof(int), hipMemcpyDeviceToHost, s));
        c->Nt = G.N + R.nm;
        c->rhs.alloc(c->Nt);
        c->xa.alloc(c->Nt);
        c->xb.alloc(c->Nt);
        c->part.alloc(2 * ((size_t)8 * ad_tiles(G).per + 4096));
        IBM_HIP(hipStreamSynchronize(s));
        IBM_REQUIRE(herr == 0, IBM_EGEOM, "cut link without ghost");
        *out = c.release();
    });
}

extern "C" int32_t ibm_ad_apply(ibm_ad_ctx *c, const double *x_dev, double *y_dev, void *stream)
{
    return guarded([&] {
        IBM_REQUIRE(c && x_dev && y_dev && x_dev != y_dev, IBM_EINVAL, "bad argument");
        AdJoin j(*c, (hipStream_t)stream);
        ad_operator(*c, false, 0.0, x_dev, y_dev, c->cs);
    });
}

extern "C" int32_t ibm_ad_solve(ibm_ad_ctx *c, const double *f_dev, const double *g_dev, double *u_dev,
                                ibm_ad_stats *stats, void *stream)
{
    return guarded([&] {
        IBM_REQUIRE(c && f_dev && u_dev, IBM_EINVAL, "null argument");
        AdJoin j(*c, (hipStream_t)stream);
        hipStream_t s = c->cs;
        IBM_HIP(hipEventRecord(c->e0, s));
        const long long Nt = c->Nt;
        k_ad_rhs<<<4096, ATPB, 0, s>>>(c->G, c->flags.p, f_dev, c->rhs.p);
        if (c->R.nrows) k_ad_rhs_rows<<<sparse_blocks_ad(c->R.nrows), ATPB, 0, s>>>(c->G, c->R, g_dev, c->rhs.p);
        IBM_HIP(hipMemcpyAsync(c->xa.p, u_dev, Nt * sizeof(double), hipMemcpyDeviceToDevice, s));
        k_ad_zero_solid<<<4096, ATPB, 0, s>>>(c->G, c->flags.p, c->xa.p);
        IBM_HIP(hipMemcpyAsync(c->xb.p, c->xa.p, Nt * sizeof(double), hipMemcpyDeviceToDevice, s));
        IBM_LAUNCH_CHECK();
        double *x = c->xa.p, *y = c->xb.p;
        double rel = ad_residual(*c, x, s);
        int cyc = 0, rc = rel <= c->opts.tol ? IBM_OK : IBM_ENOCONV;
        const int m = (int)c->omega.size();
        while (rc != IBM_OK && cyc < c->opts.max_cycles) {
            for (int q = 0; q < m; ++q) {
                ad_operator(*c, true, c->omega[q], x, y, s);
                std::swap(x, y);
            }
            ++cyc;
            rel = ad_residual(*c, x, s);
            if (!std::isfinite(rel)) { rc = IBM_EBREAKDOWN; break; }
            if (rel <= c->opts.tol) rc = IBM_OK;
        }
        IBM_HIP(hipMemcpyAsync(u_dev, x, Nt * sizeof(double), hipMemcpyDeviceToDevice, s));
        IBM_HIP(hipEventRecord(c->e1, s));
        IBM_HIP(hipStreamSynchronize(s));
        if (stats) {
            float ms = 0.f;
            IBM_HIP(hipEventElapsedTime(&ms, c->e0, c->e1));
            stats->cycles = cyc;
            stats->sweeps = cyc * m;
            stats->status = rc;
            stats->rel_residual = rel;
            stats->solve_ms = ms;
        }
        if (rc == IBM_ENOCONV) throw Error(IBM_ENOCONV, "cycle limit reached");
        if (rc == IBM_EBREAKDOWN) throw Error(IBM_EBREAKDOWN, "non-finite residual");
    });
}

extern "C" void ibm_ad_destroy(ibm_ad_ctx *c)
{
    if (c) {
        (void)hipStreamSynchronize(c->cs);
        delete c;
    }
}
