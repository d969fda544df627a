// PPE solver (Sec. 2.1: BiCGStab on the pressure Poisson equation; Sec. 2.5
// module 3: matrix-free bulk plus ELLPACK rows for the irregular part) with a
// geometric-multigrid V-cycle as right preconditioner, FP64 or mixed
// precision (FP32 inner BiCGSTAB and V-cycle, BF16 coarse right-hand sides,
// FP64 iterative refinement).
//
// Pinned system: the singular Neumann operator has its first fluid
// non-membrane-ghost cell's row replaced by -s x = 0.  The preconditioner is
// V-cycle(b') with b' = b minus the volume-weighted net of b placed at the
// pin as a sink, run on the unpinned operator, followed by a shift of its
// output to a zero pin value; the shift is folded into the consumers (the
// operator writes 0 on the pin row, the x update subtracts the pin values).
//
// All vectors are held in the red/black split layout (kernels.hpp); the C
// ABI takes and returns natural x-fastest arrays, converted at the boundary.

#include "kernels.hpp"
#include "setup.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <type_traits>

namespace ibm {
namespace {

// The Krylov vector updates run one block per 256 groups of four unknowns up
// to W4MAXB blocks (a 512^3 vector: 131072 blocks, one group per thread):
// against a 4096-block walk this measured 3% (x/r update) to 11% (p update)
// faster in FP64 and 11-14% in FP32.  Their block partials set the stride.
constexpr int W4MAXB = 131072;
constexpr int PSTRIDE = W4MAXB + 2048;  // partial slots per reduction: stencil or walk blocks, then sparse blocks
constexpr int XB = 1024;               // cap on blocks of the sparse row kernels

inline int sparse_blocks(long long n) { return (int)std::max<long long>(1, std::min<long long>(XB, (n + TPB - 1) / TPB)); }

struct Level {
    int n[3] = {0, 0, 0};
    int H = 0;
    long long N = 0, Nh = 0;
    DBuf<double> cp[3], cm[3], w[3];
    DBuf<uint8_t> m;                 // split layout: coarse mask (CM_* bits); level 0 flags
    DBuf<int> pi[3];                 // prolongation map from the coarse parent
    DBuf<double> pt[3];
    double volA = 0.0;               // volume of the active cells
    long long n_inactive = 0;        // coarse levels: inactive cells (inside bodies)
    Geo geo;                         // tiles over (h, j, k) of one colour
    Geo geo2;                        // level 0: 64 x 8 tiles of the FP64 half-sweep (two rows per thread)
    Geo geon;                        // tiles over (i, j, k): restriction into this level
    Walk walk;                       // over 2 Nh slots
    DBuf<double> x64, b64;
    DBuf<float> x32;
    DBuf<bf16> b16;
    Lv lv;
    PMap pm;
    std::vector<double> hc[3], hw[3];
};

void level_geometry(Level &L, const std::vector<double> *f, hipStream_t s)
{
    for (int d = 0; d < 3; ++d) {
        int n = L.n[d];
        L.hc[d].resize(n);
        L.hw[d].resize(n);
        std::vector<double> cp(n), cm(n);
        for (int i = 0; i < n; ++i) {
            L.hc[d][i] = 0.5 * (f[d][i] + f[d][i + 1]);
            L.hw[d][i] = f[d][i + 1] - f[d][i];
        }
        for (int i = 0; i < n; ++i) {
            cp[i] = (i + 1 < n) ? 1.0 / (L.hw[d][i] * (L.hc[d][i + 1] - L.hc[d][i])) : 0.0;
            cm[i] = (i > 0) ? 1.0 / (L.hw[d][i] * (L.hc[d][i] - L.hc[d][i - 1])) : 0.0;
        }
        upload(L.cp[d], cp, s);
        upload(L.cm[d], cm, s);
        upload(L.w[d], L.hw[d], s);
    }
    L.N = (long long)L.n[0] * L.n[1] * L.n[2];
    L.H = (L.n[0] + 1) / 2;
    L.Nh = (long long)L.H * L.n[1] * L.n[2];
    // levels below 2^26 cells take half the blocks (twice the planes per
    // thread): their per-thread set-up is then spread over more planes
    const int maxb = L.N < (1LL << 26) ? 4096 : 8192;
    L.geo = make_geo(L.H, L.n[1], L.n[2], maxb);
    L.geon = make_geo_nat(L.n[0], L.n[1], L.n[2], maxb);
    L.walk = make_walk(2 * L.Nh);
}

// LDS layout of one tail level (mask, iterate, RHS), 16-byte aligned pieces
inline void tail_layout(long long Nh, size_t tsz, int &off, int &moff, int &xoff, int &boff)
{
    auto al = [](long long v) { return (int)((v + 15) / 16 * 16); };
    moff = off;
    off = al(off + 2 * Nh);
    xoff = off;
    off = al(off + 2 * Nh * (long long)tsz);
    boff = off;
    off = al(off + 2 * Nh * (long long)tsz);
}

// slot of natural cell (i,j,k) in a level with half-width H
inline long long host_slot(int H, int ny, long long Nh, int i, int j, int k)
{
    return (long long)((i + j + k) & 1) * Nh + (i >> 1) + (long long)H * (j + (long long)ny * k);
}

}  // namespace
}  // namespace ibm

using namespace ibm;

namespace ibm {
namespace {
// Pinned host slots for the per-context scalar read-back, cut from chunks
// that live until the process ends: freeing pinned memory synchronises the
// device, which a graph capture running in another thread does not allow.
std::mutex g_pin_mu;
std::vector<double *> g_pin_free;
double *pinned_slot()
{
    std::lock_guard<std::mutex> lk(g_pin_mu);
    if (g_pin_free.empty()) {
        constexpr int per = 64;
        double *chunk = nullptr;
        std::shared_lock<std::shared_mutex> cl(capture_mutex());
        IBM_HIP(hipHostMalloc((void **)&chunk, per * S_COUNT * sizeof(double), hipHostMallocDefault));
        for (int q = per - 1; q >= 0; --q) g_pin_free.push_back(chunk + q * S_COUNT);
    }
    double *p = g_pin_free.back();
    g_pin_free.pop_back();
    return p;
}
void pinned_release(double *p)
{
    std::lock_guard<std::mutex> lk(g_pin_mu);
    g_pin_free.push_back(p);
}
}  // namespace
}  // namespace ibm

struct poisson_ctx {
    poisson_opts opts;
    HostGrid g;
    long long N = 0, nm = 0, ng = 0, nrows = 0, n_fallback = 0, pin = 0;
    long long N2 = 0, Nt = 0;  // 2 Nh cell slots, + membrane unknowns
    double vol_fluid = 0.0, vol_pin = 0.0;
    int tail0 = 1;             // first level of the single-workgroup tail (FP32 levels in the mixed form)
    int tail0d = 1;            // the same for FP64 levels
    std::vector<double> srj_w; // SRJ relaxation factors in application order
    DBuf<int32_t> rslot, rcol, mslot, mcol, mcolor;
    DBuf<int32_t> rmrow;  // membrane cell behind each ghost-row column
    DBuf<double> rw, rsG, rdlb;
    std::vector<Level> lv;
    Sp sp;
    Walk W0;   // over Nt unknowns
    Walk W4;   // over ceil(Nt / 4) groups of 4 unknowns
    Walk Wc;   // over 2 Nh cell slots
    DBuf<double> x, r, rh, p, v, ph, sh, t, rsp, b;
    DBuf<float> fr, frh, fp, fv, fph, fsh, ft, frsp;
    // mixed: the inner solution accumulates in FP64 (a smooth correction
    // rounded to FP32 loses its small Laplacian: the operator multiplies the
    // rounding by up to |A| ~ 12/h^2)
    DBuf<double> d64;
    DBuf<double> r2;           // mixed: right-hand side of the FP64 fallback solve
    DBuf<double> gtmp, mtmp, sc, part;  // ghost and membrane staging; scalars; partials
    DBuf<double> ssum;          // set-up sums (fluid volume, active volume per level)
    DBuf<int> serr;             // set-up error flag
    DBuf<uint8_t> hact[2];      // set-up: natural-order coarse active/cut bits of two consecutive levels
    double *hsc = nullptr;
    hipStream_t cs = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr, ej = nullptr;
    hipGraphExec_t g64 = nullptr, g32 = nullptr;
    hipGraphExec_t g64w = nullptr;  // FP64 iteration on the correction (solves from a guess)
    size_t bytes = 0;
    bool mixed = false;
    // per-launch timing of one kernel (HIP events on the solve stream)
    int prof_kernel = -1;
    bool capturing = false;
    std::vector<hipEvent_t> prof_ev;
    int prof_used = 0;
    double prof_ms = 0.0;
    long long prof_count = 0;

    const Lv &L0() const { return lv[0].lv; }

    ~poisson_ctx()
    {
        if (g64) (void)hipGraphExecDestroy(g64);
        if (g32) (void)hipGraphExecDestroy(g32);
        if (g64w) (void)hipGraphExecDestroy(g64w);
        if (hsc) pinned_release(hsc);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (ej) (void)hipEventDestroy(ej);
        if (cs) (void)hipStreamDestroy(cs);
        for (auto e : prof_ev) (void)hipEventDestroy(e);
    }
};

namespace ibm {
namespace {

// IBM_LOG=1 logs each solve's refinement steps to stderr, IBM_LOG=2 every iteration
int log_level()
{
    static const int lvl = [] {
        const char *e = getenv("IBM_LOG");
        return (e && *e) ? atoi(e) : 0;
    }();
    return lvl;
}
inline bool log_enabled() { return log_level() > 0; }

// kernel ids of the timing hook
enum { PK_SWEEP0 = 0, PK_APPLY0 = 1, PK_XR = 2 };

inline void prof_begin(poisson_ctx &c, int kid, hipStream_t s)
{
    if (c.prof_kernel != kid || c.capturing) return;
    if ((int)c.prof_ev.size() < 2 * (c.prof_used + 1)) {
        hipEvent_t a, b;
        IBM_HIP(hipEventCreate(&a));
        IBM_HIP(hipEventCreate(&b));
        c.prof_ev.push_back(a);
        c.prof_ev.push_back(b);
    }
    IBM_HIP(hipEventRecord(c.prof_ev[2 * c.prof_used], s));
}

inline void prof_end(poisson_ctx &c, int kid, hipStream_t s)
{
    if (c.prof_kernel != kid || c.capturing) return;
    IBM_HIP(hipEventRecord(c.prof_ev[2 * c.prof_used + 1], s));
    ++c.prof_used;
}

inline void prof_harvest(poisson_ctx &c)
{
    for (int i = 0; i < c.prof_used; ++i) {
        float ms = 0.f;
        IBM_HIP(hipEventElapsedTime(&ms, c.prof_ev[2 * i], c.prof_ev[2 * i + 1]));
        c.prof_ms += ms;
        ++c.prof_count;
    }
    c.prof_used = 0;
}

inline void fin(poisson_ctx &c, int n, int op, int dst, double aux, hipStream_t s)
{
    k_fin<<<1, 1024, 0, s>>>(c.part.p, PSTRIDE, n, op, dst, aux, c.sc.p);
    IBM_LAUNCH_CHECK();
}

// y = A x (or y = b - A x) on level 0, with dots; returns the partial count
template <class T>
int launch_apply(poisson_ctx &c, int mode, bool res, int nd, const T *x, T *y, const T *b, const double *sink,
                 const T *u1, const T *u2, hipStream_t s)
{
    const Level &L = c.lv[0];
    double *P = c.part.p;
    const int nsp = (int)(c.nrows + c.nm);
    const int sb = sparse_blocks(nsp);
    const int gb = L.geo.nb;
#define AP(MODE, RES, ND)                                                                                        \
    k0_apply2<T, MODE, RES, ND><<<gb, TPB, 0, s>>>(L.lv, L.geo, c.pin, x, y, b, sink, u1, u2, P, PSTRIDE);     \
    if (nsp) k0_sparse<T, RES, ND><<<sb, TPB, 0, s>>>(L.lv, c.sp, x, y, b, u1, u2, P, PSTRIDE, gb);
    if (res) {
        if (mode == M_PINNED && nd == 2) { AP(M_PINNED, true, 2) }
        else if (mode == M_UNPINNED && nd == 0) { AP(M_UNPINNED, true, 0) }
        else throw Error(IBM_EINVAL, "apply variant");
    } else {
        if (mode == M_PINZERO && nd == 1) { AP(M_PINZERO, false, 1) }
        else if (mode == M_PINZERO && nd == 2) { AP(M_PINZERO, false, 2) }
        else if (mode == M_PINNED && nd == 0) { AP(M_PINNED, false, 0) }
        else throw Error(IBM_EINVAL, "apply variant");
    }
#undef AP
    IBM_LAUNCH_CHECK();
    return gb + (nsp ? sb : 0);
}

template <class T>
struct Store;
template <>
struct Store<double> {
    typedef double Tc;
    typedef double TB;
    static Tc *x(Level &L) { return L.x64.p; }
    static TB *b(Level &L) { return L.b64.p; }
};
template <>
struct Store<float> {
    typedef float Tc;
    typedef bf16 TB;
    static Tc *x(Level &L) { return L.x32.p; }
    static TB *b(Level &L) { return L.b16.p; }
};

// prolongation of coarse level C onto F; the renormalised form only where C
// has inactive cells
template <bool FINE, class Tc, class Tf>
void launch_prolong(const Level &F, const Level &C, bool skip_red, const Tc *xc, Tf *xf, hipStream_t s)
{
    const bool rn = C.n_inactive > 0;
    if (skip_red && rn)
        k_prolong_z<FINE, Tc, Tf, true, true><<<C.geon.nb, TPB, 0, s>>>(F.lv, C.lv, F.pm, C.geon, xc, xf);
    else if (skip_red)
        k_prolong_z<FINE, Tc, Tf, true, false><<<C.geon.nb, TPB, 0, s>>>(F.lv, C.lv, F.pm, C.geon, xc, xf);
    else if (rn)
        k_prolong_z<FINE, Tc, Tf, false, true><<<C.geon.nb, TPB, 0, s>>>(F.lv, C.lv, F.pm, C.geon, xc, xf);
    else
        k_prolong_z<FINE, Tc, Tf, false, false><<<C.geon.nb, TPB, 0, s>>>(F.lv, C.lv, F.pm, C.geon, xc, xf);
}

// level-0 smoothing step: for red then black, the dense half-sweep, the
// membrane-adjacent cells of that colour, then Jacobi on all ghost unknowns
template <class T>
void fine_smooth(poisson_ctx &c, T *x, const T *b, const double *sink, bool from_zero, hipStream_t s)
{
    const Level &L = c.lv[0];
    const int mb = sparse_blocks(c.nm), gb = sparse_blocks(c.nrows + c.nm);
    for (int color = 0; color < 2; ++color) {
        if (from_zero && color == 0) {
            // the other colour is zeroed too: ghost rows and membrane rows read it before its sweep
            const long long pin_s = (sink && c.pin < L.Nh) ? c.pin : -1;
            k0_sweep_zero<T><<<L.geo.nb, TPB, 0, s>>>(L.lv, L.geo, pin_s, x, x + L.Nh, b, L.lv.f, sink, 0);
            if (c.nm) {
                Walk Wt = make_walk(c.nm);
                k_fill<T><<<Wt.nb, TPB, 0, s>>>(Wt, x + c.N2, 0.0);
            }
        } else {
            // (from zero, the black slots were zeroed by the red sweep; ghost
            // values set since then must survive, so this is an ordinary sweep)
            const long long co = (long long)color * L.Nh;
            const long long pin_s = (sink && c.pin >= co && c.pin < co + L.Nh) ? c.pin - co : -1;
            if (!from_zero) prof_begin(c, PK_SWEEP0, s);
            const Geo &G = std::is_same<T, double>::value ? L.geo2 : L.geo;  // FP64: two rows per thread
            k0_sweep<T><<<G.nb, TPB, 0, s>>>(L.lv, G, pin_s, x + co, x + (L.Nh - co), b + co, L.lv.f + co, sink,
                                             color);
            if (!from_zero) prof_end(c, PK_SWEEP0, s);
        }
        if (c.nm) k0_msweep<T><<<mb, TPB, 0, s>>>(L.lv, c.sp, x, b, color, c.mtmp.p);
        if (c.nrows) {
            k0_mscat_gjac<T><<<gb, TPB, 0, s>>>(c.sp, x, b, color, c.mtmp.p, c.gtmp.p);
            k0_gscat<T><<<gb, TPB, 0, s>>>(c.sp, x, c.gtmp.p);
        }
    }
    IBM_LAUNCH_CHECK();
}

template <class Tc, class TB>
void coarse_smooth(Level &L, int steps, bool from_zero, const double *mean, hipStream_t s)
{
    Tc *x = Store<Tc>::x(L);
    const TB *b = Store<Tc>::b(L);
    for (int it = 0; it < steps; ++it) {
        if (it == 0 && from_zero) {
            k_csweep<Tc, TB, 1><<<L.geo.nb, TPB, 0, s>>>(L.lv, L.geo, x, b, mean, 0);
            k_csweep<Tc, TB, 2><<<L.geo.nb, TPB, 0, s>>>(L.lv, L.geo, x, b, mean, 1);
        } else {
            k_csweep<Tc, TB, 0><<<L.geo.nb, TPB, 0, s>>>(L.lv, L.geo, x, b, mean, 0);
            k_csweep<Tc, TB, 0><<<L.geo.nb, TPB, 0, s>>>(L.lv, L.geo, x, b, mean, 1);
        }
    }
    IBM_LAUNCH_CHECK();
}

// x = V-cycle(b) on the unpinned operator with the sink at the pin; x unshifted
template <class T>
void vcycle(poisson_ctx &c, const T *b, T *x, const double *sink, hipStream_t s)
{
    typedef typename Store<T>::Tc Tc;
    typedef typename Store<T>::TB TB;
    const int nl = (int)c.lv.size();
    const poisson_opts &o = c.opts;
    for (int it = 0; it < o.nu1; ++it) fine_smooth<T>(c, x, b, sink, it == 0, s);
    if (nl > 1) {
        // level-0 residual: the sparse rows into r0, then the regular rows
        // computed and restricted in one pass
        T *r0 = std::is_same<T, double>::value ? (T *)c.rsp.p : (T *)c.frsp.p;
        const int nsp = (int)(c.nrows + c.nm);
        if (nsp) k0_sparse_res<T><<<sparse_blocks(nsp), TPB, 0, s>>>(c.lv[0].lv, c.sp, x, b, r0);
        Level &L1 = c.lv[1];
        k0_restrict_res<T, TB><<<L1.geon.nb, TPB, 0, s>>>(c.lv[0].lv, L1.lv, L1.geon, c.pin, x, b, sink, r0,
                                                         Store<T>::b(L1), c.part.p);
        IBM_LAUNCH_CHECK();
        fin(c, L1.geon.nb, FIN_MEAN, S_MEAN0 + 1, L1.volA, s);
        const int lt = std::is_same<T, double>::value ? c.tail0d : c.tail0;
        for (int l = 1; l < lt; ++l) {
            Level &L = c.lv[l];
            const double *mean = c.sc.p + S_MEAN0 + l;
            if (l == nl - 1) {
                coarse_smooth<Tc, TB>(L, o.coarse_sweeps, true, mean, s);
                break;
            }
            coarse_smooth<Tc, TB>(L, o.nu1, true, mean, s);
            Level &C = c.lv[l + 1];
            k_restrict<false, Tc, TB, TB><<<C.geon.nb, TPB, 0, s>>>(L.lv, C.lv, C.geon, -1, Store<T>::x(L),
                                                                   Store<T>::b(L), mean, (const Tc *)nullptr,
                                                                   Store<T>::b(C), c.part.p);
            IBM_LAUNCH_CHECK();
            fin(c, C.geon.nb, FIN_MEAN, S_MEAN0 + l + 1, C.volA, s);
        }
        if (lt < nl) {
            Tail tl;
            tl.n = nl - lt;
            tl.nu1 = o.nu1;
            tl.nu2 = o.nu2;
            tl.ncs = o.coarse_sweeps;
            int off = 0;
            for (int q = 0; q < tl.n; ++q) {
                Level &L = c.lv[lt + q];
                tl.t[q].L = L.lv;
                tl.t[q].M = L.pm;
                tl.t[q].volA = L.volA;
                tl.t[q].xg = Store<T>::x(L);
                tl.t[q].bg = Store<T>::b(L);
                tail_layout(L.Nh, sizeof(Tc), off, tl.t[q].moff, tl.t[q].xoff, tl.t[q].boff);
            }
            tl.coff = off;
            for (int q = 0; q < tl.n; ++q) {
                const Level &L = c.lv[lt + q];
                off += tail_coef_bytes(L.n[0], L.n[1], L.n[2]);
            }
            k_tail<Tc, TB><<<1, TAIL_T, off, s>>>(tl, c.sc.p + S_MEAN0 + lt);
            IBM_LAUNCH_CHECK();
        }
        for (int l = std::min(lt, nl - 1) - 1; l >= 1; --l) {
            Level &L = c.lv[l];
            Level &C = c.lv[l + 1];
            launch_prolong<false>(L, C, o.nu2 > 0, Store<T>::x(C), Store<T>::x(L), s);
            coarse_smooth<Tc, TB>(L, o.nu2, false, c.sc.p + S_MEAN0 + l, s);
        }
        Level &L0v = c.lv[0];
        launch_prolong<true>(L0v, L1, o.nu2 > 0, Store<T>::x(L1), x, s);
        IBM_LAUNCH_CHECK();
    }
    for (int it = 0; it < o.nu2; ++it) fine_smooth<T>(c, x, b, sink, false, s);
}

// SRJ schedule: the reciprocals of the roots of the degree-m Chebyshev
// polynomial on [kmin, 2], kmin = 16/m^2 (the minimax factors for the
// amplification prod (1 - w k) over the spectrum of D^-1 A), in the order
// smallest, largest, second smallest, ...
std::vector<double> srj_schedule(int m)
{
    const double kmin = 16.0 / ((double)m * m), pi = 3.14159265358979323846;
    std::vector<double> w(m), out;
    for (int j = 1; j <= m; ++j)
        w[j - 1] = 1.0 / (0.5 * (2.0 + kmin) - 0.5 * (2.0 - kmin) * std::cos(pi * (2 * j - 1) / (2.0 * m)));
    std::sort(w.begin(), w.end());
    for (int lo = 0, hi = m - 1; lo <= hi; ++lo, --hi) {
        out.push_back(w[lo]);
        if (hi != lo) out.push_back(w[hi]);
    }
    return out;
}

// x = SRJ(b): the scheduled sweeps from zero, alternating between x and the
// residual scratch (the starting buffer is chosen so the last sweep lands in x)
template <class T>
void srj_apply(poisson_ctx &c, const T *b, T *x, hipStream_t s)
{
    T *tmp = std::is_same<T, double>::value ? (T *)c.rsp.p : (T *)c.frsp.p;
    const Level &L = c.lv[0];
    const int m = (int)c.srj_w.size(), nsp = (int)(c.nrows + c.nm);
    T *xo = (m % 2) ? tmp : x, *xn = (m % 2) ? x : tmp;
    k_fill<T><<<c.W0.nb, TPB, 0, s>>>(c.W0, xo, 0.0);
    for (int q = 0; q < m; ++q) {
        k0_jacobi<T><<<L.geo.nb, TPB, 0, s>>>(L.lv, L.geo, c.pin, xo, xn, b, c.srj_w[q]);
        if (nsp) k0_jacobi_sparse<T><<<sparse_blocks(nsp), TPB, 0, s>>>(L.lv, c.sp, xo, xn, b, c.srj_w[q]);
        std::swap(xo, xn);
    }
    IBM_LAUNCH_CHECK();
}

// x = M^-1 b: the V-cycle (with the pin sink) or SRJ; the output is not yet
// shifted to a zero pin value (its consumers do that)
template <class T>
void precond(poisson_ctx &c, const T *b, T *x, const double *sink, hipStream_t s)
{
    if (c.opts.precond == IBM_PRECOND_SRJ) srj_apply<T>(c, b, x, s);
    else vcycle<T>(c, b, x, sink, s);
}

// One BiCGSTAB iteration (van der Vorst 1992, right preconditioning): all
// scalars stay on the device.
template <class T, class TX>
void bicg_iteration(poisson_ctx &c, TX *y, T *r, T *rh, T *p, T *v, T *ph, T *sh, T *t, hipStream_t s)
{
    const Walk &W = c.W4;
    const Lv &L = c.L0();
    k_p_update4<T><<<W.nb, TPB, 0, s>>>(L, W, c.Nt, r, p, v, c.sc.p, c.part.p);
    fin(c, W.nb, FIN_SINK, S_SINKP, 0.0, s);
    precond<T>(c, p, ph, c.sc.p + S_SINKP, s);
    prof_begin(c, PK_APPLY0, s);
    int np = launch_apply<T>(c, M_PINZERO, false, 1, ph, v, nullptr, nullptr, rh, nullptr, s);
    prof_end(c, PK_APPLY0, s);
    fin(c, np, FIN_ALPHA, 0, 0.0, s);
    k_s_update4<T><<<W.nb, TPB, 0, s>>>(L, W, c.Nt, r, v, c.sc.p, c.part.p);
    fin(c, W.nb, FIN_SINK, S_SINKS, 0.0, s);
    precond<T>(c, r, sh, c.sc.p + S_SINKS, s);
    np = launch_apply<T>(c, M_PINZERO, false, 2, sh, t, nullptr, nullptr, r, nullptr, s);
    fin(c, np, FIN_OMEGA, 0, 0.0, s);
    prof_begin(c, PK_XR, s);
    k_xr_update4<T, TX><<<W.nb, TPB, 0, s>>>(L, W, c.Nt, c.pin, y, ph, sh, r, t, rh, c.sc.p, c.part.p,
                                              PSTRIDE);
    prof_end(c, PK_XR, s);
    IBM_LAUNCH_CHECK();
    fin(c, W.nb, FIN_RHO, 0, 0.0, s);
}

void read_scalars(poisson_ctx &c, hipStream_t s)
{
    IBM_HIP(hipMemcpyAsync(c.hsc, c.sc.p, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    prof_harvest(c);
}

// Right-preconditioned BiCGSTAB on A y = rhs; y starts at zero.  rhs may be
// in a wider type than the vectors (the FP64 residual of a refinement step
// feeding an FP32 inner solve: it is rounded on the way in).  Returns the
// iteration count; *rc gets the status.
constexpr int INNER_STALL = 12;

template <class T, class TX, class TR>
int bicgstab(poisson_ctx &c, const TR *rhs, TX *y, T *r, T *rh, T *p, T *v, T *ph, T *sh, T *t, double tol, int maxit,
             bool true_check, hipGraphExec_t *graph, hipStream_t s, int *rc, double *relout)
{
    const Walk &W = c.W0;
    k_fill<TX><<<W.nb, TPB, 0, s>>>(W, y, 0.0);
    k_fill<T><<<W.nb, TPB, 0, s>>>(W, p, 0.0);
    k_fill<T><<<W.nb, TPB, 0, s>>>(W, v, 0.0);
    k_copy_norm4<TR, T><<<c.W4.nb, TPB, 0, s>>>(c.W4, c.Nt, rhs, r, rh, c.part.p);
    IBM_LAUNCH_CHECK();
    fin(c, c.W4.nb, FIN_INIT, 0, 0.0, s);
    read_scalars(c, s);
    *rc = IBM_ENOCONV;
    if (c.hsc[S_BN2] == 0.0) {
        *rc = IBM_OK;
        *relout = 0.0;
        return 0;
    }
    const bool use_graph = c.opts.use_graph && c.prof_kernel < 0;
    if (use_graph && !*graph) {
        // a failure inside the capture still ends it, so the stream never
        // stays in capture mode (the user's stream joins it afterwards)
        struct Capture {
            poisson_ctx &c;
            hipStream_t s;
            hipGraph_t gr = nullptr;
            bool open = false;
            ~Capture()
            {
                if (open) {
                    hipGraph_t g2 = nullptr;
                    if (hipStreamEndCapture(s, &g2) == hipSuccess && g2) (void)hipGraphDestroy(g2);
                    (void)hipGetLastError();
                }
                if (gr) (void)hipGraphDestroy(gr);
                c.capturing = false;
            }
        } cap{c, s};
        {
            std::unique_lock<std::shared_mutex> lk(capture_mutex());
            c.capturing = true;
            IBM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            cap.open = true;
            bicg_iteration<T, TX>(c, y, r, rh, p, v, ph, sh, t, s);
            cap.open = false;
            IBM_HIP(hipStreamEndCapture(s, &cap.gr));
        }
        IBM_HIP(hipGraphInstantiate(graph, cap.gr, nullptr, nullptr, 0));
    }
    int it = 0;
    double rel = 1.0;
    // inner solves stop once they no longer halve their residual within
    // INNER_STALL iterations: FP32 vectors cannot resolve corrections below
    // about kappa * u32, and refinement then continues in FP64
    double mark = 1.0;
    int mark_it = 0;
    while (it < maxit) {
        ++it;
        if (use_graph) IBM_HIP(hipGraphLaunch(*graph, s));
        else bicg_iteration<T, TX>(c, y, r, rh, p, v, ph, sh, t, s);
        read_scalars(c, s);
        const double st = c.hsc[S_STATUS];
        rel = c.hsc[S_REL];
        if (log_level() >= 2)
            fprintf(stderr, "[ibm]   it %d rel %.3e status %g alpha %.3e omega %.3e sinks %.3e %.3e\n", it, rel, st,
                    c.hsc[S_ALPHA], c.hsc[S_OMEGA], c.hsc[S_SINKP], c.hsc[S_SINKS]);
        if (st >= 2.0 || !std::isfinite(rel)) { *rc = IBM_EBREAKDOWN; break; }
        if (rel <= tol) {
            if constexpr (!std::is_same<T, TX>::value || !std::is_same<TR, T>::value) {
                *rc = IBM_OK;  // inner solves: no true check
                break;
            } else {
                if (!true_check) { *rc = IBM_OK; break; }
                int np = launch_apply<T>(c, M_PINNED, true, 2, (const T *)y, t, rhs, nullptr, rh, nullptr, s);
                k_fin<<<1, 1024, 0, s>>>(c.part.p + PSTRIDE, PSTRIDE, np, FIN_SUM, S_TMP, 0.0, c.sc.p);
                read_scalars(c, s);
                double trel = std::sqrt(c.hsc[S_TMP] / c.hsc[S_BN2]);
                rel = trel;
                if (trel <= tol) { *rc = IBM_OK; break; }
                // residual replacement
                k_copy<T, T><<<W.nb, TPB, 0, s>>>(W, t, r);
                k_dot2<T><<<W.nb, TPB, 0, s>>>(W, rh, r, c.part.p, PSTRIDE);
                fin(c, W.nb, FIN_REPLACE, 0, 0.0, s);
                continue;
            }
        }
        if constexpr (!std::is_same<T, TX>::value) {
            if (rel < 0.5 * mark) {
                mark = rel;
                mark_it = it;
            } else if (it - mark_it >= INNER_STALL) {
                if (log_enabled()) fprintf(stderr, "[ibm]   inner stagnation at %.3e after %d iterations\n", rel, it);
                break;  // *rc stays IBM_ENOCONV
            }
        }
        if (st == 1.0) {  // rho breakdown: restart with rh = r
            k_fill<T><<<W.nb, TPB, 0, s>>>(W, p, 0.0);
            k_fill<T><<<W.nb, TPB, 0, s>>>(W, v, 0.0);
            k_copy_norm<T, T><<<W.nb, TPB, 0, s>>>(W, r, rh, (T *)nullptr, c.part.p);
            fin(c, W.nb, FIN_RESTART, 0, 0.0, s);
        }
    }
    *relout = rel;
    return it;
}

// ------------------------------------------------------------------ RHS, gauge (split layout)
__global__ void __launch_bounds__(TPB) k_rhs(Lv L, Walk W, long long pin, const double *fs, const double *sc,
                                             int slot_, double *b)
{
    const double mean = sc[slot_];
    WALK_BEGIN(W, p)
        if (p >= 2 * L.Nh) { b[p] = 0.0; continue; }
        const uint8_t fl = L.f[p];
        b[p] = ((fl & F_SOLID) || p == pin) ? 0.0 : fs[p] - mean;
    WALK_END
}

__global__ void __launch_bounds__(TPB) k_rhs_ghost(Sp S, const double *dlb, const double *g, double *b)
{
    for (int r = blockIdx.x * TPB + threadIdx.x; r < S.nrows; r += gridDim.x * TPB)
        b[ghost_unknown(S, r)] = g ? S.rsG[r] * dlb[r] * g[r] : 0.0;
}

__global__ void __launch_bounds__(TPB) k_gauge(Lv L, Walk W, const double *x, const double *sc, int slot_, double *out)
{
    const double mean = sc[slot_];
    WALK_BEGIN(W, p)
        const bool act = p >= 2 * L.Nh || active0(L.f[p]);
        out[p] = act ? x[p] - mean : 0.0;
    WALK_END
}

template <class T>
__global__ void __launch_bounds__(TPB) k_shift(Lv L, Walk W, long long pin, T *x)
{
    const double c = ld(x, pin);
    WALK_BEGIN(W, p)
        if (p != pin && (p >= 2 * L.Nh || active0(L.f[p]))) st(x, p, ld(x, p) - c);
    WALK_END
}

__global__ void k_shift_pin(long long pin, double *x) { x[pin] = 0.0; }

// unpinned residual at the pin (the inconsistency the pin absorbs)
__global__ void k_pinres(Lv L, long long pin, const double *x, double *sc)
{
    if (threadIdx.x || blockIdx.x) return;
    int c, h, j, k, i;
    decode_slot(L, pin, c, h, j, k, i);
    double dg;
    const double off = nbsum<true>(L, x + (long long)(1 - c) * L.Nh, L.f + (long long)(1 - c) * L.Nh, h, j, k, i,
                                   L.f[pin], dg);
    sc[S_TMP] = off - dg * x[pin];
}

}  // namespace

// ------------------------------------------------------------------ setup
size_t estimate_bytes(int nx, int ny, int nz, long long nrows, int precision)
{
    long long Nh = (long long)((nx + 1) / 2) * ny * nz;
    long long Nt = 2 * Nh + nrows;
    size_t b = (size_t)2 * Nh;  // flags
    b += (size_t)nrows * (8 * 4 + 8 * 8 + 16 + 8 + 4 + 6 * 4 + 4 + 8 * 4 + 8);
    b += (size_t)Nt * 8 * (precision == IBM_PREC_MIXED ? 4 : 10);
    if (precision == IBM_PREC_MIXED) b += (size_t)Nt * (4 * 8 + 8);
    long long Nc = 2 * Nh;
    size_t coarse = 0;
    while (true) {
        Nc /= 8;
        if (Nc < 8) break;
        coarse += (size_t)Nc * (precision == IBM_PREC_MIXED ? (4 + 2 + 1) : (8 * 2 + 1));
    }
    b += coarse;
    b += (size_t)PSTRIDE * 4 * 8;
    return b;
}

// grow-only device buffer: reallocated (contents dropped) when too small
template <class T>
void reserve(DBuf<T> &b, size_t n)
{
    if (!b.p || b.n < n) b.alloc(n);
}

// Flag-dependent parts of a context -- level-0 flags, ghost and membrane rows
// in slot numbering, fluid and pin volumes, coarse masks, vectors sized by
// the unknown count -- built on the device from the classification and the
// ghost-row table.  Runs at set-up and again when bodies move.
void setup_geometry(poisson_ctx &c, const uint8_t *flags, const ibm_stencils *st)
{
    const HostGrid &g = c.g;
    for (int d = 0; d < 3; ++d) IBM_REQUIRE(g.n[d] == st->n[d], IBM_EINVAL, "stencil table of another grid");
    IBM_REQUIRE(st->pin >= 0 && st->pin < c.N, IBM_EGEOM, "no fluid cell to pin");
    // row columns are int32 slots: the cell slots (with row padding), then the membrane ghost unknowns
    IBM_REQUIRE(c.N2 + st->nm < (1LL << 31), IBM_EINVAL, "more than 2^31 unknowns with padding and membrane ghosts");
    hipStream_t s = c.cs;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int nl = (int)c.lv.size();
    Level &Z = c.lv[0];
    c.ng = st->ng;
    c.nm = st->nm;
    c.nrows = st->ng + st->nm;
    c.n_fallback = st->nfallback;
    const long long R = c.nrows, nm = c.nm, N = c.N;
    const SlotMap sm{nx, ny, Z.H, Z.Nh, N, c.N2};
    {
        const long long p = st->pin;
        const int i = (int)(p % nx), j = (int)((p / nx) % ny), k = (int)(p / ((long long)nx * ny));
        c.pin = host_slot(Z.H, ny, Z.Nh, i, j, k);
        c.vol_pin = Z.hw[0][i] * Z.hw[1][j] * Z.hw[2][k];
    }
    // the captured iterations and the vectors below may change
    IBM_HIP(hipStreamSynchronize(s));
    if (c.g64) { (void)hipGraphExecDestroy(c.g64); c.g64 = nullptr; }
    if (c.g32) { (void)hipGraphExecDestroy(c.g32); c.g32 = nullptr; }
    if (c.g64w) { (void)hipGraphExecDestroy(c.g64w); c.g64w = nullptr; }
    k_setup_flags0<<<Z.walk.nb, TPB, 0, s>>>(Z.lv, Z.walk, flags, Z.m.p);
    // ghost and membrane rows
    const long long R1 = std::max<long long>(R, 1), M1 = std::max<long long>(nm, 1);
    reserve(c.rslot, std::max<long long>(c.ng, 1));
    reserve(c.rcol, R1 * 8);
    reserve(c.rw, R1 * 8);
    reserve(c.rsG, R1);
    reserve(c.rdlb, R1);
    reserve(c.gtmp, R1);
    reserve(c.mtmp, M1);
    reserve(c.rmrow, R1 * 8);
    reserve(c.mslot, M1);
    reserve(c.mcol, M1 * 6);
    reserve(c.mcolor, M1);
    auto blocks = [](long long n) { return (int)std::min<long long>(std::max<long long>((n + TPB - 1) / TPB, 1), 4096); };
    if (R) {
        k_setup_rows<<<blocks(8 * R), TPB, 0, s>>>(sm, c.ng, R, st->cell.p, st->col.p, c.rslot.p, c.rcol.p);
        IBM_HIP(hipMemcpyAsync(c.rw.p, st->w.p, R * 64, hipMemcpyDeviceToDevice, s));
        IBM_HIP(hipMemcpyAsync(c.rsG.p, st->sG.p, R * 8, hipMemcpyDeviceToDevice, s));
        IBM_HIP(hipMemcpyAsync(c.rdlb.p, st->dlb.p, R * 8, hipMemcpyDeviceToDevice, s));
    }
    IBM_HIP(hipMemsetAsync(c.serr.p, 0, sizeof(int), s));
    if (nm)
        k_setup_membrane<<<blocks(nm), TPB, 0, s>>>(sm, nz, nm, st->cell.p + c.ng, flags, c.mslot.p, c.mcol.p,
                                                    c.mcolor.p, c.serr.p);
    if (R && nm)
        k_map_mrows<<<blocks(8 * R), TPB, 0, s>>>(8 * R, st->col.p, N, flags, st->cell.p + c.ng, nm, c.rmrow.p);
    // the slots those rows read (the first half-sweep of a V-cycle zeroes
    // these, not every black slot)
    if (R) k_mark_read<<<blocks(8 * R), TPB, 0, s>>>(8 * R, c.rcol.p, c.N2, Z.m.p);
    if (nm) k_mark_read<<<blocks(6 * nm), TPB, 0, s>>>(6 * nm, c.mcol.p, c.N2, Z.m.p);
    // fluid volume, then the coarse masks level by level with their active volumes
    k_fluid_volume<<<Z.walk.nb, TPB, 0, s>>>(Z.lv, Z.walk, c.part.p);
    k_fin<<<1, 1024, 0, s>>>(c.part.p, PSTRIDE, Z.walk.nb, FIN_SUM, 0, 0.0, c.ssum.p);
    for (int l = 1; l < nl; ++l) {
        Level &F = c.lv[l - 1], &C = c.lv[l];
        const uint8_t *fine = l == 1 ? flags : c.hact[l & 1].p;
        uint8_t *ha = c.hact[(l + 1) & 1].p;
        k_coarse_active<<<blocks(C.N), TPB, 0, s>>>(F.n[0], F.n[1], C.n[0], C.n[1], C.N, fine, l == 1, ha);
        k_coarse_mask<<<C.walk.nb, TPB, 0, s>>>(C.lv, C.walk, ha, C.m.p, c.part.p, PSTRIDE);
        k_fin<<<1, 1024, 0, s>>>(c.part.p, PSTRIDE, C.walk.nb, FIN_SUM, l, 0.0, c.ssum.p);
        k_fin<<<1, 1024, 0, s>>>(c.part.p + PSTRIDE, PSTRIDE, C.walk.nb, FIN_SUM, 16 + l, 0.0, c.ssum.p);
    }
    IBM_LAUNCH_CHECK();
    double hs[32];
    int herr = 0;
    IBM_HIP(hipMemcpyAsync(hs, c.ssum.p, 32 * sizeof(double), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipMemcpyAsync(&herr, c.serr.p, sizeof(int), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    IBM_REQUIRE(herr == 0, IBM_EGEOM, "cut link without ghost");
    c.vol_fluid = hs[0];
    for (int l = 1; l < nl; ++l) {
        c.lv[l].volA = hs[l];
        c.lv[l].n_inactive = (long long)hs[16 + l];
    }
    Sp &S = c.sp;
    S.N2 = c.N2;
    S.pin = c.pin;
    S.nrows = (int)R;
    S.ng = (int)c.ng;
    S.rslot = c.rslot.p; S.rcol = c.rcol.p; S.rw = c.rw.p; S.rsG = c.rsG.p;
    S.nm = (int)nm;
    S.mslot = c.mslot.p; S.mcol = c.mcol.p; S.mcolor = c.mcolor.p;
    S.rmrow = c.rmrow.p;
    // vectors over the unknowns: exact size at set-up; when an update needs
    // more, every held vector is reallocated with headroom for later updates
    const long long Nt = c.N2 + nm;
    const bool first = !c.x.p;
    c.Nt = Nt;
    c.W0 = make_walk(Nt);
    c.W4 = make_walk((Nt + 3) / 4, W4MAXB);
    const long long cap = first ? Nt : Nt + nm / 4 + 1024;
    DBuf<double> *dv[] = {&c.x, &c.r, &c.b, &c.t, &c.rh, &c.p, &c.v, &c.ph, &c.sh, &c.rsp, &c.d64, &c.r2};
    DBuf<float> *fv[] = {&c.fr, &c.frh, &c.fp, &c.fv, &c.fph, &c.fsh, &c.ft, &c.frsp};
    if (first) {
        c.x.alloc(Nt); c.r.alloc(Nt); c.b.alloc(Nt); c.t.alloc(Nt);
        if (!c.mixed) {
            c.rh.alloc(Nt); c.p.alloc(Nt); c.v.alloc(Nt); c.ph.alloc(Nt); c.sh.alloc(Nt); c.rsp.alloc(Nt);
        } else {
            c.d64.alloc(Nt); c.fr.alloc(Nt); c.frh.alloc(Nt); c.fp.alloc(Nt); c.fv.alloc(Nt);
            c.fph.alloc(Nt); c.fsh.alloc(Nt); c.ft.alloc(Nt); c.frsp.alloc(Nt);
        }
    } else {
        for (auto *q : dv)
            if (q->p && (long long)q->n < Nt) q->alloc(cap);
        for (auto *q : fv)
            if (q->p && (long long)q->n < Nt) q->alloc(cap);
    }
    std::vector<double> sc0(S_COUNT, 0.0);
    sc0[S_VPIN] = c.vol_pin;
    IBM_HIP(hipMemcpyAsync(c.sc.p, sc0.data(), S_COUNT * 8, hipMemcpyHostToDevice, s));
    IBM_HIP(hipStreamSynchronize(s));
    c.bytes = estimate_bytes(nx, ny, nz, c.nrows, c.opts.precision);
    IBM_REQUIRE(c.W0.nb <= PSTRIDE - 2048, IBM_EINVAL, "grid too large");
}

poisson_ctx *setup(const ibm_grid *grid, const uint8_t *flags, const ibm_stencils *st, const poisson_opts *opts)
{
    IBM_REQUIRE(flags && st, IBM_EINVAL, "null argument");
    std::unique_ptr<poisson_ctx> c(new poisson_ctx());
    if (opts) c->opts = *opts; else poisson_default_opts(&c->opts);
    poisson_opts &o = c->opts;
    IBM_REQUIRE(o.tol > 0 && o.max_iter > 0 && o.nu1 >= 1 && o.nu2 >= 0 && o.coarse_sweeps >= 1, IBM_EINVAL,
                "bad solver options");
    IBM_REQUIRE(o.precond == IBM_PRECOND_MG || (o.precond == IBM_PRECOND_SRJ && o.srj_sweeps >= 1 &&
                                                 o.srj_sweeps <= IBM_SRJ_MAX_SWEEPS),
                IBM_EINVAL, "bad preconditioner options");
    c->mixed = o.precision == IBM_PREC_MIXED;
    if (o.precond == IBM_PRECOND_SRJ) c->srj_w = srj_schedule(o.srj_sweeps);
    c->g = read_grid(grid);
    for (int d = 0; d < 3; ++d) IBM_REQUIRE(c->g.n[d] == st->n[d], IBM_EINVAL, "stencil table of another grid");
    IBM_HIP(hipStreamCreateWithFlags(&c->cs, hipStreamNonBlocking));
    IBM_HIP(hipEventCreate(&c->e0));
    IBM_HIP(hipEventCreate(&c->e1));
    IBM_HIP(hipEventCreateWithFlags(&c->ej, hipEventDisableTiming));
    c->hsc = pinned_slot();
    hipStream_t s = c->cs;
    const HostGrid &g = c->g;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    c->N = (long long)nx * ny * nz;
    // levels: halve while every dimension is even and the smallest exceeds 4
    int nl = 1;
    {
        int n[3] = {nx, ny, nz};
        while (nl < 16) {
            bool even = n[0] % 2 == 0 && n[1] % 2 == 0 && n[2] % 2 == 0;
            int mn = std::min(n[0], std::min(n[1], n[2]));
            if (!even || mn <= 4) break;
            for (int d = 0; d < 3; ++d) n[d] /= 2;
            ++nl;
        }
    }
    c->lv.resize(nl);
    std::vector<double> faces[3];
    for (int d = 0; d < 3; ++d) faces[d] = g.f[d];
    for (int l = 0; l < nl; ++l) {
        Level &L = c->lv[l];
        for (int d = 0; d < 3; ++d) L.n[d] = g.n[d] >> l;
        if (l > 0)
            for (int d = 0; d < 3; ++d) {
                std::vector<double> cf(L.n[d] + 1);
                for (int i = 0; i <= L.n[d]; ++i) cf[i] = faces[d][2 * i];
                faces[d] = cf;
            }
        level_geometry(L, faces, s);
    }
    // level 0: shorter plane runs per thread (more tiles) measured faster;
    // the half-sweep addresses a tile's planes with 32-bit byte offsets
    c->lv[0].geo = make_geo(c->lv[0].H, c->lv[0].n[1], c->lv[0].n[2], 16384);
    c->lv[0].geo2 = make_geo_rows2(c->lv[0].H, c->lv[0].n[1], c->lv[0].n[2], 8192);
    IBM_REQUIRE(plane_span_ok((long long)c->lv[0].H * c->lv[0].n[1], std::max(c->lv[0].geo.kz, c->lv[0].geo2.kz),
                              sizeof(double)),
                IBM_EINVAL, "grid planes too large for the level-0 sweep's 32-bit offsets");
    c->N2 = 2 * c->lv[0].Nh;
    // prolongation maps of each level from its coarse parent
    for (int l = 1; l < nl; ++l) {
        Level &F = c->lv[l - 1], &C = c->lv[l];
        for (int d = 0; d < 3; ++d) {
            int nf = F.n[d], nc = C.n[d];
            std::vector<int> pi(nf);
            std::vector<double> pt(nf);
            for (int i = 0; i < nf; ++i) {
                double x = F.hc[d][i];
                x = std::min(std::max(x, C.hc[d][0]), C.hc[d][nc - 1]);
                int I0 = 0;
                while (I0 + 1 <= nc - 2 && C.hc[d][I0 + 1] <= x) ++I0;
                pi[i] = I0;
                pt[i] = (x - C.hc[d][I0]) / (C.hc[d][I0 + 1] - C.hc[d][I0]);
            }
            upload(F.pi[d], pi, s);
            upload(F.pt[d], pt, s);
        }
    }
    // tail start (the coarsest levels that fit one workgroup's LDS)
    for (int pass = 0; pass < 2; ++pass) {
        const size_t tsz = pass ? sizeof(double) : sizeof(float);
        int &t0 = pass ? c->tail0d : c->tail0;
        t0 = nl;
        int off = 0;
        for (int l = nl - 1; l >= 1 && (nl - l) <= 8; --l) {
            int m, xo, bo, o2 = off;
            tail_layout(c->lv[l].Nh, tsz, o2, m, xo, bo);
            o2 += tail_coef_bytes(c->lv[l].n[0], c->lv[l].n[1], c->lv[l].n[2]);
            if (o2 > TAIL_LDS) break;
            off = o2;
            t0 = l;
        }
    }
    if (!c->mixed) c->tail0 = c->tail0d;
    // device views, masks and coarse storage
    for (int l = 0; l < nl; ++l) {
        Level &L = c->lv[l];
        L.m.alloc(2 * L.Nh);
        Lv &v = L.lv;
        v.nx = L.n[0]; v.ny = L.n[1]; v.nz = L.n[2]; v.H = L.H; v.Nh = L.Nh;
        v.fH = make_fdiv(L.H);
        v.fy = make_fdiv(L.n[1]);
        for (int d = 0; d < 3; ++d) { v.cp[d] = L.cp[d].p; v.cm[d] = L.cm[d].p; v.w[d] = L.w[d].p; }
        v.f = L.m.p;
        for (int d = 0; d < 3; ++d) { L.pm.pi[d] = L.pi[d].p; L.pm.pt[d] = L.pt[d].p; }
        if (l > 0) {
            if (c->mixed) { L.x32.alloc(2 * L.Nh); L.b16.alloc(2 * L.Nh); }
            else { L.x64.alloc(2 * L.Nh); L.b64.alloc(2 * L.Nh); }
        }
    }
    IBM_REQUIRE(c->lv[0].geo.nb <= PSTRIDE - 2048, IBM_EINVAL, "grid too large");
    for (auto &L : c->lv) {
        IBM_REQUIRE(L.geo.nb <= PSTRIDE && L.geon.nb <= PSTRIDE, IBM_EINVAL, "grid too large");
        IBM_REQUIRE(plane_span_ok((long long)L.H * L.n[1], L.geo.kz, sizeof(double)), IBM_EINVAL,
                    "grid planes too large for the sweeps' 32-bit offsets");
    }
    c->Wc = make_walk(c->N2);
    c->sc.alloc(S_COUNT);
    c->part.alloc((size_t)PSTRIDE * 4);
    c->ssum.alloc(32);
    c->serr.alloc(1);
    if (nl > 1) {
        c->hact[0].alloc(c->lv[1].N);
        if (nl > 2) c->hact[1].alloc(c->lv[2].N);
    }
    setup_geometry(*c, flags, st);
    return c.release();
}

// ------------------------------------------------------------------ solve
struct StreamJoin {
    poisson_ctx &c;
    hipStream_t user;
    StreamJoin(poisson_ctx &cc, hipStream_t u) : c(cc), user(u)
    {
        IBM_HIP(hipEventRecord(c.ej, user));
        IBM_HIP(hipStreamWaitEvent(c.cs, c.ej, 0));
    }
    ~StreamJoin()
    {
        (void)hipEventRecord(c.ej, c.cs);
        (void)hipStreamWaitEvent(user, c.ej, 0);
    }
};

namespace {

void to_split(poisson_ctx &c, const double *nat, double *spl, long long tail, hipStream_t s)
{
    k_to_split<double, double><<<c.W0.nb, TPB, 0, s>>>(c.L0(), c.W0, nat, spl, tail);
    IBM_LAUNCH_CHECK();
}

void from_split(poisson_ctx &c, const double *spl, double *nat, long long tail, hipStream_t s)
{
    k_from_split<double, double><<<c.W0.nb, TPB, 0, s>>>(c.L0(), c.W0, spl, nat, tail);
    IBM_LAUNCH_CHECK();
}

// b (split) from raw natural f and optional g
void assemble_rhs(poisson_ctx &c, const double *f, const double *gval, double *b, hipStream_t s)
{
    to_split(c, f, c.t.p, 0, s);
    k_vsum<double, false><<<c.Wc.nb, TPB, 0, s>>>(c.L0(), c.Wc, c.t.p, c.part.p);
    fin(c, c.Wc.nb, FIN_MEAN, S_TMP, c.vol_fluid, s);
    k_rhs<<<c.W0.nb, TPB, 0, s>>>(c.L0(), c.W0, c.pin, c.t.p, c.sc.p, S_TMP, b);
    if (c.nrows) k_rhs_ghost<<<sparse_blocks(c.nrows), TPB, 0, s>>>(c.sp, c.rdlb.p, gval, b);
    IBM_LAUNCH_CHECK();
}

// FP64 storage of a mixed context, allocated on first need: the coarse FP64
// levels and the FP64 Krylov vectors (the FP64 cycle uses its own tail start)
void ensure_fp64(poisson_ctx &c)
{
    for (size_t l = 1; l < c.lv.size(); ++l) {
        Level &L = c.lv[l];
        if (!L.x64.p) L.x64.alloc(2 * L.Nh);
        if (!L.b64.p) L.b64.alloc(2 * L.Nh);
    }
    DBuf<double> *v[] = {&c.rh, &c.p, &c.v, &c.ph, &c.sh, &c.rsp, &c.r2};
    for (DBuf<double> *b : v)
        if (!b->p) b->alloc(c.Nt);
}

// true relative residual ||b - A x|| / ||b|| of the FP64 iterate (c.t is
// overwritten); for FP64 solves that end without a checked residual
double true_rel_residual(poisson_ctx &c, hipStream_t s)
{
    const Walk &W = c.W0;
    k_dot2<double><<<W.nb, TPB, 0, s>>>(W, c.b.p, c.b.p, c.part.p, PSTRIDE);
    k_fin<<<1, 1024, 0, s>>>(c.part.p, PSTRIDE, W.nb, FIN_SUM, S_TMP2, 0.0, c.sc.p);
    int np = launch_apply<double>(c, M_PINNED, true, 2, c.x.p, c.t.p, c.b.p, nullptr, c.b.p, nullptr, s);
    k_fin<<<1, 1024, 0, s>>>(c.part.p + PSTRIDE, PSTRIDE, np, FIN_SUM, S_TMP, 0.0, c.sc.p);
    IBM_LAUNCH_CHECK();
    read_scalars(c, s);
    const double bn2 = c.hsc[S_TMP2];
    return bn2 > 0.0 ? std::sqrt(c.hsc[S_TMP] / bn2) : 0.0;
}

// solve A x = b (assembled, in c.b, split) into c.x; returns status.  warm:
// c.x holds an initial guess (zero on inactive slots, zero at the pin)
int solve_core(poisson_ctx &c, poisson_stats *stats, hipStream_t s, bool warm = false)
{
    const poisson_opts &o = c.opts;
    int rc = IBM_ENOCONV, its = 0, outer = 0;
    double rel = 1.0;
    if (!c.mixed && !warm) {
        its = bicgstab<double, double>(c, c.b.p, c.x.p, c.r.p, c.rh.p, c.p.p, c.v.p, c.ph.p, c.sh.p, c.t.p, o.tol, o.max_iter,
                               true, &c.g64, s, &rc, &rel);
        if (log_enabled()) fprintf(stderr, "[ibm] fp64: %d iterations to %.3e (rc %d)\n", its, rel, rc);
    } else if (!c.mixed) {
        // FP64 from an initial guess: BiCGSTAB on the correction, A d = b - A x0
        const Walk &W = c.W0;
        reserve(c.d64, c.Nt);
        reserve(c.r2, c.Nt);
        k_dot2<double><<<W.nb, TPB, 0, s>>>(W, c.b.p, c.b.p, c.part.p, PSTRIDE);
        k_fin<<<1, 1024, 0, s>>>(c.part.p, PSTRIDE, W.nb, FIN_SUM, S_TMP2, 0.0, c.sc.p);
        int np = launch_apply<double>(c, M_PINNED, true, 2, c.x.p, c.r2.p, c.b.p, nullptr, c.b.p, nullptr, s);
        k_fin<<<1, 1024, 0, s>>>(c.part.p + PSTRIDE, PSTRIDE, np, FIN_SUM, S_TMP, 0.0, c.sc.p);
        IBM_LAUNCH_CHECK();
        read_scalars(c, s);
        const double bn2 = c.hsc[S_TMP2];
        const double rel0 = bn2 > 0.0 ? std::sqrt(c.hsc[S_TMP] / bn2) : 0.0;
        if (!std::isfinite(rel0)) {
            rc = IBM_EBREAKDOWN;
        } else if (bn2 == 0.0) {
            k_fill<double><<<W.nb, TPB, 0, s>>>(W, c.x.p, 0.0);
            rc = IBM_OK;
            rel = 0.0;
        } else if (rel0 <= o.tol) {
            rc = IBM_OK;
            rel = rel0;
        } else {
            double r1;
            its = bicgstab<double, double>(c, c.r2.p, c.d64.p, c.r.p, c.rh.p, c.p.p, c.v.p, c.ph.p, c.sh.p, c.t.p,
                                           o.tol / rel0, o.max_iter, true, &c.g64w, s, &rc, &r1);
            k_add<double><<<W.nb, TPB, 0, s>>>(W, c.x.p, c.d64.p);
            IBM_LAUNCH_CHECK();
            rel = r1 * rel0;
        }
        if (log_enabled())
            fprintf(stderr, "[ibm] fp64 from a guess (rel %.3e): %d iterations to %.3e (rc %d)\n", rel0, its, rel, rc);
    } else {
        // FP64 iterative refinement around FP32 inner solves
        const Walk &W = c.W0;
        if (!warm) k_fill<double><<<W.nb, TPB, 0, s>>>(W, c.x.p, 0.0);
        k_dot2<double><<<W.nb, TPB, 0, s>>>(W, c.b.p, c.b.p, c.part.p, PSTRIDE);
        k_fin<<<1, 1024, 0, s>>>(c.part.p, PSTRIDE, W.nb, FIN_SUM, S_TMP2, 0.0, c.sc.p);
        IBM_LAUNCH_CHECK();
        read_scalars(c, s);
        const double bn2 = c.hsc[S_TMP2];
        double prev = HUGE_VAL;
        bool inner_failed = false;
        for (outer = 0; outer <= o.max_outer; ++outer) {
            if (bn2 == 0.0) {
                k_fill<double><<<W.nb, TPB, 0, s>>>(W, c.x.p, 0.0);
                rc = IBM_OK;
                rel = 0.0;
                break;
            }
            // r64 = b - A x (pinned) and its norm
            int np = launch_apply<double>(c, M_PINNED, true, 2, c.x.p, c.r.p, c.b.p, nullptr, c.b.p, nullptr, s);
            k_fin<<<1, 1024, 0, s>>>(c.part.p + PSTRIDE, PSTRIDE, np, FIN_SUM, S_TMP, 0.0, c.sc.p);
            IBM_LAUNCH_CHECK();
            read_scalars(c, s);
            rel = std::sqrt(c.hsc[S_TMP] / bn2);
            if (!std::isfinite(rel)) { rc = IBM_EBREAKDOWN; break; }
            if (rel <= o.tol) { rc = IBM_OK; break; }
            if (rel > prev || inner_failed) {
                // refinement has stalled: either the FP32 correction made the
                // FP64 residual larger (the FP32 solves cannot resolve this
                // system: the condition number times the FP32 unit roundoff is
                // not small; that correction is undone), or the FP32 solve ran
                // out of iterations before its tolerance.  Finish with an FP64
                // BiCGSTAB on the remaining residual.
                const bool grew = rel > prev;
                if (grew) {
                    k_add<double><<<W.nb, TPB, 0, s>>>(W, c.x.p, c.d64.p, -1.0);
                    IBM_LAUNCH_CHECK();
                }
                const double base = grew ? prev : rel;
                if (log_enabled())
                    fprintf(stderr, "[ibm] outer %d: rel %.3e (previous %.3e, inner %s), refinement stalled: FP64 fallback\n",
                            outer, rel, prev, inner_failed ? "unconverged" : "converged");
                ensure_fp64(c);
                launch_apply<double>(c, M_PINNED, true, 2, c.x.p, c.r2.p, c.b.p, nullptr, c.b.p, nullptr, s);
                int frc;
                double frel;
                its += bicgstab<double, double>(c, c.r2.p, c.d64.p, c.r.p, c.rh.p, c.p.p, c.v.p, c.ph.p, c.sh.p,
                                                c.t.p, o.tol / base, o.max_iter, true, &c.g64, s, &frc, &frel);
                k_add<double><<<W.nb, TPB, 0, s>>>(W, c.x.p, c.d64.p);
                int np = launch_apply<double>(c, M_PINNED, true, 2, c.x.p, c.r.p, c.b.p, nullptr, c.b.p, nullptr, s);
                k_fin<<<1, 1024, 0, s>>>(c.part.p + PSTRIDE, PSTRIDE, np, FIN_SUM, S_TMP, 0.0, c.sc.p);
                IBM_LAUNCH_CHECK();
                read_scalars(c, s);
                rel = std::sqrt(c.hsc[S_TMP] / bn2);
                rc = frc == IBM_EBREAKDOWN ? frc : (rel <= o.tol ? IBM_OK : IBM_ENOCONV);
                if (log_enabled()) fprintf(stderr, "[ibm] fp64 fallback: rel %.3e (rc %d)\n", rel, rc);
                break;
            }
            if (outer == o.max_outer) { rc = IBM_ENOCONV; break; }
            prev = rel;
            // inner FP32 solve of A d = r64 (the inner residual vector starts as r64
            // rounded to FP32); it asks only for the reduction still needed,
            // never less than inner_tol
            int irc;
            double irel;
            const double itol = std::max(o.inner_tol, 0.5 * o.tol / rel);
            const int n_in = bicgstab<float, double>(c, (const double *)c.r.p, c.d64.p, c.fr.p, c.frh.p, c.fp.p, c.fv.p,
                                                     c.fph.p, c.fsh.p, c.ft.p, itol, o.max_iter, false, &c.g32, s,
                                                     &irc, &irel);
            its += n_in;
            if (log_enabled())
                fprintf(stderr, "[ibm] outer %d: rel %.3e, inner tol %.1e: %d iterations to %.2e (rc %d)\n", outer, rel,
                        itol, n_in, irel, irc);
            if (irc == IBM_EBREAKDOWN) { rc = irc; break; }
            inner_failed = irc == IBM_ENOCONV;
            k_add<double><<<W.nb, TPB, 0, s>>>(W, c.x.p, c.d64.p);
            IBM_LAUNCH_CHECK();
        }
    }
    // an FP64 solve that stopped at its iteration limit or at a breakdown
    // holds the recursively updated residual, not the true one
    if (!c.mixed && rc != IBM_OK && std::isfinite(rel)) rel = true_rel_residual(c, s);
    if (stats) {
        stats->iterations = its;
        stats->outer_steps = outer;
        stats->rel_residual = rel;
        stats->status = rc;
        stats->levels = (int)c.lv.size();
        stats->n_fallback = c.n_fallback;
    }
    return rc;
}

}  // namespace
}  // namespace ibm

// ------------------------------------------------------------------ C ABI
extern "C" void poisson_default_opts(poisson_opts *o)
{
    if (!o) return;
    o->precision = IBM_PREC_FP64;
    o->tol = 1e-10;
    o->max_iter = 200;
    o->nu1 = 2;
    o->nu2 = 2;
    o->coarse_sweeps = 32;
    o->inner_tol = 1e-3;
    o->max_outer = 10;
    o->use_graph = 1;
    o->precond = IBM_PRECOND_MG;
    o->srj_sweeps = 16;
}

extern "C" int32_t poisson_workspace_estimate(int32_t nx, int32_t ny, int32_t nz, int64_t n_rows, int32_t precision,
                                              size_t *bytes)
{
    return guarded([&] {
        IBM_REQUIRE(bytes && nx > 0 && ny > 0 && nz > 0, IBM_EINVAL, "bad arguments");
        *bytes = estimate_bytes(nx, ny, nz, n_rows, precision);
    });
}

extern "C" int32_t poisson_setup(const ibm_grid *grid, const uint8_t *flags_dev, const ibm_stencils *st,
                                 const poisson_opts *opts, size_t *workspace_bytes, poisson_ctx **out)
{
    return guarded([&] {
        IBM_REQUIRE(out, IBM_EINVAL, "null output");
        poisson_ctx *c = setup(grid, flags_dev, st, opts);
        if (workspace_bytes) *workspace_bytes = c->bytes;
        *out = c;
    });
}

extern "C" int32_t poisson_solve(poisson_ctx *c, const double *f_dev, const double *g_dev, double *x_dev,
                                 poisson_stats *stats, void *stream)
{
    return guarded([&] {
        IBM_REQUIRE(c && f_dev && x_dev, IBM_EINVAL, "null argument");
        StreamJoin j(*c, (hipStream_t)stream);
        hipStream_t s = c->cs;
        IBM_HIP(hipEventRecord(c->e0, s));
        assemble_rhs(*c, f_dev, g_dev, c->b.p, s);
        int rc = solve_core(*c, stats, s);
        // gauge: volume-weighted fluid mean removed from fluid, ghost and membrane-ghost values
        k_pinres<<<1, 64, 0, s>>>(c->L0(), c->pin, c->x.p, c->sc.p);
        k_vsum<double, false><<<c->Wc.nb, TPB, 0, s>>>(c->L0(), c->Wc, c->x.p, c->part.p);
        fin(*c, c->Wc.nb, FIN_MEAN, S_TMP2, c->vol_fluid, s);
        k_gauge<<<c->W0.nb, TPB, 0, s>>>(c->L0(), c->W0, c->x.p, c->sc.p, S_TMP2, c->t.p);
        from_split(*c, c->t.p, x_dev, c->nm, s);
        IBM_HIP(hipEventRecord(c->e1, s));
        read_scalars(*c, s);
        if (stats) {
            float ms = 0.f;
            IBM_HIP(hipEventElapsedTime(&ms, c->e0, c->e1));
            stats->solve_ms = ms;
            stats->pin_residual = c->hsc[S_TMP];
        }
        if (rc == IBM_ENOCONV) throw Error(IBM_ENOCONV, "iteration limit reached");
        if (rc == IBM_EBREAKDOWN) throw Error(IBM_EBREAKDOWN, "BiCGSTAB breakdown or non-finite values");
    });
}

extern "C" int32_t poisson_solve_from(poisson_ctx *c, const double *f_dev, const double *g_dev, const double *x0_dev,
                                      int64_t n_x0, double *x_dev, poisson_stats *stats, void *stream)
{
    return guarded([&] {
        IBM_REQUIRE(c && f_dev && x0_dev && x_dev, IBM_EINVAL, "null argument");
        IBM_REQUIRE(n_x0 == c->N || n_x0 == c->N + c->nm, IBM_EINVAL, "initial guess must hold N or N + n_mghost values");
        StreamJoin j(*c, (hipStream_t)stream);
        hipStream_t s = c->cs;
        IBM_HIP(hipEventRecord(c->e0, s));
        assemble_rhs(*c, f_dev, g_dev, c->b.p, s);
        // initial guess: the cells (and membrane ghost unknowns when given)
        // from x0, inactive slots zero, shifted to a zero pin value
        const bool ghosts = n_x0 > c->N;
        k_to_split<double, double><<<c->W0.nb, TPB, 0, s>>>(c->L0(), c->W0, x0_dev, c->x.p, ghosts ? c->nm : 0);
        if (c->nm && !ghosts)
            k_warm_membrane<<<(int)std::min<long long>((c->nm + TPB - 1) / TPB, 4096), TPB, 0, s>>>(c->sp, c->x.p);
        k_zero_inactive<<<c->Wc.nb, TPB, 0, s>>>(c->L0(), c->Wc, c->x.p);
        k_shift<double><<<c->W0.nb, TPB, 0, s>>>(c->L0(), c->W0, c->pin, c->x.p);
        k_shift_pin<<<1, 1, 0, s>>>(c->pin, c->x.p);
        IBM_LAUNCH_CHECK();
        int rc = solve_core(*c, stats, s, true);
        k_pinres<<<1, 64, 0, s>>>(c->L0(), c->pin, c->x.p, c->sc.p);
        k_vsum<double, false><<<c->Wc.nb, TPB, 0, s>>>(c->L0(), c->Wc, c->x.p, c->part.p);
        fin(*c, c->Wc.nb, FIN_MEAN, S_TMP2, c->vol_fluid, s);
        k_gauge<<<c->W0.nb, TPB, 0, s>>>(c->L0(), c->W0, c->x.p, c->sc.p, S_TMP2, c->t.p);
        from_split(*c, c->t.p, x_dev, c->nm, s);
        IBM_HIP(hipEventRecord(c->e1, s));
        read_scalars(*c, s);
        if (stats) {
            float ms = 0.f;
            IBM_HIP(hipEventElapsedTime(&ms, c->e0, c->e1));
            stats->solve_ms = ms;
            stats->pin_residual = c->hsc[S_TMP];
        }
        if (rc == IBM_ENOCONV) throw Error(IBM_ENOCONV, "iteration limit reached");
        if (rc == IBM_EBREAKDOWN) throw Error(IBM_EBREAKDOWN, "BiCGSTAB breakdown or non-finite values");
    });
}

extern "C" int32_t poisson_update(poisson_ctx *c, const uint8_t *flags_dev, const ibm_stencils *st)
{
    return guarded([&] {
        IBM_REQUIRE(c && flags_dev && st, IBM_EINVAL, "null argument");
        setup_geometry(*c, flags_dev, st);
    });
}

extern "C" int32_t ibm_fill_fresh(const ibm_grid *grid, const uint8_t *flags_old_dev, const uint8_t *flags_new_dev,
                                  double *x_dev, int64_t *n_fresh, void *stream)
{
    return guarded([&] {
        IBM_REQUIRE(grid && flags_old_dev && flags_new_dev && x_dev, IBM_EINVAL, "null argument");
        const HostGrid g = read_grid(grid);
        const long long N = (long long)g.n[0] * g.n[1] * g.n[2];
        hipStream_t s = (hipStream_t)stream;
        DBuf<int> cnt(1);
        IBM_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int), s));
        const int nb = (int)std::min<long long>(std::max<long long>((N + TPB - 1) / TPB, 1), 8192);
        k_fill_fresh<<<nb, TPB, 0, s>>>(g.n[0], g.n[1], g.n[2], flags_old_dev, flags_new_dev, x_dev, cnt.p);
        IBM_LAUNCH_CHECK();
        int h = 0;
        IBM_HIP(hipMemcpyAsync(&h, cnt.p, sizeof(int), hipMemcpyDeviceToHost, s));
        IBM_HIP(hipStreamSynchronize(s));
        if (n_fresh) *n_fresh = h;
    });
}

extern "C" int32_t poisson_solve_assembled(poisson_ctx *c, const double *b_dev, double *x_dev, poisson_stats *stats,
                                           void *stream)
{
    return guarded([&] {
        IBM_REQUIRE(c && b_dev && x_dev, IBM_EINVAL, "null argument");
        StreamJoin j(*c, (hipStream_t)stream);
        hipStream_t s = c->cs;
        IBM_HIP(hipEventRecord(c->e0, s));
        to_split(*c, b_dev, c->b.p, c->nm, s);
        int rc = solve_core(*c, stats, s);
        from_split(*c, c->x.p, x_dev, c->nm, s);
        IBM_HIP(hipEventRecord(c->e1, s));
        IBM_HIP(hipStreamSynchronize(s));
        if (stats) {
            float ms = 0.f;
            IBM_HIP(hipEventElapsedTime(&ms, c->e0, c->e1));
            stats->solve_ms = ms;
        }
        if (rc != IBM_OK) throw Error(rc, rc == IBM_ENOCONV ? "iteration limit reached" : "breakdown");
    });
}

extern "C" int32_t poisson_apply(poisson_ctx *c, const double *x_dev, double *y_dev, void *stream)
{
    return guarded([&] {
        IBM_REQUIRE(c && x_dev && y_dev, IBM_EINVAL, "null argument");
        StreamJoin j(*c, (hipStream_t)stream);
        hipStream_t s = c->cs;
        to_split(*c, x_dev, c->r.p, c->nm, s);
        launch_apply<double>(*c, M_PINNED, false, 0, c->r.p, c->t.p, nullptr, nullptr, nullptr, nullptr, s);
        from_split(*c, c->t.p, y_dev, c->nm, s);
    });
}

extern "C" int32_t poisson_assemble_rhs(poisson_ctx *c, const double *f_dev, const double *g_dev, double *b_dev,
                                        void *stream)
{
    return guarded([&] {
        IBM_REQUIRE(c && f_dev && b_dev, IBM_EINVAL, "null argument");
        StreamJoin j(*c, (hipStream_t)stream);
        hipStream_t s = c->cs;
        assemble_rhs(*c, f_dev, g_dev, c->r.p, s);
        from_split(*c, c->r.p, b_dev, c->nm, s);
    });
}

extern "C" int32_t poisson_precond(poisson_ctx *c, const double *b_dev, double *x_dev, void *stream)
{
    return guarded([&] {
        IBM_REQUIRE(c && b_dev && x_dev, IBM_EINVAL, "null argument");
        IBM_REQUIRE(!c->mixed, IBM_EINVAL, "poisson_precond needs an FP64 context");
        StreamJoin j(*c, (hipStream_t)stream);
        hipStream_t s = c->cs;
        to_split(*c, b_dev, c->r.p, c->nm, s);
        k_vsum<double, true><<<c->Wc.nb, TPB, 0, s>>>(c->L0(), c->Wc, c->r.p, c->part.p);
        fin(*c, c->Wc.nb, FIN_SINK, S_SINKP, 0.0, s);
        precond<double>(*c, c->r.p, c->t.p, c->sc.p + S_SINKP, s);
        // shift: every active unknown minus the pin value, then the pin itself
        k_shift<double><<<c->W0.nb, TPB, 0, s>>>(c->L0(), c->W0, c->pin, c->t.p);
        k_shift_pin<<<1, 1, 0, s>>>(c->pin, c->t.p);
        from_split(*c, c->t.p, x_dev, c->nm, s);
        IBM_LAUNCH_CHECK();
    });
}

extern "C" int32_t poisson_kernel_timing(poisson_ctx *c, int32_t kernel, int32_t reset, double *total_ms,
                                         int64_t *launches)
{
    return guarded([&] {
        IBM_REQUIRE(c, IBM_EINVAL, "null context");
        IBM_REQUIRE(kernel >= -1 && kernel <= PK_XR, IBM_EINVAL, "unknown kernel id");
        if (total_ms) *total_ms = c->prof_ms;
        if (launches) *launches = c->prof_count;
        if (reset) { c->prof_ms = 0.0; c->prof_count = 0; c->prof_used = 0; }
        c->prof_kernel = kernel;
    });
}

extern "C" int32_t poisson_level_info(poisson_ctx *c, int32_t *levels, int64_t *n_unknowns, int64_t *n_ghost,
                                      int64_t *n_mghost)
{
    return guarded([&] {
        IBM_REQUIRE(c, IBM_EINVAL, "null context");
        if (levels) *levels = (int32_t)c->lv.size();
        if (n_unknowns) *n_unknowns = c->N + c->nm;
        if (n_ghost) *n_ghost = c->ng;
        if (n_mghost) *n_mghost = c->nm;
    });
}

namespace ibm {
namespace {
// the context's large per-call scratch (Krylov vectors, level iterates and
// right-hand sides): every buffer currently held, in a fixed order
template <class F>
void for_scratch(poisson_ctx &c, F &&f)
{
    DBuf<double> *d[] = {&c.x, &c.r, &c.b, &c.t, &c.rh, &c.p, &c.v, &c.ph, &c.sh, &c.rsp, &c.d64, &c.r2};
    for (auto *q : d) f(*q);
    DBuf<float> *fl[] = {&c.fr, &c.frh, &c.fp, &c.fv, &c.fph, &c.fsh, &c.ft, &c.frsp};
    for (auto *q : fl) f(*q);
    for (size_t l = 1; l < c.lv.size(); ++l) {
        f(c.lv[l].x64);
        f(c.lv[l].b64);
        f(c.lv[l].x32);
        f(c.lv[l].b16);
    }
}
constexpr size_t WS_ALIGN = 256;
size_t ws_round(size_t b) { return (b + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN; }
}  // namespace
}  // namespace ibm

extern "C" int32_t poisson_workspace_size(poisson_ctx *c, size_t *bytes)
{
    return guarded([&] {
        IBM_REQUIRE(c && bytes, IBM_EINVAL, "null argument");
        size_t total = 0;
        for_scratch(*c, [&](auto &b) { total += ws_round(b.bytes()); });
        *bytes = total;
    });
}

extern "C" int32_t poisson_bind_workspace(poisson_ctx *c, void *ws_dev, size_t bytes)
{
    return guarded([&] {
        IBM_REQUIRE(c && ws_dev, IBM_EINVAL, "null argument");
        IBM_REQUIRE(((uintptr_t)ws_dev % WS_ALIGN) == 0, IBM_EINVAL, "workspace must be 256-byte aligned");
        size_t need = 0;
        for_scratch(*c, [&](auto &b) { need += ws_round(b.bytes()); });
        IBM_REQUIRE(bytes >= need, IBM_ENOMEM, "workspace too small: " + std::to_string(bytes) + " < " +
                                                   std::to_string(need));
        IBM_HIP(hipStreamSynchronize(c->cs));
        // captured iterations hold the old addresses
        if (c->g64) { (void)hipGraphExecDestroy(c->g64); c->g64 = nullptr; }
        if (c->g32) { (void)hipGraphExecDestroy(c->g32); c->g32 = nullptr; }
        if (c->g64w) { (void)hipGraphExecDestroy(c->g64w); c->g64w = nullptr; }
        char *base = (char *)ws_dev;
        size_t off = 0;
        for_scratch(*c, [&](auto &b) {
            if (!b.n) return;
            const size_t n = b.n, sz = ws_round(b.bytes());
            typedef typename std::remove_reference<decltype(*b.p)>::type E;
            b.view(reinterpret_cast<E *>(base + off), n);
            off += sz;
        });
    });
}

extern "C" void poisson_destroy(poisson_ctx *c)
{
    if (c) {
        (void)hipStreamSynchronize(c->cs);
        delete c;
    }
}
