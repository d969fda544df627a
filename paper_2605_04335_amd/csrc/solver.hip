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

#include "kernels.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <type_traits>

namespace ibm {

namespace {

constexpr int PSTRIDE = MAXB + 4096;  // partial slots: bulk blocks, then ghost and membrane blocks
constexpr int XB = 1024;              // cap on blocks of the sparse row kernels

inline int sparse_blocks(long long n) { return (int)std::max<long long>(1, std::min<long long>(XB, (n + TPB - 1) / TPB)); }

struct Level {
    int n[3] = {0, 0, 0};
    long long N = 0;
    DBuf<double> c[3], w[3], cp[3], cm[3];
    DBuf<uint8_t> m;                   // coarse: bit0 active, bits1-3 open, bits4-6 cut
    DBuf<int> pi[3];                   // transfer map from the coarse parent (levels < last)
    DBuf<double> pt[3];
    double volA = 0.0;                 // volume of the active cells
    Walk walk;
    DBuf<double> x64, b64, r64;
    DBuf<float> x32, r32;
    DBuf<bf16> b16;
    LC lc;
    PMap pm;
    std::vector<uint8_t> hm;           // host copy of the coarse mask (setup only)
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
        upload(L.c[d], L.hc[d], s);
        upload(L.w[d], L.hw[d], s);
        upload(L.cp[d], cp, s);
        upload(L.cm[d], cm, s);
    }
    L.N = (long long)L.n[0] * L.n[1] * L.n[2];
    L.walk = make_walk(L.N);
}

}  // namespace
}  // namespace ibm

using namespace ibm;

struct poisson_ctx {
    poisson_opts opts;
    HostGrid g;
    long long N = 0, nm = 0, ng = 0, nrows = 0, n_fallback = 0, pin = 0;
    double vol_fluid = 0.0, vol_pin = 0.0;
    DBuf<uint8_t> flags;
    DBuf<int32_t> rcell, rcol, mcol;
    DBuf<double> rw, rsG, rdlb;
    std::vector<Level> lv;
    L0 l0;
    Walk W0;   // over N + nm unknowns
    Walk Wc;   // over N cells
    // FP64 Krylov vectors
    DBuf<double> x, r, rh, p, v, ph, sh, t, r0, b;
    // mixed: FP32 inner vectors
    DBuf<float> fd, fr, frh, fp, fv, fph, fsh, ft, fr0;
    DBuf<double> gtmp, sc, part;
    double *hsc = nullptr;  // pinned host mirror of the scalars
    hipStream_t cs = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr, ej = nullptr;
    hipGraphExec_t g64 = nullptr, g32 = nullptr;
    size_t bytes = 0;
    bool mixed = false;
    // per-launch timing of one kernel (HIP events on the solve stream)
    int prof_kernel = -1;
    bool capturing = false;
    std::vector<hipEvent_t> prof_ev;
    int prof_used = 0;
    double prof_ms = 0.0;
    long long prof_count = 0;

    ~poisson_ctx()
    {
        if (g64) (void)hipGraphExecDestroy(g64);
        if (g32) (void)hipGraphExecDestroy(g32);
        if (hsc) (void)hipHostFree(hsc);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (ej) (void)hipEventDestroy(ej);
        if (cs) (void)hipStreamDestroy(cs);
        for (auto e : prof_ev) (void)hipEventDestroy(e);
    }
};

namespace ibm {
namespace {

// ------------------------------------------------------------------ launch helpers
inline L0 &l0(poisson_ctx &c) { return c.l0; }

template <class T>
void launch_apply(poisson_ctx &c, int mode, bool res, int nd, const T *x, T *y, const T *b, const double *sink,
                  const T *u1, const T *u2, hipStream_t s, int *nparts)
{
    const Walk &W = c.Wc;
    double *P = c.part.p;
    const int gb = sparse_blocks(c.nrows), mb = sparse_blocks(c.nm);
#define AP(MODE, RES, ND)                                                                                       \
    k0_apply<T, MODE, RES, ND><<<W.nb, TPB, 0, s>>>(c.l0, W, x, y, b, sink, u1, u2, P, PSTRIDE);              \
    if (c.nrows) k0_ghost<T, RES, ND><<<gb, TPB, 0, s>>>(c.l0, x, y, b, u1, u2, P, PSTRIDE, W.nb);           \
    if (c.nm) k0_mrow<T, RES, ND><<<mb, TPB, 0, s>>>(c.l0, x, y, b, u1, u2, P, PSTRIDE, W.nb + gb);
    if (res) {
        if (mode == M_UNPINNED && nd == 0) { AP(M_UNPINNED, true, 0) }
        else if (mode == M_PINNED && nd == 2) { AP(M_PINNED, true, 2) }
        else throw Error(IBM_EINVAL, "apply variant");
    } else {
        if (mode == M_PINZERO && nd == 1) { AP(M_PINZERO, false, 1) }
        else if (mode == M_PINZERO && nd == 2) { AP(M_PINZERO, false, 2) }
        else if (mode == M_PINNED && nd == 0) { AP(M_PINNED, false, 0) }
        else throw Error(IBM_EINVAL, "apply variant");
    }
#undef AP
    IBM_LAUNCH_CHECK();
    if (nparts) *nparts = W.nb + (c.nrows ? gb : 0) + (c.nm ? mb : 0);
}

inline void fin(poisson_ctx &c, int n, int op, int dst, double aux, hipStream_t s)
{
    k_fin<<<1, 1024, 0, s>>>(c.part.p, PSTRIDE, n, op, dst, aux, c.sc.p);
    IBM_LAUNCH_CHECK();
}

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

// after a stream synchronisation: accumulate the recorded launch times
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

// storage of each level for a precision
template <class T>
struct Store;
template <>
struct Store<double> {
    typedef double Tc;
    typedef double TB;
    typedef double TR;
    static Tc *x(Level &L) { return L.x64.p; }
    static TB *b(Level &L) { return L.b64.p; }
    static TR *r(Level &L) { return L.r64.p; }
};
template <>
struct Store<float> {
    typedef float Tc;
    typedef bf16 TB;
    typedef float TR;
    static Tc *x(Level &L) { return L.x32.p; }
    static TB *b(Level &L) { return L.b16.p; }
    static TR *r(Level &L) { return L.r32.p; }
};

template <class Tc, class TB>
void coarse_smooth(poisson_ctx &c, Level &L, int steps, bool from_zero, const double *mean, hipStream_t s)
{
    Tc *x = Store<Tc>::x(L);
    const TB *b = Store<Tc>::b(L);
    for (int it = 0; it < steps; ++it) {
        if (it == 0 && from_zero)
            kc_sweep<Tc, TB, true><<<L.walk.nb, TPB, 0, s>>>(L.lc, L.walk, x, b, mean, 0);
        else
            kc_sweep<Tc, TB, false><<<L.walk.nb, TPB, 0, s>>>(L.lc, L.walk, x, b, mean, 0);
        kc_sweep<Tc, TB, false><<<L.walk.nb, TPB, 0, s>>>(L.lc, L.walk, x, b, mean, 1);
    }
    IBM_LAUNCH_CHECK();
}

template <class T>
void fine_smooth(poisson_ctx &c, T *x, const T *b, const double *sink, bool from_zero, hipStream_t s)
{
    const Walk &W = c.Wc;
    const int gb = sparse_blocks(c.nrows), mb = sparse_blocks(c.nm);
    for (int color = 0; color < 2; ++color) {
        if (from_zero && color == 0) {
            k0_sweep<T, true><<<W.nb, TPB, 0, s>>>(c.l0, W, x, b, sink, 0);
            if (c.nm) {
                Walk Wt = make_walk(c.nm);
                k_fill<T><<<Wt.nb, TPB, 0, s>>>(Wt, x + c.N, 0.0);
            }
        } else {
            prof_begin(c, PK_SWEEP0, s);
            k0_sweep<T, false><<<W.nb, TPB, 0, s>>>(c.l0, W, x, b, sink, color);
            prof_end(c, PK_SWEEP0, s);
        }
        if (c.nm) k0_msweep<T><<<mb, TPB, 0, s>>>(c.l0, x, b, color);
    }
    if (c.nrows) {
        k0_gjac<T><<<gb, TPB, 0, s>>>(c.l0, x, b, c.gtmp.p);
        k0_gscat<T><<<gb, TPB, 0, s>>>(c.l0, x, c.gtmp.p);
    }
    IBM_LAUNCH_CHECK();
}

// x = V-cycle(b) on the unpinned operator with the sink at the pin; x unshifted
template <class T>
void vcycle(poisson_ctx &c, const T *b, T *x, const double *sink, hipStream_t s)
{
    typedef typename Store<T>::Tc Tc;
    typedef typename Store<T>::TB TB;
    typedef typename Store<T>::TR TR;
    const int nl = (int)c.lv.size();
    const poisson_opts &o = c.opts;
    for (int it = 0; it < o.nu1; ++it) fine_smooth<T>(c, x, b, sink, it == 0, s);
    if (o.nu1 == 0) {
        k_fill<T><<<c.W0.nb, TPB, 0, s>>>(c.W0, x, 0.0);
        IBM_LAUNCH_CHECK();
    }
    if (nl > 1) {
        T *r0 = std::is_same<T, double>::value ? (T *)c.r0.p : (T *)c.fr0.p;
        launch_apply<T>(c, M_UNPINNED, true, 0, x, r0, b, sink, nullptr, nullptr, s, nullptr);
        LC dummy{};
        Level &L1 = c.lv[1];
        k_restrict<T, TB, true><<<L1.walk.nb, TPB, 0, s>>>(c.l0, dummy, L1.lc, L1.walk, r0, Store<T>::b(L1), c.part.p);
        fin(c, L1.walk.nb, FIN_MEAN, S_MEAN0 + 1, L1.volA, s);
        for (int l = 1; l < nl; ++l) {
            Level &L = c.lv[l];
            const double *mean = c.sc.p + S_MEAN0 + l;
            if (l == nl - 1) {
                coarse_smooth<Tc, TB>(c, L, o.coarse_sweeps, true, mean, s);
                break;
            }
            coarse_smooth<Tc, TB>(c, L, std::max(o.nu1, 1), true, mean, s);
            kc_resid<Tc, TB, TR><<<L.walk.nb, TPB, 0, s>>>(L.lc, L.walk, Store<T>::x(L), Store<T>::b(L), mean,
                                                           Store<T>::r(L));
            Level &C = c.lv[l + 1];
            k_restrict<TR, TB, false><<<C.walk.nb, TPB, 0, s>>>(c.l0, L.lc, C.lc, C.walk, Store<T>::r(L),
                                                                Store<T>::b(C), c.part.p);
            fin(c, C.walk.nb, FIN_MEAN, S_MEAN0 + l + 1, C.volA, s);
        }
        for (int l = nl - 2; l >= 1; --l) {
            Level &L = c.lv[l];
            Level &C = c.lv[l + 1];
            k_prolong<Tc, Tc, false><<<L.walk.nb, TPB, 0, s>>>(c.l0, L.lc, C.lc, L.pm, L.walk, Store<T>::x(C),
                                                               Store<T>::x(L));
            coarse_smooth<Tc, TB>(c, L, o.nu2, false, c.sc.p + S_MEAN0 + l, s);
        }
        LC dummy2{};
        Level &L0v = c.lv[0];
        k_prolong<Tc, T, true><<<c.Wc.nb, TPB, 0, s>>>(c.l0, dummy2, c.lv[1].lc, L0v.pm, c.Wc, Store<T>::x(c.lv[1]), x);
        IBM_LAUNCH_CHECK();
    }
    for (int it = 0; it < o.nu2; ++it) fine_smooth<T>(c, x, b, sink, false, s);
}

// One BiCGSTAB iteration (van der Vorst 1992, right preconditioning): all
// scalars stay on the device.
template <class T, class TX>
void bicg_iteration(poisson_ctx &c, T *x, T *r, T *rh, T *p, T *v, T *ph, T *sh, T *t, TX *xx, hipStream_t s)
{
    const Walk &W = c.W0;
    k_p_update<T><<<W.nb, TPB, 0, s>>>(c.l0, W, r, p, v, c.sc.p, c.part.p);
    fin(c, W.nb, FIN_SINK, S_SINKP, 0.0, s);
    vcycle<T>(c, p, ph, c.sc.p + S_SINKP, s);
    int np;
    prof_begin(c, PK_APPLY0, s);
    launch_apply<T>(c, M_PINZERO, false, 1, ph, v, nullptr, nullptr, rh, nullptr, s, &np);
    prof_end(c, PK_APPLY0, s);
    fin(c, np, FIN_ALPHA, 0, 0.0, s);
    k_s_update<T><<<W.nb, TPB, 0, s>>>(c.l0, W, r, v, c.sc.p, c.part.p);
    fin(c, W.nb, FIN_SINK, S_SINKS, 0.0, s);
    vcycle<T>(c, r, sh, c.sc.p + S_SINKS, s);
    launch_apply<T>(c, M_PINZERO, false, 2, sh, t, nullptr, nullptr, r, nullptr, s, &np);
    fin(c, np, FIN_OMEGA, 0, 0.0, s);
    prof_begin(c, PK_XR, s);
    k_xr_update<T, TX><<<W.nb, TPB, 0, s>>>(c.l0, W, xx, ph, sh, r, t, rh, c.sc.p, c.part.p, PSTRIDE);
    prof_end(c, PK_XR, s);
    IBM_LAUNCH_CHECK();
    fin(c, W.nb, FIN_RHO, 0, 0.0, s);
    (void)x;
}

void read_scalars(poisson_ctx &c, hipStream_t s)
{
    IBM_HIP(hipMemcpyAsync(c.hsc, c.sc.p, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    prof_harvest(c);
}

__global__ void k_replace_fin(const double *part, int pstride, int n, double *sc)
{
    double s0 = block_sum_all(part, n);
    double s1 = block_sum_all(part + pstride, n);
    if (threadIdx.x) return;
    // residual replacement: rho = (rh, r_true), beta from the previous rho
    sc[S_RHO] = s0;
    sc[S_RR] = s1;
    sc[S_REL] = sqrt(s1 / sc[S_BN2]);
    const double om = sc[S_OMEGA], ro = sc[S_RHO_OLD];
    sc[S_BETA] = (om != 0.0 && ro != 0.0) ? (s0 / ro) * (sc[S_ALPHA] / om) : 0.0;
}

template <class T>
__global__ void __launch_bounds__(TPB) k_dot2(Walk W, const T *a, const T *b, double *part, int pstride)
{
    Acc<2> acc;
    acc.v[0] = acc.v[1] = 0.0;
    WALK_BEGIN(W, p)
        const double bv = ld(b, p);
        acc.v[0] += ld(a, p) * bv;
        acc.v[1] += bv * bv;
    WALK_END
    block_reduce<2>(acc, part, pstride, blockIdx.x);
}

// Right-preconditioned BiCGSTAB on A y = rhs (vectors of type T); y is the
// solution (zero start).  Returns iterations; status code in *rc.
template <class T>
int bicgstab(poisson_ctx &c, const T *rhs, T *y, T *r, T *rh, T *p, T *v, T *ph, T *sh, T *t, double tol, int maxit,
             bool true_check, hipGraphExec_t *graph, hipStream_t s, int *rc, double *relout)
{
    const Walk &W = c.W0;
    k_fill<T><<<W.nb, TPB, 0, s>>>(W, y, 0.0);
    k_fill<T><<<W.nb, TPB, 0, s>>>(W, p, 0.0);
    k_fill<T><<<W.nb, TPB, 0, s>>>(W, v, 0.0);
    k_copy_norm<T, T><<<W.nb, TPB, 0, s>>>(W, rhs, r, rh, c.part.p);
    IBM_LAUNCH_CHECK();
    fin(c, W.nb, FIN_INIT, 0, 0.0, s);
    read_scalars(c, s);
    *rc = IBM_ENOCONV;
    if (c.hsc[S_BN2] == 0.0) {
        *rc = IBM_OK;
        *relout = 0.0;
        return 0;
    }
    const bool use_graph = c.opts.use_graph && c.prof_kernel < 0;
    if (use_graph && !*graph) {
        hipGraph_t gr;
        c.capturing = true;
        IBM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        bicg_iteration<T, T>(c, y, r, rh, p, v, ph, sh, t, y, s);
        IBM_HIP(hipStreamEndCapture(s, &gr));
        c.capturing = false;
        IBM_HIP(hipGraphInstantiate(graph, gr, nullptr, nullptr, 0));
        IBM_HIP(hipGraphDestroy(gr));
    }
    int it = 0;
    double rel = 1.0;
    while (it < maxit) {
        ++it;
        if (use_graph) IBM_HIP(hipGraphLaunch(*graph, s));
        else bicg_iteration<T, T>(c, y, r, rh, p, v, ph, sh, t, y, s);
        read_scalars(c, s);
        const double st = c.hsc[S_STATUS];
        rel = c.hsc[S_REL];
        if (st >= 2.0 || !std::isfinite(rel)) { *rc = IBM_EBREAKDOWN; break; }
        if (rel <= tol) {
            if (!true_check) { *rc = IBM_OK; break; }
            // true residual in FP64 terms of this precision
            int np;
            launch_apply<T>(c, M_PINNED, true, 2, y, t, rhs, nullptr, rh, nullptr, s, &np);
            k_fin<<<1, 1024, 0, s>>>(c.part.p + PSTRIDE, PSTRIDE, np, FIN_SUM, S_TMP, 0.0, c.sc.p);
            read_scalars(c, s);
            double trel = std::sqrt(c.hsc[S_TMP] / c.hsc[S_BN2]);
            rel = trel;
            if (trel <= tol) { *rc = IBM_OK; break; }
            // residual replacement
            k_copy<T, T><<<W.nb, TPB, 0, s>>>(W, t, r);
            k_dot2<T><<<W.nb, TPB, 0, s>>>(W, rh, r, c.part.p, PSTRIDE);
            k_replace_fin<<<1, 1024, 0, s>>>(c.part.p, PSTRIDE, W.nb, c.sc.p);
            IBM_LAUNCH_CHECK();
            continue;
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

// ------------------------------------------------------------------ RHS, gauge
__global__ void __launch_bounds__(TPB) k_rhs(L0 L, Walk W, const double *f, const double *sc, int slot, double *b)
{
    const double mean = sc[slot];
    WALK_BEGIN(W, p)
        const uint8_t fl = L.flags[p];
        b[p] = (fl & (F_SOLID | F_PIN)) ? 0.0 : f[p] - mean;
    WALK_END
}

__global__ void __launch_bounds__(TPB) k_rhs_ghost(L0 L, const double *dlb, const double *g, double *b)
{
    for (int r = blockIdx.x * TPB + threadIdx.x; r < L.nrows; r += gridDim.x * TPB) {
        const long long u = r < L.ng ? (long long)L.rcell[r] : (long long)L.N + (r - L.ng);
        b[u] = g ? L.rsG[r] * dlb[r] * g[r] : 0.0;
    }
}

__global__ void __launch_bounds__(TPB) k_gauge(L0 L, Walk W, const double *x, const double *sc, int slot, double *out)
{
    const double mean = sc[slot];
    WALK_BEGIN(W, p)
        bool act = p >= L.N || active0(L.flags[p]);
        out[p] = act ? x[p] - mean : 0.0;
    WALK_END
}

template <class T>
__global__ void __launch_bounds__(TPB) k_shift(L0 L, Walk W, T *x)
{
    const double c = ld(x, L.pin);
    __syncthreads();
    WALK_BEGIN(W, p)
        if (p != L.pin && (p >= L.N || active0(L.flags[p]))) st(x, p, ld(x, p) - c);
    WALK_END
}

__global__ void k_shift_pin(L0 L, double *x) { x[L.pin] = 0.0; }

// unpinned residual at the pin (the inconsistency the pin absorbs)
__global__ void k_pinres(L0 L, const double *x, double *sc)
{
    if (threadIdx.x || blockIdx.x) return;
    int i, j, k;
    long long p = L.pin;
    decode((uint32_t)p, L.nx, L.ny, L.fx, L.fy, i, j, k);
    double s;
    sc[S_TMP] = row7(L, x, p, i, j, k, x[p], s);
}

}  // namespace

// ------------------------------------------------------------------ setup
size_t estimate_bytes(int nx, int ny, int nz, long long nrows, int precision)
{
    long long N = (long long)nx * ny * nz;
    long long Nt = N + nrows;
    size_t b = (size_t)N;                       // flags
    b += (size_t)nrows * (8 * 4 + 8 * 8 + 16 + 8 + 4 + 6 * 4);
    b += (size_t)Nt * 8 * (precision == IBM_PREC_MIXED ? 3 : 10);
    if (precision == IBM_PREC_MIXED) b += (size_t)Nt * 4 * 9;
    long long Nc = N;
    size_t coarse = 0;
    while (true) {
        Nc /= 8;
        if (Nc < 8) break;
        coarse += (size_t)Nc * (precision == IBM_PREC_MIXED ? (4 + 2 + 4 + 1) : (8 * 3 + 1));
    }
    b += coarse;
    b += (size_t)PSTRIDE * 4 * 8;
    return b;
}

poisson_ctx *setup(const ibm_grid *grid, const uint8_t *flags, const ibm_stencils *st, const poisson_opts *opts)
{
    IBM_REQUIRE(flags && st, IBM_EINVAL, "null argument");
    std::unique_ptr<poisson_ctx> c(new poisson_ctx());
    if (opts) c->opts = *opts; else poisson_default_opts(&c->opts);
    poisson_opts &o = c->opts;
    IBM_REQUIRE(o.tol > 0 && o.max_iter > 0 && o.nu1 >= 1 && o.nu2 >= 0 && o.coarse_sweeps >= 1, IBM_EINVAL,
                "bad solver options");
    c->mixed = o.precision == IBM_PREC_MIXED;
    c->g = read_grid(grid);
    for (int d = 0; d < 3; ++d) IBM_REQUIRE(c->g.n[d] == st->n[d], IBM_EINVAL, "stencil table of another grid");
    IBM_HIP(hipStreamCreateWithFlags(&c->cs, hipStreamNonBlocking));
    IBM_HIP(hipEventCreate(&c->e0));
    IBM_HIP(hipEventCreate(&c->e1));
    IBM_HIP(hipEventCreateWithFlags(&c->ej, hipEventDisableTiming));
    IBM_HIP(hipHostMalloc((void **)&c->hsc, S_COUNT * sizeof(double), hipHostMallocDefault));
    hipStream_t s = c->cs;
    const HostGrid &g = c->g;
    const long long N = (long long)g.n[0] * g.n[1] * g.n[2];
    c->N = N;
    c->ng = st->ng;
    c->nm = st->nm;
    c->nrows = st->ng + st->nm;
    c->n_fallback = st->nfallback;
    c->pin = st->pin;
    const long long Nt = N + c->nm;
    // level 0 copies
    c->flags.alloc(N);
    IBM_HIP(hipMemcpyAsync(c->flags.p, flags, N, hipMemcpyDeviceToDevice, s));
    std::vector<uint8_t> hf(N);
    IBM_HIP(hipMemcpyAsync(hf.data(), flags, N, hipMemcpyDeviceToHost, s));
    const long long R = std::max<long long>(c->nrows, 1);
    c->rcell.alloc(R); c->rcol.alloc(R * 8); c->rw.alloc(R * 8); c->rsG.alloc(R); c->rdlb.alloc(R);
    if (c->nrows) {
        IBM_HIP(hipMemcpyAsync(c->rcell.p, st->cell.p, c->nrows * 4, hipMemcpyDeviceToDevice, s));
        IBM_HIP(hipMemcpyAsync(c->rcol.p, st->col.p, c->nrows * 32, hipMemcpyDeviceToDevice, s));
        IBM_HIP(hipMemcpyAsync(c->rw.p, st->w.p, c->nrows * 64, hipMemcpyDeviceToDevice, s));
        IBM_HIP(hipMemcpyAsync(c->rsG.p, st->sG.p, c->nrows * 8, hipMemcpyDeviceToDevice, s));
        IBM_HIP(hipMemcpyAsync(c->rdlb.p, st->dlb.p, c->nrows * 8, hipMemcpyDeviceToDevice, s));
    }
    std::vector<int32_t> mcell(std::max<long long>(c->nm, 1));
    if (c->nm) IBM_HIP(hipMemcpyAsync(mcell.data(), st->cell.p + c->ng, c->nm * 4, hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    // levels
    int nl = 1;
    {
        int n[3] = {g.n[0], g.n[1], g.n[2]};
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
    // membrane rows: neighbour columns (-x,+x,-y,+y,-z,+z), ghost unknown across cut links
    {
        std::vector<int32_t> mc(std::max<long long>(c->nm, 1) * 6, -1);
        const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
        for (long long m = 0; m < c->nm; ++m) {
            long long p = mcell[m];
            int ci[3] = {(int)(p % nx), (int)((p / nx) % ny), (int)(p / ((long long)nx * ny))};
            long long strd[3] = {1, nx, (long long)nx * ny};
            int nn[3] = {nx, ny, nz};
            for (int d = 0; d < 3; ++d)
                for (int sg = 0; sg < 2; ++sg) {
                    int c2 = ci[d] + (sg ? 1 : -1);
                    if (c2 < 0 || c2 >= nn[d]) continue;
                    long long q = p + (sg ? strd[d] : -strd[d]);
                    long long lo = sg ? p : q;
                    long long col = q;
                    if (hf[lo] & (F_CUTX << d)) {
                        auto it = std::lower_bound(mcell.begin(), mcell.begin() + c->nm, (int32_t)q);
                        IBM_REQUIRE(it != mcell.begin() + c->nm && *it == q, IBM_EGEOM, "cut link without ghost");
                        col = N + (it - mcell.begin());
                    }
                    mc[6 * m + 2 * d + sg] = (int32_t)col;
                }
        }
        upload(c->mcol, mc, s);
    }
    // fluid volume, pin volume
    {
        Level &L = c->lv[0];
        double sv = 0.0;
        for (int k = 0; k < g.n[2]; ++k)
            for (int j = 0; j < g.n[1]; ++j)
                for (int i = 0; i < g.n[0]; ++i) {
                    long long p = i + (long long)g.n[0] * (j + (long long)g.n[1] * k);
                    if (!(hf[p] & F_SOLID)) sv += L.hw[0][i] * L.hw[1][j] * L.hw[2][k];
                }
        c->vol_fluid = sv;
        long long p = c->pin;
        int i = (int)(p % g.n[0]), j = (int)((p / g.n[0]) % g.n[1]), k = (int)(p / ((long long)g.n[0] * g.n[1]));
        c->vol_pin = L.hw[0][i] * L.hw[1][j] * L.hw[2][k];
    }
    // coarse masks (host, setup only): active, cut, open
    for (int l = 1; l < nl; ++l) {
        Level &F = c->lv[l - 1], &C = c->lv[l];
        C.hm.assign(C.N, 0);
        const int fnx = F.n[0], fny = F.n[1];
        for (int K = 0; K < C.n[2]; ++K)
            for (int J = 0; J < C.n[1]; ++J)
                for (int I = 0; I < C.n[0]; ++I) {
                    uint8_t act = 0, cut = 0;
                    for (int q = 0; q < 8; ++q) {
                        int dx = q & 1, dy = (q >> 1) & 1, dz = (q >> 2) & 1;
                        long long p = (2 * I + dx) + (long long)fnx * ((2 * J + dy) + (long long)fny * (2 * K + dz));
                        uint8_t a, cb;
                        if (l == 1) {
                            uint8_t f = hf[p];
                            a = (!(f & F_SOLID) || (f & F_GHOST)) ? 1 : 0;
                            cb = (f >> 4) & 7;
                        } else {
                            a = F.hm[p] & 1;
                            cb = (F.hm[p] >> 4) & 7;
                        }
                        act |= a;
                        if (dx && (cb & 1)) cut |= 16;
                        if (dy && (cb & 2)) cut |= 32;
                        if (dz && (cb & 4)) cut |= 64;
                    }
                    C.hm[I + (long long)C.n[0] * (J + (long long)C.n[1] * K)] = act | cut;
                }
        double va = 0.0;
        for (int K = 0; K < C.n[2]; ++K)
            for (int J = 0; J < C.n[1]; ++J)
                for (int I = 0; I < C.n[0]; ++I) {
                    long long P = I + (long long)C.n[0] * (J + (long long)C.n[1] * K);
                    if (!(C.hm[P] & 1)) continue;
                    va += C.hw[0][I] * C.hw[1][J] * C.hw[2][K];
                    long long strd[3] = {1, C.n[0], (long long)C.n[0] * C.n[1]};
                    int ci[3] = {I, J, K};
                    for (int d = 0; d < 3; ++d)
                        if (ci[d] + 1 < C.n[d] && (C.hm[P + strd[d]] & 1) && !(C.hm[P] & (16 << d)))
                            C.hm[P] |= (uint8_t)(2 << d);
                }
        C.volA = va;
        upload(C.m, C.hm, s);
        // transfer maps of F from C
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
    // device views
    for (int l = 0; l < nl; ++l) {
        Level &L = c->lv[l];
        LC &v = L.lc;
        v.nx = L.n[0]; v.ny = L.n[1]; v.nz = L.n[2];
        v.N = (uint32_t)L.N;
        v.nxy = (uint32_t)((long long)L.n[0] * L.n[1]);
        v.fx = make_fdiv(L.n[0]);
        v.fy = make_fdiv(L.n[1]);
        for (int d = 0; d < 3; ++d) { v.cp[d] = L.cp[d].p; v.cm[d] = L.cm[d].p; v.w[d] = L.w[d].p; }
        v.m = L.m.p;
        for (int d = 0; d < 3; ++d) { L.pm.pi[d] = L.pi[d].p; L.pm.pt[d] = L.pt[d].p; }
        if (l > 0) {
            if (c->mixed) { L.x32.alloc(L.N); L.r32.alloc(L.N); L.b16.alloc(L.N); }
            else { L.x64.alloc(L.N); L.r64.alloc(L.N); L.b64.alloc(L.N); }
        }
    }
    L0 &z = c->l0;
    z.nx = g.n[0]; z.ny = g.n[1]; z.nz = g.n[2];
    z.N = (uint32_t)N;
    z.nxy = (uint32_t)((long long)g.n[0] * g.n[1]);
    z.fx = make_fdiv(g.n[0]);
    z.fy = make_fdiv(g.n[1]);
    for (int d = 0; d < 3; ++d) { z.cp[d] = c->lv[0].cp[d].p; z.cm[d] = c->lv[0].cm[d].p; z.w[d] = c->lv[0].w[d].p; }
    z.flags = c->flags.p;
    z.pin = (uint32_t)c->pin;
    z.nrows = (int)c->nrows;
    z.ng = (int)c->ng;
    z.rcell = c->rcell.p; z.rcol = c->rcol.p; z.rw = c->rw.p; z.rsG = c->rsG.p;
    z.nm = (int)c->nm;
    z.mcell = c->rcell.p + c->ng;
    z.mcol = c->mcol.p;
    c->W0 = make_walk(Nt);
    c->Wc = make_walk(N);
    // vectors
    c->x.alloc(Nt); c->r.alloc(Nt); c->b.alloc(Nt);
    if (!c->mixed) {
        c->rh.alloc(Nt); c->p.alloc(Nt); c->v.alloc(Nt); c->ph.alloc(Nt); c->sh.alloc(Nt); c->t.alloc(Nt);
        c->r0.alloc(Nt);
    } else {
        c->fd.alloc(Nt); c->fr.alloc(Nt); c->frh.alloc(Nt); c->fp.alloc(Nt); c->fv.alloc(Nt);
        c->fph.alloc(Nt); c->fsh.alloc(Nt); c->ft.alloc(Nt); c->fr0.alloc(Nt);
    }
    c->gtmp.alloc(R);
    c->sc.alloc(S_COUNT);
    c->part.alloc((size_t)PSTRIDE * 4);
    std::vector<double> sc0(S_COUNT, 0.0);
    sc0[S_VPIN] = c->vol_pin;
    IBM_HIP(hipMemcpyAsync(c->sc.p, sc0.data(), S_COUNT * 8, hipMemcpyHostToDevice, s));
    IBM_HIP(hipStreamSynchronize(s));
    c->bytes = estimate_bytes(g.n[0], g.n[1], g.n[2], c->nrows, o.precision);
    for (auto &L : c->lv) { L.hm.clear(); L.hm.shrink_to_fit(); }
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

void assemble_rhs(poisson_ctx &c, const double *f, const double *gval, double *b, hipStream_t s)
{
    k_vsum_fluid<double><<<c.Wc.nb, TPB, 0, s>>>(c.l0, c.Wc, f, c.part.p);
    fin(c, c.Wc.nb, FIN_MEAN, S_TMP, c.vol_fluid, s);
    k_rhs<<<c.Wc.nb, TPB, 0, s>>>(c.l0, c.Wc, f, c.sc.p, S_TMP, b);
    if (c.nrows) k_rhs_ghost<<<sparse_blocks(c.nrows), TPB, 0, s>>>(c.l0, c.rdlb.p, gval, b);
    IBM_LAUNCH_CHECK();
}

// solve A x = b (assembled, in c.b) into c.x; returns status
int solve_core(poisson_ctx &c, poisson_stats *stats, hipStream_t s)
{
    const poisson_opts &o = c.opts;
    int rc = IBM_ENOCONV, its = 0, outer = 0;
    double rel = 1.0;
    if (!c.mixed) {
        its = bicgstab<double>(c, c.b.p, c.x.p, c.r.p, c.rh.p, c.p.p, c.v.p, c.ph.p, c.sh.p, c.t.p, o.tol, o.max_iter,
                               true, &c.g64, s, &rc, &rel);
    } else {
        // FP64 iterative refinement around FP32 inner solves
        const Walk &W = c.W0;
        k_fill<double><<<W.nb, TPB, 0, s>>>(W, c.x.p, 0.0);
        IBM_LAUNCH_CHECK();
        for (outer = 0; outer <= o.max_outer; ++outer) {
            // r64 = b - A x (pinned), ||r64||^2 and ||b||^2
            int np;
            launch_apply<double>(c, M_PINNED, true, 2, c.x.p, c.r.p, c.b.p, nullptr, c.b.p, nullptr, s, &np);
            k_fin<<<1, 1024, 0, s>>>(c.part.p + PSTRIDE, PSTRIDE, np, FIN_SUM, S_TMP, 0.0, c.sc.p);
            IBM_LAUNCH_CHECK();
            double bn2;
            {
                k_dot2<double><<<W.nb, TPB, 0, s>>>(W, c.b.p, c.b.p, c.part.p, PSTRIDE);
                k_fin<<<1, 1024, 0, s>>>(c.part.p, PSTRIDE, W.nb, FIN_SUM, S_TMP + 1, 0.0, c.sc.p);
                read_scalars(c, s);
                bn2 = c.hsc[S_TMP + 1];
            }
            if (bn2 == 0.0) { rc = IBM_OK; rel = 0.0; break; }
            rel = std::sqrt(c.hsc[S_TMP] / bn2);
            if (!std::isfinite(rel)) { rc = IBM_EBREAKDOWN; break; }
            if (rel <= o.tol) { rc = IBM_OK; break; }
            if (outer == o.max_outer) { rc = IBM_ENOCONV; break; }
            // inner FP32 solve of A d = r64 (the inner residual vector starts as r64)
            k_copy<double, float><<<W.nb, TPB, 0, s>>>(W, c.r.p, c.fr.p);
            IBM_LAUNCH_CHECK();
            int irc;
            double irel;
            its += bicgstab<float>(c, c.fr.p, c.fd.p, c.fr.p, c.frh.p, c.fp.p, c.fv.p, c.fph.p, c.fsh.p, c.ft.p,
                                   o.inner_tol, o.max_iter, false, &c.g32, s, &irc, &irel);
            if (irc == IBM_EBREAKDOWN) { rc = irc; break; }
            k_add<float><<<W.nb, TPB, 0, s>>>(W, c.x.p, c.fd.p);
            IBM_LAUNCH_CHECK();
        }
    }
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
    o->inner_tol = 1e-5;
    o->max_outer = 10;
    o->use_graph = 1;
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
    int rc = IBM_OK;
    int32_t g = guarded([&] {
        IBM_REQUIRE(c && f_dev && x_dev, IBM_EINVAL, "null argument");
        StreamJoin j(*c, (hipStream_t)stream);
        hipStream_t s = c->cs;
        IBM_HIP(hipEventRecord(c->e0, s));
        assemble_rhs(*c, f_dev, g_dev, c->b.p, s);
        rc = solve_core(*c, stats, s);
        // gauge: volume-weighted fluid mean removed from fluid, ghost and membrane-ghost values
        k_pinres<<<1, 64, 0, s>>>(c->l0, c->x.p, c->sc.p);
        k_vsum_fluid<double><<<c->Wc.nb, TPB, 0, s>>>(c->l0, c->Wc, c->x.p, c->part.p);
        fin(*c, c->Wc.nb, FIN_MEAN, S_TMP + 1, c->vol_fluid, s);
        k_gauge<<<c->W0.nb, TPB, 0, s>>>(c->l0, c->W0, c->x.p, c->sc.p, S_TMP + 1, x_dev);
        IBM_LAUNCH_CHECK();
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
    return g;
}

extern "C" int32_t poisson_solve_assembled(poisson_ctx *c, const double *b_dev, double *x_dev, poisson_stats *stats,
                                           void *stream)
{
    return guarded([&] {
        IBM_REQUIRE(c && b_dev && x_dev, IBM_EINVAL, "null argument");
        StreamJoin j(*c, (hipStream_t)stream);
        hipStream_t s = c->cs;
        IBM_HIP(hipEventRecord(c->e0, s));
        k_copy<double, double><<<c->W0.nb, TPB, 0, s>>>(c->W0, b_dev, c->b.p);
        IBM_LAUNCH_CHECK();
        int rc = solve_core(*c, stats, s);
        k_copy<double, double><<<c->W0.nb, TPB, 0, s>>>(c->W0, c->x.p, x_dev);
        IBM_LAUNCH_CHECK();
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
        launch_apply<double>(*c, M_PINNED, false, 0, x_dev, y_dev, nullptr, nullptr, nullptr, nullptr, c->cs, nullptr);
    });
}

extern "C" int32_t poisson_assemble_rhs(poisson_ctx *c, const double *f_dev, const double *g_dev, double *b_dev,
                                        void *stream)
{
    return guarded([&] {
        IBM_REQUIRE(c && f_dev && b_dev, IBM_EINVAL, "null argument");
        StreamJoin j(*c, (hipStream_t)stream);
        assemble_rhs(*c, f_dev, g_dev, b_dev, c->cs);
    });
}

extern "C" int32_t poisson_precond(poisson_ctx *c, const double *b_dev, double *x_dev, void *stream)
{
    return guarded([&] {
        IBM_REQUIRE(c && b_dev && x_dev, IBM_EINVAL, "null argument");
        IBM_REQUIRE(!c->mixed, IBM_EINVAL, "poisson_precond needs an FP64 context");
        StreamJoin j(*c, (hipStream_t)stream);
        hipStream_t s = c->cs;
        k_vsum_active<double><<<c->Wc.nb, TPB, 0, s>>>(c->l0, c->Wc, b_dev, c->part.p);
        fin(*c, c->Wc.nb, FIN_SINK, S_SINKP, 0.0, s);
        vcycle<double>(*c, b_dev, x_dev, c->sc.p + S_SINKP, s);
        // shift: every active unknown minus the pin value, then the pin itself
        {
            Walk W = c->W0;
            k_shift<double><<<W.nb, TPB, 0, s>>>(c->l0, W, x_dev);
            k_shift_pin<<<1, 1, 0, s>>>(c->l0, x_dev);
        }
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

extern "C" void poisson_destroy(poisson_ctx *c)
{
    if (c) {
        (void)hipStreamSynchronize(c->cs);
        delete c;
    }
}
