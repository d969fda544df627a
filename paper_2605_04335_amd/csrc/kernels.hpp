// Device kernels of the PPE solve (templated on storage precision).
//
// Level 0 is the ghost-cell system: a matrix-free 7-point cell-centred
// operator for regular fluid cells (per-axis 1-D coefficient arrays, walls
// have zero flux), ELL rows for closed ghosts and membrane ghost unknowns
// (8 image-point weights, FP64 in every precision), membrane-adjacent fluid
// rows that see the neighbour's ghost unknown across a cut link, and the pin.
// Coarse levels are plain 7-point operators with per-cell open-face bits.
//
// All kernels walk cells with a 1-D, XCD-aware chunk map: the grid's blocks
// are dealt to the 8 XCDs round-robin, so block b serves XCD b%8 and each XCD
// marches through its own contiguous slab of the field, keeping the +-x, +-y
// and +-z neighbours of a cell in that XCD's L2.  Reductions are
// deterministic: wave64 shuffles, then LDS across the waves of a block, then
// per-block partials summed in a fixed order by one finalising block.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace ibm {

typedef __bf16 bf16;

template <class T>
__device__ __forceinline__ double ld(const T *a, long long i) { return (double)a[i]; }
template <class T>
__device__ __forceinline__ void st(T *a, long long i, double v) { a[i] = (T)v; }
template <>
__device__ __forceinline__ void st<bf16>(bf16 *a, long long i, double v) { a[i] = (bf16)(float)v; }
template <>
__device__ __forceinline__ double ld<bf16>(const bf16 *a, long long i) { return (double)(float)a[i]; }

// division by a runtime-invariant 32-bit divisor (round-up multiplier)
struct FDiv {
    uint32_t d, m, s;
};
inline FDiv make_fdiv(uint32_t d)
{
    FDiv f;
    f.d = d;
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    f.s = l;
    f.m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
    return f;
}
__device__ __forceinline__ uint32_t fdiv(uint32_t n, FDiv f)
{
    return (uint32_t)(((uint64_t)__umulhi(n, f.m) + n) >> f.s);
}

constexpr int TPB = 256;   // threads per block
constexpr int MAXB = 4096; // blocks per launch (multiple of 8)

// XCD-aware chunk walk over [0, n): chunk c covers [c*TPB, c*TPB + TPB)
struct Walk {
    long long n;       // elements
    long long chunks;  // ceil(n / TPB)
    long long per;     // chunks per XCD
    int nb;            // blocks (multiple of 8)
};
inline Walk make_walk(long long n)
{
    Walk w;
    w.n = n;
    w.chunks = (n + TPB - 1) / TPB;
    long long b = (w.chunks + 7) / 8 * 8;
    if (b > MAXB) b = MAXB;
    if (b < 8) b = 8;
    w.nb = (int)b;
    w.per = (w.chunks + 7) / 8;
    return w;
}
#define WALK_BEGIN(W, p)                                                                      \
    {                                                                                         \
        const long long xcd_ = blockIdx.x & 7, lane_blk_ = blockIdx.x >> 3;                   \
        const long long c0_ = xcd_ * (W).per, c1_ = min((W).chunks, c0_ + (W).per);           \
        for (long long c_ = c0_ + lane_blk_; c_ < c1_; c_ += ((W).nb >> 3)) {                 \
            const long long p = c_ * TPB + threadIdx.x;                                       \
            if (p >= (W).n) continue;
#define WALK_END \
    }            \
    }

// ---------------------------------------------------------------- reductions
template <int K>
struct Acc {
    double v[K];
};

// block sum of K values into part[slot*stride + blk] (fixed order)
template <int K>
__device__ __forceinline__ void block_reduce(Acc<K> a, double *part, int stride, int blk)
{
    __shared__ double sm[K][TPB / 64];
#pragma unroll
    for (int q = 0; q < K; ++q) {
        double v = a.v[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        a.v[q] = v;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < K; ++q) sm[q][wid] = a.v[q];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < K; ++q) {
            double s = 0.0;
            for (int w = 0; w < TPB / 64; ++w) s += sm[q][w];
            part[(long long)q * stride + blk] = s;
        }
}

// ---------------------------------------------------------------- level data
struct L0 {
    int nx, ny, nz;
    uint32_t N, nxy;
    FDiv fx, fy;
    const double *cp[3], *cm[3], *w[3];
    const uint8_t *flags;
    uint32_t pin;
    int nrows, ng;
    const int32_t *rcell, *rcol;
    const double *rw, *rsG;
    int nm;
    const int32_t *mcell, *mcol;
};

struct LC {
    int nx, ny, nz;
    uint32_t N, nxy;
    FDiv fx, fy;
    const double *cp[3], *cm[3], *w[3];
    const uint8_t *m;  // bit0 active, bits1-3 open +x/+y/+z
};

// transfer maps of a fine level from its coarse parent
struct PMap {
    const int *pi[3];
    const double *pt[3];
};

__device__ __forceinline__ void decode(uint32_t p, uint32_t nx, uint32_t ny, FDiv fx, FDiv fy, int &i, int &j, int &k)
{
    uint32_t q = fdiv(p, fx);
    i = (int)(p - q * nx);
    uint32_t r = fdiv(q, fy);
    j = (int)(q - r * ny);
    k = (int)r;
}

__device__ __forceinline__ bool active0(uint8_t f) { return !(f & F_SOLID) || (f & F_GHOST); }

// sum_c c (x_nb - xp) over the six faces of a regular level-0 cell, plus its diagonal s
template <class T>
__device__ __forceinline__ double row7(const L0 &L, const T *x, long long p, int i, int j, int k, double xp, double &s)
{
    double acc = 0.0;
    s = 0.0;
    if (i + 1 < L.nx) { double c = L.cp[0][i]; acc += c * (ld(x, p + 1) - xp); s += c; }
    if (i > 0) { double c = L.cm[0][i]; acc += c * (ld(x, p - 1) - xp); s += c; }
    if (j + 1 < L.ny) { double c = L.cp[1][j]; acc += c * (ld(x, p + L.nx) - xp); s += c; }
    if (j > 0) { double c = L.cm[1][j]; acc += c * (ld(x, p - L.nx) - xp); s += c; }
    if (k + 1 < L.nz) { double c = L.cp[2][k]; acc += c * (ld(x, p + L.nxy) - xp); s += c; }
    if (k > 0) { double c = L.cm[2][k]; acc += c * (ld(x, p - L.nxy) - xp); s += c; }
    return acc;
}

// the same for a membrane-adjacent cell whose cut links see ghost unknowns
template <class T>
__device__ __forceinline__ double rowm(const L0 &L, const T *x, int m, int i, int j, int k, double xp, double &s)
{
    const int32_t *mc = L.mcol + 6 * m;
    const double c[6] = {L.cm[0][i], L.cp[0][i], L.cm[1][j], L.cp[1][j], L.cm[2][k], L.cp[2][k]};
    double acc = 0.0;
    s = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        if (mc[q] >= 0) { acc += c[q] * (ld(x, mc[q]) - xp); s += c[q]; }
    return acc;
}

enum { M_PINNED = 0, M_PINZERO = 1, M_UNPINNED = 2 };

// ---------------------------------------------------------------- operator
// y = A x over regular cells (RES: y = b - A x with the pin sink); dots of y
// with u1, u2 and itself according to ND.
template <class T, int MODE, bool RES, int ND>
__global__ void __launch_bounds__(TPB) k0_apply(L0 L, Walk W, const T *x, T *y, const T *b, const double *sink,
                                                const T *u1, const T *u2, double *part, int pstride)
{
    Acc<3> a;
    a.v[0] = a.v[1] = a.v[2] = 0.0;
    WALK_BEGIN(W, p)
        const uint8_t f = L.flags[p];
        if (f & F_MGHOST) continue;
        double out;
        if (f & F_SOLID) {
            out = 0.0;
        } else {
            int i, j, k;
            decode((uint32_t)p, L.nx, L.ny, L.fx, L.fy, i, j, k);
            const double xp = ld(x, p);
            double s;
            double ax = row7(L, x, p, i, j, k, xp, s);
            if (p == L.pin && MODE == M_PINNED) ax = -s * xp;
            if (p == L.pin && MODE == M_PINZERO) ax = 0.0;
            if (RES) {
                double bb = ld(b, p);
                if (p == L.pin && sink) bb -= sink[0];
                out = bb - ax;
            } else {
                out = ax;
            }
        }
        st(y, p, out);
        const double yo = ld(y, p);
        if (ND >= 1) a.v[0] += ld(u1, p) * yo;
        if (ND >= 2) a.v[1] += (u2 ? ld(u2, p) : yo) * yo;
        if (ND >= 3) a.v[2] += yo * yo;
    WALK_END
    if constexpr (ND > 0) {
        Acc<ND> b;
#pragma unroll
        for (int q = 0; q < ND; ++q) b.v[q] = a.v[q];
        block_reduce<ND>(b, part, pstride, blockIdx.x);
    }
}

// ghost rows: y[u] = sG (sum w x[col] - x[u]); dots over these rows
template <class T, bool RES, int ND>
__global__ void __launch_bounds__(TPB) k0_ghost(L0 L, const T *x, T *y, const T *b, const T *u1, const T *u2,
                                                double *part, int pstride, int poff)
{
    Acc<3> a;
    a.v[0] = a.v[1] = a.v[2] = 0.0;
    for (int r = blockIdx.x * TPB + threadIdx.x; r < L.nrows; r += gridDim.x * TPB) {
        const long long u = r < L.ng ? (long long)L.rcell[r] : (long long)L.N + (r - L.ng);
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int32_t c = L.rcol[8 * r + m];
            if (c >= 0) acc += L.rw[8 * r + m] * ld(x, c);
        }
        double ax = L.rsG[r] * (acc - ld(x, u));
        double out = RES ? ld(b, u) - ax : ax;
        st(y, u, out);
        const double yo = ld(y, u);
        if (ND >= 1) a.v[0] += ld(u1, u) * yo;
        if (ND >= 2) a.v[1] += (u2 ? ld(u2, u) : yo) * yo;
        if (ND >= 3) a.v[2] += yo * yo;
    }
    if constexpr (ND > 0) {
        Acc<ND> b;
#pragma unroll
        for (int q = 0; q < ND; ++q) b.v[q] = a.v[q];
        block_reduce<ND>(b, part, pstride, poff + blockIdx.x);
    }
}

// membrane-adjacent fluid rows
template <class T, bool RES, int ND>
__global__ void __launch_bounds__(TPB) k0_mrow(L0 L, const T *x, T *y, const T *b, const T *u1, const T *u2,
                                               double *part, int pstride, int poff)
{
    Acc<3> a;
    a.v[0] = a.v[1] = a.v[2] = 0.0;
    for (int m = blockIdx.x * TPB + threadIdx.x; m < L.nm; m += gridDim.x * TPB) {
        const long long p = L.mcell[m];
        int i, j, k;
        decode((uint32_t)p, L.nx, L.ny, L.fx, L.fy, i, j, k);
        double s;
        double ax = rowm(L, x, m, i, j, k, ld(x, p), s);
        double out = RES ? ld(b, p) - ax : ax;
        st(y, p, out);
        const double yo = ld(y, p);
        if (ND >= 1) a.v[0] += ld(u1, p) * yo;
        if (ND >= 2) a.v[1] += (u2 ? ld(u2, p) : yo) * yo;
        if (ND >= 3) a.v[2] += yo * yo;
    }
    if constexpr (ND > 0) {
        Acc<ND> b;
#pragma unroll
        for (int q = 0; q < ND; ++q) b.v[q] = a.v[q];
        block_reduce<ND>(b, part, pstride, poff + blockIdx.x);
    }
}

// ---------------------------------------------------------------- level-0 smoother
// Gauss-Seidel half-sweep over regular cells of one colour ((i+j+k)&1 ==
// color).  ZERO: the iterate starts at zero, so every other cell is written 0.
template <class T, bool ZERO>
__global__ void __launch_bounds__(TPB) k0_sweep(L0 L, Walk W, T *x, const T *b, const double *sink, int color)
{
    WALK_BEGIN(W, p)
        int i, j, k;
        decode((uint32_t)p, L.nx, L.ny, L.fx, L.fy, i, j, k);
        const uint8_t f = L.flags[p];
        if ((((i + j + k) & 1) != color) || (f & (F_SOLID | F_MGHOST))) {
            if (ZERO) st(x, p, 0.0);
            continue;
        }
        double bb = ld(b, p);
        if (p == L.pin && sink) bb -= sink[0];
        double s;
        if (ZERO) {
            s = L.cp[0][i] + L.cm[0][i] + L.cp[1][j] + L.cm[1][j] + L.cp[2][k] + L.cm[2][k];
            st(x, p, -bb / s);
        } else {
            const double xp = ld(x, p);
            double r = row7(L, x, p, i, j, k, xp, s);
            st(x, p, (r + s * xp - bb) / s);
        }
    WALK_END
}

template <class T>
__global__ void __launch_bounds__(TPB) k0_msweep(L0 L, T *x, const T *b, int color)
{
    for (int m = blockIdx.x * TPB + threadIdx.x; m < L.nm; m += gridDim.x * TPB) {
        const long long p = L.mcell[m];
        int i, j, k;
        decode((uint32_t)p, L.nx, L.ny, L.fx, L.fy, i, j, k);
        if (((i + j + k) & 1) != color) continue;
        const double xp = ld(x, p);
        double s;
        double r = rowm(L, x, m, i, j, k, xp, s);
        st(x, p, (r + s * xp - ld(b, p)) / s);
    }
}

// Jacobi on every ghost unknown: staged so all rows read the same iterate
template <class T>
__global__ void __launch_bounds__(TPB) k0_gjac(L0 L, const T *x, const T *b, double *tmp)
{
    for (int r = blockIdx.x * TPB + threadIdx.x; r < L.nrows; r += gridDim.x * TPB) {
        const long long u = r < L.ng ? (long long)L.rcell[r] : (long long)L.N + (r - L.ng);
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int32_t c = L.rcol[8 * r + m];
            if (c >= 0) acc += L.rw[8 * r + m] * ld(x, c);
        }
        tmp[r] = acc - ld(b, u) / L.rsG[r];
    }
}

template <class T>
__global__ void __launch_bounds__(TPB) k0_gscat(L0 L, T *x, const double *tmp)
{
    for (int r = blockIdx.x * TPB + threadIdx.x; r < L.nrows; r += gridDim.x * TPB) {
        const long long u = r < L.ng ? (long long)L.rcell[r] : (long long)L.N + (r - L.ng);
        st(x, u, tmp[r]);
    }
}

// ---------------------------------------------------------------- coarse levels
template <class T>
__device__ __forceinline__ double rowc(const LC &L, const T *x, long long p, int i, int j, int k, double &dg)
{
    const uint8_t mp = L.m[p];
    double acc = 0.0;
    dg = 0.0;
    if (mp & 2) { double c = L.cp[0][i]; acc += c * ld(x, p + 1); dg += c; }
    if (i > 0 && (L.m[p - 1] & 2)) { double c = L.cm[0][i]; acc += c * ld(x, p - 1); dg += c; }
    if (mp & 4) { double c = L.cp[1][j]; acc += c * ld(x, p + L.nx); dg += c; }
    if (j > 0 && (L.m[p - L.nx] & 4)) { double c = L.cm[1][j]; acc += c * ld(x, p - L.nx); dg += c; }
    if (mp & 8) { double c = L.cp[2][k]; acc += c * ld(x, p + L.nxy); dg += c; }
    if (k > 0 && (L.m[p - L.nxy] & 8)) { double c = L.cm[2][k]; acc += c * ld(x, p - L.nxy); dg += c; }
    return acc;
}

template <class T, class TB, bool ZERO>
__global__ void __launch_bounds__(TPB) kc_sweep(LC L, Walk W, T *x, const TB *b, const double *mean, int color)
{
    const double mu = mean[0];
    WALK_BEGIN(W, p)
        int i, j, k;
        decode((uint32_t)p, L.nx, L.ny, L.fx, L.fy, i, j, k);
        const uint8_t mp = L.m[p];
        if ((((i + j + k) & 1) != color) || !(mp & 1)) {
            if (ZERO) st(x, p, 0.0);
            continue;
        }
        double dg;
        double off = ZERO ? 0.0 : rowc(L, x, p, i, j, k, dg);
        if (ZERO) {
            dg = 0.0;
            if (mp & 2) dg += L.cp[0][i];
            if (i > 0 && (L.m[p - 1] & 2)) dg += L.cm[0][i];
            if (mp & 4) dg += L.cp[1][j];
            if (j > 0 && (L.m[p - L.nx] & 4)) dg += L.cm[1][j];
            if (mp & 8) dg += L.cp[2][k];
            if (k > 0 && (L.m[p - L.nxy] & 8)) dg += L.cm[2][k];
        }
        const double bb = ld(b, p) - mu;
        st(x, p, dg > 0.0 ? (off - bb) / dg : 0.0);
    WALK_END
}

template <class T, class TB, class TR>
__global__ void __launch_bounds__(TPB) kc_resid(LC L, Walk W, const T *x, const TB *b, const double *mean, TR *r)
{
    const double mu = mean[0];
    WALK_BEGIN(W, p)
        int i, j, k;
        decode((uint32_t)p, L.nx, L.ny, L.fx, L.fy, i, j, k);
        if (!(L.m[p] & 1)) { st(r, p, 0.0); continue; }
        double dg;
        double off = rowc(L, x, p, i, j, k, dg);
        st(r, p, ld(b, p) - mu - (off - dg * ld(x, p)));
    WALK_END
}

// restriction: coarse RHS = volume-weighted mean of the active children's
// residuals; partial sums of V_C * b_C for the coarse mean projection.
template <class TR, class TBc, bool FINE0>
__global__ void __launch_bounds__(TPB) k_restrict(L0 F0, LC F, LC C, Walk W, const TR *r, TBc *bc, double *part)
{
    Acc<1> a;
    a.v[0] = 0.0;
    const int fnx = FINE0 ? F0.nx : F.nx;
    const uint32_t fnxy = FINE0 ? F0.nxy : F.nxy;
    const double *const *fw = FINE0 ? F0.w : F.w;
    WALK_BEGIN(W, P)
        int I, J, K;
        decode((uint32_t)P, C.nx, C.ny, C.fx, C.fy, I, J, K);
        double sv = 0.0, svr = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int i = 2 * I + (c & 1), j = 2 * J + ((c >> 1) & 1), k = 2 * K + ((c >> 2) & 1);
            const long long p = (long long)i + (long long)fnx * j + (long long)fnxy * k;
            const bool act = FINE0 ? active0(F0.flags[p]) : (F.m[p] & 1);
            if (!act) continue;
            const double V = fw[0][i] * fw[1][j] * fw[2][k];
            sv += V;
            svr += V * ld(r, p);
        }
        const double v = sv > 0.0 ? svr / sv : 0.0;
        st(bc, P, v);
        if (C.m[P] & 1) a.v[0] += C.w[0][I] * C.w[1][J] * C.w[2][K] * ld(bc, P);
    WALK_END
    block_reduce<1>(a, part, 0, blockIdx.x);
}

// prolongation: trilinear in physical coordinates from the coarse parent,
// added to the active cells of the fine level
template <class Tc, class Tf, bool FINE0>
__global__ void __launch_bounds__(TPB) k_prolong(L0 F0, LC F, LC C, PMap M, Walk W, const Tc *xc, Tf *xf)
{
    const int fnx = FINE0 ? F0.nx : F.nx, fny = FINE0 ? F0.ny : F.ny;
    const FDiv ffx = FINE0 ? F0.fx : F.fx, ffy = FINE0 ? F0.fy : F.fy;
    WALK_BEGIN(W, p)
        const bool act = FINE0 ? active0(F0.flags[p]) : (F.m[p] & 1);
        if (!act) continue;
        int i, j, k;
        decode((uint32_t)p, fnx, fny, ffx, ffy, i, j, k);
        const int I = M.pi[0][i], J = M.pi[1][j], K = M.pi[2][k];
        const double tx = M.pt[0][i], ty = M.pt[1][j], tz = M.pt[2][k];
        const long long q = (long long)I + (long long)C.nx * J + (long long)C.nxy * K;
        const double v = (1 - tz) * ((1 - ty) * ((1 - tx) * ld(xc, q) + tx * ld(xc, q + 1)) +
                                     ty * ((1 - tx) * ld(xc, q + C.nx) + tx * ld(xc, q + C.nx + 1))) +
                         tz * ((1 - ty) * ((1 - tx) * ld(xc, q + C.nxy) + tx * ld(xc, q + C.nxy + 1)) +
                               ty * ((1 - tx) * ld(xc, q + C.nxy + C.nx) + tx * ld(xc, q + C.nxy + C.nx + 1)));
        st(xf, p, ld(xf, p) + v);
    WALK_END
}

// ---------------------------------------------------------------- Krylov vector kernels
// scalar slots on the device
enum {
    S_RHO = 0, S_RHO_OLD, S_ALPHA, S_OMEGA, S_BETA, S_RR, S_BN2, S_REL, S_SINKP, S_SINKS,
    S_RV, S_TS, S_TT, S_STATUS, S_VPIN, S_TMP, S_MEAN0 = 16, S_COUNT = 40
};

__device__ __forceinline__ double cell_volume(const L0 &L, long long p)
{
    int i, j, k;
    decode((uint32_t)p, L.nx, L.ny, L.fx, L.fy, i, j, k);
    return L.w[0][i] * L.w[1][j] * L.w[2][k];
}

// p = r + beta (p - omega v); partial sum of V p over the active cells (sink)
template <class T>
__global__ void __launch_bounds__(TPB) k_p_update(L0 L, Walk W, const T *r, T *pv, const T *v, const double *sc,
                                                  double *part)
{
    const double beta = sc[S_BETA], omega = sc[S_OMEGA];
    Acc<1> a;
    a.v[0] = 0.0;
    WALK_BEGIN(W, p)
        st(pv, p, ld(r, p) + beta * (ld(pv, p) - omega * ld(v, p)));
        if (p < L.N && active0(L.flags[p])) a.v[0] += cell_volume(L, p) * ld(pv, p);
    WALK_END
    block_reduce<1>(a, part, 0, blockIdx.x);
}

// r <- s = r - alpha v; partial sum of V s (sink of the second V-cycle)
template <class T>
__global__ void __launch_bounds__(TPB) k_s_update(L0 L, Walk W, T *r, const T *v, const double *sc, double *part)
{
    const double alpha = sc[S_ALPHA];
    Acc<1> a;
    a.v[0] = 0.0;
    WALK_BEGIN(W, p)
        st(r, p, ld(r, p) - alpha * ld(v, p));
        if (p < L.N && active0(L.flags[p])) a.v[0] += cell_volume(L, p) * ld(r, p);
    WALK_END
    block_reduce<1>(a, part, 0, blockIdx.x);
}

// x += alpha (ph - ph_pin) + omega (sh - sh_pin) on active unknowns (the
// preconditioner's shift to the pinned subspace, applied here instead of in
// an extra pass); r = s - omega t; partials of (rh, r) and (r, r)
template <class T, class TX>
__global__ void __launch_bounds__(TPB) k_xr_update(L0 L, Walk W, TX *x, const T *ph, const T *sh, T *r, const T *t,
                                                   const T *rh, const double *sc, double *part, int pstride)
{
    const double alpha = sc[S_ALPHA], omega = sc[S_OMEGA];
    const double cp = ld(ph, L.pin), cs = ld(sh, L.pin);
    Acc<2> a;
    a.v[0] = a.v[1] = 0.0;
    WALK_BEGIN(W, p)
        const bool act = p >= L.N || active0(L.flags[p]);
        if (act) st(x, p, ld(x, p) + alpha * (ld(ph, p) - cp) + omega * (ld(sh, p) - cs));
        st(r, p, ld(r, p) - omega * ld(t, p));
        const double rv = ld(r, p);
        a.v[0] += ld(rh, p) * rv;
        a.v[1] += rv * rv;
    WALK_END
    block_reduce<2>(a, part, pstride, blockIdx.x);
}

// generic helpers
template <class T>
__global__ void __launch_bounds__(TPB) k_fill(Walk W, T *a, double v)
{
    WALK_BEGIN(W, p)
        st(a, p, v);
    WALK_END
}

template <class TA, class TB>
__global__ void __launch_bounds__(TPB) k_copy(Walk W, const TA *a, TB *b)
{
    WALK_BEGIN(W, p)
        st(b, p, ld(a, p));
    WALK_END
}

// b = a (converted), partials of (a, a)
template <class TA, class TB>
__global__ void __launch_bounds__(TPB) k_copy_norm(Walk W, const TA *a, TB *b, TB *b2, double *part)
{
    Acc<1> s;
    s.v[0] = 0.0;
    WALK_BEGIN(W, p)
        st(b, p, ld(a, p));
        if (b2) st(b2, p, ld(a, p));
        const double v = ld(b, p);
        s.v[0] += v * v;
    WALK_END
    block_reduce<1>(s, part, 0, blockIdx.x);
}

// x64 += d (pinned subspace already), used by the mixed outer refinement
template <class T>
__global__ void __launch_bounds__(TPB) k_add(Walk W, double *x, const T *d)
{
    WALK_BEGIN(W, p)
        x[p] += ld(d, p);
    WALK_END
}

// volume-weighted sum of a over fluid cells (gauge, RHS projection)
template <class T>
__global__ void __launch_bounds__(TPB) k_vsum_fluid(L0 L, Walk W, const T *a, double *part)
{
    Acc<1> s;
    s.v[0] = 0.0;
    WALK_BEGIN(W, p)
        if (!(L.flags[p] & F_SOLID)) s.v[0] += cell_volume(L, p) * ld(a, p);
    WALK_END
    block_reduce<1>(s, part, 0, blockIdx.x);
}

// volume-weighted sum over the active cells (the preconditioner's sink)
template <class T>
__global__ void __launch_bounds__(TPB) k_vsum_active(L0 L, Walk W, const T *a, double *part)
{
    Acc<1> s;
    s.v[0] = 0.0;
    WALK_BEGIN(W, p)
        if (active0(L.flags[p])) s.v[0] += cell_volume(L, p) * ld(a, p);
    WALK_END
    block_reduce<1>(s, part, 0, blockIdx.x);
}

// ---------------------------------------------------------------- finalisers (one block)
__device__ double block_sum_all(const double *part, int n)
{
    __shared__ double sm[1024];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
        __syncthreads();
    }
    double r = sm[0];
    __syncthreads();
    return r;
}

enum { FIN_SUM = 0, FIN_SINK, FIN_ALPHA, FIN_OMEGA, FIN_RHO, FIN_MEAN, FIN_INIT, FIN_RESTART };

// op: FIN_SUM sc[dst] = sum slot0; FIN_SINK sc[dst] = sum/V_pin; FIN_ALPHA;
// FIN_OMEGA (slots ts, tt); FIN_RHO (slots rhonew, rr); FIN_MEAN sc[dst] =
// sum/aux; FIN_INIT (slot rr: rho = rr = bn2); FIN_RESTART (rho = rr).
__global__ void __launch_bounds__(1024) k_fin(const double *part, int pstride, int n, int op, int dst, double aux,
                                              double *sc)
{
    double s0 = block_sum_all(part, n);
    double s1 = (op == FIN_OMEGA || op == FIN_RHO) ? block_sum_all(part + pstride, n) : 0.0;
    if (threadIdx.x != 0) return;
    switch (op) {
    case FIN_SUM: sc[dst] = s0; break;
    case FIN_SINK: sc[dst] = s0 / sc[S_VPIN]; break;
    case FIN_MEAN: sc[dst] = aux > 0.0 ? s0 / aux : 0.0; break;
    case FIN_ALPHA: {
        sc[S_RV] = s0;
        if (s0 == 0.0 || !isfinite(s0)) { sc[S_STATUS] = 2.0; sc[S_ALPHA] = 0.0; }
        else sc[S_ALPHA] = sc[S_RHO] / s0;
        break;
    }
    case FIN_OMEGA: {
        sc[S_TS] = s0; sc[S_TT] = s1;
        sc[S_OMEGA] = s1 > 0.0 ? s0 / s1 : 0.0;
        if (!(s1 > 0.0)) sc[S_STATUS] = 3.0;
        break;
    }
    case FIN_RHO: {
        const double rho = sc[S_RHO], rhon = s0;
        sc[S_RR] = s1;
        sc[S_REL] = sqrt(s1 / sc[S_BN2]);
        sc[S_RHO_OLD] = rho;
        sc[S_RHO] = rhon;
        const double om = sc[S_OMEGA];
        sc[S_BETA] = (om != 0.0 && rho != 0.0) ? (rhon / rho) * (sc[S_ALPHA] / om) : 0.0;
        if (!isfinite(s1)) sc[S_STATUS] = 4.0;
        else if (fabs(rhon) < 1e-300 * sc[S_BN2]) sc[S_STATUS] = 1.0;  // restart wanted
        break;
    }
    case FIN_INIT: {
        sc[S_BN2] = s0; sc[S_RR] = s0; sc[S_RHO] = s0; sc[S_RHO_OLD] = 1.0;
        sc[S_ALPHA] = 1.0; sc[S_OMEGA] = 1.0; sc[S_BETA] = 0.0;
        sc[S_REL] = s0 > 0.0 ? 1.0 : 0.0; sc[S_STATUS] = 0.0;
        break;
    }
    case FIN_RESTART: {
        sc[S_RR] = s0; sc[S_RHO] = s0; sc[S_BETA] = 0.0; sc[S_STATUS] = 0.0;
        sc[S_REL] = sqrt(s0 / sc[S_BN2]);
        break;
    }
    }
}

}  // namespace ibm
