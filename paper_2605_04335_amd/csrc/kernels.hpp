// Device kernels of the PPE solve (templated on storage precision).
//
// Storage: every solver vector lives in a red/black split layout.  Cell
// (i,j,k) has colour c = (i+j+k)&1 and half-index h = i>>1; its slot is
// c*Nh + h + H*(j + ny*k) with H = ceil(nx/2), Nh = H*ny*nz (when nx is odd
// one slot per row is padding, flagged inactive).  A red/black half-sweep
// then reads exactly the other colour's array plus its own right-hand side
// and writes its own colour, with unit-stride rows: no cache line carries
// values the kernel does not use.  The y, z neighbours of a slot sit at the
// same (h) in the other colour's neighbouring rows; the x neighbours at h+p
// and h+p-1 with p = (c+j+k)&1; the 8 children of a coarse cell (I,J,K) all
// sit at h = I.  Membrane ghost unknowns follow the 2*Nh cell slots.
//
// Level 0 is the ghost-cell system: a matrix-free 7-point cell-centred
// operator for regular fluid cells (per-axis 1-D coefficient arrays; walls
// have zero flux), ELL rows for closed ghosts and membrane ghost unknowns
// (8 image-point weights, FP64 in every precision), membrane-adjacent fluid
// rows that see the neighbour's ghost unknown across a cut link, and the pin.
// Coarse levels are plain 7-point operators with per-cell open-face bits.
//
// Launches are 1-D grids remapped so that the blocks of each XCD (blocks are
// dealt to the 8 XCDs round-robin) cover one contiguous z-slab, keeping the
// y and z neighbours of a slot in that XCD's L2.  Reductions are
// deterministic: wave64 shuffles, LDS across the waves of a block, per-block
// partials summed in a fixed order by one finalising block.
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

constexpr int TPB = 256;    // threads per block
constexpr int MAXB = 4096;  // blocks of an element-wise launch (multiple of 8)

// ---------------------------------------------------------------- element-wise walk
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

// ---------------------------------------------------------------- 3-D stencil launch
// block = 64 x 4 threads over (h, j); each thread walks kz planes in k.
struct Geo {
    int gx, gy, gz;  // tiles in h, j, k
    int kz;          // planes per tile
    int nb;          // launched blocks (multiple of 8, >= gx*gy*gz)
    int H, ny, nz;
};
inline Geo make_geo(int H, int ny, int nz)
{
    Geo g;
    g.H = H; g.ny = ny; g.nz = nz;
    g.gx = (H + 63) / 64;
    g.gy = (ny + 3) / 4;
    long long xy = (long long)g.gx * g.gy;
    int kz = 1;
    while (xy * ((nz + kz - 1) / kz) > 8192 && kz < nz) kz *= 2;
    g.kz = kz;
    g.gz = (nz + kz - 1) / kz;
    long long n = xy * g.gz;
    g.nb = (int)((n + 7) / 8 * 8);
    return g;
}
// Tile of this block (XCD-contiguous remap); false for padding blocks.
__device__ __forceinline__ bool geo_tile(const Geo &G, int &h, int &j, int &k0, int &k1)
{
    const int b = blockIdx.x;
    const int L = (b & 7) * (G.nb >> 3) + (b >> 3);
    const int bx = L % G.gx;
    const int r = L / G.gx;
    const int by = r % G.gy;
    const int bz = r / G.gy;
    if (bz >= G.gz) return false;
    h = bx * 64 + (threadIdx.x & 63);
    j = by * 4 + (threadIdx.x >> 6);
    k0 = bz * G.kz;
    k1 = min(G.nz, k0 + G.kz);
    return h < G.H && j < G.ny;
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
    __syncthreads();
}

// ---------------------------------------------------------------- levels
struct Lv {
    int nx, ny, nz, H;
    long long Nh;                       // slots per colour
    FDiv fH, fy;                        // for slot decoding
    const double *cp[3], *cm[3], *w[3];
    const uint8_t *f;                   // per slot: level 0 flags (padding = SOLID); coarse: bit0 active, bits1-3 open
};

__device__ __forceinline__ long long slot(const Lv &L, int c, int h, int j, int k)
{
    return (long long)c * L.Nh + h + (long long)L.H * (j + (long long)L.ny * k);
}

// decode a slot index (< 2 Nh) into colour, h, j, k and the cell's i
__device__ __forceinline__ void decode_slot(const Lv &L, long long s, int &c, int &h, int &j, int &k, int &i)
{
    c = s >= L.Nh ? 1 : 0;
    uint32_t q = (uint32_t)(s - (c ? L.Nh : 0));
    uint32_t row = fdiv(q, L.fH);
    h = (int)(q - row * (uint32_t)L.H);
    uint32_t kk = fdiv(row, L.fy);
    j = (int)(row - kk * (uint32_t)L.ny);
    k = (int)kk;
    i = 2 * h + ((c + j + k) & 1);
}

__device__ __forceinline__ bool active0(uint8_t f) { return !(f & F_SOLID) || (f & F_GHOST); }

// Sum over the open faces of coefficient * neighbour value, and the diagonal.
// xo is the other colour's array (base of that colour).  FINE: the faces of a
// regular level-0 cell are open inside the domain; coarse: open-face bits.
template <bool FINE, class T>
__device__ __forceinline__ double nbsum(const Lv &L, const T *xo, const uint8_t *fo, int h, int j, int k, int i,
                                        uint8_t fm, double &dg)
{
    const int p = i & 1;  // (c + j + k) & 1
    const long long row = (long long)L.H * (j + (long long)L.ny * k);
    double acc = 0.0, d = 0.0;
    if (FINE) {
        if (i + 1 < L.nx) { double c = L.cp[0][i]; acc += c * ld(xo, row + h + p); d += c; }
        if (i > 0) { double c = L.cm[0][i]; acc += c * ld(xo, row + h + p - 1); d += c; }
        if (j + 1 < L.ny) { double c = L.cp[1][j]; acc += c * ld(xo, row + h + L.H); d += c; }
        if (j > 0) { double c = L.cm[1][j]; acc += c * ld(xo, row + h - L.H); d += c; }
        const long long pl = (long long)L.H * L.ny;
        if (k + 1 < L.nz) { double c = L.cp[2][k]; acc += c * ld(xo, row + h + pl); d += c; }
        if (k > 0) { double c = L.cm[2][k]; acc += c * ld(xo, row + h - pl); d += c; }
    } else {
        const long long pl = (long long)L.H * L.ny;
        if (fm & 2) { double c = L.cp[0][i]; acc += c * ld(xo, row + h + p); d += c; }
        if (i > 0 && (fo[row + h + p - 1] & 2)) { double c = L.cm[0][i]; acc += c * ld(xo, row + h + p - 1); d += c; }
        if (fm & 4) { double c = L.cp[1][j]; acc += c * ld(xo, row + h + L.H); d += c; }
        if (j > 0 && (fo[row + h - L.H] & 4)) { double c = L.cm[1][j]; acc += c * ld(xo, row + h - L.H); d += c; }
        if (fm & 8) { double c = L.cp[2][k]; acc += c * ld(xo, row + h + pl); d += c; }
        if (k > 0 && (fo[row + h - pl] & 8)) { double c = L.cm[2][k]; acc += c * ld(xo, row + h - pl); d += c; }
    }
    dg = d;
    return acc;
}

// the diagonal alone (no vector is read): sum of the open faces' coefficients
template <bool FINE>
__device__ __forceinline__ double diag_only(const Lv &L, const uint8_t *fo, int h, int j, int k, int i, uint8_t fm)
{
    const int p = i & 1;
    const long long row = (long long)L.H * (j + (long long)L.ny * k);
    const long long pl = (long long)L.H * L.ny;
    double d = 0.0;
    if (FINE) {
        if (i + 1 < L.nx) d += L.cp[0][i];
        if (i > 0) d += L.cm[0][i];
        if (j + 1 < L.ny) d += L.cp[1][j];
        if (j > 0) d += L.cm[1][j];
        if (k + 1 < L.nz) d += L.cp[2][k];
        if (k > 0) d += L.cm[2][k];
    } else {
        if (fm & 2) d += L.cp[0][i];
        if (i > 0 && (fo[row + h + p - 1] & 2)) d += L.cm[0][i];
        if (fm & 4) d += L.cp[1][j];
        if (j > 0 && (fo[row + h - L.H] & 4)) d += L.cm[1][j];
        if (fm & 8) d += L.cp[2][k];
        if (k > 0 && (fo[row + h - pl] & 8)) d += L.cm[2][k];
    }
    return d;
}

// sparse level-0 rows (ghosts, membrane-adjacent cells, pin)
struct Sp {
    long long N2;          // 2 Nh: first membrane ghost unknown
    long long pin;         // pin slot
    int nrows, ng;         // ghost rows: ng closed (slot) then membrane unknowns (N2 + m)
    const int32_t *rslot;  // [ng] slots of the closed ghosts (membrane rows: unknown N2 + r - ng)
    const int32_t *rcol;   // [nrows*8] slot / unknown columns
    const double *rw, *rsG;
    int nm;
    const int32_t *mslot;  // [nm] slots of the membrane-adjacent cells
    const int32_t *mcol;   // [nm*6] -x,+x,-y,+y,-z,+z neighbour unknowns (-1: wall)
    const int32_t *mcolor; // [nm] colour of each membrane cell (0/1)
};

__device__ __forceinline__ long long ghost_unknown(const Sp &S, int r)
{
    return r < S.ng ? (long long)S.rslot[r] : S.N2 + (r - S.ng);
}

template <class T>
__device__ __forceinline__ double ghost_sum(const Sp &S, const T *x, int r)
{
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int32_t c = S.rcol[8 * r + m];
        if (c >= 0) acc += S.rw[8 * r + m] * ld(x, c);
    }
    return acc;
}

// fluid row of membrane cell m: sum c (x_nb - xp) and its diagonal
template <class T>
__device__ __forceinline__ double mrow(const Lv &L, const Sp &S, const T *x, int m, double xp, double &s)
{
    int c, h, j, k, i;
    decode_slot(L, S.mslot[m], c, h, j, k, i);
    const int32_t *mc = S.mcol + 6 * m;
    const double cf[6] = {L.cm[0][i], L.cp[0][i], L.cm[1][j], L.cp[1][j], L.cm[2][k], L.cp[2][k]};
    double acc = 0.0;
    s = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        if (mc[q] >= 0) { acc += cf[q] * (ld(x, mc[q]) - xp); s += cf[q]; }
    return acc;
}

enum { M_PINNED = 0, M_PINZERO = 1, M_UNPINNED = 2 };

// ---------------------------------------------------------------- level-0 operator
// y = A x on regular cells (RES: y = b - A x, with the sink at the pin);
// skips membrane cells; solid cells (incl. ghosts, padding) get 0.  Dots of
// y with u1 / u2 (u2 NULL: with y itself).
template <class T, int MODE, bool RES, int ND>
__global__ void __launch_bounds__(TPB) k0_apply(Lv L, Geo G, long long pin, const T *x, T *y, const T *b,
                                                const double *sink, const T *u1, const T *u2, double *part,
                                                int pstride)
{
    Acc<3> a;
    a.v[0] = a.v[1] = a.v[2] = 0.0;
    int h, j, k0, k1;
    if (geo_tile(G, h, j, k0, k1)) {
        for (int k = k0; k < k1; ++k)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const long long s = slot(L, c, h, j, k);
                const uint8_t f = L.f[s];
                if (f & F_MGHOST) continue;
                double out;
                if (f & F_SOLID) {
                    out = 0.0;
                } else {
                    const int i = 2 * h + ((c + j + k) & 1);
                    const double xp = ld(x, s);
                    double dg;
                    double ax = nbsum<true>(L, x + (1 - c) * L.Nh, L.f + (1 - c) * L.Nh, h, j, k, i, f, dg) - dg * xp;
                    if (s == pin && MODE == M_PINNED) ax = -dg * xp;
                    if (s == pin && MODE == M_PINZERO) ax = 0.0;
                    if (RES) {
                        double bb = ld(b, s);
                        if (s == pin && sink) bb -= sink[0];
                        out = bb - ax;
                    } else {
                        out = ax;
                    }
                }
                st(y, s, out);
                const double yo = ld(y, s);
                if (ND >= 1) a.v[0] += ld(u1, s) * yo;
                if (ND >= 2) a.v[1] += (u2 ? ld(u2, s) : yo) * yo;
                if (ND >= 3) a.v[2] += yo * yo;
            }
    }
    if constexpr (ND > 0) {
        Acc<ND> r;
#pragma unroll
        for (int q = 0; q < ND; ++q) r.v[q] = a.v[q];
        block_reduce<ND>(r, part, pstride, blockIdx.x);
    }
}

// ghost rows and membrane rows of the operator (one launch for both)
template <class T, bool RES, int ND>
__global__ void __launch_bounds__(TPB) k0_sparse(Lv L, Sp S, const T *x, T *y, const T *b, const T *u1,
                                                 const T *u2, double *part, int pstride, int poff)
{
    Acc<3> a;
    a.v[0] = a.v[1] = a.v[2] = 0.0;
    const int n = S.nrows + S.nm;
    for (int r = blockIdx.x * TPB + threadIdx.x; r < n; r += gridDim.x * TPB) {
        long long u;
        double ax;
        if (r < S.nrows) {
            u = ghost_unknown(S, r);
            ax = S.rsG[r] * (ghost_sum(S, x, r) - ld(x, u));
        } else {
            const int m = r - S.nrows;
            u = S.mslot[m];
            double s;
            ax = mrow(L, S, x, m, ld(x, u), s);
        }
        const double out = RES ? ld(b, u) - ax : ax;
        st(y, u, out);
        const double yo = ld(y, u);
        if (ND >= 1) a.v[0] += ld(u1, u) * yo;
        if (ND >= 2) a.v[1] += (u2 ? ld(u2, u) : yo) * yo;
        if (ND >= 3) a.v[2] += yo * yo;
    }
    if constexpr (ND > 0) {
        Acc<ND> rr;
#pragma unroll
        for (int q = 0; q < ND; ++q) rr.v[q] = a.v[q];
        block_reduce<ND>(rr, part, pstride, poff + blockIdx.x);
    }
}

// ---------------------------------------------------------------- smoother
// Gauss-Seidel half-sweep of colour c over the regular cells of a level.
// ZMODE 1: first red sweep from a zero iterate (neighbours are zero, every
// slot of the colour is written); ZMODE 2: first black sweep (reads the new
// red values, writes zeros to skipped slots).  bsh: FINE - the sink at the
// pin slot; coarse - the level mean subtracted from every active RHS.
template <bool FINE, class T, class TB, int ZMODE>
__global__ void __launch_bounds__(TPB) k_sweep(Lv L, Geo G, long long pin, T *x, const TB *b, const double *bsh,
                                               int c, int zero_other = 0)
{
    int h, j, k0, k1;
    if (!geo_tile(G, h, j, k0, k1)) return;
    const double mu = (!FINE && bsh) ? bsh[0] : 0.0;
    T *xc = x + (long long)c * L.Nh;
    const T *xo = x + (long long)(1 - c) * L.Nh;
    const uint8_t *fc = L.f + (long long)c * L.Nh, *fo = L.f + (long long)(1 - c) * L.Nh;
    const TB *bc = b + (long long)c * L.Nh;
    for (int k = k0; k < k1; ++k) {
        const long long s = h + (long long)L.H * (j + (long long)L.ny * k);
        // from zero with membrane rows: the other colour must read as zero
        // before its own sweep (membrane rows of this colour read it)
        if (ZMODE == 1 && zero_other) st(x + (long long)(1 - c) * L.Nh, s, 0.0);
        const uint8_t f = fc[s];
        const int i = 2 * h + ((c + j + k) & 1);
        const bool skip = FINE ? (f & (F_SOLID | F_MGHOST)) != 0 : !(f & 1);
        if (skip || i >= L.nx) {
            if (ZMODE) st(xc, s, 0.0);
            continue;
        }
        double bb = ld(bc, s) - mu;
        if (FINE && bsh && s + (long long)c * L.Nh == pin) bb -= bsh[0];
        double dg, off;
        if (ZMODE == 1) {
            off = 0.0;
            dg = diag_only<FINE>(L, fo, h, j, k, i, f);
        } else {
            off = nbsum<FINE>(L, xo, fo, h, j, k, i, f, dg);
        }
        st(xc, s, dg > 0.0 ? (off - bb) / dg : 0.0);
    }
}

// membrane-adjacent cells of one colour (after the dense half-sweep): across
// a cut link the neighbour's ghost unknown is eliminated, i.e. replaced by
// the current value of its stencil, sum w x - b/sG
template <class T>
__global__ void __launch_bounds__(TPB) k0_msweep(Lv L, Sp S, T *x, const T *b, int color)
{
    for (int m = blockIdx.x * TPB + threadIdx.x; m < S.nm; m += gridDim.x * TPB) {
        if (S.mcolor[m] != color) continue;
        const long long u = S.mslot[m];
        int c, h, j, k, i;
        decode_slot(L, u, c, h, j, k, i);
        const int32_t *mc = S.mcol + 6 * m;
        const double cf[6] = {L.cm[0][i], L.cp[0][i], L.cm[1][j], L.cp[1][j], L.cm[2][k], L.cp[2][k]};
        double off = 0.0, s = 0.0;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int32_t col = mc[q];
            if (col < 0) continue;
            double v;
            if (col >= S.N2) {
                const int r = S.ng + (int)(col - S.N2);
                v = ghost_sum(S, x, r) - ld(b, col) / S.rsG[r];
            } else {
                v = ld(x, col);
            }
            off += cf[q] * v;
            s += cf[q];
        }
        st(x, u, (off - ld(b, u)) / s);
    }
}

// Jacobi on every ghost unknown, staged so that all rows read the same iterate
template <class T>
__global__ void __launch_bounds__(TPB) k0_gjac(Sp S, const T *x, const T *b, double *tmp)
{
    for (int r = blockIdx.x * TPB + threadIdx.x; r < S.nrows; r += gridDim.x * TPB)
        tmp[r] = ghost_sum(S, x, r) - ld(b, ghost_unknown(S, r)) / S.rsG[r];
}

template <class T>
__global__ void __launch_bounds__(TPB) k0_gscat(Sp S, T *x, const double *tmp)
{
    for (int r = blockIdx.x * TPB + threadIdx.x; r < S.nrows; r += gridDim.x * TPB) st(x, ghost_unknown(S, r), tmp[r]);
}

// residual of the sparse level-0 rows (unpinned; no row is the pin) into rsp
template <class T>
__global__ void __launch_bounds__(TPB) k0_sparse_res(Lv L, Sp S, const T *x, const T *b, T *rsp)
{
    const int n = S.nrows + S.nm;
    for (int r = blockIdx.x * TPB + threadIdx.x; r < n; r += gridDim.x * TPB) {
        if (r < S.nrows) {
            const long long u = ghost_unknown(S, r);
            if (u >= S.N2) continue;  // membrane ghost unknowns are not restricted
            st(rsp, u, ld(b, u) - S.rsG[r] * (ghost_sum(S, x, r) - ld(x, u)));
        } else {
            const int m = r - S.nrows;
            const long long u = S.mslot[m];
            double s;
            st(rsp, u, ld(b, u) - mrow(L, S, x, m, ld(x, u), s));
        }
    }
}

// ---------------------------------------------------------------- transfers
// residual of one fine slot, computed on the fly (regular cells) or read
// from rsp (irregular level-0 rows)
template <bool FINE, class T, class TB>
__device__ __forceinline__ bool child_res(const Lv &F, long long pin, const T *x, const TB *b, const double *bsh,
                                          const T *rsp, int cf, int h, int j, int k, double &r)
{
    const long long so = (long long)cf * F.Nh;
    const long long s = h + (long long)F.H * (j + (long long)F.ny * k);
    const uint8_t f = F.f[so + s];
    const int i = 2 * h + ((cf + j + k) & 1);
    if (FINE) {
        if ((f & F_SOLID) && !(f & F_GHOST)) return false;
        if (f & (F_GHOST | F_MGHOST)) { r = ld(rsp, so + s); return true; }
        double dg;
        double off = nbsum<true>(F, x + (long long)(1 - cf) * F.Nh, F.f + (long long)(1 - cf) * F.Nh, h, j, k, i, f, dg);
        double bb = ld(b, so + s);
        if (so + s == pin && bsh) bb -= bsh[0];
        r = bb - (off - dg * ld(x, so + s));
        return true;
    } else {
        if (!(f & 1)) return false;
        double dg;
        double off = nbsum<false>(F, x + (long long)(1 - cf) * F.Nh, F.f + (long long)(1 - cf) * F.Nh, h, j, k, i, f, dg);
        r = ld(b, so + s) - (bsh ? bsh[0] : 0.0) - (off - dg * ld(x, so + s));
        return true;
    }
}

// fused residual + restriction: coarse RHS = volume-weighted mean of the
// active children's residuals; partial sums of V_C b_C for the coarse mean
template <bool FINE, class T, class TB, class TBc>
__device__ __forceinline__ double restrict_one(const Lv &F, const Lv &C, long long pin, const T *x, const TB *b,
                                               const double *bsh, const T *rsp, TBc *bc, int cc, int hc, int J,
                                               int K)
{
    const long long sc = slot(C, cc, hc, J, K);
    const int I = 2 * hc + ((cc + J + K) & 1);
    if (I >= C.nx) { st(bc, sc, 0.0); return 0.0; }
    double sv = 0.0, svr = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int dx = q & 1, dy = (q >> 1) & 1, dz = (q >> 2) & 1;
        const int j = 2 * J + dy, k = 2 * K + dz, i = 2 * I + dx;
        double r;
        if (!child_res<FINE>(F, pin, x, b, bsh, rsp, (dx + dy + dz) & 1, I, j, k, r)) continue;
        const double V = F.w[0][i] * F.w[1][j] * F.w[2][k];
        sv += V;
        svr += V * r;
    }
    st(bc, sc, sv > 0.0 ? svr / sv : 0.0);
    return (C.f[sc] & 1) ? C.w[0][I] * C.w[1][J] * C.w[2][K] * ld(bc, sc) : 0.0;
}

template <bool FINE, class T, class TB, class TBc>
__global__ void __launch_bounds__(TPB) k_restrict(Lv F, Lv C, Geo Gc, long long pin, const T *x, const TB *b,
                                                  const double *bsh, const T *rsp, TBc *bc, double *part)
{
    Acc<1> a;
    a.v[0] = 0.0;
    int h, j, k0, k1;
    if (geo_tile(Gc, h, j, k0, k1))
        for (int k = k0; k < k1; ++k)
            for (int c = 0; c < 2; ++c) a.v[0] += restrict_one<FINE>(F, C, pin, x, b, bsh, rsp, bc, c, h, j, k);
    block_reduce<1>(a, part, 0, blockIdx.x);
}

// prolongation maps of a fine level from its coarse parent
struct PMap {
    const int *pi[3];
    const double *pt[3];
};

template <class Tc>
__device__ __forceinline__ double coarse_val(const Lv &C, const Tc *xc, int I, int J, int K)
{
    return ld(xc, slot(C, (I + J + K) & 1, I >> 1, J, K));
}

// trilinear interpolation (physical coordinates) of the coarse correction at one fine cell
template <class Tc>
__device__ __forceinline__ double interp(const Lv &C, const PMap &M, const Tc *xc, int i, int j, int k)
{
    const int I = M.pi[0][i], J = M.pi[1][j], K = M.pi[2][k];
    const double tx = M.pt[0][i], ty = M.pt[1][j], tz = M.pt[2][k];
    return (1 - tz) * ((1 - ty) * ((1 - tx) * coarse_val(C, xc, I, J, K) + tx * coarse_val(C, xc, I + 1, J, K)) +
                       ty * ((1 - tx) * coarse_val(C, xc, I, J + 1, K) + tx * coarse_val(C, xc, I + 1, J + 1, K))) +
           tz * ((1 - ty) * ((1 - tx) * coarse_val(C, xc, I, J, K + 1) + tx * coarse_val(C, xc, I + 1, J, K + 1)) +
                 ty * ((1 - tx) * coarse_val(C, xc, I, J + 1, K + 1) + tx * coarse_val(C, xc, I + 1, J + 1, K + 1)));
}

template <bool FINE, class Tc, class Tf>
__device__ __forceinline__ void prolong_one(const Lv &F, const Lv &C, const PMap &M, const Tc *xc, Tf *xf, int c,
                                            int h, int j, int k)
{
    const long long s = slot(F, c, h, j, k);
    const int i = 2 * h + ((c + j + k) & 1);
    if (i >= F.nx) return;
    const uint8_t f = F.f[s];
    if (FINE ? !active0(f) : !(f & 1)) return;
    st(xf, s, ld(xf, s) + interp(C, M, xc, i, j, k));
}

template <bool FINE, class Tc, class Tf>
__global__ void __launch_bounds__(TPB) k_prolong(Lv F, Lv C, PMap M, Geo G, const Tc *xc, Tf *xf)
{
    int h, j, k0, k1;
    if (!geo_tile(G, h, j, k0, k1)) return;
    for (int k = k0; k < k1; ++k)
        for (int c = 0; c < 2; ++c) prolong_one<FINE>(F, C, M, xc, xf, c, h, j, k);
}

// ---------------------------------------------------------------- coarse tail in one workgroup
// The smallest levels (each <= TAIL_MAX cells) run as one 1024-thread block:
// same operations as the grid kernels, separated by block barriers; the
// coarse means are block reductions.
constexpr int TAIL_MAX = 32768;
constexpr int TAIL_T = 1024;

struct TailLevel {
    Lv L;
    PMap M;          // prolongation onto this level from the next one
    double volA;
    void *x, *b, *r; // typed by the caller
};
struct Tail {
    int n;           // levels in the tail (>= 1)
    TailLevel t[8];
    int nu1, nu2, ncs;
};

__device__ double tail_sum(double v)
{
    __shared__ double sm[TAIL_T / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sm[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sm[w];
    __syncthreads();
    return s;
}

template <class Tc, class TB>
__device__ void tail_sweep(const Lv &L, Tc *x, const TB *b, double mu, int c, bool zero)
{
    const long long n = (long long)L.H * L.ny * L.nz;
    for (long long q = threadIdx.x; q < n; q += blockDim.x) {
        const int h = (int)(q % L.H);
        const long long row = q / L.H;
        const int j = (int)(row % L.ny), k = (int)(row / L.ny);
        const long long s = (long long)c * L.Nh + q;
        const uint8_t f = L.f[s];
        const int i = 2 * h + ((c + j + k) & 1);
        if (!(f & 1) || i >= L.nx) {
            if (zero) st(x, s, 0.0);
            continue;
        }
        double dg, off;
        if (zero && c == 0) {
            off = 0.0;
            dg = diag_only<false>(L, L.f + L.Nh, h, j, k, i, f);
        } else {
            off = nbsum<false>(L, x + (long long)(1 - c) * L.Nh, L.f + (long long)(1 - c) * L.Nh, h, j, k, i, f, dg);
        }
        st(x, s, dg > 0.0 ? (off - (ld(b, s) - mu)) / dg : 0.0);
    }
    __syncthreads();
}

template <class Tc, class TB>
__global__ void __launch_bounds__(TAIL_T) k_tail(Tail T, const double *mean0)
{
    __shared__ double mus[8];
    // level t[0]'s RHS was restricted by the caller; its mean is mean0
    if (threadIdx.x == 0) mus[0] = mean0[0];
    __syncthreads();
    for (int l = 0; l < T.n; ++l) {
        const Lv &L = T.t[l].L;
        Tc *x = (Tc *)T.t[l].x;
        const TB *b = (const TB *)T.t[l].b;
        const double mu = mus[l];
        const bool last = l == T.n - 1;
        const int steps = last ? T.ncs : T.nu1;
        for (int it = 0; it < steps; ++it) {
            tail_sweep<Tc, TB>(L, x, b, mu, 0, it == 0);
            tail_sweep<Tc, TB>(L, x, b, mu, 1, it == 0);
        }
        if (last) break;
        // restriction to the next level with the block-reduced coarse mean
        const Lv &C = T.t[l + 1].L;
        TB *bc = (TB *)T.t[l + 1].b;
        const long long nc = (long long)C.H * C.ny * C.nz;
        double part = 0.0;
        for (long long q = threadIdx.x; q < 2 * nc; q += blockDim.x) {
            const int cc = q >= nc ? 1 : 0;
            const long long qq = q - cc * nc;
            const int hc = (int)(qq % C.H);
            const long long row = qq / C.H;
            const int J = (int)(row % C.ny), K = (int)(row / C.ny);
            double mub = mu;
            part += restrict_one<false, Tc, TB, TB>(L, C, -1, x, b, &mub, (const Tc *)nullptr, bc, cc, hc, J, K);
        }
        const double tot = tail_sum(part);
        if (threadIdx.x == 0) mus[l + 1] = T.t[l + 1].volA > 0.0 ? tot / T.t[l + 1].volA : 0.0;
        __syncthreads();
    }
    for (int l = T.n - 2; l >= 0; --l) {
        const Lv &L = T.t[l].L, &C = T.t[l + 1].L;
        Tc *x = (Tc *)T.t[l].x;
        const Tc *xc = (const Tc *)T.t[l + 1].x;
        const long long n = (long long)L.H * L.ny * L.nz;
        for (long long q = threadIdx.x; q < 2 * n; q += blockDim.x) {
            const int c = q >= n ? 1 : 0;
            const long long qq = q - c * n;
            const int h = (int)(qq % L.H);
            const long long row = qq / L.H;
            prolong_one<false>(L, C, T.t[l].M, xc, x, c, h, (int)(row % L.ny), (int)(row / L.ny));
        }
        __syncthreads();
        const TB *b = (const TB *)T.t[l].b;
        for (int it = 0; it < T.nu2; ++it) {
            tail_sweep<Tc, TB>(L, x, b, mus[l], 0, false);
            tail_sweep<Tc, TB>(L, x, b, mus[l], 1, false);
        }
    }
}

// ---------------------------------------------------------------- Krylov vector kernels
enum {
    S_RHO = 0, S_RHO_OLD, S_ALPHA, S_OMEGA, S_BETA, S_RR, S_BN2, S_REL, S_SINKP, S_SINKS,
    S_RV, S_TS, S_TT, S_STATUS, S_VPIN, S_TMP, S_TMP2, S_MEAN0 = 20, S_COUNT = 48
};

__device__ __forceinline__ double slot_volume(const Lv &L, long long s, bool &act)
{
    int c, h, j, k, i;
    decode_slot(L, s, c, h, j, k, i);
    act = i < L.nx && active0(L.f[s]);
    return act ? L.w[0][i] * L.w[1][j] * L.w[2][k] : 0.0;
}

// p = r + beta (p - omega v); partial sum of V p over active cells (sink)
template <class T>
__global__ void __launch_bounds__(TPB) k_p_update(Lv L, Walk W, const T *r, T *pv, const T *v, const double *sc,
                                                  double *part)
{
    const double beta = sc[S_BETA], omega = sc[S_OMEGA];
    Acc<1> a;
    a.v[0] = 0.0;
    const long long N2 = 2 * L.Nh;
    WALK_BEGIN(W, p)
        st(pv, p, ld(r, p) + beta * (ld(pv, p) - omega * ld(v, p)));
        if (p < N2) {
            bool act;
            const double V = slot_volume(L, p, act);
            if (act) a.v[0] += V * ld(pv, p);
        }
    WALK_END
    block_reduce<1>(a, part, 0, blockIdx.x);
}

// r <- s = r - alpha v; partial sum of V s (sink of the second V-cycle)
template <class T>
__global__ void __launch_bounds__(TPB) k_s_update(Lv L, Walk W, T *r, const T *v, const double *sc, double *part)
{
    const double alpha = sc[S_ALPHA];
    Acc<1> a;
    a.v[0] = 0.0;
    const long long N2 = 2 * L.Nh;
    WALK_BEGIN(W, p)
        st(r, p, ld(r, p) - alpha * ld(v, p));
        if (p < N2) {
            bool act;
            const double V = slot_volume(L, p, act);
            if (act) a.v[0] += V * ld(r, p);
        }
    WALK_END
    block_reduce<1>(a, part, 0, blockIdx.x);
}

// x += alpha (ph - ph_pin) + omega (sh - sh_pin) on the active unknowns (the
// preconditioner's shift to the pinned subspace, folded in here); r = s -
// omega t; partials of (rh, r) and (r, r)
template <class T, class TX>
__global__ void __launch_bounds__(TPB) k_xr_update(Lv L, Walk W, long long pin, TX *x, const T *ph, const T *sh,
                                                   T *r, const T *t, const T *rh, const double *sc, double *part,
                                                   int pstride)
{
    const double alpha = sc[S_ALPHA], omega = sc[S_OMEGA];
    const double cp = ld(ph, pin), cs = ld(sh, pin);
    const long long N2 = 2 * L.Nh;
    Acc<2> a;
    a.v[0] = a.v[1] = 0.0;
    WALK_BEGIN(W, p)
        const bool act = p >= N2 || active0(L.f[p]);
        if (act) st(x, p, ld(x, p) + alpha * (ld(ph, p) - cp) + omega * (ld(sh, p) - cs));
        st(r, p, ld(r, p) - omega * ld(t, p));
        const double rv = ld(r, p);
        a.v[0] += ld(rh, p) * rv;
        a.v[1] += rv * rv;
    WALK_END
    block_reduce<2>(a, part, pstride, blockIdx.x);
}

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

// b = a (converted), b2 = a (may be NULL); partials of (b, b)
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

template <class T>
__global__ void __launch_bounds__(TPB) k_add(Walk W, double *x, const T *d)
{
    WALK_BEGIN(W, p)
        x[p] += ld(d, p);
    WALK_END
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

// volume-weighted sum of a over the cells selected by the flag test
// (FLUID: not solid; ACTIVE: fluid or closed ghost)
template <class T, bool ACTIVE>
__global__ void __launch_bounds__(TPB) k_vsum(Lv L, Walk W, const T *a, double *part)
{
    Acc<1> s;
    s.v[0] = 0.0;
    WALK_BEGIN(W, p)
        int c, h, j, k, i;
        decode_slot(L, p, c, h, j, k, i);
        const uint8_t f = L.f[p];
        const bool use = i < L.nx && (ACTIVE ? active0(f) : !(f & F_SOLID));
        if (use) s.v[0] += L.w[0][i] * L.w[1][j] * L.w[2][k] * ld(a, p);
    WALK_END
    block_reduce<1>(s, part, 0, blockIdx.x);
}

// ---------------------------------------------------------------- layout conversion
// natural (x fastest) <-> split slots; membrane tail copied as is
template <class TA, class TB>
__global__ void __launch_bounds__(TPB) k_to_split(Lv L, Walk W, const TA *nat, TB *spl, long long tail)
{
    WALK_BEGIN(W, p)
        if (p < 2 * L.Nh) {
            int c, h, j, k, i;
            decode_slot(L, p, c, h, j, k, i);
            st(spl, p, i < L.nx ? ld(nat, (long long)i + (long long)L.nx * (j + (long long)L.ny * k)) : 0.0);
        } else if (p - 2 * L.Nh < tail) {
            st(spl, p, ld(nat, (long long)L.nx * L.ny * L.nz + (p - 2 * L.Nh)));
        }
    WALK_END
}

template <class TA, class TB>
__global__ void __launch_bounds__(TPB) k_from_split(Lv L, Walk W, const TA *spl, TB *nat, long long tail)
{
    WALK_BEGIN(W, p)
        if (p < 2 * L.Nh) {
            int c, h, j, k, i;
            decode_slot(L, p, c, h, j, k, i);
            if (i < L.nx) st(nat, (long long)i + (long long)L.nx * (j + (long long)L.ny * k), ld(spl, p));
        } else if (p - 2 * L.Nh < tail) {
            st(nat, (long long)L.nx * L.ny * L.nz + (p - 2 * L.Nh), ld(spl, p));
        }
    WALK_END
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

enum { FIN_SUM = 0, FIN_SINK, FIN_ALPHA, FIN_OMEGA, FIN_RHO, FIN_MEAN, FIN_INIT, FIN_RESTART, FIN_REPLACE };

__global__ void __launch_bounds__(1024) k_fin(const double *part, int pstride, int n, int op, int dst, double aux,
                                              double *sc)
{
    const bool two = op == FIN_OMEGA || op == FIN_RHO || op == FIN_REPLACE;
    double s0 = block_sum_all(part, n);
    double s1 = two ? block_sum_all(part + pstride, n) : 0.0;
    if (threadIdx.x != 0) return;
    switch (op) {
    case FIN_SUM: sc[dst] = s0; break;
    case FIN_SINK: sc[dst] = s0 / sc[S_VPIN]; break;
    case FIN_MEAN: sc[dst] = aux > 0.0 ? s0 / aux : 0.0; break;
    case FIN_ALPHA:
        sc[S_RV] = s0;
        if (s0 == 0.0 || !isfinite(s0)) { sc[S_STATUS] = 2.0; sc[S_ALPHA] = 0.0; }
        else sc[S_ALPHA] = sc[S_RHO] / s0;
        break;
    case FIN_OMEGA:
        sc[S_TS] = s0; sc[S_TT] = s1;
        sc[S_OMEGA] = s1 > 0.0 ? s0 / s1 : 0.0;
        if (!(s1 > 0.0)) sc[S_STATUS] = 3.0;
        break;
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
    case FIN_INIT:
        sc[S_BN2] = s0; sc[S_RR] = s0; sc[S_RHO] = s0; sc[S_RHO_OLD] = 1.0;
        sc[S_ALPHA] = 1.0; sc[S_OMEGA] = 1.0; sc[S_BETA] = 0.0;
        sc[S_REL] = s0 > 0.0 ? 1.0 : 0.0; sc[S_STATUS] = 0.0;
        break;
    case FIN_RESTART:
        sc[S_RR] = s0; sc[S_RHO] = s0; sc[S_BETA] = 0.0; sc[S_STATUS] = 0.0;
        sc[S_REL] = sqrt(s0 / sc[S_BN2]);
        break;
    case FIN_REPLACE: {
        // residual replacement: rho = (rh, r_true); beta from the previous rho
        sc[S_RHO] = s0;
        sc[S_RR] = s1;
        sc[S_REL] = sqrt(s1 / sc[S_BN2]);
        const double om = sc[S_OMEGA], ro = sc[S_RHO_OLD];
        sc[S_BETA] = (om != 0.0 && ro != 0.0) ? (s0 / ro) * (sc[S_ALPHA] / om) : 0.0;
        break;
    }
    }
}

}  // namespace ibm
