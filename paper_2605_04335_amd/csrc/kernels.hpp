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

// load at a block-uniform base plus a 32-bit element offset (the compiler
// then addresses with a scalar base and one 32-bit VGPR per load)
template <class T>
__device__ __forceinline__ T ldu(const T *base, uint32_t i)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + i * (uint32_t)sizeof(T));
}

// v rounded to the precision of storage type T
template <class T>
__device__ __forceinline__ double round_to(double v) { return (double)(T)v; }
template <>
__device__ __forceinline__ double round_to<bf16>(double v) { return (double)(float)(bf16)(float)v; }

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
inline Walk make_walk(long long n, long long maxb = MAXB)
{
    Walk w;
    w.n = n;
    w.chunks = (n + TPB - 1) / TPB;
    long long b = (w.chunks + 7) / 8 * 8;
    if (b > maxb) b = maxb;
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
inline Geo make_geo(int H, int ny, int nz, int maxb = 8192)
{
    Geo g;
    g.H = H; g.ny = ny; g.nz = nz;
    g.gx = (H + 63) / 64;
    g.gy = (ny + 3) / 4;
    long long xy = (long long)g.gx * g.gy;
    int kz = 1;
    while (xy * ((nz + kz - 1) / kz) > maxb && kz < nz) kz *= 2;
    g.kz = kz;
    g.gz = (nz + kz - 1) / kz;
    long long n = xy * g.gz;
    g.nb = (int)((n + 7) / 8 * 8);
    return g;
}
// tiles of 64 half-indices x 8 rows for a kernel whose threads take two
// consecutive rows each (the FP64 level-0 half-sweep)
inline Geo make_geo_rows2(int H, int ny, int nz, int maxb = 8192)
{
    Geo g = make_geo(H, ny, nz, maxb);
    g.gy = (ny + 7) / 8;
    const long long xy = (long long)g.gx * g.gy;
    int kz = 1;
    while (xy * ((nz + kz - 1) / kz) > maxb && kz < nz) kz *= 2;
    g.kz = kz;
    g.gz = (nz + kz - 1) / kz;
    g.nb = (int)((xy * g.gz + 7) / 8 * 8);
    return g;
}
// tiles over cells in natural x order (nx instead of H): the restriction
inline Geo make_geo_nat(int nx, int ny, int nz, int maxb = 8192) { return make_geo(nx, ny, nz, maxb); }

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

// coarse-level mask bits: active cell, then the six faces that are open
// (both cells active and no membrane cut between them), each stored in both
// cells so a row needs only its own byte
enum : uint8_t { CM_ACT = 1, CM_PX = 2, CM_PY = 4, CM_PZ = 8, CM_MX = 16, CM_MY = 32, CM_MZ = 64 };

// Sum over the open faces of coefficient * neighbour value, and the diagonal.
// xo is the other colour's array (base of that colour).  FINE: the faces of a
// regular level-0 cell are open inside the domain; coarse: the cell's own
// open-face bits (fo is not read).
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
        if (fm & CM_PX) { double c = L.cp[0][i]; acc += c * ld(xo, row + h + p); d += c; }
        if (fm & CM_MX) { double c = L.cm[0][i]; acc += c * ld(xo, row + h + p - 1); d += c; }
        if (fm & CM_PY) { double c = L.cp[1][j]; acc += c * ld(xo, row + h + L.H); d += c; }
        if (fm & CM_MY) { double c = L.cm[1][j]; acc += c * ld(xo, row + h - L.H); d += c; }
        if (fm & CM_PZ) { double c = L.cp[2][k]; acc += c * ld(xo, row + h + pl); d += c; }
        if (fm & CM_MZ) { double c = L.cm[2][k]; acc += c * ld(xo, row + h - pl); d += c; }
    }
    dg = d;
    return acc;
}

// nbsum<false> without branches: every neighbour value and coefficient is
// loaded (a closed face reads the cell's own slot in the other colour) and a
// closed face's coefficient is replaced by zero, so all six loads are in
// flight together.  Adding a zero product or a zero coefficient leaves the
// sums unchanged (the sums are never -0), so the result is nbsum's.  Used
// where the level is LDS-resident (the coarse tail).
template <class T>
__device__ __forceinline__ double nbsum_all(const Lv &L, const T *xo, int h, int j, int k, int i, uint8_t fm,
                                            double &dg)
{
    const int p = i & 1;
    const int pl = L.H * L.ny, base = h + L.H * j + pl * k;
    const bool o[6] = {(fm & CM_PX) != 0, (fm & CM_MX) != 0, (fm & CM_PY) != 0,
                       (fm & CM_MY) != 0, (fm & CM_PZ) != 0, (fm & CM_MZ) != 0};
    const int dx[6] = {p, p - 1, L.H, -L.H, pl, -pl};
    const double cv[6] = {L.cp[0][i], L.cm[0][i], L.cp[1][j], L.cm[1][j], L.cp[2][k], L.cm[2][k]};
    double xv[6];
#pragma unroll
    for (int t = 0; t < 6; ++t) xv[t] = ld(xo, base + (o[t] ? dx[t] : 0));
    double acc = 0.0, d = 0.0;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        const double c = o[t] ? cv[t] : 0.0;
        acc += c * xv[t];
        d += c;
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
        if (fm & CM_PX) d += L.cp[0][i];
        if (fm & CM_MX) d += L.cm[0][i];
        if (fm & CM_PY) d += L.cp[1][j];
        if (fm & CM_MY) d += L.cm[1][j];
        if (fm & CM_PZ) d += L.cp[2][k];
        if (fm & CM_MZ) d += L.cm[2][k];
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
    const int32_t *rmrow;  // [nrows*8] membrane cell behind each stencil column (-1: none)
};

__device__ __forceinline__ long long ghost_unknown(const Sp &S, int r)
{
    return r < S.ng ? (long long)S.rslot[r] : S.N2 + (r - S.ng);
}

// Sum of w x over the 8 stencil columns of ghost row r (a column < 0 is
// absent).  The columns and weights are read first (16-byte loads), then
// every value (an absent column reads unknown 0, unused), then the sum in
// column order: one dependent step instead of one per column.
template <class T>
__device__ __forceinline__ double ghost_sum(const Sp &S, const T *x, int r)
{
    const int4 *c4 = reinterpret_cast<const int4 *>(S.rcol + 8 * (long long)r);
    const double2 *w2 = reinterpret_cast<const double2 *>(S.rw + 8 * (long long)r);
    int32_t gc[8];
    double gw[8], xv[8];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int4 q = c4[t];
        gc[4 * t] = q.x; gc[4 * t + 1] = q.y; gc[4 * t + 2] = q.z; gc[4 * t + 3] = q.w;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const double2 q = w2[t];
        gw[2 * t] = q.x; gw[2 * t + 1] = q.y;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) xv[t] = ld(x, gc[t] >= 0 ? (long long)gc[t] : 0LL);
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < 8; ++t)
        if (gc[t] >= 0) acc += gw[t] * xv[t];
    return acc;
}

// fluid row of membrane cell m: sum c (x_nb - xp) and its diagonal; the six
// neighbour values are loaded together (a wall reads unknown 0, unused)
template <class T>
__device__ __forceinline__ double mrow(const Lv &L, const Sp &S, const T *x, int m, double xp, double &s)
{
    int c, h, j, k, i;
    decode_slot(L, S.mslot[m], c, h, j, k, i);
    int32_t mc[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) mc[q] = S.mcol[6 * m + q];
    const double cf[6] = {L.cm[0][i], L.cp[0][i], L.cm[1][j], L.cp[1][j], L.cm[2][k], L.cp[2][k]};
    double xv[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) xv[q] = ld(x, mc[q] >= 0 ? (long long)mc[q] : 0LL);
    double acc = 0.0;
    s = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        if (mc[q] >= 0) { acc += cf[q] * (xv[q] - xp); s += cf[q]; }
    return acc;
}

enum { M_PINNED = 0, M_PINZERO = 1, M_UNPINNED = 2 };

// ---------------------------------------------------------------- level-0 operator
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

// Per-column constants of a level-0 stencil walk in one colour: x
// coefficients and neighbour offsets for both parities of i (which
// alternates with k), y coefficients and offsets.  Walls carry a zero
// coefficient and a clamped (in-bounds) offset, so loads need no branches.
struct Col0 {
    double cpx[2], cmx[2], cpy, cmy;
    int oxp[2], oxm[2];
    long long oyp, oym;
};
__device__ __forceinline__ Col0 col0(const Lv &L, int c, int h, int j)
{
    Col0 q;
    const int pa = (c + j) & 1;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int p = pa ^ t;
        const int i = 2 * h + p;
        const bool xp = i + 1 < L.nx, xm = i > 0 && i < L.nx;
        q.cpx[t] = xp ? L.cp[0][i] : 0.0;
        q.cmx[t] = xm ? L.cm[0][i] : 0.0;
        q.oxp[t] = xp ? p : 0;
        q.oxm[t] = xm ? p - 1 : 0;
    }
    q.cpy = j + 1 < L.ny ? L.cp[1][j] : 0.0;
    q.cmy = j > 0 ? L.cm[1][j] : 0.0;
    q.oyp = j + 1 < L.ny ? (long long)L.H : 0;
    q.oym = j > 0 ? -(long long)L.H : 0;
    return q;
}

// sum of coefficient * other-colour neighbour at slot s of plane k, and the diagonal
template <class T>
__device__ __forceinline__ double col0_sum(const Lv &L, const Col0 &q, const T *__restrict__ xo, long long s, int k,
                                           long long pl, double &dg)
{
    // parity of i alternates with k: select (constant indices keep q in registers)
    const bool t = k & 1;
    const double cpx = t ? q.cpx[1] : q.cpx[0], cmx = t ? q.cmx[1] : q.cmx[0];
    const int oxp = t ? q.oxp[1] : q.oxp[0], oxm = t ? q.oxm[1] : q.oxm[0];
    const double czp = L.cp[2][k], czm = L.cm[2][k];  // zero at the walls
    const long long ozp = k + 1 < L.nz ? pl : 0, ozm = k > 0 ? -pl : 0;
    dg = cpx + cmx + q.cpy + q.cmy + czp + czm;
    return cpx * ld(xo, s + oxp) + cmx * ld(xo, s + oxm) + q.cpy * ld(xo, s + q.oyp) + q.cmy * ld(xo, s + q.oym) +
           czp * ld(xo, s + ozp) + czm * ld(xo, s + ozm);
}

// Coarse-level Gauss-Seidel half-sweep of colour c over the active cells,
// with the level mean mu subtracted from every RHS.  Faces are taken from the
// cell's own mask byte: a closed face gets a zero coefficient and reads an
// in-range slot, so every load of a plane is issued before any arithmetic.
// ZMODE 1: first red sweep from a zero iterate (diagonal only; every slot of
// the colour is written); ZMODE 2: first black sweep (skipped slots get 0).
__device__ __forceinline__ double cmask_sum_dg(const Lv &L, const Col0 &q, uint8_t f, int k, double &cpx,
                                               double &cmx, double &cpy, double &cmy, double &czp, double &czm)
{
    const bool t = k & 1;
    const double zp = L.cp[2][k], zm = L.cm[2][k];  // loaded whatever the mask (no wait on it)
    cpx = (f & CM_PX) ? (t ? q.cpx[1] : q.cpx[0]) : 0.0;
    cmx = (f & CM_MX) ? (t ? q.cmx[1] : q.cmx[0]) : 0.0;
    cpy = (f & CM_PY) ? q.cpy : 0.0;
    cmy = (f & CM_MY) ? q.cmy : 0.0;
    czp = (f & CM_PZ) ? zp : 0.0;
    czm = (f & CM_MZ) ? zm : 0.0;
    return cpx + cmx + cpy + cmy + czp + czm;
}

constexpr int UC = 2;
template <class T, class TB, int ZMODE>
__global__ void __launch_bounds__(TPB) k_csweep(Lv L, Geo G, T *__restrict__ x, const TB *__restrict__ b,
                                                const double *__restrict__ bsh, int c)
{
    int h, j, k0, k1;
    if (!geo_tile(G, h, j, k0, k1)) return;
    const double mu = bsh ? bsh[0] : 0.0;
    T *xc = x + (long long)c * L.Nh;
    const T *xo = x + (long long)(1 - c) * L.Nh;
    const uint8_t *fc = L.f + (long long)c * L.Nh;
    const TB *bc = b + (long long)c * L.Nh;
    const Col0 q = col0(L, c, h, j);
    if constexpr (ZMODE == 0) {
        // ordinary sweep: the other colour's values at (h, j) in planes k-1,
        // k, k+1 kept in registers (the centre is an x neighbour, the planes
        // above and below the z neighbours), every load of a step issued
        // unconditionally before any arithmetic (the planes beyond the walls
        // read clamped indices: their mask bits close those faces), 32-bit
        // offsets from plane-uniform bases.  Same arithmetic as below.
        constexpr int UW = 2;
        const uint32_t pl = (uint32_t)(L.H * L.ny);
        const int kb = max(k0 - 1, 0);
        const T *xb = xo + (long long)pl * kb;
        const TB *bp = bc + (long long)pl * kb;
        const uint8_t *fb = fc + (long long)pl * kb;
        T *xw = xc + (long long)pl * kb;
        const uint32_t col = (uint32_t)(h + L.H * j);
        const int ox0 = q.oxp[0] + q.oxm[0], ox1 = q.oxp[1] + q.oxm[1];
        auto zs = [&](int k) { return col + pl * (uint32_t)(k - kb); };
        double cprev = ldu(xb, zs(max(k0 - 1, 0))), ccur = ldu(xb, zs(k0));
        for (int ks = k0; ks < k1; ks += UW) {
            double cn[UW], xs[UW], yp[UW], ym[UW], bb[UW], zp[UW], zm[UW];
            uint8_t fl[UW];
#pragma unroll
            for (int u = 0; u < UW; ++u) {
                const int k = min(ks + u, k1 - 1);
                const uint32_t s = zs(k);
                cn[u] = ldu(xb, zs(min(k + 1, L.nz - 1)));
                xs[u] = ldu(xb, s + (uint32_t)((k & 1) ? ox1 : ox0));
                yp[u] = ldu(xb, s + (uint32_t)(int)q.oyp);
                ym[u] = ldu(xb, s + (uint32_t)(int)q.oym);
                fl[u] = ldu(fb, s);
                bb[u] = ld(bp, (long long)s);
                zp[u] = L.cp[2][k];
                zm[u] = L.cm[2][k];
            }
#pragma unroll
            for (int u = 0; u < UW; ++u) {
                const int k = ks + u;
                if (k >= k1) continue;
                const double cc = u == 0 ? ccur : cn[u - 1];
                const double cmv = u == 0 ? cprev : (u == 1 ? ccur : cn[u - 2]);
                const uint32_t s = zs(k);
                const int i = 2 * h + ((c + j + k) & 1);
                const uint8_t f = fl[u];
                if (!(f & CM_ACT) || i >= L.nx) continue;
                const bool t = k & 1;
                const double cpx = (f & CM_PX) ? (t ? q.cpx[1] : q.cpx[0]) : 0.0;
                const double cmx = (f & CM_MX) ? (t ? q.cmx[1] : q.cmx[0]) : 0.0;
                const double cpy = (f & CM_PY) ? q.cpy : 0.0, cmy = (f & CM_MY) ? q.cmy : 0.0;
                const double czp = (f & CM_PZ) ? zp[u] : 0.0, czm = (f & CM_MZ) ? zm[u] : 0.0;
                const int oxp = t ? q.oxp[1] : q.oxp[0], oxm = t ? q.oxm[1] : q.oxm[0];
                const double xpv = oxp == 0 ? cc : xs[u], xmv = oxm == 0 ? cc : xs[u];
                const double dg = cpx + cmx + cpy + cmy + czp + czm;
                const double nb = cpx * xpv + cmx * xmv + cpy * yp[u] + cmy * ym[u] + czp * cn[u] + czm * cmv;
                st(xw, (long long)s, dg > 0.0 ? (nb - (bb[u] - mu)) / dg : 0.0);
            }
            cprev = cn[UW - 2];
            ccur = cn[UW - 1];
        }
        return;
    }
    const long long pl = (long long)L.H * L.ny;
    const long long col = h + (long long)L.H * j;
    for (int kb = k0; kb < k1; kb += UC) {
        double nb[UC], bb[UC], dg[UC];
        uint8_t fl[UC];
#pragma unroll
        for (int u = 0; u < UC; ++u) {
            const int k = min(kb + u, k1 - 1);
            const long long s = col + pl * k;
            fl[u] = fc[s];
            bb[u] = ld(bc, s);
            double cpx, cmx, cpy, cmy, czp, czm;
            dg[u] = cmask_sum_dg(L, q, fl[u], k, cpx, cmx, cpy, cmy, czp, czm);
            if (ZMODE == 1) {
                nb[u] = 0.0;
            } else {
                const bool t = k & 1;
                const int oxp = t ? q.oxp[1] : q.oxp[0], oxm = t ? q.oxm[1] : q.oxm[0];
                const long long ozp = k + 1 < L.nz ? pl : 0, ozm = k > 0 ? -pl : 0;
                nb[u] = cpx * ld(xo, s + oxp) + cmx * ld(xo, s + oxm) + cpy * ld(xo, s + q.oyp) +
                        cmy * ld(xo, s + q.oym) + czp * ld(xo, s + ozp) + czm * ld(xo, s + ozm);
            }
        }
#pragma unroll
        for (int u = 0; u < UC; ++u) {
            const int k = kb + u;
            if (k >= k1) continue;
            const long long s = col + pl * k;
            const int i = 2 * h + ((c + j + k) & 1);
            if (!(fl[u] & CM_ACT) || i >= L.nx) {
                if (ZMODE) st(xc, s, 0.0);
                continue;
            }
            st(xc, s, dg[u] > 0.0 ? (nb[u] - (bb[u] - mu)) / dg[u] : 0.0);
        }
    }
}

// Level-0 Gauss-Seidel half-sweep of colour c (ordinary mode): xc, bc, fc
// are this colour's arrays, xo the other colour's.  The other colour's slot
// at the same (h, j, k) is an x neighbour of the cell in plane k and its z
// neighbour in planes k-1 and k+1, so each thread walks its planes with a
// three-plane window of those values in registers.  SWP planes per step
// (two in FP64, four in FP32), every load of a step issued before any
// arithmetic and none of them conditional: the plane above is read from a
// clamped index (its coefficient is zero at the top wall) and the z
// coefficients are loaded with the values.  Addresses are 32-bit offsets
// from block-uniform bases at the tile's first plane (the tile spans at most
// kz + 1 planes; plane_span_ok() holds for every level-0 geometry).  The new
// values are written with non-temporal stores: the next kernel to read them
// is a later half-sweep, long after a level-0 vector has left the caches.
// pin_s: the pin's slot within this colour (or -1), whose RHS carries the sink.
template <class T>
__device__ __forceinline__ void st_nt(T *p, T v) { __builtin_nontemporal_store(v, p); }

// FP64: each thread updates two consecutive rows j0, j0 + 1 of its column
// (tiles of 64 x 8 from make_geo_rows2).  The other colour's centres of both
// rows are in the window, and they are row j0's y+ neighbour and row j0+1's
// y- neighbour, so a step loads 10 values for 2 cells instead of 12
// (5.5% faster at 512^3; FP32 is faster with the one-row form).  Same
// arithmetic, in the same order, per cell.
__device__ __forceinline__ bool geo_tile2(const Geo &G, int &h, int &j0, int &k0, int &k1)
{
    const int b = blockIdx.x;
    const int L = (b & 7) * (G.nb >> 3) + (b >> 3);
    const int bx = L % G.gx, r = L / G.gx, by = r % G.gy, bz = r / G.gy;
    if (bz >= G.gz) return false;
    h = bx * 64 + (threadIdx.x & 63);
    j0 = by * 8 + 2 * (threadIdx.x >> 6);
    k0 = bz * G.kz;
    k1 = min(G.nz, k0 + G.kz);
    return h < G.H && j0 < G.ny;
}

template <class T>
__device__ __forceinline__ void sweep_rows2(const Lv &L, const Geo &G, long long pin_s, T *__restrict__ xc,
                                            const T *__restrict__ xo, const T *__restrict__ bc,
                                            const uint8_t *__restrict__ fc, const double *__restrict__ sink, int c)
{
    constexpr int UP = 2;
    int h, j0, k0, k1;
    if (!geo_tile2(G, h, j0, k0, k1)) return;
    const bool two = j0 + 1 < L.ny;  // an odd last row is updated alone
    const int j1 = two ? j0 + 1 : j0;
    const Col0 qa = col0(L, c, h, j0), qb = col0(L, c, h, j1);
    const uint32_t pl = (uint32_t)(L.H * L.ny);
    const int kb = max(k0 - 1, 0);
    const T *xb = xo + (long long)pl * kb;
    const T *bp = bc + (long long)pl * kb;
    const uint8_t *fb = fc + (long long)pl * kb;
    T *xw = xc + (long long)pl * kb;
    const uint32_t ca = (uint32_t)(h + L.H * j0), cb = (uint32_t)(h + L.H * j1);
    const int oxa0 = qa.oxp[0] + qa.oxm[0], oxa1 = qa.oxp[1] + qa.oxm[1];
    const int oxb0 = qb.oxp[0] + qb.oxm[0], oxb1 = qb.oxp[1] + qb.oxm[1];
    const int oyma = (int)qa.oym, oypb = (int)qb.oyp;  // the two loaded y neighbours
    const long long pin_rel = pin_s >= 0 ? pin_s - (long long)pl * kb : -1;
    // centres of both rows in planes k-1 and k
    double pa = k0 > 0 ? (double)ldu(xb, ca + pl * (uint32_t)(k0 - 1 - kb)) : 0.0;
    double pb = k0 > 0 ? (double)ldu(xb, cb + pl * (uint32_t)(k0 - 1 - kb)) : 0.0;
    double ua = ldu(xb, ca + pl * (uint32_t)(k0 - kb));
    double ub = ldu(xb, cb + pl * (uint32_t)(k0 - kb));
    for (int ks = k0; ks < k1; ks += UP) {
        double na[UP], nb2[UP], xa[UP], xbb[UP], ym[UP], yp[UP], ba[UP], bb[UP], czp[UP], czm[UP];
        uint8_t fa[UP], fbb[UP];
#pragma unroll
        for (int u = 0; u < UP; ++u) {
            const int k = min(ks + u, k1 - 1);
            const int kn = min(k + 1, L.nz - 1);
            const uint32_t sa = ca + pl * (uint32_t)(k - kb), sb = cb + pl * (uint32_t)(k - kb);
            const bool t = k & 1;
            na[u] = ldu(xb, ca + pl * (uint32_t)(kn - kb));  // centres of plane k+1
            nb2[u] = ldu(xb, cb + pl * (uint32_t)(kn - kb));
            xa[u] = ldu(xb, sa + (uint32_t)(t ? oxa1 : oxa0));
            xbb[u] = ldu(xb, sb + (uint32_t)(t ? oxb1 : oxb0));
            ym[u] = ldu(xb, sa + (uint32_t)oyma);
            yp[u] = ldu(xb, sb + (uint32_t)oypb);
            fa[u] = ldu(fb, sa);
            fbb[u] = ldu(fb, sb);
            ba[u] = ldu(bp, sa);
            bb[u] = ldu(bp, sb);
            czp[u] = L.cp[2][k];  // zero at the walls
            czm[u] = L.cm[2][k];
        }
#pragma unroll
        for (int u = 0; u < UP; ++u) {
            const int k = ks + u;
            const double cca = u == 0 ? ua : na[u - 1], ccb = u == 0 ? ub : nb2[u - 1];
            const double cma = u == 0 ? pa : (u == 1 ? ua : na[u - 2]);
            const double cmb = u == 0 ? pb : (u == 1 ? ub : nb2[u - 2]);
            if (k >= k1) continue;
            const bool t = k & 1;
            {   // row j0: its y+ neighbour is row j1's centre (its own centre when alone)
                const uint32_t s = ca + pl * (uint32_t)(k - kb);
                const double cpx = t ? qa.cpx[1] : qa.cpx[0], cmx = t ? qa.cmx[1] : qa.cmx[0];
                const int oxp = t ? qa.oxp[1] : qa.oxp[0], oxm = t ? qa.oxm[1] : qa.oxm[0];
                const double xpv = oxp == 0 ? cca : xa[u], xmv = oxm == 0 ? cca : xa[u];
                const double ypk = two ? ccb : cca;
                const double dg = cpx + cmx + qa.cpy + qa.cmy + czp[u] + czm[u];
                const double nb = cpx * xpv + cmx * xmv + qa.cpy * ypk + qa.cmy * ym[u] + czp[u] * na[u] + czm[u] * cma;
                if (!(fa[u] & (F_SOLID | F_MGHOST))) {
                    double b0 = ba[u];
                    if ((long long)s == pin_rel) b0 -= sink[0];
                    st_nt(xw + s, (T)((nb - b0) / dg));
                }
            }
            if (two) {  // row j1: its y- neighbour is row j0's centre
                const uint32_t s = cb + pl * (uint32_t)(k - kb);
                const double cpx = t ? qb.cpx[1] : qb.cpx[0], cmx = t ? qb.cmx[1] : qb.cmx[0];
                const int oxp = t ? qb.oxp[1] : qb.oxp[0], oxm = t ? qb.oxm[1] : qb.oxm[0];
                const double xpv = oxp == 0 ? ccb : xbb[u], xmv = oxm == 0 ? ccb : xbb[u];
                const double dg = cpx + cmx + qb.cpy + qb.cmy + czp[u] + czm[u];
                const double nb = cpx * xpv + cmx * xmv + qb.cpy * yp[u] + qb.cmy * cca + czp[u] * nb2[u] + czm[u] * cmb;
                if (!(fbb[u] & (F_SOLID | F_MGHOST))) {
                    double b0 = bb[u];
                    if ((long long)s == pin_rel) b0 -= sink[0];
                    st_nt(xw + s, (T)((nb - b0) / dg));
                }
            }
        }
        pa = na[UP - 2];
        pb = nb2[UP - 2];
        ua = na[UP - 1];
        ub = nb2[UP - 1];
    }
}

template <class T>
struct SweepPlanes {
    static constexpr int n = 2;
};
template <>
struct SweepPlanes<float> {
    static constexpr int n = 4;
};

// byte offsets of a tile's planes fit in 32 bits
inline bool plane_span_ok(long long plane_slots, int kz, size_t elem) { return plane_slots * (kz + 2) * (long long)elem < (1LL << 32); }

template <class T>
__global__ void __launch_bounds__(TPB) k0_sweep(Lv L, Geo G, long long pin_s, T *__restrict__ xc,
                                                const T *__restrict__ xo, const T *__restrict__ bc,
                                                const uint8_t *__restrict__ fc, const double *__restrict__ sink, int c)
{
    if constexpr (sizeof(T) == 8) {  // G: 64 x 8 tiles (make_geo_rows2)
        sweep_rows2<T>(L, G, pin_s, xc, xo, bc, fc, sink, c);
        return;
    }
    constexpr int UP = SweepPlanes<T>::n;
    // FP32: the x and y neighbours of plane k+1 are loaded with plane k+1's
    // centre, one step ahead of their use, so a step's loads all fall in the
    // planes being fetched then (4% faster at 512^3; FP64 gained nothing)
    constexpr bool AHEAD = sizeof(T) == 4;
    int h, j, k0, k1;
    if (!geo_tile(G, h, j, k0, k1)) return;
    const Col0 q = col0(L, c, h, j);
    const uint32_t pl = (uint32_t)(L.H * L.ny);
    const int kb = max(k0 - 1, 0);
    const T *xb = xo + (long long)pl * kb;
    const T *bp = bc + (long long)pl * kb;
    const uint8_t *fb = fc + (long long)pl * kb;
    T *xw = xc + (long long)pl * kb;
    const uint32_t col = (uint32_t)(h + L.H * j);
    const int ox0 = q.oxp[0] + q.oxm[0], ox1 = q.oxp[1] + q.oxm[1];  // the x neighbour that is not the centre
    const int oyp = (int)q.oyp, oym = (int)q.oym;
    const long long pin_rel = pin_s >= 0 ? pin_s - (long long)pl * kb : -1;
    // centres of planes k-1 and k (zero coefficient outside the grid)
    double cprev = k0 > 0 ? (double)ldu(xb, col + pl * (uint32_t)(k0 - 1 - kb)) : 0.0;
    double ccur = ldu(xb, col + pl * (uint32_t)(k0 - kb));
    // x and y neighbours of the next plane to update (used only ahead of time)
    double xsa = 0.0, ypa = 0.0, yma = 0.0;
    if constexpr (AHEAD) {
        const uint32_t s = col + pl * (uint32_t)(k0 - kb);
        xsa = ldu(xb, s + (uint32_t)((k0 & 1) ? ox1 : ox0));
        ypa = ldu(xb, s + (uint32_t)oyp);
        yma = ldu(xb, s + (uint32_t)oym);
    }
    for (int ks = k0; ks < k1; ks += UP) {
        double cn[UP], xs[UP], yp[UP], ym[UP], bb[UP], czp[UP], czm[UP];
        uint8_t fl[UP];
#pragma unroll
        for (int u = 0; u < UP; ++u) {
            const int k = min(ks + u, k1 - 1);
            const int kn = min(k + 1, L.nz - 1);
            const uint32_t s = col + pl * (uint32_t)(k - kb), sn = col + pl * (uint32_t)(kn - kb);
            const bool t = k & 1;
            cn[u] = ldu(xb, sn);  // centre of plane k+1
            if constexpr (AHEAD) {  // plane k+1's neighbours
                xs[u] = ldu(xb, sn + (uint32_t)((kn & 1) ? ox1 : ox0));
                yp[u] = ldu(xb, sn + (uint32_t)oyp);
                ym[u] = ldu(xb, sn + (uint32_t)oym);
            } else {  // plane k's
                xs[u] = ldu(xb, s + (uint32_t)(t ? ox1 : ox0));
                yp[u] = ldu(xb, s + (uint32_t)oyp);
                ym[u] = ldu(xb, s + (uint32_t)oym);
            }
            fl[u] = ldu(fb, s);
            bb[u] = ldu(bp, s);
            czp[u] = L.cp[2][k];  // zero at the walls
            czm[u] = L.cm[2][k];
        }
#pragma unroll
        for (int u = 0; u < UP; ++u) {
            const int k = ks + u;
            const double cc = u == 0 ? ccur : cn[u - 1];
            const double cm = u == 0 ? cprev : (u == 1 ? ccur : cn[u - 2]);
            const double xk = !AHEAD ? xs[u] : (u == 0 ? xsa : xs[u - 1]);
            const double ypk = !AHEAD ? yp[u] : (u == 0 ? ypa : yp[u - 1]);
            const double ymk = !AHEAD ? ym[u] : (u == 0 ? yma : ym[u - 1]);
            if (k >= k1) continue;
            const uint32_t s = col + pl * (uint32_t)(k - kb);
            const bool t = k & 1;
            const double cpx = t ? q.cpx[1] : q.cpx[0], cmx = t ? q.cmx[1] : q.cmx[0];
            const int oxp = t ? q.oxp[1] : q.oxp[0], oxm = t ? q.oxm[1] : q.oxm[0];
            const double xpv = oxp == 0 ? cc : xk, xmv = oxm == 0 ? cc : xk;
            const double dg = cpx + cmx + q.cpy + q.cmy + czp[u] + czm[u];
            const double nb = cpx * xpv + cmx * xmv + q.cpy * ypk + q.cmy * ymk + czp[u] * cn[u] + czm[u] * cm;
            if (fl[u] & (F_SOLID | F_MGHOST)) continue;
            double b0 = bb[u];
            if ((long long)s == pin_rel) b0 -= sink[0];
            st_nt(xw + s, (T)((nb - b0) / dg));
        }
        cprev = cn[UP - 2];
        ccur = cn[UP - 1];
        if constexpr (AHEAD) {
            xsa = xs[UP - 1];
            ypa = yp[UP - 1];
            yma = ym[UP - 1];
        }
    }
}

// First level-0 half-sweep of a V-cycle, from a zero iterate: every regular
// cell of colour c gets -b/diag (its neighbours are zero), every other slot
// of colour c gets 0.  Of the other colour only the slots that something
// reads before that colour's own half-sweep are zeroed: solid and padding
// slots, membrane-adjacent cells, and the slots ghost and membrane rows read
// (F_RD); the rest is overwritten by that half-sweep unread, so its stale
// values never count (writing all of it cost a quarter of this kernel's
// bytes).  32-bit offsets from the tile's first plane, non-temporal stores
// (as k0_sweep).
template <class T>
__global__ void __launch_bounds__(TPB) k0_sweep_zero(Lv L, Geo G, long long pin_s, T *__restrict__ xc,
                                                     T *__restrict__ xo, const T *__restrict__ bc,
                                                     const uint8_t *__restrict__ fc, const double *__restrict__ sink,
                                                     int c)
{
    int h, j, k0, k1;
    if (!geo_tile(G, h, j, k0, k1)) return;
    const Col0 q = col0(L, c, h, j);
    const uint32_t pl = (uint32_t)(L.H * L.ny);
    const long long base = (long long)pl * k0;
    const T *bp = bc + base;
    const uint8_t *fb = fc + base, *fo = fc + ((c ? -1 : 1) * L.Nh) + base;
    T *xw = xc + base, *xz = xo + base;
    const uint32_t col = (uint32_t)(h + L.H * j);
    const double snk = pin_s >= 0 ? sink[0] : 0.0;
    const long long pin_rel = pin_s >= 0 ? pin_s - base : -1;
    // the RHS, masks and z coefficients of UZ planes are loaded before any is used
    constexpr int UZ = 4;
    for (int kb = k0; kb < k1; kb += UZ) {
        double bv[UZ], zp[UZ], zm[UZ];
        uint8_t fv[UZ], fz[UZ];
#pragma unroll
        for (int u = 0; u < UZ; ++u) {
            const int k = min(kb + u, k1 - 1);
            const uint32_t s = col + pl * (uint32_t)(k - k0);
            bv[u] = ldu(bp, s);
            fv[u] = ldu(fb, s);
            fz[u] = ldu(fo, s);
            zp[u] = L.cp[2][k];
            zm[u] = L.cm[2][k];
        }
#pragma unroll
        for (int u = 0; u < UZ; ++u) {
            const int k = kb + u;
            if (k >= k1) continue;
            const uint32_t s = col + pl * (uint32_t)(k - k0);
            const bool t = k & 1;
            const double dg = (t ? q.cpx[1] : q.cpx[0]) + (t ? q.cmx[1] : q.cmx[0]) + q.cpy + q.cmy + zp[u] + zm[u];
            double b0 = bv[u];
            if ((long long)s == pin_rel) b0 -= snk;
            st_nt(xw + s, (T)((fv[u] & (F_SOLID | F_MGHOST)) ? 0.0 : -b0 / dg));
            if (fz[u] & (F_SOLID | F_MGHOST | F_RD)) st_nt(xz + s, (T)0.0);
        }
    }
}

// Level-0 operator on the regular cells of both colours: y = A x, or
// y = b - A x with the sink at the pin (RES); membrane cells are left to the
// sparse kernel, solid cells get 0.  Dots of y with u1, u2 (u2 NULL: with y
// itself).
template <int MODE, bool RES>
__device__ __forceinline__ bool apply_out(uint8_t f, double xv, double nsum, double dg, double bv, bool is_pin,
                                          const double *sink, double &out)
{
    if (f & F_MGHOST) return false;
    if (f & F_SOLID) {
        out = 0.0;
        return true;
    }
    double axv = nsum - dg * xv;
    if (is_pin && MODE == M_PINNED) axv = -dg * xv;
    if (is_pin && MODE == M_PINZERO) axv = 0.0;
    if (RES) {
        if (is_pin && sink) bv -= sink[0];
        out = bv - axv;
    } else {
        out = axv;
    }
    return true;
}

// Each thread walks the planes of its (h, j) column for both colours.  The
// cell of one colour and the other colour's slot at the same (h, j, k) are x
// neighbours, and the other colour's slots at (h, j, k -/+ 1) are its z
// neighbours, so the centres of both colours in planes k-1, k, k+1 stay in
// registers and a plane costs one new centre per colour plus the outer x
// neighbour and the two y neighbours.  As in the half-sweep, every load of a
// step is issued unconditionally before any arithmetic (a wall reads the
// cell's partner slot, with a zero coefficient), and addresses are 32-bit
// offsets from block-uniform bases; this keeps the kernel at about 100
// VGPRs in FP64 (4-5 waves per SIMD) where indexing each neighbour with
// 64-bit addresses took over 130 (3 waves).  Two planes per step.  The outer x and
// the y neighbours of plane k+1 are loaded with its centres, one step ahead
// of their use, so that a step's loads fall in the plane being fetched
// (equal time in FP64, 2% faster in FP32, fewer bytes from HBM in both).
template <class T, int MODE, bool RES, int ND>
__global__ void __launch_bounds__(TPB) k0_apply2(Lv L, Geo G, long long pin, const T *__restrict__ x, T *__restrict__ y,
                                                 const T *__restrict__ b, const double *__restrict__ sink,
                                                 const T *__restrict__ u1, const T *__restrict__ u2, double *part,
                                                 int pstride)
{
    constexpr int UA = 2;
    double a0 = 0.0, a1 = 0.0;
    int h, j, k0, k1;
    if (geo_tile(G, h, j, k0, k1)) {
        const uint32_t pl = (uint32_t)(L.H * L.ny);
        const int kb = max(k0 - 1, 0);
        const long long base = (long long)pl * kb, Nh = L.Nh;
        const T *xb[2] = {x + base, x + Nh + base};
        const uint8_t *fb[2] = {L.f + base, L.f + Nh + base};
        // (pointers of operands a variant does not read are never dereferenced)
        const T *ub[2] = {ND >= 1 ? u1 + base : x + base, ND >= 1 ? u1 + Nh + base : x + Nh + base};
        const T *u2p = ND >= 2 ? (u2 ? u2 : u1) : x;  // without u2 the second dot reads u1 again (unused)
        const T *vb[2] = {u2p + base, u2p + Nh + base};
        const T *bb[2] = {RES ? b + base : x + base, RES ? b + Nh + base : x + Nh + base};
        T *yb[2] = {y + base, y + Nh + base};
        const long long prel[2] = {pin - base, pin - Nh - base};
        const uint32_t col = (uint32_t)(h + L.H * j);
        // x coefficients of the pair's cells i = 2h + e and the offset of
        // each one's outer x neighbour (0: the partner, at a wall)
        double cpe[2], cme[2];
        int ope[2], ome[2], oxe[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int i = 2 * h + e;
            const bool xp = i + 1 < L.nx, xm = i > 0 && i < L.nx;
            cpe[e] = xp ? L.cp[0][i] : 0.0;
            cme[e] = xm ? L.cm[0][i] : 0.0;
            ope[e] = xp ? e : 0;
            ome[e] = xm ? e - 1 : 0;
            oxe[e] = ope[e] + ome[e];
        }
        const double cpy = j + 1 < L.ny ? L.cp[1][j] : 0.0, cmy = j > 0 ? L.cm[1][j] : 0.0;
        const int oyp = j + 1 < L.ny ? L.H : 0, oym = j > 0 ? -L.H : 0;
        auto zo = [&](int kk) { return pl * (uint32_t)(kk - kb); };
        // both colours' centres in planes k-1 and k (below the bottom wall:
        // plane k itself)
        double cm0[2], cc0[2], xa[2], ypa[2], yma[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            cm0[c] = ldu(xb[c], col + zo(max(k0 - 1, 0)));
            cc0[c] = ldu(xb[c], col + zo(k0));
        }
        {
            // x and y neighbours of plane k0 (later planes' come one step ahead)
            const uint32_t s = col + zo(k0);
            const int p0 = (j ^ k0) & 1;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int e = c ? 1 - p0 : p0;
                xa[c] = ldu(xb[1 - c], s + (uint32_t)oxe[e]);
                ypa[c] = ldu(xb[1 - c], s + (uint32_t)oyp);
                yma[c] = ldu(xb[1 - c], s + (uint32_t)oym);
            }
        }
        for (int ks = k0; ks < k1; ks += UA) {
            double cn[UA][2], xo[UA][2], yp[UA][2], ym[UA][2], uv[UA][2], wv[UA][2], bv[UA][2], czp[UA], czm[UA];
            uint8_t fv[UA][2];
#pragma unroll
            for (int u = 0; u < UA; ++u) {
                const int k = min(ks + u, k1 - 1);
                const int kn = min(k + 1, L.nz - 1);
                const uint32_t s = col + zo(k), sn = col + zo(kn);
                const int pn = (j ^ kn) & 1;
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int en = c ? 1 - pn : pn;
                    cn[u][c] = ldu(xb[c], sn);  // centre of plane k+1
                    xo[u][c] = ldu(xb[1 - c], sn + (uint32_t)oxe[en]);  // plane k+1's neighbours
                    yp[u][c] = ldu(xb[1 - c], sn + (uint32_t)oyp);
                    ym[u][c] = ldu(xb[1 - c], sn + (uint32_t)oym);
                    fv[u][c] = ldu(fb[c], s);
                    uv[u][c] = ND >= 1 ? (double)ldu(ub[c], s) : 0.0;
                    wv[u][c] = ND >= 2 ? (double)ldu(vb[c], s) : 0.0;
                    bv[u][c] = RES ? (double)ldu(bb[c], s) : 0.0;
                }
                czp[u] = L.cp[2][k];  // zero at the walls
                czm[u] = L.cm[2][k];
            }
#pragma unroll
            for (int u = 0; u < UA; ++u) {
                const int k = ks + u;
                if (k >= k1) continue;
                const uint32_t s = col + zo(k);
                const int p0 = (j ^ k) & 1;
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int e = c ? 1 - p0 : p0;
                    const int o = 1 - c;
                    // the other colour's centres: plane k (x partner), k-1 and k+1 (z)
                    const double pc = u == 0 ? cc0[o] : cn[u - 1][o];
                    const double pm = u == 0 ? cm0[o] : (u == 1 ? cc0[o] : cn[u - 2][o]);
                    const double pp = cn[u][o];
                    const double xk = u == 0 ? xa[c] : xo[u - 1][c];
                    const double ypk = u == 0 ? ypa[c] : yp[u - 1][c], ymk = u == 0 ? yma[c] : ym[u - 1][c];
                    const double xpv = ope[e] == 0 ? pc : xk, xmv = ome[e] == 0 ? pc : xk;
                    const double nsum = cpe[e] * xpv + cme[e] * xmv + cpy * ypk + cmy * ymk + czp[u] * pp +
                                        czm[u] * pm;
                    const double dg = cpe[e] + cme[e] + cpy + cmy + czp[u] + czm[u];
                    const double xv = u == 0 ? cc0[c] : cn[u - 1][c];
                    double out;
                    if (apply_out<MODE, RES>(fv[u][c], xv, nsum, dg, bv[u][c], (long long)s == prel[c], sink, out)) {
                        st_nt(yb[c] + s, (T)out);  // y is next read by another kernel, long after it left the caches
                        const double yo = round_to<T>(out);  // the stored value
                        if (ND >= 1) a0 += uv[u][c] * yo;
                        if (ND >= 2) a1 += (u2 ? wv[u][c] : yo) * yo;
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                cm0[c] = cn[UA - 2][c];
                cc0[c] = cn[UA - 1][c];
                xa[c] = xo[UA - 1][c];
                ypa[c] = yp[UA - 1][c];
                yma[c] = ym[UA - 1][c];
            }
        }
    }
    if constexpr (ND == 1) {
        Acc<1> r;
        r.v[0] = a0;
        block_reduce<1>(r, part, pstride, blockIdx.x);
    } else if constexpr (ND == 2) {
        Acc<2> r;
        r.v[0] = a0;
        r.v[1] = a1;
        block_reduce<2>(r, part, pstride, blockIdx.x);
    }
}

// One weighted-Jacobi sweep of the pinned system on the regular level-0
// rows of both colours: xn = xo + w (b - A xo) / diag(A), diag = -(sum of the
// face coefficients); solid cells and padding get 0; ghost and membrane rows
// are left to k0_jacobi_sparse.  Every row reads xo only.
template <class T>
__global__ void __launch_bounds__(TPB) k0_jacobi(Lv L, Geo G, long long pin, const T *__restrict__ xo,
                                                 T *__restrict__ xn, const T *__restrict__ b, double w)
{
    int h, j, k0, k1;
    if (!geo_tile(G, h, j, k0, k1)) return;
    const long long pl = (long long)L.H * L.ny, Nh = L.Nh;
    const long long col = h + (long long)L.H * j;
    const Col0 q0 = col0(L, 0, h, j), q1 = col0(L, 1, h, j);
    constexpr int UJ = 2;
    for (int kb = k0; kb < k1; kb += UJ) {
        uint8_t f[UJ][2];
        double xv[UJ][2], nb[UJ][2], dg[UJ][2], bv[UJ][2];
#pragma unroll
        for (int u = 0; u < UJ; ++u) {
            const int k = min(kb + u, k1 - 1);
            const long long s = col + pl * k, t = Nh + s;
            f[u][0] = L.f[s];
            f[u][1] = L.f[t];
            xv[u][0] = ld(xo, s);
            xv[u][1] = ld(xo, t);
            nb[u][0] = col0_sum(L, q0, xo + Nh, s, k, pl, dg[u][0]);
            nb[u][1] = col0_sum(L, q1, xo, s, k, pl, dg[u][1]);
            bv[u][0] = ld(b, s);
            bv[u][1] = ld(b, t);
        }
#pragma unroll
        for (int u = 0; u < UJ; ++u) {
            if (kb + u >= k1) continue;
            const long long s0 = col + pl * (kb + u);
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
                const long long sc = s0 + (cc ? Nh : 0);
                const uint8_t ff = f[u][cc];
                if (ff & F_MGHOST) continue;
                if (ff & F_SOLID) {
                    if (!(ff & F_GHOST)) st(xn, sc, 0.0);
                    continue;
                }
                const double ax = sc == pin ? -dg[u][cc] * xv[u][cc] : nb[u][cc] - dg[u][cc] * xv[u][cc];
                st(xn, sc, xv[u][cc] + w * (bv[u][cc] - ax) / (-dg[u][cc]));
            }
        }
    }
}

// the same sweep on the ghost rows (diag -sG) and the membrane rows
template <class T>
__global__ void __launch_bounds__(TPB) k0_jacobi_sparse(Lv L, Sp S, const T *xo, T *xn, const T *b, double w)
{
    const int n = S.nrows + S.nm;
    for (int r = blockIdx.x * TPB + threadIdx.x; r < n; r += gridDim.x * TPB) {
        if (r < S.nrows) {
            const long long u = ghost_unknown(S, r);
            const double xu = ld(xo, u);
            const double ax = S.rsG[r] * (ghost_sum(S, xo, r) - xu);
            st(xn, u, xu + w * (ld(b, u) - ax) / (-S.rsG[r]));
        } else {
            const int m = r - S.nrows;
            const long long u = S.mslot[m];
            const double xu = ld(xo, u);
            double sd;
            const double ax = mrow(L, S, xo, m, xu, sd);
            st(xn, u, xu + w * (ld(b, u) - ax) / (-sd));
        }
    }
}

// stencil of ghost row r (8 columns, 8 weights) by 16-byte loads
__device__ __forceinline__ void ghost_stencil(const Sp &S, int r, int32_t (&gc)[8], double (&gw)[8])
{
    const int4 *c4 = reinterpret_cast<const int4 *>(S.rcol + 8 * (long long)r);
    const double2 *w2 = reinterpret_cast<const double2 *>(S.rw + 8 * (long long)r);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int4 q = c4[t];
        gc[4 * t] = q.x; gc[4 * t + 1] = q.y; gc[4 * t + 2] = q.z; gc[4 * t + 3] = q.w;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const double2 q = w2[t];
        gw[2 * t] = q.x; gw[2 * t + 1] = q.y;
    }
}

// sum w x over a preloaded ghost stencil, in column order (as ghost_sum)
template <class T>
__device__ __forceinline__ double stencil_sum(const T *x, long long fallback, const int32_t (&gc)[8], const double (&gw)[8])
{
    double xv[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) xv[t] = ld(x, gc[t] >= 0 ? (long long)gc[t] : fallback);
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < 8; ++t)
        if (gc[t] >= 0) acc += gw[t] * xv[t];
    return acc;
}

// membrane-adjacent cells of one colour (after the dense half-sweep): across
// a cut link the neighbour's ghost unknown is eliminated, i.e. replaced by
// the current value of its stencil, sum w x - b/sG
// All cells of the colour read the same iterate (their eliminated stencils
// may reach each other): new values go to tmp, k0_mscat_gjac writes them.
// The loads go out in batches (the row's indices; the direct neighbours and
// the stencils of its first two cut links; the stencil values), so a row
// waits on three dependent steps rather than on one per neighbour; a third
// or later cut link takes the plain path.  The arithmetic and its order are
// those of ghost_sum.
template <class T>
__global__ void __launch_bounds__(TPB) k0_msweep(Lv L, Sp S, const T *x, const T *b, int color, double *tmp)
{
    for (int m = blockIdx.x * TPB + threadIdx.x; m < S.nm; m += gridDim.x * TPB) {
        const int mcl = S.mcolor[m];
        const long long u = S.mslot[m];
        int32_t mc[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) mc[q] = S.mcol[6 * m + q];
        if (mcl != color) continue;
        int c, h, j, k, i;
        decode_slot(L, u, c, h, j, k, i);
        const double cf[6] = {L.cm[0][i], L.cp[0][i], L.cm[1][j], L.cp[1][j], L.cm[2][k], L.cp[2][k]};
        const double bu = ld(b, u);
        // direct neighbours (a wall or cut link reads the row's own slot, unused)
        // and the ghost rows of the first two cut links
        double v[6];
        int ra = -1, rb = -1;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int32_t col = mc[q];
            v[q] = ld(x, col >= 0 && col < S.N2 ? (long long)col : u);
            if (col >= S.N2) {
                const int r = S.ng + (int)(col - S.N2);
                if (ra < 0) ra = r;
                else if (rb < 0) rb = r;
            }
        }
        int32_t ca[8], cb[8];
        double wa[8], wb[8], ba = 0.0, bb = 0.0, sa = 1.0, sb = 1.0;
        if (ra >= 0) {
            ghost_stencil(S, ra, ca, wa);
            ba = ld(b, S.N2 + (ra - S.ng));
            sa = S.rsG[ra];
        }
        if (rb >= 0) {
            ghost_stencil(S, rb, cb, wb);
            bb = ld(b, S.N2 + (rb - S.ng));
            sb = S.rsG[rb];
        }
        const double va = ra >= 0 ? stencil_sum(x, u, ca, wa) - ba / sa : 0.0;
        const double vb = rb >= 0 ? stencil_sum(x, u, cb, wb) - bb / sb : 0.0;
        double off = 0.0, s = 0.0;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int32_t col = mc[q];
            if (col < 0) continue;
            double val = v[q];
            if (col >= S.N2) {
                const int r = S.ng + (int)(col - S.N2);
                val = r == ra ? va : r == rb ? vb : ghost_sum(S, x, r) - ld(b, col) / S.rsG[r];
            }
            off += cf[q] * val;
            s += cf[q];
        }
        tmp[m] = (off - bu) / s;
    }
}

// After the membrane cells of one colour: their new values (staged in mtmp
// by k0_msweep) are written to x, and in the same launch one Jacobi update
// of every ghost unknown is staged in gtmp (k0_gscat writes it).  The ghost
// rows must see the colour's new membrane values, which other threads of
// this launch are writing: a stencil column that is a membrane cell of the
// colour (rmrow) takes its value from mtmp, rounded to T as the store
// rounds it, so the result is that of scattering first.  Sum in column
// order (as ghost_sum).
template <class T>
__global__ void __launch_bounds__(TPB) k0_mscat_gjac(Sp S, T *x, const T *b, int color, const double *mtmp,
                                                     double *gtmp)
{
    const int n = S.nrows + S.nm;
    const long long Nh = S.N2 >> 1;
    for (int r = blockIdx.x * TPB + threadIdx.x; r < n; r += gridDim.x * TPB) {
        if (r >= S.nrows) {
            const int m = r - S.nrows;
            if (S.mcolor[m] == color) st(x, S.mslot[m], mtmp[m]);
            continue;
        }
        const double bv = ld(b, ghost_unknown(S, r)), sg = S.rsG[r];
        int32_t gc[8], gm[8];
        double gw[8], xv[8];
        ghost_stencil(S, r, gc, gw);
        if (S.nm) {
            const int4 *m4 = reinterpret_cast<const int4 *>(S.rmrow + 8 * (long long)r);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int4 q = m4[t];
                gm[4 * t] = q.x; gm[4 * t + 1] = q.y; gm[4 * t + 2] = q.z; gm[4 * t + 3] = q.w;
            }
        } else {
#pragma unroll
            for (int t = 0; t < 8; ++t) gm[t] = -1;
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const bool fresh = gm[t] >= 0 && (gc[t] >= Nh) == (color == 1);
            xv[t] = fresh ? round_to<T>(mtmp[gm[t]]) : ld(x, gc[t] >= 0 ? (long long)gc[t] : 0LL);
        }
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (gc[t] >= 0) acc += gw[t] * xv[t];
        gtmp[r] = acc - bv / sg;
    }
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
        double off = nbsum_all(F, x + (long long)(1 - cf) * F.Nh, h, j, k, i, f, dg);
        r = ld(b, so + s) - (bsh ? bsh[0] : 0.0) - (off - dg * ld(x, so + s));
        return true;
    }
}

// fused residual + restriction: coarse RHS = the volume integral of the
// active children's residuals divided by the full coarse-cell volume (the
// coarse operator is per full volume); partial sums of V_C b_C for the
// coarse mean
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
    const double VC = C.w[0][I] * C.w[1][J] * C.w[2][K];
    st(bc, sc, sv > 0.0 ? svr / VC : 0.0);
    return (C.f[sc] & 1) ? VC * ld(bc, sc) : 0.0;
}

// restrict_one<false> for a coarse level in global memory, with the loads of
// all 8 children issued before any is used: the 2x2x2 box, the 3 outer face
// neighbours of each child (outside the level: the child itself, whose face
// is closed in the mask), their RHS and masks, and the coefficients.  Same
// arithmetic in the same order.
template <class T, class TB, class TBc>
__device__ __forceinline__ double restrict_box(const Lv &F, const Lv &C, const T *x, const TB *b, double mu, TBc *bc,
                                               int cc, int hc, int J, int K)
{
    const long long sc = slot(C, cc, hc, J, K);
    const int I = 2 * hc + ((cc + J + K) & 1);
    if (I >= C.nx) {
        st(bc, sc, 0.0);
        return 0.0;
    }
    const uint8_t fC = C.f[sc];
    const long long H = F.H, ny = F.ny;
    T xb[8], xn[8][3];
    uint8_t fb[8];
    double bb[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int dx = q & 1, dy = (q >> 1) & 1, dz = q >> 2;
        const int i = 2 * I + dx, j = 2 * J + dy, k = 2 * K + dz;
        const int c = (dx + dy + dz) & 1;
        const long long so = (long long)(1 - c) * F.Nh;
        const long long s = (long long)c * F.Nh + I + H * (j + ny * k);
        const int io = dx ? i + 1 : i - 1, jo = dy ? j + 1 : j - 1, ko = dz ? k + 1 : k - 1;
        const long long sx = io >= 0 && io < F.nx ? so + (io >> 1) + H * (j + ny * k) : s;
        const long long sy = jo >= 0 && jo < F.ny ? so + I + H * (jo + ny * k) : s;
        const long long sz = ko >= 0 && ko < F.nz ? so + I + H * (j + ny * ko) : s;
        xb[q] = x[s];
        fb[q] = F.f[s];
        bb[q] = ld(b, s);
        xn[q][0] = x[sx];
        xn[q][1] = x[sy];
        xn[q][2] = x[sz];
    }
    double cpx[2], cmx[2], cpy[2], cmy[2], cpz[2], cmz[2], w0[2], w1[2], w2[2];
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        cpx[d] = F.cp[0][2 * I + d];
        cmx[d] = F.cm[0][2 * I + d];
        cpy[d] = F.cp[1][2 * J + d];
        cmy[d] = F.cm[1][2 * J + d];
        cpz[d] = F.cp[2][2 * K + d];
        cmz[d] = F.cm[2][2 * K + d];
        w0[d] = F.w[0][2 * I + d];
        w1[d] = F.w[1][2 * J + d];
        w2[d] = F.w[2][2 * K + d];
    }
    double sv = 0.0, svr = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int dx = q & 1, dy = (q >> 1) & 1, dz = q >> 2;
        const uint8_t f = fb[q];
        if (!(f & 1)) continue;
        // face values in the order of nbsum: +x, -x, +y, -y, +z, -z
        const double vpx = dx ? (double)xn[q][0] : (double)xb[q ^ 1], vmx = dx ? (double)xb[q ^ 1] : (double)xn[q][0];
        const double vpy = dy ? (double)xn[q][1] : (double)xb[q ^ 2], vmy = dy ? (double)xb[q ^ 2] : (double)xn[q][1];
        const double vpz = dz ? (double)xn[q][2] : (double)xb[q ^ 4], vmz = dz ? (double)xb[q ^ 4] : (double)xn[q][2];
        double acc = 0.0, d = 0.0;
        if (f & CM_PX) { acc += cpx[dx] * vpx; d += cpx[dx]; }
        if (f & CM_MX) { acc += cmx[dx] * vmx; d += cmx[dx]; }
        if (f & CM_PY) { acc += cpy[dy] * vpy; d += cpy[dy]; }
        if (f & CM_MY) { acc += cmy[dy] * vmy; d += cmy[dy]; }
        if (f & CM_PZ) { acc += cpz[dz] * vpz; d += cpz[dz]; }
        if (f & CM_MZ) { acc += cmz[dz] * vmz; d += cmz[dz]; }
        const double r = bb[q] - mu - (acc - d * (double)xb[q]);
        const double V = w0[dx] * w1[dy] * w2[dz];
        sv += V;
        svr += V * r;
    }
    const double VC = C.w[0][I] * C.w[1][J] * C.w[2][K];
    st(bc, sc, sv > 0.0 ? svr / VC : 0.0);
    return (fC & 1) ? VC * ld(bc, sc) : 0.0;
}

// one thread per coarse cell in natural x order (Gc tiles I over C.nx), so a
// wave reads the children's rows with unit stride
template <bool FINE, class T, class TB, class TBc>
__global__ void __launch_bounds__(TPB) k_restrict(Lv F, Lv C, Geo Gc, long long pin, const T *x, const TB *b,
                                                  const double *bsh, const T *rsp, TBc *bc, double *part)
{
    Acc<1> a;
    a.v[0] = 0.0;
    int I, J, k0, k1;
    if (geo_tile(Gc, I, J, k0, k1)) {
        const double mu = FINE ? 0.0 : (bsh ? bsh[0] : 0.0);
        for (int K = k0; K < k1; ++K) {
            const int cc = (I + J + K) & 1;
            if constexpr (FINE)
                a.v[0] += restrict_one<FINE>(F, C, pin, x, b, bsh, rsp, bc, cc, I >> 1, J, K);
            else
                a.v[0] += restrict_box(F, C, x, b, mu, bc, cc, I >> 1, J, K);
        }
    }
    block_reduce<1>(a, part, 0, blockIdx.x);
}

// Level-0 residual of the unpinned system (sink at the pin) fused with its
// restriction into level 1: one thread per coarse (I, J) column walks its K
// range; the 8 children of coarse cell (I, J, K) are half-index I of both
// colours in rows 2J, 2J+1 and planes 2K, 2K+1.  The thread steps through
// the fine planes with both colours' values of the two rows in planes k-1,
// k, k+1 in registers (one new plane per step); the outer x and y
// neighbours of a plane's four children are loaded one plane ahead, with the
// window plane they lie in (loaded a step later they missed the L2 and the
// kernel read 1.36x its algorithmic bytes; now 1.09x).  Children that carry
// a ghost or membrane row take their residual from rsp (written by
// k0_sparse_res).  Coarse RHS = volume-weighted mean over the active
// children, added in child order; partial sums of V_C b_C for the coarse
// mean.
template <class T, class TBc>
__global__ void __launch_bounds__(TPB) k0_restrict_res(Lv F, Lv C, Geo Gc, long long pin, const T *__restrict__ x,
                                                       const T *__restrict__ b, const double *__restrict__ sink,
                                                       const T *__restrict__ rsp, TBc *__restrict__ bc, double *part)
{
    Acc<1> a;
    a.v[0] = 0.0;
    int I, J, k0, k1;
    if (geo_tile(Gc, I, J, k0, k1)) {
        J = __builtin_amdgcn_readfirstlane(J);  // one coarse row per wave
        const long long Nh = F.Nh, H = F.H, pl = H * F.ny;
        typedef T R;  // arithmetic in the precision of the level-0 vectors
        const R snk = sink ? (R)sink[0] : (R)0;
        // x: coefficients of the two cells i = 2I + dx; the outer neighbour of
        // i = 2I is half I-1, of i = 2I+1 half I+1 (clamped, zero coefficient)
        R cpx[2], cmx[2], wx[2];
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
            const int i = 2 * I + dx;
            cpx[dx] = i + 1 < F.nx ? (R)F.cp[0][i] : (R)0;
            cmx[dx] = i > 0 ? (R)F.cm[0][i] : (R)0;
            wx[dx] = (R)F.w[0][i];
        }
        const int hm = I > 0 ? I - 1 : I, hp = 2 * I + 2 < F.nx ? I + 1 : I;
        R cpy[2], cmy[2], wy[2];
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
            const int j = 2 * J + dy;
            cpy[dy] = j + 1 < F.ny ? (R)F.cp[1][j] : (R)0;
            cmy[dy] = j > 0 ? (R)F.cm[1][j] : (R)0;
            wy[dy] = (R)F.w[1][j];
        }
        // every load of this thread is within fine planes [kb, 2 k1]: block-uniform
        // per-colour bases and 32-bit offsets from them
        const int kb = max(2 * k0 - 1, 0);
        const T *xb[2] = {x + pl * kb, x + Nh + pl * kb};
        const T *bb[2] = {b + pl * kb, b + Nh + pl * kb};
        const T *rb[2] = {rsp + pl * kb, rsp + Nh + pl * kb};
        const uint8_t *fb[2] = {F.f + pl * kb, F.f + Nh + pl * kb};
        const uint32_t rowm = (uint32_t)(H * max(2 * J - 1, 0)), row0 = (uint32_t)(H * (2 * J)),
                       row1 = (uint32_t)(H * (2 * J + 1)), rowp = (uint32_t)(H * min(2 * J + 2, F.ny - 1));
        const uint32_t pl32 = (uint32_t)pl;
        auto zoff = [&](int kk) { return pl32 * (uint32_t)(min(max(kk, 0), F.nz - 1) - kb); };
        // w[c][dy][t]: colour c, row 2J+dy, fine planes k-1, k, k+1 of the
        // current fine plane k (clamped at the walls, zero coefficient)
        T w[2][2][3];
        auto ldcol = [&](int kk, int t) {
            const uint32_t z = zoff(kk);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                w[c][0][t] = ldu(xb[c], I + row0 + z);
                w[c][1][t] = ldu(xb[c], I + row1 + z);
            }
        };
        ldcol(2 * k0 - 1, 0);
        ldcol(2 * k0, 1);
        // outer x and y neighbours of the 4 children of a fine plane, loaded
        // one plane ahead (with the window plane they lie in)
        auto ldnb = [&](int kk, int par, T (&xo4)[4], T (&yo4)[4]) {
            const uint32_t zk = zoff(kk);
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const int dx = qq & 1, dy = qq >> 1;
                const int o = 1 - ((dx + dy + par) & 1);
                xo4[qq] = ldu(xb[o], (dx ? hp : hm) + (dy ? row1 : row0) + zk);
                yo4[qq] = ldu(xb[o], I + (dy ? rowp : rowm) + zk);
            }
        };
        T xa[4], ya[4];
        ldnb(2 * k0, 0, xa, ya);
        const double wIJ = C.w[0][I] * C.w[1][J];
        for (int K = k0; K < k1; ++K) {
            const long long sc = slot(C, (I + J + K) & 1, I >> 1, J, K);
            const uint8_t fc = C.f[sc];
            const double wK = C.w[2][K];
            R sv = 0, svr = 0;
#pragma unroll
            for (int dz = 0; dz < 2; ++dz) {
                const int k = 2 * K + dz;
                ldcol(k + 1, 2);
                T xn[4], yn[4];
                ldnb(k + 1, (dz + 1) & 1, xn, yn);
                const R czp = (R)F.cp[2][k], czm = (R)F.cm[2][k], wz = (R)F.w[2][k];  // zero at the walls
                const uint32_t zk = zoff(k);
                uint8_t fq[4];
                T bq[4], xq[4], yq[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int dx = q & 1, dy = q >> 1;
                    const int c = (dx + dy + dz) & 1, o = 1 - c;
                    const uint32_t s = I + (dy ? row1 : row0) + zk;
                    fq[q] = ldu(fb[c], s);
                    bq[q] = ldu(bb[c], s);
                    xq[q] = xa[q];
                    yq[q] = ya[q];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int dx = q & 1, dy = q >> 1;
                    const int c = (dx + dy + dz) & 1, o = 1 - c;
                    const uint8_t f = fq[q];
                    if (!active0(f)) continue;
                    R r;
                    const uint32_t s = I + (dy ? row1 : row0) + zk;
                    if (f & (F_GHOST | F_MGHOST)) {
                        r = ldu(rb[c], s);
                    } else {
                        const R xv = w[c][dy][1];
                        const R xin = w[o][dy][1];
                        const R xout = xq[q];
                        const R xpx = dx ? xout : xin, xmx = dx ? xin : xout;
                        const R xpy = dy ? yq[q] : w[o][1][1];
                        const R xmy = dy ? w[o][0][1] : yq[q];
                        const R xpz = w[o][dy][2], xmz = w[o][dy][0];
                        const R dg = cpx[dx] + cmx[dx] + cpy[dy] + cmy[dy] + czp + czm;
                        const R n = cpx[dx] * xpx + cmx[dx] * xmx + cpy[dy] * xpy + cmy[dy] * xmy + czp * xpz +
                                    czm * xmz;
                        R bv = bq[q];
                        if (c * Nh + pl * kb + s == pin) bv -= snk;
                        r = bv - (n - dg * xv);
                    }
                    const R V = wx[dx] * wy[dy] * wz;
                    sv += V;
                    svr += V * r;
                }
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int d = 0; d < 2; ++d) {
                        w[c][d][0] = w[c][d][1];
                        w[c][d][1] = w[c][d][2];
                    }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    xa[q] = xn[q];
                    ya[q] = yn[q];
                }
            }
            const double vc = wIJ * wK;  // coarse cell volume
            st(bc, sc, sv > 0 ? (double)(svr / (R)vc) : 0.0);
            if (fc & 1) a.v[0] += vc * ld(bc, sc);
        }
    }
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

template <class Tc>
__device__ __forceinline__ double coarse_act(const Lv &C, int I, int J, int K)
{
    return (C.f[slot(C, (I + J + K) & 1, I >> 1, J, K)] & 1) ? 1.0 : 0.0;
}

// trilinear interpolation (physical coordinates) of the coarse correction at
// one fine cell over the active coarse nodes, weights renormalised (an
// inactive node, inside a body, carries no correction)
template <class Tc>
__device__ __forceinline__ double interp(const Lv &C, const PMap &M, const Tc *xc, int i, int j, int k)
{
    const int I = M.pi[0][i], J = M.pi[1][j], K = M.pi[2][k];
    const double tx = M.pt[0][i], ty = M.pt[1][j], tz = M.pt[2][k];
    double num = 0.0, den = 0.0;
    int na = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int dx = q & 1, dy = (q >> 1) & 1, dz = q >> 2;
        const double w = (dz ? tz : 1 - tz) * (dy ? ty : 1 - ty) * (dx ? tx : 1 - tx);
        const double a = coarse_act<Tc>(C, I + dx, J + dy, K + dz);
        num += w * a * coarse_val(C, xc, I + dx, J + dy, K + dz);
        den += w * a;
        na += a > 0.0;
    }
    if (na < 8) return den > 0.0 ? num / den : 0.0;
    // all nodes active: the plain trilinear form (its weights sum to one)
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

// Prolongation by coarse column: one thread per coarse (I, J) column walks
// its K range with the 3x3 coarse neighbourhoods of planes K-1, K, K+1 in
// registers (one new plane per step) and corrects the 8 children of each
// coarse cell: trilinear in physical coordinates over the active coarse
// nodes (weights renormalised), clamped at the walls, in the precision of
// the fine iterate.
// SKIP_RED: the red half-sweep that follows overwrites every regular red
// cell without reading it, so only black slots (and, on level 0, the red
// ghost and membrane cells, which later rows read) receive the correction.
// RENORM: the coarse level has inactive cells, so weights are renormalised
// over the active nodes (without inactive cells the plain trilinear weights
// are the same and the activity loads are skipped).
template <bool FINE, class Tc, class Tf, bool SKIP_RED, bool RENORM>
__global__ void __launch_bounds__(TPB) k_prolong_z(Lv F, Lv C, PMap M, Geo Gc, const Tc *__restrict__ xc,
                                                   Tf *__restrict__ xf)
{
    typedef Tf R;
    int I, J, k0, k1;
    if (!geo_tile(Gc, I, J, k0, k1)) return;
    const int Ie[3] = {max(I - 1, 0), I, min(I + 1, C.nx - 1)};
    const int Jb[3] = {max(J - 1, 0), J, min(J + 1, C.ny - 1)};
    // coarse values (zero where inactive) and activity (0/1) of the 3x3
    // neighbourhoods of planes K-1, K, K+1
    R va[3][3], vb[3][3], vn[3][3], aa[3][3], ab[3][3], an[3][3];
    auto plane = [&](int kk, R (&v)[3][3], R (&a)[3][3]) {
        const long long zo = (long long)C.H * C.ny * kk;
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                const long long sc = (((Ie[e] + Jb[b] + kk) & 1) ? C.Nh : 0) + (Ie[e] >> 1) +
                                     (long long)C.H * Jb[b] + zo;
                if constexpr (RENORM) {
                    a[b][e] = (C.f[sc] & 1) ? (R)1 : (R)0;
                    v[b][e] = a[b][e] * (R)ld(xc, sc);
                } else {
                    v[b][e] = (R)ld(xc, sc);
                }
            }
    };
    // per child direction: does the 2-point box start at the cell (offset 1)
    // or at its lower neighbour (offset 0), and the weight of the upper point
    bool ex[2], ey[2];
    R tx[2], ty[2];
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        ex[d] = M.pi[0][2 * I + d] != I - 1;
        tx[d] = (R)M.pt[0][2 * I + d];
        ey[d] = M.pi[1][2 * J + d] != J - 1;
        ty[d] = (R)M.pt[1][2 * J + d];
    }
    const long long fpl = (long long)F.H * F.ny;
    plane(max(k0 - 1, 0), va, aa);
    plane(k0, vb, ab);
    for (int K = k0; K < k1; ++K) {
        plane(min(K + 1, C.nz - 1), vn, an);
        // flags of the 8 children and the values to be corrected, issued
        // together (red values only when they are corrected at all)
        uint8_t fq[8];
        Tf xq[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int dx = q & 1, dy = (q >> 1) & 1, dz = q >> 2;
            const int cf = (dx + dy + dz) & 1;
            const long long s = (long long)cf * F.Nh + I + (long long)F.H * (2 * J + dy) + fpl * (2 * K + dz);
            fq[q] = F.f[s];
            if (!SKIP_RED || cf == 1) xq[q] = xf[s];
        }
#pragma unroll
        for (int dz = 0; dz < 2; ++dz) {
            const int k = 2 * K + dz;
            const bool ez = M.pi[2][k] != K - 1;
            const R tz = (R)M.pt[2][k];
            // z, then y, then x, for the values and for the weights
            R zz[3][3], zw[3][3];
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    zz[b][e] = ez ? (1 - tz) * vb[b][e] + tz * vn[b][e] : (1 - tz) * va[b][e] + tz * vb[b][e];
                    if constexpr (RENORM)
                        zw[b][e] = ez ? (1 - tz) * ab[b][e] + tz * an[b][e] : (1 - tz) * aa[b][e] + tz * ab[b][e];
                }
#pragma unroll
            for (int dy = 0; dy < 2; ++dy) {
                R yy[3], yw[3];
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    yy[e] = ey[dy] ? (1 - ty[dy]) * zz[1][e] + ty[dy] * zz[2][e]
                                   : (1 - ty[dy]) * zz[0][e] + ty[dy] * zz[1][e];
                    if constexpr (RENORM)
                        yw[e] = ey[dy] ? (1 - ty[dy]) * zw[1][e] + ty[dy] * zw[2][e]
                                       : (1 - ty[dy]) * zw[0][e] + ty[dy] * zw[1][e];
                }
#pragma unroll
                for (int dx = 0; dx < 2; ++dx) {
                    const int q = dx + 2 * dy + 4 * dz;
                    const int cf = (dx + dy + dz) & 1;
                    const long long s = (long long)cf * F.Nh + I + (long long)F.H * (2 * J + dy) + fpl * k;
                    const uint8_t f = fq[q];
                    if (FINE ? !active0(f) : !(f & 1)) continue;
                    Tf xv;
                    if (SKIP_RED && cf == 0) {
                        if (!FINE || !(f & (F_GHOST | F_MGHOST))) continue;
                        xv = xf[s];
                    } else {
                        xv = xq[q];
                    }
                    const R num = ex[dx] ? (1 - tx[dx]) * yy[1] + tx[dx] * yy[2] : (1 - tx[dx]) * yy[0] + tx[dx] * yy[1];
                    if constexpr (RENORM) {
                        const R den = ex[dx] ? (1 - tx[dx]) * yw[1] + tx[dx] * yw[2]
                                             : (1 - tx[dx]) * yw[0] + tx[dx] * yw[1];
                        xf[s] = (Tf)((R)xv + (den > (R)0 ? num / den : (R)0));
                    } else {
                        xf[s] = (Tf)((R)xv + num);
                    }
                }
            }
        }
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                va[b][e] = vb[b][e];
                vb[b][e] = vn[b][e];
                if constexpr (RENORM) {
                    aa[b][e] = ab[b][e];
                    ab[b][e] = an[b][e];
                }
            }
    }
}

// ---------------------------------------------------------------- coarse tail in one workgroup
// The smallest levels run as one 1024-thread block with their masks, iterates
// and right-hand sides staged in LDS: the same operations as the grid
// kernels, separated by block barriers; the coarse means are block
// reductions.  Only the first tail level's RHS comes from global memory and
// only its iterate goes back.
constexpr int TAIL_T = 1024;
static_assert(TAIL_T >= 8 * 128, "the tail stages each of up to 8 levels with 128 threads");
constexpr int TAIL_LDS = 60 * 1024;  // bytes of dynamic LDS the tail may use

struct TailLevel {
    Lv L;             // global views (coefficients, maps); L.f is replaced by the LDS mask
    PMap M;           // prolongation onto this level from the next one
    double volA;
    void *xg;         // global iterate of the first tail level
    const void *bg;   // global RHS of the first tail level
    int moff, xoff, boff;  // LDS byte offsets
};
struct Tail {
    int n;            // levels in the tail (>= 1)
    TailLevel t[8];
    int nu1, nu2, ncs;
    int coff;         // LDS byte offset of the levels' coefficient copies
};

// LDS bytes of one tail level's coefficient copies: cp, cm, w and the
// prolongation weights pt (double), then the map pi (int), per axis
__host__ __device__ inline int tail_coef_bytes(int nx, int ny, int nz)
{
    return (36 * (nx + ny + nz) + 15) / 16 * 16;
}

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

template <class Tc>
__device__ void tail_sweep(const Lv &L, Tc *x, const Tc *b, double mu, int c, bool zero)
{
    const int n = L.H * L.ny * L.nz;  // a tail level fits in LDS: 32-bit indices
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        const int row = (int)fdiv((uint32_t)q, L.fH), h = q - row * L.H;
        const int k = (int)fdiv((uint32_t)row, L.fy), j = row - k * L.ny;
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
            off = nbsum_all(L, x + (long long)(1 - c) * L.Nh, h, j, k, i, f, dg);
        }
        st(x, s, dg > 0.0 ? (off - (ld(b, s) - mu)) / dg : 0.0);
    }
    __syncthreads();
}

// A coarsest level of at most 64 cells per colour runs its sweeps in one
// wavefront: each lane keeps its cell's open-face neighbour offsets, face
// coefficients, diagonal and b - mu in registers, and the half-sweeps are
// separated by wavefront barriers instead of block barriers.  Same
// operations, in the same order, as tail_sweep.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class Tc>
__device__ void tail_coarsest_wave(const Lv &L, Tc *x, const Tc *b, double mu, int steps)
{
    const int lane = threadIdx.x & 63;
    const int n = L.H * L.ny * L.nz;  // <= 64
    // a closed face keeps the cell's own slot with a zero coefficient, so the
    // six loads of a half-sweep go out without branches (adding zero
    // products leaves the sum as it was)
    int nb[2][6];
    double cf[2][6], dg[2], bm[2];
    bool act[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        act[c] = false;
        dg[c] = bm[c] = 0.0;
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            nb[c][t] = c * (int)L.Nh;
            cf[c][t] = 0.0;
        }
        if (lane >= n) continue;
        const int row = (int)fdiv((uint32_t)lane, L.fH), h = lane - row * L.H;
        const int k = (int)fdiv((uint32_t)row, L.fy), j = row - k * L.ny;
        const int s = c * (int)L.Nh + lane;
        const uint8_t f = L.f[s];
        const int i = 2 * h + ((c + j + k) & 1);
        if (!(f & 1) || i >= L.nx) continue;
        act[c] = true;
        const int p = i & 1, o = (1 - c) * (int)L.Nh + L.H * (j + L.ny * k) + h;
        const int pl = L.H * L.ny;
        const uint8_t bit[6] = {CM_PX, CM_MX, CM_PY, CM_MY, CM_PZ, CM_MZ};
        const int off[6] = {p, p - 1, L.H, -L.H, pl, -pl};
        const double cv[6] = {L.cp[0][i], L.cm[0][i], L.cp[1][j], L.cm[1][j], L.cp[2][k], L.cm[2][k]};
        double d = 0.0;
#pragma unroll
        for (int t = 0; t < 6; ++t)
            if (f & bit[t]) {
                nb[c][t] = o + off[t];
                cf[c][t] = cv[t];
                d += cv[t];
            } else {
                nb[c][t] = o;
            }
        dg[c] = d;
        bm[c] = ld(b, s) - mu;
    }
    for (int it = 0; it < steps; ++it) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (act[c]) {
                double acc = 0.0;
                if (it > 0 || c == 1) {
                    double xv[6];
#pragma unroll
                    for (int t = 0; t < 6; ++t) xv[t] = ld(x, nb[c][t]);
#pragma unroll
                    for (int t = 0; t < 6; ++t) acc += cf[c][t] * xv[t];
                }
                st(x, c * L.Nh + lane, dg[c] > 0.0 ? (acc - bm[c]) / dg[c] : 0.0);
            } else if (it == 0 && lane < n) {
                st(x, c * L.Nh + lane, 0.0);
            }
            wave_sync();
        }
    }
}

// byte offset of tail level l's coefficient copies
__device__ __forceinline__ int tail_coef_off(const Tail &T, int l)
{
    int o = T.coff;
    for (int q = 0; q < l; ++q) o += tail_coef_bytes(T.t[q].L.nx, T.t[q].L.ny, T.t[q].L.nz);
    return o;
}

// view of tail level l whose mask and coefficients live in LDS (the
// prolongation map onto it from the next level in *M)
__device__ __forceinline__ Lv tail_lv(const Tail &T, int l, unsigned char *smem, PMap *M = nullptr)
{
    Lv L = T.t[l].L;
    L.f = (const uint8_t *)(smem + T.t[l].moff);
    const int n[3] = {L.nx, L.ny, L.nz}, nt = L.nx + L.ny + L.nz;
    double *dp = (double *)(smem + tail_coef_off(T, l));
    int *ip = (int *)(dp + 4 * nt);
    for (int d = 0; d < 3; ++d) {
        L.cp[d] = dp;
        L.cm[d] = dp + n[d];
        L.w[d] = dp + 2 * n[d];
        if (M) {
            M->pt[d] = dp + 3 * n[d];
            M->pi[d] = ip;
        }
        dp += 4 * n[d];
        ip += n[d];
    }
    return L;
}

// copy tail level l's coefficients (and, below the last level, its
// prolongation map) from global memory into LDS, threads t0, t0 + nt, ...
__device__ __forceinline__ void tail_stage_coef(const Tail &T, int l, unsigned char *smem, int t0, int nt)
{
    const Lv &G = T.t[l].L;
    const PMap &GM = T.t[l].M;
    const bool map = l < T.n - 1;
    PMap M;
    Lv L = tail_lv(T, l, smem, &M);
    const int n[3] = {G.nx, G.ny, G.nz};
    for (int d = 0; d < 3; ++d)
        for (int q = t0; q < n[d]; q += nt) {
            const_cast<double *>(L.cp[d])[q] = G.cp[d][q];
            const_cast<double *>(L.cm[d])[q] = G.cm[d][q];
            const_cast<double *>(L.w[d])[q] = G.w[d][q];
            if (map) {
                const_cast<double *>(M.pt[d])[q] = GM.pt[d][q];
                const_cast<int *>(M.pi[d])[q] = GM.pi[d][q];
            }
        }
}

template <class Tc, class TB>
__global__ void __launch_bounds__(TAIL_T) k_tail(Tail T, const double *mean0)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double mus[8];
    {
        // each level is staged by its own 128 threads (at most 8 levels), so
        // the levels' global loads are in flight together: the mask in
        // 16-byte pieces, then the coefficients
        const int l = threadIdx.x >> 7, t0 = threadIdx.x & 127;
        if (l < T.n) {
            const TailLevel &TL = T.t[l];
            uint8_t *m = (uint8_t *)(smem + TL.moff);
            const long long n2 = 2 * TL.L.Nh, n16 = n2 >> 4;
            for (long long q = t0; q < n16; q += 128)
                reinterpret_cast<uint4 *>(m)[q] = reinterpret_cast<const uint4 *>(TL.L.f)[q];
            for (long long q = 16 * n16 + t0; q < n2; q += 128) m[q] = TL.L.f[q];
            tail_stage_coef(T, l, smem, t0, 128);
        }
    }
    {
        // the first tail level's RHS, four loads per thread in flight
        Tc *b0 = (Tc *)(smem + T.t[0].boff);
        const TB *bg = (const TB *)T.t[0].bg;
        const long long n2 = 2 * T.t[0].L.Nh;
        for (long long q0 = threadIdx.x; q0 < n2; q0 += 4 * (long long)blockDim.x) {
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const long long q = q0 + u * (long long)blockDim.x;
                v[u] = q < n2 ? ld(bg, q) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const long long q = q0 + u * (long long)blockDim.x;
                if (q < n2) b0[q] = (Tc)v[u];
            }
        }
    }
    if (threadIdx.x == 0) mus[0] = mean0[0];
    __syncthreads();
    for (int l = 0; l < T.n; ++l) {
        const Lv L = tail_lv(T, l, smem);
        Tc *x = (Tc *)(smem + T.t[l].xoff);
        const Tc *b = (const Tc *)(smem + T.t[l].boff);
        const double mu = mus[l];
        const bool last = l == T.n - 1;
        const int steps = last ? T.ncs : T.nu1;
        if (last && (long long)L.H * L.ny * L.nz <= 64) {
            if (threadIdx.x < 64) tail_coarsest_wave<Tc>(L, x, b, mu, steps);
            __syncthreads();
            break;
        }
        for (int it = 0; it < steps; ++it) {
            tail_sweep<Tc>(L, x, b, mu, 0, it == 0);
            tail_sweep<Tc>(L, x, b, mu, 1, it == 0);
        }
        if (last) break;
        // residual + restriction into the next level (rounded to the coarse
        // storage precision), then its volume-weighted mean
        const Lv C = tail_lv(T, l + 1, smem);
        Tc *bc = (Tc *)(smem + T.t[l + 1].boff);
        const int nc = C.H * C.ny * C.nz;
        for (int q = threadIdx.x; q < 2 * nc; q += blockDim.x) {
            const int cc = q >= nc ? 1 : 0;
            const int qq = q - cc * nc;
            const int row = (int)fdiv((uint32_t)qq, C.fH), hc = qq - row * C.H;
            const int K = (int)fdiv((uint32_t)row, C.fy), J = row - K * C.ny;
            double mub = mu;
            restrict_one<false, Tc, Tc, Tc>(L, C, -1, x, b, &mub, (const Tc *)nullptr, bc, cc, hc, J, K);
            const long long sc = (long long)cc * C.Nh + qq;
            st(bc, sc, round_to<TB>(ld(bc, sc)));  // coarse storage precision
        }
        __syncthreads();
        double part = 0.0;
        for (int q = threadIdx.x; q < 2 * nc; q += blockDim.x) {
            if (!(C.f[q] & 1)) continue;
            const int cc = q >= nc ? 1 : 0;
            const int qq = q - cc * nc;
            const int row = (int)fdiv((uint32_t)qq, C.fH), hc = qq - row * C.H;
            const int K = (int)fdiv((uint32_t)row, C.fy), J = row - K * C.ny;
            const int I = 2 * hc + ((cc + J + K) & 1);
            part += C.w[0][I] * C.w[1][J] * C.w[2][K] * ld(bc, q);
        }
        const double tot = tail_sum(part);
        if (threadIdx.x == 0) mus[l + 1] = T.t[l + 1].volA > 0.0 ? tot / T.t[l + 1].volA : 0.0;
        __syncthreads();
    }
    for (int l = T.n - 2; l >= 0; --l) {
        PMap M;
        const Lv L = tail_lv(T, l, smem, &M), C = tail_lv(T, l + 1, smem);
        Tc *x = (Tc *)(smem + T.t[l].xoff);
        const Tc *xc = (const Tc *)(smem + T.t[l + 1].xoff);
        const int n = L.H * L.ny * L.nz;
        for (int q = threadIdx.x; q < 2 * n; q += blockDim.x) {
            const int c = q >= n ? 1 : 0;
            const int qq = q - c * n;
            const int row = (int)fdiv((uint32_t)qq, L.fH), h = qq - row * L.H;
            const int k = (int)fdiv((uint32_t)row, L.fy);
            prolong_one<false>(L, C, M, xc, x, c, h, row - k * L.ny, k);
        }
        __syncthreads();
        const Tc *b = (const Tc *)(smem + T.t[l].boff);
        for (int it = 0; it < T.nu2; ++it) {
            tail_sweep<Tc>(L, x, b, mus[l], 0, false);
            tail_sweep<Tc>(L, x, b, mus[l], 1, false);
        }
    }
    {
        const Tc *x0 = (const Tc *)(smem + T.t[0].xoff);
        Tc *xg = (Tc *)T.t[0].xg;
        const long long n2 = 2 * T.t[0].L.Nh;
        for (long long q = threadIdx.x; q < n2; q += blockDim.x) xg[q] = x0[q];
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

// ---------------------------------------------------------------- 4-wide vector walks
// The Krylov updates walk groups of 4 consecutive unknowns (one 16-byte load
// per FP32 vector, two per FP64 vector); a group that is cut by the end of
// the vector or by the first membrane unknown takes the element path.
__device__ __forceinline__ void ld4(const float *a, long long g, double (&o)[4])
{
    const float4 q = reinterpret_cast<const float4 *>(a)[g];
    o[0] = q.x; o[1] = q.y; o[2] = q.z; o[3] = q.w;
}
__device__ __forceinline__ void ld4(const double *a, long long g, double (&o)[4])
{
    const double2 q0 = reinterpret_cast<const double2 *>(a)[2 * g], q1 = reinterpret_cast<const double2 *>(a)[2 * g + 1];
    o[0] = q0.x; o[1] = q0.y; o[2] = q1.x; o[3] = q1.y;
}
__device__ __forceinline__ void st4(float *a, long long g, double (&o)[4])
{
    float4 q;
    q.x = (float)o[0]; q.y = (float)o[1]; q.z = (float)o[2]; q.w = (float)o[3];
    reinterpret_cast<float4 *>(a)[g] = q;
    o[0] = q.x; o[1] = q.y; o[2] = q.z; o[3] = q.w;  // the stored (rounded) values
}
__device__ __forceinline__ void st4(double *a, long long g, double (&o)[4])
{
    double2 q0, q1;
    q0.x = o[0]; q0.y = o[1]; q1.x = o[2]; q1.y = o[3];
    reinterpret_cast<double2 *>(a)[2 * g] = q0;
    reinterpret_cast<double2 *>(a)[2 * g + 1] = q1;
}

// volumes of the 4 cells of a group (0 for inactive slots); e0 + 3 < 2 Nh
// raw 4-wide group of a vector: loaded first, converted after every load of
// the group has been issued
template <class T>
struct Raw4;
template <>
struct Raw4<float> {
    float4 q;
    __device__ __forceinline__ void load(const float *a, long long g) { q = reinterpret_cast<const float4 *>(a)[g]; }
    __device__ __forceinline__ void get(double (&o)[4]) const
    {
        o[0] = q.x; o[1] = q.y; o[2] = q.z; o[3] = q.w;
    }
};
template <>
struct Raw4<double> {
    double2 q0, q1;
    __device__ __forceinline__ void load(const double *a, long long g)
    {
        q0 = reinterpret_cast<const double2 *>(a)[2 * g];
        q1 = reinterpret_cast<const double2 *>(a)[2 * g + 1];
    }
    __device__ __forceinline__ void get(double (&o)[4]) const
    {
        o[0] = q0.x; o[1] = q0.y; o[2] = q1.x; o[3] = q1.y;
    }
};

// Cell volumes of the group of 4 slots from e0 (0 for inactive cells), with
// the group's masks already loaded (fq) and every width loaded whatever the
// mask (index clamped to the level), so that the loads of a group need not
// wait for one another
__device__ __forceinline__ void group_volumes_q(const Lv &L, long long e0, uchar4 fq, double (&V)[4])
{
    const uint8_t f[4] = {fq.x, fq.y, fq.z, fq.w};
    int c, h, j, k, i;
    decode_slot(L, e0, c, h, j, k, i);
    if (h + 3 < L.H) {
        const int par = i & 1;
        double w0[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) w0[q] = L.w[0][min(2 * (h + q) + par, L.nx - 1)];
        const double wjk = L.w[1][j] * L.w[2][k];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int iq = 2 * (h + q) + par;
            V[q] = (iq < L.nx && active0(f[q])) ? w0[q] * wjk : 0.0;
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            bool act;
            V[q] = slot_volume(L, e0 + q, act);
        }
    }
}

// p = r + beta (p - omega v); partial sum of V p over the active cells (the
// sink of the first V-cycle).  ne unknowns, W over ceil(ne/4) groups.
template <class T>
__global__ void __launch_bounds__(TPB) k_p_update4(Lv L, Walk W, long long ne, const T *__restrict__ r,
                                                   T *__restrict__ pv, const T *__restrict__ v, const double *sc,
                                                   double *part)
{
    const double beta = sc[S_BETA], omega = sc[S_OMEGA];
    Acc<1> a;
    a.v[0] = 0.0;
    const long long N2 = 2 * L.Nh;
    WALK_BEGIN(W, g)
        const long long e0 = 4 * g;
        if (e0 + 3 < ne && (e0 + 3 < N2 || e0 >= N2)) {
            // every load of the group goes out before any arithmetic (a group
            // of membrane unknowns has no volumes: slot 0 stands in, unused)
            const bool cells = e0 < N2;
            const long long ev = cells ? e0 : 0;
            const uchar4 fq = *reinterpret_cast<const uchar4 *>(L.f + ev);
            Raw4<T> rq, pq, vq;
            rq.load(r, g);
            pq.load(pv, g);
            vq.load(v, g);
            double V[4];
            group_volumes_q(L, ev, fq, V);
            __builtin_amdgcn_sched_barrier(0);
            double rr[4], pp[4], vv[4];
            rq.get(rr);
            pq.get(pp);
            vq.get(vv);
#pragma unroll
            for (int q = 0; q < 4; ++q) pp[q] = rr[q] + beta * (pp[q] - omega * vv[q]);
            st4(pv, g, pp);
            if (cells) {
#pragma unroll
                for (int q = 0; q < 4; ++q) a.v[0] += V[q] * pp[q];
            }
        } else {
            for (long long p = e0; p < min(e0 + 4, ne); ++p) {
                st(pv, p, ld(r, p) + beta * (ld(pv, p) - omega * ld(v, p)));
                if (p < N2) {
                    bool act;
                    const double V = slot_volume(L, p, act);
                    if (act) a.v[0] += V * ld(pv, p);
                }
            }
        }
    WALK_END
    block_reduce<1>(a, part, 0, blockIdx.x);
}

// r <- s = r - alpha v; partial sum of V s (sink of the second V-cycle)
template <class T>
__global__ void __launch_bounds__(TPB) k_s_update4(Lv L, Walk W, long long ne, T *__restrict__ r,
                                                   const T *__restrict__ v, const double *sc, double *part)
{
    const double alpha = sc[S_ALPHA];
    Acc<1> a;
    a.v[0] = 0.0;
    const long long N2 = 2 * L.Nh;
    WALK_BEGIN(W, g)
        const long long e0 = 4 * g;
        if (e0 + 3 < ne && (e0 + 3 < N2 || e0 >= N2)) {
            const bool cells = e0 < N2;
            const long long ev = cells ? e0 : 0;
            const uchar4 fq = *reinterpret_cast<const uchar4 *>(L.f + ev);
            Raw4<T> rq, vq;
            rq.load(r, g);
            vq.load(v, g);
            double V[4];
            group_volumes_q(L, ev, fq, V);
            __builtin_amdgcn_sched_barrier(0);
            double rr[4], vv[4];
            rq.get(rr);
            vq.get(vv);
#pragma unroll
            for (int q = 0; q < 4; ++q) rr[q] = rr[q] - alpha * vv[q];
            st4(r, g, rr);
            if (cells) {
#pragma unroll
                for (int q = 0; q < 4; ++q) a.v[0] += V[q] * rr[q];
            }
        } else {
            for (long long p = e0; p < min(e0 + 4, ne); ++p) {
                st(r, p, ld(r, p) - alpha * ld(v, p));
                if (p < N2) {
                    bool act;
                    const double V = slot_volume(L, p, act);
                    if (act) a.v[0] += V * ld(r, p);
                }
            }
        }
    WALK_END
    block_reduce<1>(a, part, 0, blockIdx.x);
}

// x += alpha (ph - ph_pin) + omega (sh - sh_pin) on the active unknowns (the
// preconditioner's shift to the pinned subspace, folded in here); r = s -
// omega t; partials of (rh, r) and (r, r)
template <class T, class TX>
__global__ void __launch_bounds__(TPB) k_xr_update4(Lv L, Walk W, long long ne, long long pin, TX *__restrict__ x,
                                                    const T *__restrict__ ph, const T *__restrict__ sh,
                                                    T *__restrict__ r, const T *__restrict__ t,
                                                    const T *__restrict__ rh, const double *sc, double *part,
                                                    int pstride)
{
    const double alpha = sc[S_ALPHA], omega = sc[S_OMEGA];
    const double cp = ld(ph, pin), cs = ld(sh, pin);
    const long long N2 = 2 * L.Nh;
    Acc<2> a;
    a.v[0] = a.v[1] = 0.0;
    WALK_BEGIN(W, g)
        const long long e0 = 4 * g;
        if (e0 + 3 < ne && (e0 + 3 < N2 || e0 >= N2)) {
            double xx[4], pp[4], ss[4], rr[4], tt[4], hh[4];
            ld4(x, g, xx);
            ld4(ph, g, pp);
            ld4(sh, g, ss);
            ld4(r, g, rr);
            ld4(t, g, tt);
            ld4(rh, g, hh);
            bool act[4] = {true, true, true, true};
            if (e0 < N2) {
                const uchar4 fq = *reinterpret_cast<const uchar4 *>(L.f + e0);
                act[0] = active0(fq.x); act[1] = active0(fq.y); act[2] = active0(fq.z); act[3] = active0(fq.w);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (act[q]) xx[q] = xx[q] + alpha * (pp[q] - cp) + omega * (ss[q] - cs);
                rr[q] = rr[q] - omega * tt[q];
            }
            st4(x, g, xx);
            st4(r, g, rr);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a.v[0] += hh[q] * rr[q];
                a.v[1] += rr[q] * rr[q];
            }
        } else {
            for (long long p = e0; p < min(e0 + 4, ne); ++p) {
                const bool act = p >= N2 || active0(L.f[p]);
                if (act) st(x, p, ld(x, p) + alpha * (ld(ph, p) - cp) + omega * (ld(sh, p) - cs));
                st(r, p, ld(r, p) - omega * ld(t, p));
                const double rv = ld(r, p);
                a.v[0] += ld(rh, p) * rv;
                a.v[1] += rv * rv;
            }
        }
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

// b = b2 = a (converted to TB) and the partial sums of the stored b^2, in
// groups of 4 (the last group of the vector element by element); W walks
// ceil(ne/4) groups
template <class TA, class TB>
__global__ void __launch_bounds__(TPB) k_copy_norm4(Walk W, long long ne, const TA *__restrict__ a,
                                                    TB *__restrict__ b, TB *__restrict__ b2, double *part)
{
    Acc<1> s;
    s.v[0] = 0.0;
    WALK_BEGIN(W, g)
        const long long e0 = 4 * g;
        if (e0 + 3 < ne) {
            Raw4<TA> aq;
            aq.load(a, g);
            double v[4];
            aq.get(v);
            st4(b, g, v);  // v now holds the stored values
            st4(b2, g, v);
#pragma unroll
            for (int q = 0; q < 4; ++q) s.v[0] += v[q] * v[q];
        } else {
            for (long long p = e0; p < ne; ++p) {
                st(b, p, ld(a, p));
                st(b2, p, ld(a, p));
                const double v = ld(b, p);
                s.v[0] += v * v;
            }
        }
    WALK_END
    block_reduce<1>(s, part, 0, blockIdx.x);
}

template <class T>
__global__ void __launch_bounds__(TPB) k_add(Walk W, double *x, const T *d, double a = 1.0)
{
    WALK_BEGIN(W, p)
        x[p] += a * ld(d, p);
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
    // four independent running sums per thread keep four loads in flight
    // (up to ~130k partials); fixed order, so the result is reproducible
    const int bd = blockDim.x;
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    int i = threadIdx.x;
    for (; i + 3 * bd < n; i += 4 * bd) {
        s4[0] += part[i];
        s4[1] += part[i + bd];
        s4[2] += part[i + 2 * bd];
        s4[3] += part[i + 3 * bd];
    }
    for (; i < n; i += bd) s4[0] += part[i];
    sm[threadIdx.x] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
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
