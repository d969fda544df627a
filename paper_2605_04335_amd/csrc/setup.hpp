// Device kernels of the solver set-up that depend on the classification:
// level-0 flags in split layout, ghost and membrane rows in slot numbering,
// the fluid volume, and the coarse-level masks of the multigrid hierarchy.
// They run once per set-up and again whenever moving bodies change the
// classification, so every O(N) step stays on the device.
#pragma once

#include "kernels.hpp"

namespace ibm {
namespace {

// natural cell index -> split slot on level 0
struct SlotMap {
    int nx, ny, H;
    long long Nh, N, N2;
};
__device__ __forceinline__ long long cell_slot(const SlotMap &m, long long cell)
{
    const long long i = cell % m.nx, r = cell / m.nx, j = r % m.ny, k = r / m.ny;
    return ((i + j + k) & 1) * m.Nh + (i >> 1) + (long long)m.H * (j + (long long)m.ny * k);
}
// unknown of a ghost-stencil column: a cell, or membrane ghost unknown N + m
__device__ __forceinline__ long long col_unknown(const SlotMap &m, long long col)
{
    return col < m.N ? cell_slot(m, col) : m.N2 + (col - m.N);
}

// level-0 flags in split layout; padding slots (i == nx on odd nx) are solid
__global__ void __launch_bounds__(TPB) k_setup_flags0(Lv L, Walk W, const uint8_t *__restrict__ nat,
                                                      uint8_t *__restrict__ spl)
{
    WALK_BEGIN(W, p)
        int c, h, j, k, i;
        decode_slot(L, p, c, h, j, k, i);
        spl[p] = i < L.nx ? nat[(long long)i + (long long)L.nx * (j + (long long)L.ny * k)] : (uint8_t)F_SOLID;
    WALK_END
}

// ghost rows: slot of each closed ghost cell, unknowns of every stencil column
__global__ void __launch_bounds__(TPB) k_setup_rows(SlotMap m, long long ng, long long R,
                                                    const int32_t *__restrict__ cell, const int32_t *__restrict__ col,
                                                    int32_t *__restrict__ rslot, int32_t *__restrict__ rcol)
{
    for (long long q = blockIdx.x * (long long)TPB + threadIdx.x; q < 8 * R; q += (long long)gridDim.x * TPB) {
        const int32_t v = col[q];
        rcol[q] = v >= 0 ? (int32_t)col_unknown(m, v) : -1;
        if ((q & 7) == 0 && (q >> 3) < ng) rslot[q >> 3] = (int32_t)cell_slot(m, cell[q >> 3]);
    }
}

// membrane cell behind each ghost-row stencil column: its index in the
// sorted membrane cell list, or -1 (not a grid cell, or not a membrane cell)
__global__ void __launch_bounds__(TPB) k_map_mrows(long long n, const int32_t *__restrict__ col, long long N,
                                                   const uint8_t *__restrict__ flags,
                                                   const int32_t *__restrict__ mcell, long long nm,
                                                   int32_t *__restrict__ out)
{
    for (long long q = blockIdx.x * (long long)TPB + threadIdx.x; q < n; q += (long long)gridDim.x * TPB) {
        const int32_t v = col[q];
        int32_t o = -1;
        if (v >= 0 && v < N && (flags[v] & F_MGHOST)) {
            long long a = 0, e = nm;  // first index with mcell >= v
            while (a < e) {
                const long long h = (a + e) >> 1;
                if (mcell[h] < v) a = h + 1;
                else e = h;
            }
            if (a < nm && mcell[a] == v) o = (int32_t)a;
        }
        out[q] = o;
    }
}

// membrane-adjacent cells: slot, colour, and the unknown behind each face
// (-x, +x, -y, +y, -z, +z): the neighbour cell, or the neighbour's ghost
// unknown when the link is cut (-1 at a wall).  mcell is sorted; a cut link
// whose far cell has no ghost row sets *err.
__global__ void __launch_bounds__(TPB) k_setup_membrane(SlotMap m, int nz, long long nm,
                                                        const int32_t *__restrict__ mcell,
                                                        const uint8_t *__restrict__ flags, int32_t *__restrict__ ms,
                                                        int32_t *__restrict__ mc, int32_t *__restrict__ mk,
                                                        int *__restrict__ err)
{
    for (long long q = blockIdx.x * (long long)TPB + threadIdx.x; q < nm; q += (long long)gridDim.x * TPB) {
        const long long p = mcell[q];
        const int ci[3] = {(int)(p % m.nx), (int)((p / m.nx) % m.ny), (int)(p / ((long long)m.nx * m.ny))};
        const int nd[3] = {m.nx, m.ny, nz};
        const long long strd[3] = {1, m.nx, (long long)m.nx * m.ny};
        ms[q] = (int32_t)cell_slot(m, p);
        mk[q] = (ci[0] + ci[1] + ci[2]) & 1;
        for (int d = 0; d < 3; ++d)
            for (int sg = 0; sg < 2; ++sg) {
                int32_t out = -1;
                const int c2 = ci[d] + (sg ? 1 : -1);
                if (c2 >= 0 && c2 < nd[d]) {
                    const long long nb = p + (sg ? strd[d] : -strd[d]);
                    const long long lo = sg ? p : nb;
                    if (flags[lo] & (F_CUTX << d)) {
                        long long a = 0, b = nm;  // first index with mcell >= nb
                        while (a < b) {
                            const long long h = (a + b) >> 1;
                            if (mcell[h] < nb) a = h + 1;
                            else b = h;
                        }
                        if (a < nm && mcell[a] == nb) out = (int32_t)(m.N2 + a);
                        else *err = 1;
                    } else {
                        out = (int32_t)cell_slot(m, nb);
                    }
                }
                mc[6 * q + 2 * d + sg] = out;
            }
    }
}

// mark (F_RD) the level-0 slots that the given row columns read (ghost
// stencils: 8 per row; membrane cells: 6 neighbours); several threads may set
// the bit of one slot, all writing the same byte
__global__ void __launch_bounds__(TPB) k_mark_read(long long n, const int32_t *__restrict__ cols, long long N2,
                                                   uint8_t *__restrict__ spl)
{
    for (long long q = blockIdx.x * (long long)TPB + threadIdx.x; q < n; q += (long long)gridDim.x * TPB) {
        const int32_t v = cols[q];
        if (v >= 0 && v < N2) spl[v] = (uint8_t)(spl[v] | F_RD);
    }
}

// volume of the fluid cells (per-block partial sums)
__global__ void __launch_bounds__(TPB) k_fluid_volume(Lv L, Walk W, double *part)
{
    Acc<1> s;
    s.v[0] = 0.0;
    WALK_BEGIN(W, p)
        int c, h, j, k, i;
        decode_slot(L, p, c, h, j, k, i);
        if (i < L.nx && !(L.f[p] & F_SOLID)) s.v[0] += L.w[0][i] * L.w[1][j] * L.w[2][k];
    WALK_END
    block_reduce<1>(s, part, 0, blockIdx.x);
}

// coarse cell (natural order): bit 0 active (a child is active), bits 4-6 a
// child link across the cell's +x/+y/+z half-way plane is cut -- from the
// level-0 flags (level 1) or the finer level's bits
__global__ void __launch_bounds__(TPB) k_coarse_active(int fnx, int fny, int cnx, int cny, long long CN,
                                                       const uint8_t *__restrict__ fine, int from_flags,
                                                       uint8_t *__restrict__ ha)
{
    for (long long P = blockIdx.x * (long long)TPB + threadIdx.x; P < CN; P += (long long)gridDim.x * TPB) {
        const long long I = P % cnx, r = P / cnx, J = r % cny, K = r / cny;
        uint8_t act = 0, cut = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int dx = q & 1, dy = (q >> 1) & 1, dz = (q >> 2) & 1;
            const long long p = (2 * I + dx) + (long long)fnx * ((2 * J + dy) + (long long)fny * (2 * K + dz));
            const uint8_t f = fine[p];
            const uint8_t a = from_flags ? (uint8_t)active0(f) : (uint8_t)(f & 1);
            const uint8_t cb = (f >> 4) & 7;
            act |= a;
            if (dx && (cb & 1)) cut |= 16;
            if (dy && (cb & 2)) cut |= 32;
            if (dz && (cb & 4)) cut |= 64;
        }
        ha[P] = act | cut;
    }
}

// coarse mask in split layout (CM_* bits: active, open +faces, open -faces),
// the volume of the active cells and the count of inactive cells (partials
// at part and part + pstride).  A face is open when both cells are active and
// no child link across it is cut.
__global__ void __launch_bounds__(TPB) k_coarse_mask(Lv L, Walk W, const uint8_t *__restrict__ ha,
                                                     uint8_t *__restrict__ sm, double *part, int pstride)
{
    Acc<2> s;
    s.v[0] = 0.0;
    s.v[1] = 0.0;
    WALK_BEGIN(W, p)
        int c, h, j, k, i;
        decode_slot(L, p, c, h, j, k, i);
        uint8_t out = 0;
        if (i < L.nx) {
            const long long P = (long long)i + (long long)L.nx * (j + (long long)L.ny * k);
            const uint8_t a = ha[P];
            if (!(a & 1)) s.v[1] += 1.0;
            if (a & 1) {
                out = CM_ACT;
                s.v[0] += L.w[0][i] * L.w[1][j] * L.w[2][k];
                const int ci[3] = {i, j, k}, nd[3] = {L.nx, L.ny, L.nz};
                const long long strd[3] = {1, L.nx, (long long)L.nx * L.ny};
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    if (ci[d] + 1 < nd[d] && (ha[P + strd[d]] & 1) && !(a & (16 << d))) out |= (uint8_t)(CM_PX << d);
                    if (ci[d] > 0) {
                        const uint8_t b = ha[P - strd[d]];
                        if ((b & 1) && !(b & (16 << d))) out |= (uint8_t)(CM_MX << d);
                    }
                }
            }
        }
        sm[p] = out;
    WALK_END
    block_reduce<2>(s, part, pstride, blockIdx.x);
}

}  // namespace
}  // namespace ibm

namespace ibm {
namespace {

// warm start without ghost values: a membrane ghost unknown (the field of
// the other side at this cell) starts from the mean of the cells across this
// cell's cut links, i.e. the other side's nearest values
__global__ void __launch_bounds__(TPB) k_warm_membrane(Sp S, double *x)
{
    for (int m = blockIdx.x * TPB + threadIdx.x; m < S.nm; m += gridDim.x * TPB) {
        double acc = 0.0;
        int cnt = 0;
        for (int q = 0; q < 6; ++q) {
            const long long col = S.mcol[6 * m + q];
            if (col >= S.N2) {
                acc += x[S.mslot[col - S.N2]];
                ++cnt;
            }
        }
        x[S.N2 + m] = cnt ? acc / cnt : x[S.mslot[m]];
    }
}

// warm start: unknowns of inactive (solid, non-ghost) and padding slots are zero
__global__ void __launch_bounds__(TPB) k_zero_inactive(Lv L, Walk W, double *x)
{
    WALK_BEGIN(W, p)
        int c, h, j, k, i;
        decode_slot(L, p, c, h, j, k, i);
        if (!(i < L.nx && active0(L.f[p]))) x[p] = 0.0;
    WALK_END
}

// fresh cells of a moving-body step (fluid now, solid before): the mean of
// the face neighbours that are fluid at both steps, in the order -x, +x, -y,
// +y, -z, +z; unchanged when there is none.  Those neighbours are never
// fresh themselves, so the update is in place.
__global__ void __launch_bounds__(TPB) k_fill_fresh(int nx, int ny, int nz, const uint8_t *__restrict__ fo,
                                                    const uint8_t *__restrict__ fn, double *x, int *count)
{
    const long long N = (long long)nx * ny * nz;
    int mine = 0;
    for (long long p = blockIdx.x * (long long)TPB + threadIdx.x; p < N; p += (long long)gridDim.x * TPB) {
        if ((fn[p] & F_SOLID) || !(fo[p] & F_SOLID)) continue;
        ++mine;
        const long long i = p % nx, r = p / nx, j = r % ny, k = r / ny;
        const long long sd[3] = {1, nx, (long long)nx * ny};
        const long long id[3] = {i, j, k}, nd[3] = {nx, ny, nz};
        double acc = 0.0;
        int cnt = 0;
        for (int d = 0; d < 3; ++d)
            for (int sg = 0; sg < 2; ++sg) {
                const long long c2 = id[d] + (sg ? 1 : -1);
                if (c2 < 0 || c2 >= nd[d]) continue;
                const long long q = p + (sg ? sd[d] : -sd[d]);
                if ((fn[q] & F_SOLID) || (fo[q] & F_SOLID)) continue;
                acc += x[q];
                ++cnt;
            }
        if (cnt) x[p] = acc / cnt;
    }
    if (mine) atomicAdd(count, mine);
}

}  // namespace
}  // namespace ibm
