// Cell classification ("iblanking", Sec. 2.5 module 1) on gfx950.
//
// Closed bodies: a cell is solid iff the ray along +x through its centre has
// crossed the body an odd number of times before reaching the centre.
// Membranes: the link between two face neighbours is cut iff an odd number of
// membrane triangles cross it (rays along x, y and z).  All predicates are
// exact int64 arithmetic on lattice coordinates q(v) = floor((v-lo)*S + 0.5),
// S = 2^16 / longest domain edge; a point exactly on a projected edge belongs
// to the triangle for which that edge is "top-left" (d_w < 0, or d_w == 0 and
// d_u > 0), the same as perturbing the ray by (+e, +e^2).
//
// GPU form: one thread per triangle walks the rays its projected bounding box
// covers, finds the first cell beyond the crossing by binary search and flips
// one bit of a toggle bitset with an integer atomic XOR; one thread per ray
// then turns toggles into parity.  This file is compiled with
// -ffp-contract=off so that the quantisation rounds exactly as written.

#include "common.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace ibm {

HostGrid read_grid(const ibm_grid *g)
{
    IBM_REQUIRE(g != nullptr, IBM_EINVAL, "null grid");
    HostGrid h;
    h.n[0] = g->nx; h.n[1] = g->ny; h.n[2] = g->nz;
    const double *f[3] = {g->xf, g->yf, g->zf};
    for (int d = 0; d < 3; ++d) {
        IBM_REQUIRE(h.n[d] >= 4, IBM_EINVAL, "grid dimension below 4");
        IBM_REQUIRE(f[d] != nullptr, IBM_EINVAL, "null face array");
        h.f[d].assign(f[d], f[d] + h.n[d] + 1);
        for (int i = 0; i < h.n[d]; ++i)
            IBM_REQUIRE(h.f[d][i + 1] > h.f[d][i], IBM_EINVAL, "face coordinates not strictly increasing");
    }
    IBM_REQUIRE((int64_t)h.n[0] * h.n[1] * h.n[2] < ((int64_t)1 << 31), IBM_EINVAL, "more than 2^31 cells");
    return h;
}

namespace {

struct Lat {
    double lo[3];
    double S;
};

__device__ __forceinline__ long long qnt(double v, double lo, double S)
{
    double t = (v - lo) * S;
    t = t + 0.5;
    return (long long)floor(t);
}

__global__ void k_quant_centres(const double *f, int n, double lo, double S, long long *q)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) q[i] = qnt(0.5 * (f[i] + f[i + 1]), lo, S);
}

__global__ void k_quant_verts(const double *v, int nv, Lat L, long long *q)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nv * 3) {
        int d = i % 3;
        q[i] = qnt(v[i], L.lo[d], L.S);
    }
}

__global__ void k_fill_u32(uint32_t *a, long long n, uint32_t v)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (long long)gridDim.x * blockDim.x) a[i] = v;
}

__global__ void k_fill_u8(uint8_t *a, long long n, uint8_t v)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (long long)gridDim.x * blockDim.x) a[i] = v;
}

__device__ __forceinline__ long long o2(const long long *U, const long long *V, const long long *P, int u, int w)
{
    return (V[u] - U[u]) * (P[w] - U[w]) - (V[w] - U[w]) * (P[u] - U[u]);
}

__device__ __forceinline__ bool owns(const long long *U, const long long *V, const long long *P, int u, int w)
{
    long long e = o2(U, V, P, u, w);
    if (e != 0) return e > 0;
    long long du = V[u] - U[u], dw = V[w] - U[w];
    return dw < 0 || (dw == 0 && du > 0);
}

__device__ __forceinline__ int lower_bound_ll(const long long *a, int n, long long v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int m = (lo + hi) >> 1;
        if (a[m] < v) lo = m + 1; else hi = m;
    }
    return lo;
}

struct RayArgs {
    const long long *qc[3];  // lattice centres per axis
    int n[3];
    const long long *qv;     // lattice vertices of the body
    const int32_t *tri;      // triangles of the body
    int nt;
    int d;                   // ray axis
    int mode;                // 0 closed parity toggles at the first cell beyond; 1 cut-link toggles
    uint32_t *bits;          // toggle bitset over cells
    uint8_t *has;            // per-ray "touched" marker (closed mode)
};

// One thread per triangle: every covered ray flips the bit of the first cell
// whose centre lies strictly beyond the crossing (closed mode), or the link
// just before it (membrane mode).
__global__ void k_rays(RayArgs A)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= A.nt) return;
    const int d = A.d, u = (d + 1) % 3, w = (d + 2) % 3;
    const long long *P0 = A.qv + 3 * A.tri[3 * t], *P1 = A.qv + 3 * A.tri[3 * t + 1], *P2 = A.qv + 3 * A.tri[3 * t + 2];
    long long e1[3], e2[3], Nn[3];
    for (int c = 0; c < 3; ++c) { e1[c] = P1[c] - P0[c]; e2[c] = P2[c] - P0[c]; }
    Nn[0] = e1[1] * e2[2] - e1[2] * e2[1];
    Nn[1] = e1[2] * e2[0] - e1[0] * e2[2];
    Nn[2] = e1[0] * e2[1] - e1[1] * e2[0];
    const long long a = Nn[d];
    if (a == 0) return;
    const long long *B = P1, *C = P2;  // counter-clockwise order in (u, w)
    if (a < 0) { B = P2; C = P1; }
    long long umin = min(P0[u], min(P1[u], P2[u])), umax = max(P0[u], max(P1[u], P2[u]));
    long long wmin = min(P0[w], min(P1[w], P2[w])), wmax = max(P0[w], max(P1[w], P2[w]));
    const int nu = A.n[u], nw = A.n[w], nr = A.n[d];
    const long long *qu = A.qc[u], *qw = A.qc[w], *qr = A.qc[d];
    const long long sa = a > 0 ? 1 : -1, aa = a > 0 ? a : -a;
    int ia0 = lower_bound_ll(qu, nu, umin), ib0 = lower_bound_ll(qw, nw, wmin);
    long long st[3] = {1, A.n[0], (long long)A.n[0] * A.n[1]};
    long long X[3];
    for (int ia = ia0; ia < nu && qu[ia] <= umax; ++ia) {
        for (int ib = ib0; ib < nw && qw[ib] <= wmax; ++ib) {
            X[u] = qu[ia];
            X[w] = qw[ib];
            if (!owns(P0, B, X, u, w) || !owns(B, C, X, u, w) || !owns(C, P0, X, u, w)) continue;
            // first i with (qr[i]-A_d)|a| + sign(a) K > 0 (centre strictly beyond the crossing)
            long long K = (X[u] - P0[u]) * Nn[u] + (X[w] - P0[w]) * Nn[w];
            long long sk = sa * K;
            int lo = 0, hi = nr;
            while (lo < hi) {
                int m = (lo + hi) >> 1;
                if ((qr[m] - P0[d]) * aa + sk > 0) hi = m; else lo = m + 1;
            }
            long long base = (long long)ia * st[u] + (long long)ib * st[w];
            if (A.mode == 0) {
                if (lo < nr) {
                    long long cell = base + (long long)lo * st[d];
                    atomicXor(&A.bits[cell >> 5], 1u << (cell & 31));
                    long long ray = d == 0 ? (long long)ia + (long long)A.n[1] * ib : 0;
                    A.has[ray] = 1;
                }
            } else if (lo >= 1 && lo <= nr - 1) {
                long long cell = base + (long long)(lo - 1) * st[d];
                atomicXor(&A.bits[cell >> 5], 1u << (cell & 31));
            }
        }
    }
}

// One thread per x-ray: prefix parity of the toggles; odd cells become solid.
__global__ void k_ray_parity(const uint32_t *bits, const uint8_t *has, int nx, long long nrays, uint8_t *flags)
{
    long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrays || !has[r]) return;
    long long base = r * nx;
    uint32_t par = 0;
    for (int i = 0; i < nx; ++i) {
        long long c = base + i;
        par ^= (bits[c >> 5] >> (c & 31)) & 1u;
        if (par) flags[c] |= F_SOLID;
    }
}

__device__ __forceinline__ bool bit(const uint32_t *b, long long c) { return (b[c >> 5] >> (c & 31)) & 1u; }

// Ghost, membrane-ghost and cut bits from the solid bits and the raw cut toggles.
__global__ void k_flags(uint8_t *flags, const uint32_t *cx, const uint32_t *cy, const uint32_t *cz, int nx, int ny,
                        int nz, int has_membrane)
{
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long N = (long long)nx * ny * nz;
    if (p >= N) return;
    int i = (int)(p % nx);
    int j = (int)((p / nx) % ny);
    int k = (int)(p / ((long long)nx * ny));
    int ci[3] = {i, j, k}, nn[3] = {nx, ny, nz};
    long long st[3] = {1, nx, (long long)nx * ny};
    const uint32_t *cut[3] = {cx, cy, cz};
    uint8_t f = flags[p] & F_SOLID;
    if (f) {
        bool g = false;
        for (int d = 0; d < 3; ++d) {
            if (ci[d] > 0 && !(flags[p - st[d]] & F_SOLID)) g = true;
            if (ci[d] + 1 < nn[d] && !(flags[p + st[d]] & F_SOLID)) g = true;
        }
        if (g) f |= F_GHOST;
    } else if (has_membrane) {
        for (int d = 0; d < 3; ++d) {
            if (ci[d] + 1 < nn[d] && bit(cut[d], p) && !(flags[p + st[d]] & F_SOLID)) f |= (uint8_t)(F_CUTX << d);
            if (ci[d] > 0 && bit(cut[d], p - st[d]) && !(flags[p - st[d]] & F_SOLID)) f |= F_MGHOST;
        }
        if (f & 0x70) f |= F_MGHOST;
    }
    flags[p] = f;
}

__global__ void k_pin(const uint8_t *flags, long long N, unsigned long long *pin)
{
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (; p < N; p += (long long)gridDim.x * blockDim.x)
        if (!(flags[p] & (F_SOLID | F_MGHOST))) {
            atomicMin(pin, (unsigned long long)p);
            return;  // later cells of this thread are larger
        }
}

__global__ void k_set_pin(uint8_t *flags, const unsigned long long *pin, long long N)
{
    if (threadIdx.x == 0 && blockIdx.x == 0 && *pin < (unsigned long long)N) flags[*pin] |= F_PIN;
}

// counts: solid, ghost, mghost, cut links (per-block partial sums with integer atomics)
__global__ void k_counts(const uint8_t *flags, long long N, unsigned long long *cnt)
{
    __shared__ unsigned long long s[4];
    if (threadIdx.x < 4) s[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long a = 0, b = 0, c = 0, e = 0;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (long long)gridDim.x * blockDim.x) {
        uint8_t f = flags[p];
        a += f & F_SOLID;
        b += (f >> 1) & 1;
        c += (f >> 2) & 1;
        e += ((f >> 4) & 1) + ((f >> 5) & 1) + ((f >> 6) & 1);
    }
    atomicAdd(&s[0], a);
    atomicAdd(&s[1], b);
    atomicAdd(&s[2], c);
    atomicAdd(&s[3], e);
    __syncthreads();
    if (threadIdx.x < 4) atomicAdd(&cnt[threadIdx.x], s[threadIdx.x]);
}

// counters of one classification: pin (minimum), then the four counts
__global__ void k_init_counters(unsigned long long *dev)
{
    if (threadIdx.x < 5) dev[threadIdx.x] = threadIdx.x == 0 ? ~0ull : 0ull;
}

// Device scratch of one classification, carved from one region in 256-byte
// aligned pieces.  A carve with a null base only measures.
struct Carve {
    char *base = nullptr;
    size_t off = 0;
    template <class T>
    T *take(size_t n)
    {
        off = (off + 255) / 256 * 256;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
};

struct BodyScratch {
    double *dv;
    int32_t *dt;
    long long *qv;
};

struct ClassifyScratch {
    double *df[3];
    long long *qc[3];
    uint32_t *tog = nullptr, *cut[3] = {nullptr, nullptr, nullptr};
    uint8_t *has = nullptr;
    unsigned long long *dev;
    std::vector<BodyScratch> body;
};

// Every device buffer a classification uses: per axis the faces and the
// quantised centres; the toggle bitset and per-ray markers (closed bodies);
// three cut-link bitsets (membranes); per body its vertices, triangles and
// quantised vertices; the five counters.
ClassifyScratch carve_classify(Carve &C, const HostGrid &g, const ibm_body *bodies, int n_body, bool any_closed,
                               bool any_mem)
{
    ClassifyScratch S;
    const long long N = (long long)g.n[0] * g.n[1] * g.n[2];
    const size_t words = (size_t)((N + 31) / 32 + 1);
    for (int d = 0; d < 3; ++d) {
        S.df[d] = C.take<double>(g.n[d] + 1);
        S.qc[d] = C.take<long long>(g.n[d]);
    }
    if (any_closed) {
        S.tog = C.take<uint32_t>(words);
        S.has = C.take<uint8_t>((size_t)g.n[1] * g.n[2]);
    }
    if (any_mem)
        for (int d = 0; d < 3; ++d) S.cut[d] = C.take<uint32_t>(words);
    for (int b = 0; b < n_body; ++b) {
        BodyScratch B;
        B.dv = C.take<double>((size_t)3 * bodies[b].n_vert);
        B.dt = C.take<int32_t>((size_t)3 * bodies[b].n_tri);
        B.qv = C.take<long long>((size_t)3 * bodies[b].n_vert);
        S.body.push_back(B);
    }
    S.dev = C.take<unsigned long long>(5);
    return S;
}

struct ClassifyPlan {
    HostGrid g;
    bool any_closed = false, any_mem = false;
    size_t bytes = 0;  // device scratch the classification needs
};

// Argument checks and the scratch size; nothing touches the device.
ClassifyPlan plan_classify(const ibm_grid *grid, const ibm_body *bodies, int n_body, const uint8_t *flags)
{
    ClassifyPlan P;
    P.g = read_grid(grid);
    const HostGrid &g = P.g;
    IBM_REQUIRE(flags != nullptr, IBM_EINVAL, "null flags");
    IBM_REQUIRE(n_body >= 0 && (n_body == 0 || bodies != nullptr), IBM_EINVAL, "bad body list");
    for (int b = 0; b < n_body; ++b) {
        const ibm_body &B = bodies[b];
        IBM_REQUIRE(B.kind == IBM_KIND_CLOSED || B.kind == IBM_KIND_MEMBRANE, IBM_EINVAL, "bad body kind");
        (B.kind == IBM_KIND_CLOSED ? P.any_closed : P.any_mem) = true;
        IBM_REQUIRE(B.n_vert >= 3 && B.n_tri >= 1 && B.vert && B.tri, IBM_EINVAL, "empty body");
        for (int v = 0; v < 3 * B.n_vert; ++v) {
            int d = v % 3;
            double x = B.vert[v];
            double Ld = g.f[d][g.n[d]] - g.f[d][0];
            IBM_REQUIRE(std::isfinite(x) && x >= g.f[d][0] - Ld && x <= g.f[d][g.n[d]] + Ld, IBM_EINVAL,
                        "body vertex more than one domain length outside the domain");
        }
        for (int t = 0; t < 3 * B.n_tri; ++t)
            IBM_REQUIRE(B.tri[t] >= 0 && B.tri[t] < B.n_vert, IBM_EGEOM, "triangle index out of range");
    }
    Carve C;
    (void)carve_classify(C, g, bodies, n_body, P.any_closed, P.any_mem);
    P.bytes = C.off;
    return P;
}

// Host orchestration of the classification; every device buffer of the call
// comes from `scratch` (at least plan.bytes, 256-byte aligned).
void classify_with(const ClassifyPlan &plan, const ibm_body *bodies, int n_body, uint8_t *flags, ibm_class_stats *st,
              char *scratch, hipStream_t s)
{
    const HostGrid &g = plan.g;
    const long long N = (long long)g.n[0] * g.n[1] * g.n[2];
    double L = 0.0;
    for (int d = 0; d < 3; ++d) L = std::max(L, g.f[d][g.n[d]] - g.f[d][0]);
    Lat lat;
    lat.S = 65536.0 / L;
    for (int d = 0; d < 3; ++d) lat.lo[d] = g.f[d][0];
    Carve C;
    C.base = scratch;
    ClassifyScratch S = carve_classify(C, g, bodies, n_body, plan.any_closed, plan.any_mem);

    for (int d = 0; d < 3; ++d) {
        IBM_HIP(hipMemcpyAsync(S.df[d], g.f[d].data(), (g.n[d] + 1) * sizeof(double), hipMemcpyHostToDevice, s));
        k_quant_centres<<<cdiv(g.n[d], 256), 256, 0, s>>>(S.df[d], g.n[d], lat.lo[d], lat.S, S.qc[d]);
        IBM_LAUNCH_CHECK();
    }
    const long long words = (N + 31) / 32 + 1;
    k_fill_u8<<<2048, 256, 0, s>>>(flags, N, 0);
    IBM_LAUNCH_CHECK();
    if (plan.any_mem)
        for (int d = 0; d < 3; ++d) {
            k_fill_u32<<<2048, 256, 0, s>>>(S.cut[d], words, 0u);
            IBM_LAUNCH_CHECK();
        }
    for (int b = 0; b < n_body; ++b) {
        const ibm_body &B = bodies[b];
        const BodyScratch &Q = S.body[b];
        IBM_HIP(hipMemcpyAsync(Q.dv, B.vert, (size_t)3 * B.n_vert * sizeof(double), hipMemcpyHostToDevice, s));
        IBM_HIP(hipMemcpyAsync(Q.dt, B.tri, (size_t)3 * B.n_tri * sizeof(int32_t), hipMemcpyHostToDevice, s));
        k_quant_verts<<<cdiv(3 * B.n_vert, 256), 256, 0, s>>>(Q.dv, B.n_vert, lat, Q.qv);
        IBM_LAUNCH_CHECK();
        RayArgs A;
        for (int d = 0; d < 3; ++d) { A.qc[d] = S.qc[d]; A.n[d] = g.n[d]; }
        A.qv = Q.qv;
        A.tri = Q.dt;
        A.nt = B.n_tri;
        if (B.kind == IBM_KIND_CLOSED) {
            k_fill_u32<<<2048, 256, 0, s>>>(S.tog, words, 0u);
            k_fill_u8<<<256, 256, 0, s>>>(S.has, (long long)g.n[1] * g.n[2], 0);
            IBM_LAUNCH_CHECK();
            A.d = 0; A.mode = 0; A.bits = S.tog; A.has = S.has;
            k_rays<<<cdiv(B.n_tri, 64), 64, 0, s>>>(A);
            IBM_LAUNCH_CHECK();
            long long nrays = (long long)g.n[1] * g.n[2];
            k_ray_parity<<<cdiv(nrays, 128), 128, 0, s>>>(S.tog, S.has, g.n[0], nrays, flags);
            IBM_LAUNCH_CHECK();
        } else {
            for (int d = 0; d < 3; ++d) {
                A.d = d; A.mode = 1; A.bits = S.cut[d]; A.has = nullptr;
                k_rays<<<cdiv(B.n_tri, 64), 64, 0, s>>>(A);
                IBM_LAUNCH_CHECK();
            }
        }
    }
    k_flags<<<cdiv(N, 256), 256, 0, s>>>(flags, S.cut[0], S.cut[1], S.cut[2], g.n[0], g.n[1], g.n[2],
                                         plan.any_mem ? 1 : 0);
    k_init_counters<<<1, 64, 0, s>>>(S.dev);
    k_pin<<<2048, 256, 0, s>>>(flags, N, S.dev);
    k_set_pin<<<1, 64, 0, s>>>(flags, S.dev, N);
    k_counts<<<1024, 256, 0, s>>>(flags, N, S.dev + 1);
    IBM_LAUNCH_CHECK();
    unsigned long long h[5];
    IBM_HIP(hipMemcpyAsync(h, S.dev, 5 * 8, hipMemcpyDeviceToHost, s));
    // the counts are needed on the host; this also ends every use of the scratch
    IBM_HIP(hipStreamSynchronize(s));
    IBM_REQUIRE(h[0] < (unsigned long long)N, IBM_EGEOM, "no fluid cell outside the membrane ghosts");
    if (st) {
        st->pin = (int64_t)h[0];
        st->n_solid = (int64_t)h[1];
        st->n_ghost = (int64_t)h[2];
        st->n_mghost = (int64_t)h[3];
        st->n_cut_links = (int64_t)h[4];
    }
}

// Scratch of ibm_classify_noalloc: one array per device, for the life of the
// process.  Its host-side name is not a device address; the address comes
// from hipGetSymbolAddress, once per device.
constexpr size_t NOALLOC_BYTES = (size_t)IBM_CLASSIFY_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

std::mutex g_scratch_mu;
std::vector<char *> g_scratch_ptr;  // per device ordinal, null until looked up

char *device_scratch()
{
    int dev = 0;
    IBM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        IBM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        IBM_REQUIRE(ptr != nullptr, IBM_EHIP, "no device address for the classification scratch");
        g_scratch_ptr[dev] = (char *)ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

void classify(const ibm_grid *grid, const ibm_body *bodies, int n_body, uint8_t *flags, ibm_class_stats *st,
              hipStream_t s)
{
    const ClassifyPlan plan = plan_classify(grid, bodies, n_body, flags);
    DBuf<char> ws(plan.bytes);
    classify_with(plan, bodies, n_body, flags, st, ws.p, s);
}

}  // namespace ibm

extern "C" int32_t ibm_classify(const ibm_grid *grid, const ibm_body *bodies, int32_t n_body, uint8_t *flags_dev,
                                ibm_class_stats *st, void *stream)
{
    return ibm::guarded([&] { ibm::classify(grid, bodies, n_body, flags_dev, st, (hipStream_t)stream); });
}

extern "C" int32_t ibm_classify_noalloc(const ibm_grid *grid, const ibm_body *bodies, int32_t n_body,
                                        uint8_t *flags_dev, ibm_class_stats *st, size_t *scratch_bytes, void *stream)
{
    return ibm::guarded([&] {
        const ibm::ClassifyPlan plan = ibm::plan_classify(grid, bodies, n_body, flags_dev);
        if (scratch_bytes) *scratch_bytes = plan.bytes;
        IBM_REQUIRE(plan.bytes <= ibm::NOALLOC_BYTES, IBM_ENOMEM,
                    "ibm_classify_noalloc: this grid and these bodies need " + std::to_string(plan.bytes) +
                        " bytes of scratch, above its fixed " + std::to_string(ibm::NOALLOC_BYTES) +
                        " (use ibm_classify)");
        ibm::classify_with(plan, bodies, n_body, flags_dev, st, ibm::device_scratch(), (hipStream_t)stream);
    });
}
