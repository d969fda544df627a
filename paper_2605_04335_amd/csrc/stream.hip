// Streaming probes of the device's HBM bandwidth ceiling.
//
// The solve's kernels are bandwidth-bound stencils and vector updates, so
// their rooflines are quoted against the HBM peak and against what plain
// streams reach on the same device: a copy (one read, one write), the
// three-read, one-write mix of a red/black half-sweep, and a read-only sum.
// Buffers are far larger than the 256 MB Infinity Cache, every lane moves
// 16 bytes per access, and blocks are mapped so that each XCD streams one
// contiguous range.
#include "common.hpp"

#include <algorithm>

namespace ibm {
namespace {

constexpr int ST_TPB = 256;
constexpr int ST_UNROLL = 4;  // 16-byte accesses in flight per lane

// [begin, end) range of 16-byte elements of this block; the blocks of one
// XCD (blocks are dealt to the 8 XCDs round-robin) cover a contiguous slab
__device__ __forceinline__ void st_range(long long n, long long &b0, long long &b1)
{
    const long long nb = gridDim.x, per_xcd = nb / 8;
    const long long L = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    const long long chunk = (n + nb - 1) / nb;
    b0 = std::min(n, L * chunk);
    b1 = std::min(n, b0 + chunk);
}

__global__ void __launch_bounds__(ST_TPB) k_st_copy(long long n, const uint4 *__restrict__ a, uint4 *__restrict__ b)
{
    long long b0, b1;
    st_range(n, b0, b1);
    for (long long e = b0 + threadIdx.x; e < b1; e += (long long)ST_TPB * ST_UNROLL) {
        uint4 v[ST_UNROLL];
#pragma unroll
        for (int u = 0; u < ST_UNROLL; ++u) {
            const long long q = e + (long long)u * ST_TPB;
            if (q < b1) v[u] = a[q];
        }
#pragma unroll
        for (int u = 0; u < ST_UNROLL; ++u) {
            const long long q = e + (long long)u * ST_TPB;
            if (q < b1) b[q] = v[u];
        }
    }
}

// d = a + b + c in FP32 lanes (three reads, one write)
__global__ void __launch_bounds__(ST_TPB) k_st_triad(long long n, const float4 *__restrict__ a,
                                                     const float4 *__restrict__ b, const float4 *__restrict__ c,
                                                     float4 *__restrict__ d)
{
    long long b0, b1;
    st_range(n, b0, b1);
    for (long long e = b0 + threadIdx.x; e < b1; e += (long long)ST_TPB * ST_UNROLL) {
        float4 va[ST_UNROLL], vb[ST_UNROLL], vc[ST_UNROLL];
#pragma unroll
        for (int u = 0; u < ST_UNROLL; ++u) {
            const long long q = e + (long long)u * ST_TPB;
            if (q < b1) {
                va[u] = a[q];
                vb[u] = b[q];
                vc[u] = c[q];
            }
        }
#pragma unroll
        for (int u = 0; u < ST_UNROLL; ++u) {
            const long long q = e + (long long)u * ST_TPB;
            if (q < b1) {
                float4 r;
                r.x = va[u].x + vb[u].x + vc[u].x;
                r.y = va[u].y + vb[u].y + vc[u].y;
                r.z = va[u].z + vb[u].z + vc[u].z;
                r.w = va[u].w + vb[u].w + vc[u].w;
                d[q] = r;
            }
        }
    }
}

// per-block sums of a (one 8-byte write per block)
__global__ void __launch_bounds__(ST_TPB) k_st_read(long long n, const float4 *__restrict__ a, double *part)
{
    long long b0, b1;
    st_range(n, b0, b1);
    float acc = 0.f;
    for (long long e = b0 + threadIdx.x; e < b1; e += (long long)ST_TPB * ST_UNROLL) {
        float4 v[ST_UNROLL];
#pragma unroll
        for (int u = 0; u < ST_UNROLL; ++u) {
            const long long q = e + (long long)u * ST_TPB;
            v[u] = q < b1 ? a[q] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < ST_UNROLL; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    __shared__ float sm[ST_TPB / 64];
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (double)(sm[0] + sm[1] + sm[2] + sm[3]);
}

__global__ void __launch_bounds__(ST_TPB) k_st_fill(long long n, float4 *a, float v)
{
    for (long long e = (long long)blockIdx.x * ST_TPB + threadIdx.x; e < n; e += (long long)gridDim.x * ST_TPB)
        a[e] = make_float4(v, v + 1.f, v + 2.f, v + 3.f);
}

}  // namespace
}  // namespace ibm

using namespace ibm;

extern "C" int32_t ibm_hbm_stream(int32_t kind, size_t bytes, int32_t reps, double *ms, double *bytes_moved,
                                  void *stream)
{
    return guarded([&] {
        IBM_REQUIRE(ms && bytes_moved && reps >= 1 && reps <= 1000, IBM_EINVAL, "bad arguments");
        IBM_REQUIRE(kind >= IBM_STREAM_COPY && kind <= IBM_STREAM_READ, IBM_EINVAL, "unknown stream kind");
        IBM_REQUIRE(bytes >= ((size_t)1 << 20) && bytes <= ((size_t)64 << 30), IBM_EINVAL,
                    "buffer size must be 1 MiB .. 64 GiB");
        hipStream_t s = (hipStream_t)stream;
        const long long n = (long long)(bytes / 16);  // 16-byte elements per buffer
        const int nbuf = kind == IBM_STREAM_TRIAD ? 4 : (kind == IBM_STREAM_COPY ? 2 : 1);
        std::vector<DBuf<uint4>> buf(nbuf);
        for (auto &b : buf) b.alloc((size_t)n);
        // 2048 blocks per launch: 8 per CU, a multiple of the 8 XCDs
        const int nb = 2048;
        DBuf<double> part(nb);
        for (int q = 0; q < nbuf; ++q)
            k_st_fill<<<8192, ST_TPB, 0, s>>>(n, (float4 *)buf[q].p, (float)q);
        IBM_LAUNCH_CHECK();
        auto launch = [&] {
            if (kind == IBM_STREAM_COPY)
                k_st_copy<<<nb, ST_TPB, 0, s>>>(n, buf[0].p, buf[1].p);
            else if (kind == IBM_STREAM_TRIAD)
                k_st_triad<<<nb, ST_TPB, 0, s>>>(n, (const float4 *)buf[0].p, (const float4 *)buf[1].p,
                                                 (const float4 *)buf[2].p, (float4 *)buf[3].p);
            else
                k_st_read<<<nb, ST_TPB, 0, s>>>(n, (const float4 *)buf[0].p, part.p);
        };
        launch();  // first touch
        hipEvent_t e0, e1;
        IBM_HIP(hipEventCreate(&e0));
        IBM_HIP(hipEventCreate(&e1));
        IBM_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) launch();
        IBM_HIP(hipEventRecord(e1, s));
        IBM_LAUNCH_CHECK();
        IBM_HIP(hipEventSynchronize(e1));
        float t = 0.f;
        IBM_HIP(hipEventElapsedTime(&t, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *ms = (double)t / reps;
        const double per = 16.0 * (double)n;
        *bytes_moved = kind == IBM_STREAM_COPY ? 2.0 * per : (kind == IBM_STREAM_TRIAD ? 4.0 * per : per);
        IBM_HIP(hipStreamSynchronize(s));
    });
}
