// Streaming probes of the device's HBM bandwidth ceiling.
//
// The solve's kernels are bandwidth-bound stencils and vector updates, so
// their rooflines are quoted against the HBM peak and against what plain
// streams reach on the same device: a copy (one read, one write), the
// three-read, one-write mix of a red/black half-sweep, and a read-only sum.
// Buffers are far larger than the 256 MB Infinity Cache and every lane moves
// 16 bytes.
#include "common.hpp"

#include <algorithm>

namespace ibm {
namespace {

constexpr int ST_TPB = 256;

// One 16-byte element per thread over a grid of n / 256 blocks: on this
// device the hardware's block dispatch streams faster than threads looping
// over a range (measured: copy 6.3 against 5.0 TB/s for a chunked loop of
// four elements per step).  Stores are non-temporal.
typedef float v4f __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(ST_TPB) k_st_copy(long long n, const v4f *__restrict__ a, v4f *__restrict__ b)
{
    const long long e = (long long)blockIdx.x * ST_TPB + threadIdx.x;
    if (e < n) __builtin_nontemporal_store(a[e], b + e);
}

// d = a + b + c in FP32 lanes (three reads, one write)
__global__ void __launch_bounds__(ST_TPB) k_st_triad(long long n, const v4f *__restrict__ a, const v4f *__restrict__ b,
                                                     const v4f *__restrict__ c, v4f *__restrict__ d)
{
    const long long e = (long long)blockIdx.x * ST_TPB + threadIdx.x;
    if (e < n) __builtin_nontemporal_store(a[e] + b[e] + c[e], d + e);
}

// per-block sums of a (one 8-byte write per block)
__global__ void __launch_bounds__(ST_TPB) k_st_read(long long n, const v4f *__restrict__ a, double *part)
{
    const long long e = (long long)blockIdx.x * ST_TPB + threadIdx.x;
    float acc = 0.f;
    if (e < n) {
        const v4f v = a[e];
        acc = (v[0] + v[1]) + (v[2] + v[3]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    __shared__ float sm[ST_TPB / 64];
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (double)(sm[0] + sm[1] + sm[2] + sm[3]);
}

__global__ void __launch_bounds__(ST_TPB) k_st_fill(long long n, v4f *a, float v)
{
    for (long long e = (long long)blockIdx.x * ST_TPB + threadIdx.x; e < n; e += (long long)gridDim.x * ST_TPB) {
        const v4f q = {v, v + 1.f, v + 2.f, v + 3.f};
        a[e] = q;
    }
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
        const long long nb = (n + ST_TPB - 1) / ST_TPB;
        IBM_REQUIRE(nb < (1LL << 31), IBM_EINVAL, "buffer too large");
        DBuf<double> part(kind == IBM_STREAM_READ ? (size_t)nb : 1);
        for (int q = 0; q < nbuf; ++q)
            k_st_fill<<<8192, ST_TPB, 0, s>>>(n, (v4f *)buf[q].p, (float)q);
        IBM_LAUNCH_CHECK();
        auto launch = [&] {
            if (kind == IBM_STREAM_COPY)
                k_st_copy<<<(unsigned)nb, ST_TPB, 0, s>>>(n, (const v4f *)buf[0].p, (v4f *)buf[1].p);
            else if (kind == IBM_STREAM_TRIAD)
                k_st_triad<<<(unsigned)nb, ST_TPB, 0, s>>>(n, (const v4f *)buf[0].p, (const v4f *)buf[1].p,
                                                           (const v4f *)buf[2].p, (v4f *)buf[3].p);
            else
                k_st_read<<<(unsigned)nb, ST_TPB, 0, s>>>(n, (const v4f *)buf[0].p, part.p);
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
