// Shared host/device helpers of libibmpoisson (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <mutex>
#include <shared_mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "ibm_poisson.h"

namespace ibm {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string &msg);

#define IBM_HIP(expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            throw ::ibm::Error(IBM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_) + " at " +   \
                                             __FILE__ + ":" + std::to_string(__LINE__));                \
    } while (0)

#define IBM_REQUIRE(cond, code, msg)                                                                    \
    do {                                                                                                \
        if (!(cond)) throw ::ibm::Error((code), (msg));                                                 \
    } while (0)

#define IBM_LAUNCH_CHECK() IBM_HIP(hipGetLastError())

// Wraps an extern "C" body: converts exceptions into return codes.
template <class F>
int32_t guarded(F &&f)
{
    try {
        f();
        return IBM_OK;
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return IBM_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return IBM_EINVAL;
    }
}

// ---------------------------------------------------------------- memory
// A graph capture in one thread excludes the library's device allocations
// and frees in every other thread (the runtime treats them as synchronising
// calls, which a capture in flight does not allow): captures hold this
// exclusively, allocations and frees share it.
inline std::shared_mutex &capture_mutex()
{
    static std::shared_mutex m;
    return m;
}

// Device blocks from the library's cache (memory.hip): cls is the block's
// size class, 0 for a block that bypassed the cache.  Both may throw Error.
void *device_alloc(size_t bytes, int &dev, size_t &cls);
void device_release(void *p, int dev, size_t cls);

// Owning device buffer (device_alloc / device_release).
template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    bool own = true;  // false: a view into caller-owned memory (never freed here)
    int dev = 0;      // device and size class of an owned block
    size_t cls = 0;
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n), own(o.own), dev(o.dev), cls(o.cls) { o.p = nullptr; o.n = 0; }
    DBuf &operator=(DBuf &&o) noexcept
    {
        if (this != &o) {
            release();
            p = o.p; n = o.n; own = o.own; dev = o.dev; cls = o.cls;
            o.p = nullptr;
            o.n = 0;
        }
        return *this;
    }
    void view(T *q, size_t count)
    {
        release();
        p = q;
        n = count;
        own = false;
    }
    ~DBuf() { release(); }
    void alloc(size_t count)
    {
        release();
        own = true;
        if (count) {
            p = (T *)device_alloc(count * sizeof(T), dev, cls);
            n = count;
        }
    }
    void release()
    {
        if (p && own) device_release(p, dev, cls);
        p = nullptr;
        n = 0;
        own = true;
    }
    size_t bytes() const { return n * sizeof(T); }
};

template <class T>
void upload(DBuf<T> &d, const std::vector<T> &h, hipStream_t s)
{
    d.alloc(h.size());
    if (!h.empty()) IBM_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

inline unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

// ---------------------------------------------------------------- grid (host)
struct HostGrid {
    int n[3];
    std::vector<double> f[3];
};

HostGrid read_grid(const ibm_grid *g);

constexpr uint8_t F_SOLID = IBM_F_SOLID, F_GHOST = IBM_F_GHOST, F_MGHOST = IBM_F_MGHOST, F_PIN = IBM_F_PIN,
                  F_CUTX = IBM_F_CUTX;
// bit 7 of the solver's own level-0 mask (never of the classification
// output): the slot is read by a ghost row or a membrane row, so it must be
// zero when those rows run after a V-cycle's first (red) half-sweep
constexpr uint8_t F_RD = 0x80;

}  // namespace ibm

// Stencil table (device-resident), shared between the geometry and the solver
// translation units.
struct ibm_stencils {
    int n[3] = {0, 0, 0};
    int64_t N = 0;
    int64_t ng = 0, nm = 0, nfallback = 0, pin = -1;
    int bc = 0;                // IBM_BC_NEUMANN or IBM_BC_DIRICHLET rows
    ibm::DBuf<int32_t> cell;   // [ng + nm] closed ghost cells then membrane ghost cells (sorted)
    ibm::DBuf<int32_t> col;    // [rows*8]
    ibm::DBuf<double> w;       // [rows*8]
    ibm::DBuf<double> sG;      // [rows]
    ibm::DBuf<double> dlb;     // [rows]
    ibm::DBuf<uint8_t> rfl;    // [rows]
    ibm::DBuf<double> geo;     // [rows*12]
};
