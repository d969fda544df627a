// Device memory of the library: a cache in front of hipMalloc / hipFree.
//
// hipFree performs an implicit hipDeviceSynchronize, so with several solves
// in flight on one device (the server runs one per stream) every release
// would stall its thread until all of them drain, and a request's set-up and
// teardown would take as long as the other requests' work.  A released block
// therefore is not freed: it joins its device's pending list.  A background
// thread synchronises the device once for everything pending and then makes
// those blocks reusable (all work that used a block was enqueued before its
// release, so it has completed by then; the same condition hipFree relies
// on).  Allocations round up to a size class (four per power of two) and take
// a reusable block of their class before calling hipMalloc.
//
// Limits: blocks larger than kDirect bytes bypass the cache (hipMalloc and a
// synchronising hipFree, as before); reusable bytes above the device's cap
// are returned to the runtime by the background thread; when hipMalloc fails
// the allocating thread waits for the pending blocks, frees every cached
// block of that device and tries once more.  The cap is IBM_MEM_CACHE_MB
// (default 16384) per device.
//
// Runtime calls that synchronise (hipDeviceSynchronize, hipFree, hipMalloc)
// hold the capture lock shared, so they never overlap a graph capture in
// another thread.

#include "common.hpp"

#include <condition_variable>
#include <cstdlib>
#include <map>
#include <thread>
#include <unordered_map>

namespace ibm {
namespace {

constexpr size_t kDirect = (size_t)2 << 30;  // larger blocks are not cached

// smallest class >= b: multiples of 4 KiB up to 16 KiB, then four classes per
// power of two (at most 25% above the request)
size_t size_class(size_t b)
{
    if (b <= 16384) return (b + 4095) / 4096 * 4096;
    const int e = 63 - __builtin_clzll((unsigned long long)(b - 1));  // 2^e < b <= 2^(e+1)
    const size_t step = (size_t)1 << (e - 2);
    return (b + step - 1) / step * step;
}

struct DevCache {
    std::unordered_map<size_t, std::vector<void *>> ready;  // class -> reusable blocks
    std::vector<std::pair<void *, size_t>> pending;          // released, not yet behind a device sync
    size_t ready_bytes = 0;
    uint64_t synced = 0;  // completed device syncs
    bool busy = false;    // the worker is synchronising this device
};

class MemCache {
public:
    static MemCache &get()
    {
        // created on first use and never destroyed: the worker may still be
        // running while static objects are torn down (see stop_at_exit)
        static MemCache *m = new MemCache();
        return *m;
    }

    void *alloc(size_t bytes, int dev, size_t &cls)
    {
        if (bytes > kDirect) {
            cls = 0;
            return raw_malloc(bytes, dev, true);
        }
        cls = size_class(bytes);
        {
            std::lock_guard<std::mutex> lk(m_);
            DevCache &d = devs_[dev];
            auto it = d.ready.find(cls);
            if (it != d.ready.end() && !it->second.empty()) {
                void *p = it->second.back();
                it->second.pop_back();
                d.ready_bytes -= cls;
                return p;
            }
        }
        return raw_malloc(cls, dev, true);
    }

    void release(void *p, int dev, size_t cls)
    {
        if (!cls) {  // direct block
            std::shared_lock<std::shared_mutex> cl(capture_mutex());
            (void)hipFree(p);
            return;
        }
        std::lock_guard<std::mutex> lk(m_);
        devs_[dev].pending.emplace_back(p, cls);
        cv_.notify_all();
    }

private:
    std::mutex m_;
    std::condition_variable cv_;
    std::map<int, DevCache> devs_;
    std::thread worker_;
    bool stop_ = false;
    size_t cap_;

    MemCache()
    {
        const char *e = getenv("IBM_MEM_CACHE_MB");
        cap_ = (size_t)(e ? std::max(0L, atol(e)) : 16384L) << 20;
        worker_ = std::thread([this] { run(); });
        // joined before the runtime's own teardown: registered after the
        // runtime was loaded, so it runs first
        std::atexit(stop_at_exit);
    }

    static void stop_at_exit()
    {
        MemCache &m = get();
        {
            std::lock_guard<std::mutex> lk(m.m_);
            m.stop_ = true;
            m.cv_.notify_all();
        }
        if (m.worker_.joinable()) m.worker_.join();
    }

    // hipMalloc; on failure (when allowed) give the device's cached blocks
    // back to the runtime and try once more
    void *raw_malloc(size_t bytes, int dev, bool retry)
    {
        void *p = nullptr;
        hipError_t e;
        {
            std::shared_lock<std::shared_mutex> cl(capture_mutex());
            e = hipMalloc(&p, bytes);
        }
        if (e == hipSuccess) return p;
        (void)hipGetLastError();
        if (retry) {
            trim_all(dev);
            return raw_malloc(bytes, dev, false);
        }
        throw Error(IBM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }

    // wait until every block pending now is reusable, then free all of them
    void trim_all(int dev)
    {
        std::vector<void *> victims;
        {
            std::unique_lock<std::mutex> lk(m_);
            DevCache &d = devs_[dev];
            // the round in progress (if any) and one more for what is pending
            const uint64_t need = d.synced + (d.busy ? 1 : 0) + (d.pending.empty() ? 0 : 1);
            if (need > d.synced) {
                cv_.notify_all();
                cv_.wait(lk, [&] { return stop_ || d.synced >= need; });
            }
            for (auto &kv : d.ready)
                for (void *p : kv.second) victims.push_back(p);
            d.ready.clear();
            d.ready_bytes = 0;
        }
        std::shared_lock<std::shared_mutex> cl(capture_mutex());
        for (void *p : victims) (void)hipFree(p);
    }

    void run()
    {
        std::unique_lock<std::mutex> lk(m_);
        while (true) {
            int dev = -1;
            for (auto &kv : devs_)
                if (!kv.second.pending.empty()) { dev = kv.first; break; }
            if (dev < 0) {
                if (stop_) return;
                cv_.wait(lk);
                continue;
            }
            DevCache &d = devs_[dev];
            std::vector<std::pair<void *, size_t>> batch;
            batch.swap(d.pending);
            d.busy = true;
            lk.unlock();
            hipError_t e;
            {
                std::shared_lock<std::shared_mutex> cl(capture_mutex());
                e = hipSetDevice(dev);
                if (e == hipSuccess) e = hipDeviceSynchronize();
            }
            std::vector<void *> excess;
            lk.lock();
            if (e != hipSuccess) {
                // the device is unusable: keep the blocks out of circulation
                (void)hipGetLastError();
            } else {
                for (auto &b : batch) {
                    d.ready[b.second].push_back(b.first);
                    d.ready_bytes += b.second;
                }
                // over the cap: return the largest blocks first
                while (d.ready_bytes > cap_) {
                    auto big = d.ready.end();
                    for (auto it = d.ready.begin(); it != d.ready.end(); ++it)
                        if (!it->second.empty() && (big == d.ready.end() || it->first > big->first)) big = it;
                    if (big == d.ready.end()) break;
                    excess.push_back(big->second.back());
                    big->second.pop_back();
                    d.ready_bytes -= big->first;
                }
            }
            d.busy = false;
            ++d.synced;
            cv_.notify_all();
            if (!excess.empty()) {
                lk.unlock();
                {
                    std::shared_lock<std::shared_mutex> cl(capture_mutex());
                    for (void *p : excess) (void)hipFree(p);
                }
                lk.lock();
            }
        }
    }
};

}  // namespace

void *device_alloc(size_t bytes, int &dev, size_t &cls)
{
    IBM_HIP(hipGetDevice(&dev));
    return MemCache::get().alloc(bytes, dev, cls);
}

void device_release(void *p, int dev, size_t cls) { MemCache::get().release(p, dev, cls); }

}  // namespace ibm
