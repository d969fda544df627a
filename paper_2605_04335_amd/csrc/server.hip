// Continuous-batching solve server: a persistent scheduler thread admits
// requests while the number of active solves is below max_slots and their
// summed device footprints fit the HBM budget (first come, first served; a
// request larger than the whole budget is refused at once).  Every admitted
// solve runs on its own worker thread and HIP stream, so solves that arrive
// while others are on the GPU join them and their kernels overlap on the
// device; a finished solve returns its slot and memory immediately.  Each
// solve keeps its multigrid hierarchy resident for its lifetime and is
// deterministic, so a result does not depend on what else is running.

#include "common.hpp"

#include <cstdio>
#include <cstdlib>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include <csignal>
#include <cstring>
#include <execinfo.h>
#include <sys/syscall.h>
#include <unistd.h>

namespace ibm {
void classify(const ibm_grid *, const ibm_body *, int, uint8_t *, ibm_class_stats *, hipStream_t);
void build_stencils(const ibm_grid *, const ibm_body *, int, const uint8_t *, ibm_stencils **, hipStream_t,
                    int bc = 0);
size_t estimate_bytes(int nx, int ny, int nz, long long nrows, int precision);
}  // namespace ibm

using namespace ibm;

namespace {

struct BodyCopy {
    int kind;
    std::vector<double> v;
    std::vector<int32_t> t;
};

struct Request {
    uint64_t id = 0;
    HostGrid g;
    std::vector<BodyCopy> bodies;
    std::vector<double> f;
    poisson_opts opts;
    std::string key;            // exact bytes of grid, bodies and options
    poisson_ctx *ctx = nullptr; // a cached set-up handed over at admission
    size_t footprint = 0;
    int state = IBM_REQ_QUEUED;
    int rc = IBM_OK;
    std::string err;
    std::vector<double> x;
    poisson_stats stats{};
    poisson_req_times times{};
};

// solver set-ups kept after their solve
struct CacheEntry {
    std::string key;
    poisson_ctx *ctx = nullptr;
    size_t bytes = 0;
    uint64_t last = 0;
    bool busy = false;
};

template <class T>
void append_bytes(std::string &k, const T *p, size_t n)
{
    k.append(reinterpret_cast<const char *>(p), n * sizeof(T));
}

double now_ms(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// ---------------------------------------------------------------- crash report
// Opt-in (IBM_CRASH_TRACE set when a server is created): a fatal SIGSEGV,
// SIGBUS or SIGFPE in any thread of the process first writes the signal, the
// faulting address, the kernel thread id and that thread's native stack to
// standard error, then passes the signal on to the disposition installed
// before (Python's faulthandler, say, or the default action).  Installed once
// per process.  The handler makes only async-signal-safe calls; backtrace is
// called once at installation so that it does not load its unwinder inside
// the handler.  A fault from stack exhaustion is not reported (no alternate
// signal stack).
constexpr int kTraceSigs[3] = {SIGSEGV, SIGBUS, SIGFPE};
struct sigaction g_prev_action[3];

void put_str(const char *t)
{
    const ssize_t r = write(2, t, strlen(t));
    (void)r;
}

void put_num(unsigned long long v, unsigned base)
{
    char buf[24];
    int n = 0;
    do {
        const unsigned d = (unsigned)(v % base);
        buf[n++] = (char)(d < 10 ? '0' + d : 'a' + d - 10);
        v /= base;
    } while (v && n < 24);
    char out[25];
    for (int q = 0; q < n; ++q) out[q] = buf[n - 1 - q];
    out[n] = 0;
    put_str(out);
}

void crash_trace(int sig, siginfo_t *si, void *)
{
    put_str("[ibm] fatal signal ");
    put_num((unsigned)sig, 10);
    put_str(" at address 0x");
    put_num((unsigned long long)(uintptr_t)(si ? si->si_addr : nullptr), 16);
    put_str(" in thread ");
    put_num((unsigned long long)syscall(SYS_gettid), 10);
    put_str("; native stack:\n");
    void *fr[64];
    backtrace_symbols_fd(fr, backtrace(fr, 64), 2);
    for (int q = 0; q < 3; ++q)
        if (kTraceSigs[q] == sig) sigaction(sig, &g_prev_action[q], nullptr);
    // blocked while this handler runs: taken by the previous disposition on
    // return (a fault would also recur there)
    raise(sig);
}

void install_crash_trace()
{
    static std::once_flag once;
    std::call_once(once, [] {
        void *fr[4];
        (void)backtrace(fr, 4);
        struct sigaction sa;
        memset(&sa, 0, sizeof sa);
        sa.sa_sigaction = crash_trace;
        sa.sa_flags = SA_SIGINFO;
        sigemptyset(&sa.sa_mask);
        for (int q = 0; q < 3; ++q) sigaction(kTraceSigs[q], &sa, &g_prev_action[q]);
    });
}

}  // namespace

struct poisson_server {
    poisson_server_opts o;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> queue;
    std::map<uint64_t, std::unique_ptr<Request>> reqs;
    std::thread sched;
    size_t used = 0;
    int active = 0;
    uint64_t next_id = 1, tick = 0;
    bool stop = false;
    std::vector<CacheEntry> cache;

    void run_request(Request *r);
    void schedule();
    CacheEntry *find_idle(const std::string &key)
    {
        for (auto &e : cache)
            if (!e.busy && e.key == key) return &e;
        return nullptr;
    }
    size_t idle_bytes() const
    {
        size_t b = 0;
        for (auto &e : cache)
            if (!e.busy) b += e.bytes;
        return b;
    }
    // drop least recently used idle set-ups until `need` more bytes fit, or
    // until at most `keep` entries remain (caller holds mu); the caller
    // destroys the returned set-ups after releasing mu
    std::vector<poisson_ctx *> evict(size_t need, size_t keep)
    {
        std::vector<poisson_ctx *> gone;
        while (!cache.empty()) {
            const bool over_budget = used + need > o.hbm_budget, over_count = cache.size() > keep;
            if (!over_budget && !over_count) break;
            int lru = -1;
            for (int q = 0; q < (int)cache.size(); ++q)
                if (!cache[q].busy && (lru < 0 || cache[q].last < cache[lru].last)) lru = q;
            if (lru < 0) break;
            gone.push_back(cache[lru].ctx);
            used -= cache[lru].bytes;
            cache.erase(cache.begin() + lru);
        }
        return gone;
    }
    ~poisson_server()
    {
        for (auto &e : cache) poisson_destroy(e.ctx);
    }
};

void poisson_server::run_request(Request *r)
{
    int rc = IBM_OK;
    std::string err;
    hipStream_t s = nullptr;
    poisson_ctx *keep = nullptr;  // set-up to cache after the solve
    double setup_ms = 0.0, solve_ms = 0.0;  // published with the result, under mu
    try {
        IBM_HIP(hipSetDevice(o.device));
        IBM_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        ibm_grid g{r->g.n[0], r->g.n[1], r->g.n[2], r->g.f[0].data(), r->g.f[1].data(), r->g.f[2].data()};
        const long long N = (long long)g.nx * g.ny * g.nz;
        poisson_ctx *ctx = r->ctx;
        const auto ts = std::chrono::steady_clock::now();
        if (!ctx) {
            std::vector<ibm_body> bd;
            for (auto &b : r->bodies)
                bd.push_back(
                    ibm_body{(int32_t)(b.v.size() / 3), (int32_t)(b.t.size() / 3), b.kind, b.v.data(), b.t.data()});
            DBuf<uint8_t> flags(N);
            classify(&g, bd.data(), (int)bd.size(), flags.p, nullptr, s);
            ibm_stencils *st = nullptr;
            build_stencils(&g, bd.data(), (int)bd.size(), flags.p, &st, s);
            std::unique_ptr<ibm_stencils> stg(st);
            size_t bytes = 0;
            int e = poisson_setup(&g, flags.p, st, &r->opts, &bytes, &ctx);
            if (e) throw Error(e, ibm_last_error());
        }
        if (!r->ctx) setup_ms = now_ms(ts);  // the temporaries' release included
        const auto tv = std::chrono::steady_clock::now();
        std::unique_ptr<poisson_ctx, void (*)(poisson_ctx *)> cg(ctx, poisson_destroy);
        int64_t nun = 0;
        IBM_REQUIRE(poisson_level_info(ctx, nullptr, &nun, nullptr, nullptr) == IBM_OK, IBM_EINVAL, "level info");
        const long long nt = nun;
        DBuf<double> df(N), dx(nt);
        IBM_HIP(hipMemcpyAsync(df.p, r->f.data(), N * 8, hipMemcpyHostToDevice, s));
        rc = poisson_solve(ctx, df.p, nullptr, dx.p, &r->stats, s);
        if (rc && rc != IBM_ENOCONV) err = ibm_last_error();
        r->x.resize(nt);
        IBM_HIP(hipMemcpyAsync(r->x.data(), dx.p, nt * 8, hipMemcpyDeviceToHost, s));
        IBM_HIP(hipStreamSynchronize(s));
        solve_ms = now_ms(tv);
        if (o.cache_entries > 0) keep = cg.release();
    } catch (const Error &e) {
        rc = e.code;
        err = e.what();
    } catch (const std::exception &e) {
        rc = IBM_EINVAL;
        err = e.what();
    }
    if (s) (void)hipStreamDestroy(s);
    if (rc != IBM_OK && getenv("IBM_LOG")) fprintf(stderr, "[ibm] request failed (%d): %s\n", rc, err.c_str());
    std::vector<poisson_ctx *> gone;
    std::unique_lock<std::mutex> lk(mu);
    r->rc = rc;
    r->err = err;
    r->stats.status = rc;
    r->state = rc == IBM_OK || rc == IBM_ENOCONV ? IBM_REQ_DONE : IBM_REQ_FAILED;
    r->times.done_ms = now_ms(t0);
    r->times.setup_ms = setup_ms;
    r->times.solve_ms = solve_ms;
    if (r->ctx) {
        // a cached set-up: back to idle (its memory stays accounted), or gone
        // if the solve failed
        for (size_t q = 0; q < cache.size(); ++q)
            if (cache[q].ctx == r->ctx) {
                if (keep) { cache[q].busy = false; cache[q].last = ++tick; }
                else { used -= cache[q].bytes; cache.erase(cache.begin() + q); }
                break;
            }
    } else if (keep) {
        CacheEntry e;
        e.key = r->key;
        e.ctx = keep;
        e.bytes = r->footprint;  // stays accounted while cached
        e.last = ++tick;
        cache.push_back(std::move(e));
        gone = evict(0, (size_t)o.cache_entries);
    } else {
        used -= r->footprint;
    }
    if (!gone.empty()) {
        // evicted set-ups are released outside the lock but before this
        // worker counts as finished, so that poisson_server_destroy returns
        // only once no worker touches the device any more
        lk.unlock();
        for (poisson_ctx *c : gone) poisson_destroy(c);
        lk.lock();
    }
    --active;
    cv.notify_all();
}

void poisson_server::schedule()
{
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        cv.wait(lk, [&] {
            if (stop) return true;
            if (queue.empty()) return false;
            Request *h = queue.front();
            if (h->footprint > o.hbm_budget) return true;
            if (active >= o.max_slots) return false;
            return find_idle(h->key) != nullptr || used - idle_bytes() + h->footprint <= o.hbm_budget;
        });
        if (stop && queue.empty()) break;
        if (stop) {  // refuse what is still queued
            for (Request *r : queue) {
                r->state = IBM_REQ_FAILED;
                r->rc = IBM_EAGAIN;
                r->err = "server stopped";
            }
            queue.clear();
            cv.notify_all();
            break;
        }
        Request *r = queue.front();
        queue.pop_front();
        if (r->footprint > o.hbm_budget) {
            r->state = IBM_REQ_FAILED;
            r->rc = IBM_ENOMEM;
            r->err = "request footprint exceeds the HBM budget";
            r->stats.status = IBM_ENOMEM;
            r->times.admit_ms = r->times.done_ms = now_ms(t0);
            cv.notify_all();
            continue;
        }
        if (CacheEntry *e = find_idle(r->key)) {
            e->busy = true;
            r->ctx = e->ctx;
            r->times.cache_hit = 1;
        } else {
            std::vector<poisson_ctx *> gone = evict(r->footprint, (size_t)o.cache_entries);
            used += r->footprint;
            if (!gone.empty()) {
                lk.unlock();
                for (poisson_ctx *c : gone) poisson_destroy(c);
                lk.lock();
            }
        }
        ++active;
        r->state = IBM_REQ_RUNNING;
        r->times.admit_ms = now_ms(t0);
        std::thread([this, r] { run_request(r); }).detach();
    }
}

extern "C" int32_t poisson_server_create(const poisson_server_opts *opts, poisson_server **out)
{
    return guarded([&] {
        IBM_REQUIRE(opts && out && opts->max_slots >= 1 && opts->hbm_budget > 0, IBM_EINVAL, "bad server options");
        if (getenv("IBM_CRASH_TRACE")) install_crash_trace();
        auto *S = new poisson_server();
        S->o = *opts;
        S->t0 = std::chrono::steady_clock::now();
        S->sched = std::thread([S] { S->schedule(); });
        *out = S;
    });
}

extern "C" int32_t poisson_submit(poisson_server *S, const poisson_request *q, uint64_t *ticket)
{
    return guarded([&] {
        IBM_REQUIRE(S && q && ticket && q->f, IBM_EINVAL, "null argument");
        IBM_REQUIRE(q->n_body >= 0 && (q->n_body == 0 || q->bodies), IBM_EINVAL, "bad body list");
        auto r = std::make_unique<Request>();
        r->g = read_grid(&q->grid);
        for (int b = 0; b < q->n_body; ++b) {
            const ibm_body &B = q->bodies[b];
            IBM_REQUIRE(B.vert && B.tri && B.n_vert > 0 && B.n_tri > 0, IBM_EINVAL, "empty body");
            BodyCopy c;
            c.kind = B.kind;
            c.v.assign(B.vert, B.vert + 3 * (size_t)B.n_vert);
            c.t.assign(B.tri, B.tri + 3 * (size_t)B.n_tri);
            r->bodies.push_back(std::move(c));
        }
        const long long N = (long long)r->g.n[0] * r->g.n[1] * r->g.n[2];
        r->f.assign(q->f, q->f + N);
        r->opts = q->opts;
        append_bytes(r->key, r->g.n, 3);
        for (int d = 0; d < 3; ++d) append_bytes(r->key, r->g.f[d].data(), r->g.f[d].size());
        for (auto &b : r->bodies) {
            append_bytes(r->key, &b.kind, 1);
            const size_t nv = b.v.size(), nt = b.t.size();
            append_bytes(r->key, &nv, 1);
            append_bytes(r->key, b.v.data(), nv);
            append_bytes(r->key, &nt, 1);
            append_bytes(r->key, b.t.data(), nt);
        }
        const poisson_opts &po = r->opts;  // field by field: no padding bytes in the key
        const double od[2] = {po.tol, po.inner_tol};
        const int32_t oi[9] = {po.precision, po.max_iter,    po.nu1,     po.nu2,       po.coarse_sweeps,
                               po.max_outer, po.use_graph, po.precond, po.srj_sweeps};
        static_assert(sizeof(poisson_opts) == 56, "poisson_opts changed: every field belongs in the cache key");
        append_bytes(r->key, od, 2);
        append_bytes(r->key, oi, 9);
        // footprint: solver workspace plus classification temporaries, with a
        // generous bound on the ghost rows (one cell in eight)
        r->footprint = estimate_bytes(r->g.n[0], r->g.n[1], r->g.n[2], N / 8, q->opts.precision) + (size_t)N +
                       (size_t)N / 2 + (size_t)16 * N;
        std::lock_guard<std::mutex> lk(S->mu);
        r->id = S->next_id++;
        r->times.submit_ms = now_ms(S->t0);
        *ticket = r->id;
        S->queue.push_back(r.get());
        S->reqs[r->id] = std::move(r);
        S->cv.notify_all();
    });
}

extern "C" int32_t poisson_poll(poisson_server *S, uint64_t ticket, double *x_out, int64_t x_len,
                                poisson_stats *stats, poisson_req_times *times, int32_t *state)
{
    int rc = IBM_OK;
    int32_t g = guarded([&] {
        IBM_REQUIRE(S, IBM_EINVAL, "null server");
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->reqs.find(ticket);
        if (it == S->reqs.end()) throw Error(IBM_ENOTFOUND, "unknown ticket");
        Request *r = it->second.get();
        if (state) *state = r->state;
        if (times) *times = r->times;
        if (r->state == IBM_REQ_QUEUED || r->state == IBM_REQ_RUNNING) { rc = IBM_EAGAIN; return; }
        if (times) times->n_unknowns = (int64_t)r->x.size();
        if (stats) *stats = r->stats;
        if (x_out && !r->x.empty()) {
            IBM_REQUIRE(x_len >= (int64_t)r->x.size(), IBM_EINVAL, "x_out too short");
            std::copy(r->x.begin(), r->x.end(), x_out);
        }
        rc = r->rc;
        std::string err = r->err;
        S->reqs.erase(it);
        if (rc) throw Error(rc, err);
    });
    if (g) return g;
    return rc;
}

extern "C" int32_t poisson_server_drain(poisson_server *S)
{
    return guarded([&] {
        IBM_REQUIRE(S, IBM_EINVAL, "null server");
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv.wait(lk, [&] { return S->queue.empty() && S->active == 0; });
    });
}

extern "C" void poisson_server_destroy(poisson_server *S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    if (S->sched.joinable()) S->sched.join();
    {
        // detached workers finish their solve before the server goes away
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv.wait(lk, [&] { return S->active == 0; });
    }
    delete S;
}
