// Drives the solve server as a client does (test infrastructure): Poisson
// arrivals at a high rate, every request polled until it is done, requests
// that repeat a grid and options (set-up cache hits) and new ones (cache
// evictions), an HBM budget small enough that admission waits.
// usage: drive [requests] [rate per s] [budget MB] [cache entries]
//        drive crash <address>: create a server, then store through
//        <address> (0 in the test) from a thread of its own, so that the
//        crash report of IBM_CRASH_TRACE can be checked on the host
#include "ibm_poisson.h"
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <thread>
#include <vector>
int main(int argc, char **argv)
{
    if (argc > 2 && !strcmp(argv[1], "crash")) {
        poisson_server_opts so{(size_t)1 << 26, 4, 0, 0};
        poisson_server *S = nullptr;
        if (poisson_server_create(&so, &S)) { printf("create failed\n"); return 1; }
        volatile int *bad = reinterpret_cast<volatile int *>((uintptr_t)strtoull(argv[2], nullptr, 0));
        std::thread([bad] { *bad = 1; }).join();
        poisson_server_destroy(S);
        printf("no crash\n");
        return 0;
    }
    const int nreq = argc > 1 ? atoi(argv[1]) : 3000;
    const double rate = argc > 2 ? atof(argv[2]) : 2000.0;
    const size_t mb = argc > 3 ? (size_t)atoi(argv[3]) : 64;
    const int cache = argc > 4 ? atoi(argv[4]) : 8;
    poisson_server_opts so{mb << 20, 16, 0, cache};
    poisson_server *S = nullptr;
    if (poisson_server_create(&so, &S)) { printf("create failed\n"); return 1; }
    std::mt19937 rng(5);
    std::exponential_distribution<double> ex(rate);
    struct G { int n[3]; std::vector<double> f[3]; std::vector<double> rhs; };
    std::vector<G> grids(40);
    for (int q = 0; q < 40; ++q) {
        G &g = grids[q];
        for (int d = 0; d < 3; ++d) {
            g.n[d] = 8 + (int)(rng() % 24);
            g.f[d].resize(g.n[d] + 1);
            for (int i = 0; i <= g.n[d]; ++i) g.f[d][i] = i / (double)g.n[d];
        }
        g.rhs.assign((size_t)g.n[0] * g.n[1] * g.n[2], 1.0);
    }
    std::map<uint64_t, int> pending;
    auto t0 = std::chrono::steady_clock::now();
    double next = 0.0;
    int sent = 0, done = 0, failed = 0;
    while (sent < nreq || !pending.empty()) {
        const double now = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        while (sent < nreq && next <= now) {
            G &g = grids[rng() % grids.size()];
            poisson_request rq{};
            rq.grid = ibm_grid{g.n[0], g.n[1], g.n[2], g.f[0].data(), g.f[1].data(), g.f[2].data()};
            rq.bodies = nullptr;
            rq.n_body = 0;
            rq.f = g.rhs.data();
            poisson_default_opts(&rq.opts);
            rq.opts.precision = (int)(rng() % 2);
            uint64_t t;
            if (poisson_submit(S, &rq, &t) == 0) pending[t] = 1;
            ++sent;
            next += ex(rng);
        }
        for (auto it = pending.begin(); it != pending.end();) {
            poisson_stats st; poisson_req_times tm; int32_t state;
            int rc = poisson_poll(S, it->first, nullptr, 0, &st, &tm, &state);
            if (rc == IBM_EAGAIN) { ++it; continue; }
            if (rc) ++failed;
            ++done;
            it = pending.erase(it);
        }
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    poisson_server_destroy(S);
    printf("done %d failed %d\n", done, failed);
    return 0;
}
