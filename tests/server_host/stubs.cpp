// Stand-ins for the GPU work behind the solve server (test infrastructure):
// set-up and solve sleep for a while and read and write library-owned
// buffers, so that the server's scheduler and worker threads, its set-up
// cache and the device-memory cache run as they do with the real solver.
#include "common.hpp"
#include <atomic>
#include <random>
#include <thread>
using namespace ibm;
struct poisson_ctx {
    int64_t nt = 0;
    DBuf<double> a, b;
};
namespace ibm {
void classify(const ibm_grid *g, const ibm_body *, int, uint8_t *flags, ibm_class_stats *, hipStream_t)
{
    const long long N = (long long)g->nx * g->ny * g->nz;
    std::memset(flags, 0, N);
}
void build_stencils(const ibm_grid *g, const ibm_body *, int, const uint8_t *, ibm_stencils **out, hipStream_t, int)
{
    auto *s = new ibm_stencils();
    s->N = (long long)g->nx * g->ny * g->nz;
    s->cell.alloc(64);
    s->col.alloc(512);
    *out = s;
}
size_t estimate_bytes(int nx, int ny, int nz, long long nrows, int) { return (size_t)nx * ny * nz * 120 + nrows * 200; }
HostGrid read_grid(const ibm_grid *g)
{
    HostGrid h;
    h.n[0] = g->nx; h.n[1] = g->ny; h.n[2] = g->nz;
    h.f[0].assign(g->xf, g->xf + g->nx + 1);
    h.f[1].assign(g->yf, g->yf + g->ny + 1);
    h.f[2].assign(g->zf, g->zf + g->nz + 1);
    return h;
}
}  // namespace ibm
static thread_local std::mt19937 rng(std::hash<std::thread::id>()(std::this_thread::get_id()));
extern "C" int32_t poisson_setup(const ibm_grid *g, const uint8_t *, const ibm_stencils *, const poisson_opts *,
                                 size_t *bytes, poisson_ctx **out)
{
    return guarded([&] {
        auto *c = new poisson_ctx();
        c->nt = (long long)g->nx * g->ny * g->nz;
        c->a.alloc(c->nt);
        c->b.alloc(c->nt / 2 + 1);
        std::this_thread::sleep_for(std::chrono::microseconds(200 + rng() % 800));
        if (bytes) *bytes = c->nt * 24;
        *out = c;
    });
}
extern "C" int32_t poisson_level_info(poisson_ctx *c, int32_t *lv, int64_t *nun, int64_t *ng, int64_t *nm)
{
    if (lv) *lv = 3;
    if (nun) *nun = c->nt;
    if (ng) *ng = 0;
    if (nm) *nm = 0;
    return 0;
}
extern "C" int32_t poisson_solve(poisson_ctx *c, const double *f, const double *, double *x, poisson_stats *st, void *)
{
    return guarded([&] {
        DBuf<double> tmp(c->nt);
        std::memcpy(tmp.p, f, c->nt * 8);
        std::this_thread::sleep_for(std::chrono::microseconds(300 + rng() % 3000));
        std::memcpy(x, tmp.p, c->nt * 8);
        std::memcpy(c->a.p, tmp.p, c->nt * 8);
        st->iterations = 7;
        st->rel_residual = 1e-9;
    });
}
extern "C" void poisson_destroy(poisson_ctx *c)
{
    if (c) delete c;
}
extern "C" void poisson_default_opts(poisson_opts *o)
{
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-8; o->max_iter = 100; o->nu1 = 2; o->nu2 = 2; o->coarse_sweeps = 32;
}
