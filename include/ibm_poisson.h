/*
 * ibm_poisson.h -- C ABI of the MI355X (gfx950) ghost-cell immersed-boundary
 * pressure-Poisson library (libibmpoisson.so).
 *
 * The library implements the pressure Poisson equation (PPE) step of a
 * fractional-step, sharp-interface immersed-boundary flow solver (Kumar,
 * Seo, Mittal, Romero, Fatica, "GPU-Accelerated Simulations of Moving
 * Boundary Problems and Fluid-Structure Interaction at Extreme Scales",
 * arXiv 2605.04335; Sec. 2.1 fractional step and PPE by BiCGStab, Sec. 2.5
 * the three GPU modules: iblanking, ghost-cell boundary conditions, sparse
 * matrix-free + ELLPACK solvers).  Every step runs in HIP kernels on the
 * device; this header has no HIP or framework types.
 *
 * Conventions
 *   - Grid: nx*ny*nz cells, faces xf[0..nx] etc. strictly increasing, each
 *     dimension >= 4.  Fields are x-fastest: idx = i + nx*(j + ny*k).
 *   - Unknown vectors have length N + n_mghost: the N cell values followed
 *     by one ghost unknown per membrane ghost cell (in cell-index order).
 *   - "host" pointers are read during the call only (copied); "device"
 *     pointers are caller-owned device memory that must outlive the work
 *     enqueued on the given stream.  A stream argument is a hipStream_t
 *     passed as void* (NULL = the null stream).
 *   - Every function returns 0 on success or a negative IBM_E* code; the
 *     message of the last failure on the calling thread is ibm_last_error().
 *   - Device memory the library allocates for itself (contexts, stencils,
 *     temporaries) comes from a per-device cache: a released block is not
 *     returned with hipFree (which waits for the whole device) but reused
 *     by later allocations of its size class once a background thread has
 *     synchronised the device.  Blocks above 2 GiB bypass the cache.  The
 *     environment variable IBM_MEM_CACHE_MB (default 16384) caps the cached
 *     bytes per device; when hipMalloc fails, the cached blocks of that
 *     device are freed and the allocation is tried once more.
 *   - IBM_LOG set in the environment: refinement steps, fallbacks and
 *     failed server requests are reported on stderr (IBM_LOG=2 adds every
 *     BiCGSTAB iteration).
 */
#ifndef IBM_POISSON_H
#define IBM_POISSON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IBM_OK 0
#define IBM_EINVAL (-1)      /* null pointer, bad sizes, non-increasing faces, body too far out */
#define IBM_EGEOM (-2)       /* bad mesh indices, degenerate triangle, no fluid cell */
#define IBM_ENOMEM (-3)      /* device allocation failed, workspace too small, request cannot be admitted */
#define IBM_EHIP (-4)        /* HIP runtime error (message carries the HIP error string) */
#define IBM_ENOCONV (-5)     /* iteration limit reached; x holds the last iterate, stats are filled */
#define IBM_EBREAKDOWN (-6)  /* BiCGSTAB breakdown or non-finite values */
#define IBM_EAGAIN (-7)      /* poll: request not finished */
#define IBM_ENOTFOUND (-8)   /* poll: unknown ticket */

#define IBM_KIND_CLOSED 0    /* watertight, outward-oriented triangulated body */
#define IBM_KIND_MEMBRANE 1  /* zero-thickness open sheet */

/* flag bits of the classification (one byte per cell) */
#define IBM_F_SOLID 0x01
#define IBM_F_GHOST 0x02     /* solid cell with a fluid face neighbour */
#define IBM_F_MGHOST 0x04    /* fluid cell with at least one membrane-cut link */
#define IBM_F_PIN 0x08       /* the gauge cell: first fluid non-membrane-ghost cell */
#define IBM_F_CUTX 0x10      /* link (i,j,k)-(i+1,j,k) crosses a membrane */
#define IBM_F_CUTY 0x20
#define IBM_F_CUTZ 0x40

typedef struct ibm_grid {
    int32_t nx, ny, nz;
    const double *xf, *yf, *zf; /* host, lengths nx+1, ny+1, nz+1 */
} ibm_grid;

typedef struct ibm_body {
    int32_t n_vert, n_tri, kind; /* kind: IBM_KIND_* */
    const double *vert;          /* host, n_vert*3 coordinates */
    const int32_t *tri;          /* host, n_tri*3 vertex indices */
} ibm_body;

typedef struct ibm_class_stats {
    int64_t n_solid, n_ghost, n_mghost, n_cut_links, pin;
} ibm_class_stats;

typedef struct ibm_stencils ibm_stencils; /* opaque, library-owned, device-resident */
typedef struct poisson_ctx poisson_ctx;   /* opaque, library-owned */

#define IBM_PREC_FP64 0
#define IBM_PREC_MIXED 1

/* Preconditioner of the BiCGSTAB iteration.  MG: the geometric-multigrid
 * V-cycle (default).  SRJ: scheduled relaxation Jacobi, the preconditioner
 * the paper pairs with BiCGStab for the PPE (Sec. 2.1): srj_sweeps weighted
 * Jacobi sweeps from zero with relaxation factors 1/k_s, k_s the roots of the
 * degree-srj_sweeps Chebyshev polynomial on [16/srj_sweeps^2, 2] (the
 * minimax schedule for the amplification over the spectrum of D^-1 A),
 * applied smallest, largest, second smallest, ...  srj_sweeps is limited to
 * 1..IBM_SRJ_MAX_SWEEPS (IBM_EINVAL otherwise): the Neumann ghost rows give
 * D^-1 A modes, localised at the ghost cells and their fluid neighbours, that
 * longer schedules (largest factor ~ srj_sweeps^2 / 16) amplify instead of
 * damp on grids of 128^3 and more. */
#define IBM_PRECOND_MG 0
#define IBM_PRECOND_SRJ 1
#define IBM_SRJ_MAX_SWEEPS 16

typedef struct poisson_opts {
    int32_t precision;      /* IBM_PREC_FP64 or IBM_PREC_MIXED */
    double tol;             /* relative true residual ||b - A x|| / ||b|| */
    int32_t max_iter;       /* BiCGSTAB iterations (FP64) / inner iterations per outer step (mixed) */
    int32_t nu1, nu2;       /* pre/post smoothing steps of the V-cycle */
    int32_t coarse_sweeps;  /* red-black sweeps on the coarsest level */
    double inner_tol;       /* mixed: relative tolerance of each inner solve */
    int32_t max_outer;      /* mixed: outer refinement steps */
    int32_t use_graph;      /* replay each iteration as a captured HIP graph */
    int32_t precond;        /* IBM_PRECOND_MG or IBM_PRECOND_SRJ */
    int32_t srj_sweeps;     /* SRJ: Jacobi sweeps per preconditioner application */
} poisson_opts;

typedef struct poisson_stats {
    int32_t iterations;      /* BiCGSTAB iterations (summed over outer steps when mixed) */
    int32_t outer_steps;     /* mixed: refinement steps taken */
    int32_t status;          /* same code as the return value */
    int32_t levels;          /* multigrid levels */
    double rel_residual;     /* final true relative residual, FP64 (also when the
                                iteration limit or a breakdown ends the solve) */
    double pin_residual;     /* unpinned-operator residual at the pin (inconsistency of the RHS) */
    double solve_ms;         /* device time of the whole solve (events on the stream) */
    int64_t n_fallback;      /* ghost rows that took the first-order fallback */
} poisson_stats;

/* Defaults: FP64, tol 1e-10, 200 iterations, V(2,2), 32 coarse sweeps,
 * inner_tol 1e-3, max_outer 10, graphs on, multigrid preconditioner
 * (srj_sweeps 16 when SRJ is chosen).  Each inner solve of the mixed
 * form asks for max(inner_tol, tol / (2 rel)) where rel is the current FP64
 * relative residual: tighter inner tolerances buy little, because the BF16
 * rounding of the coarse right-hand sides makes the preconditioner slightly
 * non-linear and the inner Krylov iteration slows down below ~1e-3.
 * Refinement switches to an FP64 BiCGSTAB on the remaining residual when an
 * outer step makes the FP64 residual larger (that step is undone) or when an
 * inner solve stops before its tolerance: at max_iter, or when it has not
 * halved its residual within 12 iterations (FP32 vectors cannot resolve a
 * correction below about kappa * 6e-8 of the residual). */
void poisson_default_opts(poisson_opts *opts);

/*
 * ibm_classify -- "iblanking" (Sec. 2.5, module 1): voxel classification of
 * the grid against triangulated bodies.  Closed bodies: a cell is solid iff
 * the ray along +x through its centre crosses the body an odd number of
 * times before the centre, counted with exact integer predicates on a
 * 2^16-per-longest-edge lattice and a top-left tie rule.  Membranes: a link
 * between face neighbours is cut iff an odd number of membrane triangles
 * cross it.  Then ghost, membrane-ghost, cut and pin bits (see IBM_F_*).
 *   grid, bodies (host, copied); flags_dev: device uint8[N], written;
 *   st (host, may be NULL): counts.  Bodies must lie within one domain length
 *   of the domain.  Stream-ordered; synchronises once to read the counts.
 */
int32_t ibm_classify(const ibm_grid *grid, const ibm_body *bodies, int32_t n_body, uint8_t *flags_dev,
                     ibm_class_stats *st, void *stream);

/*
 * ibm_classify_noalloc -- ibm_classify for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments, results and synchronisation as
 * ibm_classify, but every device buffer of the call (faces, quantised
 * centres and vertices, toggle and cut-link bitsets, per-ray markers,
 * counters) is carved from one fixed array of IBM_CLASSIFY_NOALLOC_MAX_BYTES
 * in device memory that each GPU the library runs on holds until the process
 * ends; the call makes no hipMalloc, hipFree or other allocating call.
 *   scratch_bytes (host, may be NULL): the scratch this input needs.
 * Needs about N/8 bytes with closed bodies, 3N/8 with membranes, N/2 with
 * both (N cells), plus 48 bytes per vertex and 12 per triangle (a 512^3
 * grid with membranes takes 48 MiB of bitsets; closed bodies alone fit up to
 * about 800^3 cells).  An input that needs more
 * than the maximum returns IBM_ENOMEM with *scratch_bytes set and nothing
 * enqueued.  The array keeps the last call's contents (the call clears what
 * it needs).  Calls that overlap on one GPU (concurrent host threads, or
 * streams not ordered with each other) race on the shared array: serialise
 * them.
 */
#define IBM_CLASSIFY_NOALLOC_MAX_BYTES (64u << 20)
int32_t ibm_classify_noalloc(const ibm_grid *grid, const ibm_body *bodies, int32_t n_body, uint8_t *flags_dev,
                             ibm_class_stats *st, size_t *scratch_bytes, void *stream);

/*
 * ibm_build_ghost_stencils -- ghost-cell boundary rows (Sec. 2.5, module 2;
 * GCM of Mittal et al. 2008): for each closed ghost cell and each membrane
 * ghost unknown, the body intercept (closest point on the body surface of
 * the same kind), the image point mirrored through it, and the trilinear
 * image-point weights of a homogeneous-Neumann row, from an 8x8 FP64 LU
 * solve with partial pivoting per ghost (the batched inversions of Sec. 2.5).
 *   flags_dev: the output of ibm_classify; *out receives a library-owned
 *   table (free with ibm_stencils_free).  Synchronises to size the table.
 * Columns are int32, so cells plus membrane ghost unknowns must stay below
 * 2^31 (IBM_EINVAL otherwise).
 */
int32_t ibm_build_ghost_stencils(const ibm_grid *grid, const ibm_body *bodies, int32_t n_body,
                                 const uint8_t *flags_dev, ibm_stencils **out, void *stream);

/* Boundary condition of the ghost rows.  NEUMANN: the pressure rows above.
 * DIRICHLET: rows of the advection-diffusion step, where the value at BI is
 * the mean of the ghost and image-point values; when G is a node of the box
 * a value row at BI replaces the derivative row, giving
 * sG (sum w x + x_G) = sG (2 - beta_BI) g with dlb = 2 - beta_BI (a ghost on
 * the surface gets x_G = g, dlb = 1; the first-order fallback uses the
 * neighbour mean with dlb = 2). */
#define IBM_BC_NEUMANN 0
#define IBM_BC_DIRICHLET 1

/* ibm_build_ghost_stencils with the boundary condition chosen (IBM_EINVAL
 * for another value); ibm_build_ghost_stencils is the NEUMANN case. */
int32_t ibm_build_ghost_stencils_bc(const ibm_grid *grid, const ibm_body *bodies, int32_t n_body,
                                    const uint8_t *flags_dev, int32_t bc, ibm_stencils **out, void *stream);

/* Row counts of a stencil table (any pointer may be NULL). */
int32_t ibm_stencils_info(const ibm_stencils *s, int64_t *n_ghost, int64_t *n_mghost, int64_t *n_fallback);

/*
 * Host copies of the table, rows = n_ghost closed ghosts then n_mghost
 * membrane ghosts, both in cell order: cell[rows]; col[rows*8] value
 * columns (cell index or N + membrane index, -1 unused or derivative node);
 * w[rows*8]; sG[rows] row scale; dlb[rows] = dl - beta_BI (the row's RHS is
 * sG*dlb*g); rflags[rows] bit0 fallback, bit1 derivative row, bit2
 * degenerate distance; geo[rows*12] (may be NULL): BI, IP, n, dl, beta_BI,
 * distance.  All arrays are caller-allocated host memory.
 */
int32_t ibm_stencils_export(const ibm_stencils *s, int32_t *cell, int32_t *col, double *w, double *sG, double *dlb,
                            uint8_t *rflags, double *geo);

void ibm_stencils_free(ibm_stencils *s);

/*
 * poisson_setup -- builds the solver for one classified grid: copies the
 * flags and the ghost rows into a device-resident level-0 operator
 * (matrix-free 7-point bulk + ELL irregular rows, Sec. 2.5 module 3), the
 * multigrid hierarchy and the Krylov work vectors, all in library-owned
 * device memory.  *workspace_bytes (may be NULL) receives that footprint.
 * flags_dev and the stencil table are not referenced after the call.
 * IBM_EINVAL for bad options, a table of another grid, or more than 2^31
 * unknowns (cell slots, each x-row padded to even length, plus membrane
 * ghost unknowns: the row columns are int32).
 */
int32_t poisson_setup(const ibm_grid *grid, const uint8_t *flags_dev, const ibm_stencils *st,
                      const poisson_opts *opts, size_t *workspace_bytes, poisson_ctx **out);

/*
 * Caller-owned workspace.  poisson_workspace_size reports the bytes of the
 * context's per-call scratch (Krylov vectors, multigrid iterates and
 * right-hand sides -- everything but the operator tables, which stay
 * library-owned).  poisson_bind_workspace moves that scratch into ws_dev
 * (device memory of at least that size, 256-byte aligned, e.g. a torch uint8
 * tensor): the library frees its own copies and never frees ws_dev, which
 * must outlive the context or the next bind.  Contents of the scratch do not
 * carry over between calls, so binding never changes results.  Returns
 * IBM_ENOMEM when bytes is too small.  Not thread-safe with work in flight on
 * the context.
 */
int32_t poisson_workspace_size(poisson_ctx *ctx, size_t *bytes);
int32_t poisson_bind_workspace(poisson_ctx *ctx, void *ws_dev, size_t bytes);

/* Device bytes a poisson_setup of this grid would hold (for admission). */
int32_t poisson_workspace_estimate(int32_t nx, int32_t ny, int32_t nz, int64_t n_rows, int32_t precision,
                                   size_t *bytes);

/*
 * poisson_solve -- the PPE solve of the fractional step (Sec. 2.1: the
 * pressure Poisson equation, solved by BiCGStab with a preconditioner; Sec.
 * 2.5, module 3: matrix-free bulk rows plus ELLPACK ghost rows): RHS assembly (fluid f projected to zero
 * volume-weighted mean, pin row 0, ghost rows sG*dlb*g), right-preconditioned
 * BiCGSTAB (van der Vorst 1992) with a geometric-multigrid V-cycle on the
 * pinned system, FP64 (or mixed: FP32/BF16 inner solves inside FP64
 * iterative refinement), then the gauge (volume-weighted fluid mean removed).
 *   f_dev: device double[N]; g_dev: device double[n_ghost+n_mghost] or NULL
 *   (homogeneous Neumann); x_dev: device double[N+n_mghost], output.
 * Blocks the calling thread until done.  Returns IBM_ENOCONV with the last
 * iterate in x_dev when the iteration limit is hit.
 */
int32_t poisson_solve(poisson_ctx *ctx, const double *f_dev, const double *g_dev, double *x_dev,
                      poisson_stats *stats, void *stream);

/*
 * ibm_surface_forces -- pressure loads on the bodies (Sec. 2.3.1, Eq. fext
 * without the shear term; the surface pressure handed to the structural
 * solver each step, Sec. 2.4).  Per triangle: centroid c, area A, unit
 * normal n = (v1-v0) x (v2-v0) / |.| (vertex order; outward for closed
 * bodies), probe distance d = 2 max(w_x, w_y, w_z) of the cell holding c.
 * p+ is the trilinear interpolation of the cell pressures at c + d n (box
 * clamped to the outermost centres; nodes in solid non-ghost cells dropped,
 * remaining weights renormalised); membranes also take p- at c - d n.
 * dp = p+ - p- (membrane) or p+ (closed body, fluid outside).  Each node of
 * the triangle receives -(1/3) dp n A, summed per node in a fixed order.
 *   flags_dev: device uint8[N] (ibm_classify); p_dev: device double[>= N],
 *   cell pressures in natural order (a poisson_solve output);
 *   force_dev: device double[3 * total vertices], body by body (output);
 *   dp_dev: device double[total triangles] or NULL (output);
 *   n_lost (may be NULL): probes with no usable node (their p is 0).
 * Synchronous with stream.  IBM_EINVAL for null pointers or empty bodies,
 * IBM_EGEOM for triangle indices out of range.
 */
int32_t ibm_surface_forces(const ibm_grid *grid, const ibm_body *bodies, int32_t n_body, const uint8_t *flags_dev,
                           const double *p_dev, double *force_dev, double *dp_dev, int64_t *n_lost, void *stream);

/*
 * Advection-diffusion step (Sec. 2.1: the momentum equations of the
 * fractional step are solved with scheduled relaxed Jacobi).  One velocity
 * component: H u = u - beta L u on fluid cells, L the 7-point operator of the
 * pressure system (zero-flux walls, the far side's ghost unknown across a cut
 * membrane link), beta = nu dt (times 1/2 for Crank-Nicolson); Dirichlet
 * ghost rows from ibm_build_ghost_stencils_bc(..., IBM_BC_DIRICHLET, ...);
 * solid non-ghost unknowns are 0.  SRJ cycle: `sweeps` weighted Jacobi
 * sweeps u <- u + omega_s D^-1 (rhs - H u), D = 1 + beta sum c (fluid) or sG
 * (ghost rows), omega_s the reciprocals of the degree-`sweeps` Chebyshev
 * roots on [a, 2 - a], a = 1 / (1 + beta max sum c); the relative residual
 * ||rhs - H u|| / ||rhs|| is checked after every cycle.
 */
typedef struct ibm_ad_ctx ibm_ad_ctx; /* opaque, library-owned */

typedef struct ibm_ad_opts {
    double beta;         /* diffusion number nu dt (>= 0) */
    double tol;          /* relative residual */
    int32_t sweeps;      /* SRJ sweeps per cycle, 1..64 */
    int32_t max_cycles;  /* cycle limit */
} ibm_ad_opts;

typedef struct ibm_ad_stats {
    int32_t cycles, sweeps, status;
    double rel_residual; /* final relative residual (device reduction order) */
    double solve_ms;     /* device time of the solve */
} ibm_ad_stats;

/* Defaults: beta 0, tol 1e-10, 8 sweeps per cycle, 500 cycles. */
void ibm_ad_default_opts(ibm_ad_opts *opts);
/* Set-up from the classification (device uint8[N]) and a Dirichlet table
 * (IBM_EINVAL for a Neumann one or another grid); copies what it needs. */
int32_t ibm_ad_setup(const ibm_grid *grid, const uint8_t *flags_dev, const ibm_stencils *st, const ibm_ad_opts *opts,
                     ibm_ad_ctx **out);
/* y = H x, device double[N + n_mghost] each, natural order. */
int32_t ibm_ad_apply(ibm_ad_ctx *ctx, const double *x_dev, double *y_dev, void *stream);
/* Solve H u = rhs, rhs = f on fluid cells (device double[N]) and
 * sG dlb g on ghost rows (g_dev: device double[n_ghost + n_mghost], the wall
 * velocity at each row's BI; NULL for walls at rest).  u_dev
 * (double[N + n_mghost]) holds the initial guess on entry and the solution on
 * return.  Blocks until done; IBM_ENOCONV at the cycle limit (u holds the
 * last iterate), IBM_EBREAKDOWN for a non-finite residual. */
int32_t ibm_ad_solve(ibm_ad_ctx *ctx, const double *f_dev, const double *g_dev, double *u_dev, ibm_ad_stats *stats,
                     void *stream);
void ibm_ad_destroy(ibm_ad_ctx *ctx);

/*
 * Moving bodies (the paper's time loop, Sec. 2.4 and 2.5: every step
 * re-classifies the grid and rebuilds the ghost rows before the PPE).
 *
 * poisson_update -- re-set-up of a context after the bodies moved: the same
 * grid and options, a new classification (flags_dev, device uint8[N]) and
 * ghost-row table.  Every part of the context that depends on them (level-0
 * flags, ghost and membrane rows, pin, volumes, coarse masks of every level)
 * is rebuilt on the device; the level geometry, prolongation maps and coarse
 * storage are kept.  The vectors over the unknowns are reallocated only
 * when the new membrane ghost count needs more than they hold (with headroom
 * for later steps); such a reallocation moves them out of a caller-bound
 * workspace.  The results equal those of a fresh poisson_setup bit for bit.
 * Synchronous.  IBM_EINVAL for a table of another grid, IBM_EGEOM for a
 * classification without fluid or a cut link without a ghost row,
 * IBM_ENOMEM; after an error the context may only be destroyed.
 *
 * poisson_solve_from -- poisson_solve from an initial guess x0_dev (device
 * double[n_x0], natural order), e.g. the previous step's pressure after
 * ibm_fill_fresh.  n_x0 = N: cell values only; each membrane ghost unknown
 * (the other side's field at its cell) then starts from the mean of the
 * cells across its cell's cut links.  n_x0 = N + n_mghost: cell values and
 * membrane ghost values (a solution of this geometry).  Solid non-ghost
 * cells start from zero and the guess is shifted to a zero pin value; FP64
 * contexts then solve for the correction, mixed ones start the refinement
 * from it.  x0_dev and x_dev (double[N+n_mghost]) must not overlap.  Same
 * returns as poisson_solve, and IBM_EINVAL for another n_x0.
 *
 * ibm_fill_fresh -- initial values of fresh cells, cells that are fluid
 * under flags_new and were solid under flags_old: each gets the mean of its
 * face neighbours that are fluid under both (summed in the order -x, +x, -y,
 * +y, -z, +z), and keeps its value when there is none.  x_dev: device
 * double[N], natural order, updated in place; *n_fresh (may be NULL)
 * receives the fresh-cell count.  Synchronous with stream.
 */
int32_t poisson_update(poisson_ctx *ctx, const uint8_t *flags_dev, const ibm_stencils *st);
int32_t poisson_solve_from(poisson_ctx *ctx, const double *f_dev, const double *g_dev, const double *x0_dev,
                           int64_t n_x0, double *x_dev, poisson_stats *stats, void *stream);
int32_t ibm_fill_fresh(const ibm_grid *grid, const uint8_t *flags_old_dev, const uint8_t *flags_new_dev,
                       double *x_dev, int64_t *n_fresh, void *stream);

/* y = A x with the pinned operator (device double[N+n_mghost] each). */
int32_t poisson_apply(poisson_ctx *ctx, const double *x_dev, double *y_dev, void *stream);

/* b = assembled right-hand side for raw input f (and g or NULL). */
int32_t poisson_assemble_rhs(poisson_ctx *ctx, const double *f_dev, const double *g_dev, double *b_dev, void *stream);

/* x = M^{-1} b: one FP64 V-cycle of the preconditioner, including the
 * compensating sink at the pin and the shift to a zero pin value. */
int32_t poisson_precond(poisson_ctx *ctx, const double *b_dev, double *x_dev, void *stream);

/* Solve an already assembled pinned system A x = b (no projection, no
 * gauge); x_dev is the output.  For parity tests with manufactured b. */
int32_t poisson_solve_assembled(poisson_ctx *ctx, const double *b_dev, double *x_dev, poisson_stats *stats,
                                void *stream);

/* Per-launch device timing of one kernel of the solve, for roofline
 * reports: kernel 0 = level-0 red/black Gauss-Seidel half-sweep, 1 = level-0
 * operator apply inside BiCGSTAB, 2 = the fused x/r update; -1 = off.  While
 * a kernel is selected, solves run without graph replay and bracket each of
 * its launches with HIP events on the solve stream.  Returns (and with reset
 * != 0 clears) the accumulated milliseconds and launch count, then selects
 * `kernel` for the following solves. */
int32_t poisson_kernel_timing(poisson_ctx *ctx, int32_t kernel, int32_t reset, double *total_ms, int64_t *launches);

/*
 * ibm_hbm_stream -- the device's streaming bandwidth, the ceiling quoted
 * beside the HBM peak for the solve's bandwidth-bound kernels.  Allocates the
 * buffers (each `bytes` long, 1 MiB .. 64 GiB; use sizes far above the
 * 256 MB Infinity Cache), fills them, runs one untimed pass and then `reps`
 * (1..1000) timed passes of one stream on `stream`, bracketed by HIP events:
 *   IBM_STREAM_COPY   b = a                    (1 read : 1 write)
 *   IBM_STREAM_TRIAD  d = a + b + c, FP32      (3 reads : 1 write, the mix of a red/black half-sweep)
 *   IBM_STREAM_READ   per-block sums of a      (read only)
 * Every lane moves 16 bytes per access.  *ms gets the mean milliseconds per
 * pass and *bytes_moved the bytes read plus written per pass.  Synchronises
 * the stream before returning; the buffers are released.
 */
#define IBM_STREAM_COPY 0
#define IBM_STREAM_TRIAD 1
#define IBM_STREAM_READ 2
int32_t ibm_hbm_stream(int32_t kind, size_t bytes, int32_t reps, double *ms, double *bytes_moved, void *stream);

/* Multigrid level count and unknown counts of a context (any pointer may be NULL). */
int32_t poisson_level_info(poisson_ctx *ctx, int32_t *levels, int64_t *n_unknowns, int64_t *n_ghost,
                           int64_t *n_mghost);

void poisson_destroy(poisson_ctx *ctx);

/* ------------------------------------------------------------------ serving
 * A persistent scheduler thread owns one device and runs many solves at
 * once (continuous batching: a request that arrives while others are on the
 * GPU is admitted as soon as a slot and memory are free, and runs its whole
 * pipeline -- classification, stencils, set-up, solve -- on its own stream,
 * so its kernels interleave with those of the running solves).  Requests are
 * admitted first come, first served while the number of active solves is
 * below max_slots and the summed footprints (poisson_workspace_estimate plus
 * classification temporaries) fit hbm_budget; a request larger than the
 * whole budget fails with IBM_ENOMEM.  Finished solves release their slot and
 * memory at once.  With cache_entries > 0 a finished solve's set-up
 * (classification, ghost rows, operator, multigrid hierarchy) stays resident,
 * keyed by the exact bytes of its grid, bodies and options: a later request
 * with the same key reuses it and only runs the solve.  Cached set-ups count
 * against hbm_budget and the least recently used idle ones are freed when an
 * admission needs the memory.  Every solve is deterministic, so a result is
 * the same alone, in the mix and from the cache.
 * With the environment variable IBM_CRASH_TRACE set when a server is
 * created, a fatal SIGSEGV, SIGBUS or SIGFPE in any thread of the process
 * writes the signal, the faulting address, the thread id and that thread's
 * native stack to standard error before the signal goes on to the handler
 * installed earlier or to the default action (installed once per process).
 */
typedef struct poisson_server poisson_server;

typedef struct poisson_server_opts {
    size_t hbm_budget;      /* bytes of device memory the active solves (and cached hierarchies) may hold */
    int32_t max_slots;      /* concurrently active solves */
    int32_t device;         /* HIP device ordinal */
    int32_t cache_entries;  /* solver set-ups kept after their solve, keyed by (grid, bodies, options);
                               0 disables the cache */
} poisson_server_opts;

typedef struct poisson_request {
    ibm_grid grid;             /* host arrays, copied at submit */
    const ibm_body *bodies;    /* host, copied at submit */
    int32_t n_body;
    const double *f;           /* host double[N], copied at submit */
    poisson_opts opts;
} poisson_request;

#define IBM_REQ_QUEUED 0
#define IBM_REQ_RUNNING 1
#define IBM_REQ_DONE 2
#define IBM_REQ_FAILED 3

typedef struct poisson_req_times {
    double submit_ms, admit_ms, done_ms; /* on the server's steady clock, from server start */
    int64_t n_unknowns;                  /* length of the solution once finished (N + n_mghost), else 0 */
    int32_t cache_hit;                   /* 1: the request reused a cached set-up (no classification,
                                            ghost rows or hierarchy build) */
    double setup_ms;                     /* worker wall time in classification, ghost rows and
                                            poisson_setup (0 on a cache hit) */
    double solve_ms;                     /* worker wall time from the RHS upload to the solution on the
                                            host (poisson_solve and the copies around it) */
} poisson_req_times;

int32_t poisson_server_create(const poisson_server_opts *opts, poisson_server **out);
/* Enqueue a request; never blocks on the GPU.  *ticket identifies it. */
int32_t poisson_submit(poisson_server *srv, const poisson_request *req, uint64_t *ticket);
/* Non-blocking: IBM_EAGAIN while queued or running; on completion copies the
 * solution (host double[N + n_mghost], may be NULL) and stats, frees the
 * request and returns its solve status.  *state (may be NULL) gets IBM_REQ_*.
 * x_len is the capacity of x_out in doubles: when it is too small the call
 * returns IBM_EINVAL, keeps the request and reports the needed length in
 * times->n_unknowns. */
int32_t poisson_poll(poisson_server *srv, uint64_t ticket, double *x_out, int64_t x_len, poisson_stats *stats,
                     poisson_req_times *times, int32_t *state);
/* Block until every submitted request has finished. */
int32_t poisson_server_drain(poisson_server *srv);
void poisson_server_destroy(poisson_server *srv);

const char *ibm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* IBM_POISSON_H */
