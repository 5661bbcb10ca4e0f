/*
 * poisson.h -- C ABI of the MI355X (gfx950) preconditioned Bi-CGSTAB solver for
 * the 3D Poisson equation, after Pennati et al., "A Parallel and Highly-Portable
 * HPC Poisson Solver: Preconditioned Bi-CGSTAB with alpaka" (arXiv 2503.08935).
 *
 * Problem (Background section, eq. poisson and eq. matrix_p): -lap(u) = f on
 * an nx x ny x nz grid with spacing h, second-order central differences
 * (matrix D of eq. matrix_dirichlet, or N of eq. matrix_neuman on axes with a
 * Neumann face; see poisson_create). The matrix is never formed: A u is a 7-point stencil,
 *   (A u)_ijk = (6 u_ijk - u_{i-1} - u_{i+1} - u_{j-1} - u_{j+1} - u_{k-1} - u_{k+1}) / h^2,
 * with neighbours outside the grid zero (Dirichlet) or mirrored (Neumann).
 *
 * Layout of every vector argument: contiguous, x fastest,
 *   idx = i + nx * (j + ny * k),  0 <= i < nx, 0 <= j < ny, 0 <= k < nz;
 * grid node (i, j, k) sits at ((i+1) h, (j+1) h, (k+1) h).
 *
 * Conventions for every call:
 *   - the return value is a status code: 0 = OK, > 0 informational, < 0 error;
 *   - out-parameters are written only on success; a failed create sets *out = NULL;
 *   - no C++ exception crosses this boundary (an internal failure returns
 *     POISSON_ERR_INTERNAL);
 *   - device pointers are HIP device (or managed) allocations owned by the
 *     caller, 16-byte aligned; they must stay valid and unmodified until the
 *     call that uses them has returned (solve) or reported a final status (poll);
 *   - a context or server is not thread-safe; distinct objects are independent.
 */
#ifndef POISSON_H
#define POISSON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
enum {
    POISSON_OK = 0,
    POISSON_NOT_CONVERGED = 1,   /* maxit reached; x holds the last iterate */
    POISSON_PENDING = 2,         /* serving: request still queued or running */
    POISSON_ERR_ARG = -1,        /* invalid argument; nothing was touched */
    POISSON_ERR_NOMEM = -2,      /* device allocation failed / over budget */
    POISSON_ERR_DEVICE = -3,     /* a HIP call failed (no GPU, bad pointer, ...) */
    POISSON_ERR_UNSUPPORTED = -4,/* valid but not supported (e.g. all faces Neumann) */
    POISSON_ERR_BREAKDOWN = -5,  /* r~.A p^ = 0, t.t = 0, r~.r = 0 or omega = 0 */
    POISSON_ERR_NONFINITE = -6,  /* a NaN or Inf reached a reduction */
    POISSON_ERR_INTERNAL = -7
};

/* ---- preconditioners (Table 1 of the paper) ---------------------------- */
enum {
    POISSON_PC_NONE = 0,         /* plain Bi-CGSTAB (BiCGS) */
    POISSON_PC_JACOBI = 1,       /* point Jacobi, M^-1 = diag(A)^-1 = (h^2/6) I */
    POISSON_PC_CHEBYSHEV = 2,    /* G(CI): Chebyshev iteration (Alg. 2) of degree m on
                                    the whole grid, interval [lambda_min, lambda_max] of
                                    eqs. lambdaMin / lambdaMax */
    POISSON_PC_BLOCK_JACOBI = 3  /* BJ(CI): Chebyshev of degree m on each non-overlapping
                                    block x block x block sub-grid, neighbours across block
                                    faces read as zero (eqs. blockJacobiPreconditioner and
                                    systemBJpreconditioner), interval of one block; with
                                    POISSON_OPT_BJ_GLOBAL_INTERVAL = 1 the global interval,
                                    which is GNoComm(CI) */
};

/* ---- precision --------------------------------------------------------- */
enum {
    POISSON_FP64 = 0,            /* everything in FP64 */
    POISSON_MIXED = 1            /* FP64 outer Bi-CGSTAB; the preconditioner is applied in
                                    FP32: its input is rounded to FP32 once, its scalar
                                    coefficients (computed in FP64) are rounded to FP32
                                    once, all its arithmetic is FP32, and its output p^ / s^
                                    is stored in FP32 and widened exactly where FP64 uses it.
                                    Its A u sums the axes' second differences,
                                    ((u - u_x-) + (u - u_x+)) + ... , which keeps FP32's
                                    relative accuracy where u is smooth */
};

/* ---- options (poisson_set_option keys) ---------------------------------- */
enum {
    POISSON_OPT_PRECISION = 1,          /* POISSON_FP64 (default) or POISSON_MIXED */
    POISSON_OPT_BLOCK = 2,              /* Block-Jacobi block edge, >= 2 (default 64) */
    POISSON_OPT_LMIN_SCALE = 3,         /* lambda_min multiplier (default 1); the paper
                                           uses 100 (256^3) and 10 (64^3) */
    POISSON_OPT_LMAX_SCALE = 4,         /* lambda_max multiplier (default 1); paper: 1 - 1e-4 */
    POISSON_OPT_BJ_GLOBAL_INTERVAL = 5, /* 0 = BJ(CI) local interval (default), 1 = GNoComm(CI) */
    POISSON_OPT_GRAPH_ITERS = 6,        /* iterations per captured HIP graph / per host poll
                                           (default 8, 1..256) */
    POISSON_OPT_USE_GRAPH = 7,          /* 1 = replay captured HIP graphs (default), 0 = launch */
    POISSON_OPT_DEBUG_BREAKDOWN_AT = 8, /* testing: force omega = 0 at this iteration (-1 off) */
    POISSON_OPT_FUSE = 9,               /* Chebyshev / Block-Jacobi with degree >= 3 (FP64 or
                                           mixed): 3 (default) four steps per pass from
                                           degree 4 (steps 1-4 first, then fours, then the
                                           rest as for 2; a degree 4k+1 starts with 1-2,
                                           or 1-3 mixed, and ends on a triple) where that
                                           was measured faster: mixed Chebyshev always,
                                           mixed Block-Jacobi and FP64 Chebyshev at
                                           degrees 4-7 and below 448^3 unknowns; elsewhere
                                           as 2; 4: four steps per pass in every plan;
                                           2: three per pass where the passes are
                                           LDS-staged (the steps left over, and the first
                                           two, run as pairs or alone); two per pass (1)
                                           or one per pass (0); same arithmetic, same
                                           results */
    POISSON_OPT_TILE_ORDER = 10,        /* order in which workgroups take tiles: 0 default
                                           (natural; x-grouped for the FP32 fused Chebyshev
                                           pairs, slabs for the triples and FP64 pairs),
                                           1 x-grouped everywhere (the x-tiles of a tile row
                                           on one XCD), 2 slabs (each XCD one contiguous
                                           eighth of the tiles); same results */
    POISSON_OPT_PAIR_LDS = 11,          /* fused Chebyshev pairs of single solves: 1 (default)
                                           stage 128 x 16 (FP64) or 256 x 16 (FP32) tiles in
                                           LDS, 0 use the 64 x 16 register tiles; same
                                           arithmetic, same results */
    POISSON_OPT_FUSE_UPDATES = 12       /* Chebyshev / Block-Jacobi plans whose first pass of an
                                           apply is LDS-staged (degree >= 3, FUSE >= 1,
                                           PAIR_LDS = 1): 1 forms s = r - alpha w with s.s
                                           (Alg. 1 half step) inside the first pass of the
                                           second apply, and p = r + beta (p - omega w)
                                           inside the first pass of the next iteration's
                                           first apply, instead of in passes of their own;
                                           0 keeps the separate update passes; 2 (default)
                                           folds from 352^3 unknowns on, and from 128^3
                                           when the first pass runs four steps (mixed,
                                           degree >= 4), where it was measured faster;
                                           same arithmetic, same results */
};

/* ---- solver context ----------------------------------------------------- */
typedef struct poisson_ctx poisson_ctx;

/* Create a context for an nx x ny x nz grid with spacing h.
   bc: bit f (x-, x+, y-, y+, z-, z+) set = homogeneous Neumann on face f, clear =
   zero Dirichlet. Along an axis with a Neumann end the 1D operator is the matrix N
   of eq. matrix_neuman: the outside neighbour is the mirror image of the inside one
   (u_{-1} = u_1), so the boundary node itself is an unknown; the operator is then
   non-symmetric. The Chebyshev interval uses the closed-form spectra of D and N
   (one Neumann end: 4 sin^2((2k-1) pi/(4n)); two: 4 sin^2(k pi/(2(n-1)))).
   Host-only: no device memory is touched until the first solve. Errors:
   ERR_ARG if a size < 1, nx*ny*nz > 2^34, nx*ny >= 2^28 (kernels address a plane
   with 32-bit offsets), h not finite and > 0, bc > 63, a Neumann face on an axis of
   length 1, or out == NULL; ERR_UNSUPPORTED for bc = 63 (all
   faces Neumann: singular). Chebyshev / Block-Jacobi need lambda_min > 0, so an
   axis with two Neumann ends must be paired with a Dirichlet face elsewhere. */
int poisson_create(int nx, int ny, int nz, double h, unsigned bc, poisson_ctx **out);

/* Set an option (keys above). ERR_ARG for an unknown key or an out-of-range value. */
int poisson_set_option(poisson_ctx *c, int key, double value);

/* Stream used by every later call on this context (a hipStream_t; NULL = the
   null stream). The caller keeps the stream alive. */
int poisson_set_stream(poisson_ctx *c, void *hip_stream);

/* Solve A x = rhs with right-preconditioned Bi-CGSTAB (Alg. 1 of the paper; the
   scalar formulas and kernel order of Alg. 3).
   rhs, x : device FP64 vectors of nx*ny*nz entries; x holds the initial guess
            on entry and the solution (or the last iterate) on return.
   precond: POISSON_PC_*; degree: Chebyshev degree m = number of operator
            applications per preconditioner apply (0..64; ignored for NONE/JACOBI).
   tol    : relative tolerance in (0, 1); the stopping test is ||r||_2 < tol ||rhs||_2,
            evaluated as r.r < (tol*tol) (rhs.rhs) on the recursively updated r, both at
            the half step (s) and at the end of each iteration.
   maxit  : iteration limit >= 1.
   Synchronous on the context stream. Returns OK, NOT_CONVERGED, ERR_BREAKDOWN or
   ERR_NONFINITE (x = last iterate, stats valid), or ERR_ARG / ERR_NOMEM /
   ERR_DEVICE / ERR_UNSUPPORTED (nothing solved). rhs = 0 gives x = 0 and 0 iterations. */
int poisson_solve(poisson_ctx *c, const double *rhs, double *x, int precond, int degree,
                  double tol, int maxit);

/* Bytes of the static device scratch of poisson_solve_noalloc, per GPU. */
#define POISSON_NOALLOC_SCRATCH_BYTES (64u << 20)

/* poisson_solve for callers that cannot allocate device or pinned host memory
   (code under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc). Same arguments, kernels and results as poisson_solve: the same x,
   iterations and status bit for bit. The library keeps one static device array
   of POISSON_NOALLOC_SCRATCH_BYTES per GPU for this call (held until the process
   ends) and carves from it the problem descriptor, the scalar block, the
   reduction partials and the workspace vectors; it calls no hipMalloc, hipFree,
   hipHostMalloc or graph instantiation. Kernels are launched on the context
   stream without graphs; the descriptor and scalars cross through pageable host
   copies (synchronous). Limits: the plan's scratch must fit, e.g. up to 90^3
   unknowns for an FP64 Chebyshev plan of degree >= 5 (88 bytes per unknown plus
   the partials), otherwise ERR_NOMEM with nothing touched. No history is kept
   (poisson_stats reports history_len = 0; poisson_trace returns 0 rows);
   loop_ms is host wall time. Every call on one GPU shares that GPU's array and
   leaves its contents behind: calls that overlap on the same GPU (from several
   threads or contexts) race and must be serialised by the caller. */
int poisson_solve_noalloc(poisson_ctx *c, const double *rhs, double *x, int precond, int degree,
                          double tol, int maxit);

typedef struct {
    size_t struct_size;         /* set by the caller to sizeof(poisson_stats_t) */
    int status;                 /* status of the last solve */
    int iterations;             /* index i of the exit iteration (a half-step exit counts i) */
    int half_step_exit;         /* 1 if the solve stopped on s (Alg. 1 half step) */
    int precond, degree, precision;
    double relres_recursive;    /* sqrt(r.r / rhs.rhs) of the recursive residual at exit */
    double relres_true;         /* ||rhs - A x|| / ||rhs||, recomputed in FP64 after the solve */
    double lambda_min, lambda_max; /* interval given to the Chebyshev iteration */
    double solve_ms;            /* host wall time of poisson_solve */
    double loop_ms;             /* device time of the iteration loop (HIP events) */
    double model_bytes;         /* algorithmic HBM bytes of the iteration loop */
    double model_gbps;          /* model_bytes / loop_ms */
    int history_len;            /* number of entries of history (iterations + 1) */
    const double *history;      /* relative residual norm, [0] initial, [i] after iteration i;
                                   owned by the context, valid until the next solve/destroy */
} poisson_stats_t;

/* Statistics of the last solve. ERR_ARG if nothing was solved yet or
   out->struct_size < sizeof(poisson_stats_t). */
int poisson_stats(const poisson_ctx *c, poisson_stats_t *out);

/* Per-iteration scalars of the last solve, 4 doubles per iteration:
   alpha_i, omega_i (0 at a half-step exit), rho_{i-1}, and the squared residual
   norm tested at the exit of iteration i. Copies min(cap, iterations) rows to out
   (host memory) and returns the number of rows copied (>= 0) or an error. */
int poisson_trace(const poisson_ctx *c, double *out, int cap);

/* The interval [lambda_min, lambda_max] a Chebyshev (G(CI)) or Block-Jacobi
   (BJ(CI) / GNoComm(CI)) preconditioner of this context would use, with the
   current options (POISSON_OPT_BLOCK, _BJ_GLOBAL_INTERVAL, _LMIN_SCALE,
   _LMAX_SCALE). The spectrum of the grid operator is the sum over the axes of
   the 1D spectra divided by h^2 (eqs. eigenvaluesPoissonDirichletMatrix,
   lambdaMin and lambdaMax; the matrix N of eq. matrix_neuman on a Neumann axis);
   BJ(CI) bounds the spectra of all its diagonal blocks (eq.
   blockJacobiPreconditioner), GNoComm(CI) takes the global interval
   (Methodology section). The same values poisson_stats reports after a solve.
   Host-only: touches no device. ERR_ARG for a NULL argument, precond not
   CHEBYSHEV / BLOCK_JACOBI, or a degenerate interval (lambda_min <= 0 or
   lambda_max <= lambda_min, e.g. on a 1x1x1 grid); outputs unchanged then. */
int poisson_cheb_interval(const poisson_ctx *c, int precond, double *lambda_min,
                          double *lambda_max);

/* Release everything the context owns. NULL-safe. */
void poisson_destroy(poisson_ctx *c);

/* Static description of a status code. */
const char *poisson_strerror(int code);

/* ---- single operations (asynchronous on the context stream unless noted) --- */

/* out = A u with the grid operator of the context (u, out: device FP64). */
int poisson_apply_operator(poisson_ctx *c, const double *u, double *out);

/* out = M^-1 v, one preconditioner apply as used inside the solve, in the
   precision set by POISSON_OPT_PRECISION: out is FP64 (POISSON_FP64) or FP32
   (POISSON_MIXED). precond != NONE. v: device FP64. */
int poisson_apply_precond(poisson_ctx *c, int precond, int degree, const double *v, void *out);

/* *result = x . y over nx*ny*nz entries (device FP64), computed with the same
   double-double tile reduction as the solver. Synchronous. */
int poisson_dot(poisson_ctx *c, const double *x, const double *y, double *result);

/* Kernel identifiers for poisson_kernel_bench. */
enum {
    POISSON_KERNEL_CHEB_STEP = 0,       /* one interior Chebyshev step (Alg. 2 loop body) */
    POISSON_KERNEL_STENCIL_DOT = 1,     /* w = A p^ fused with r~.w */
    POISSON_KERNEL_UPDATE_XR = 2,       /* x and r updates fused with r~.r, r.r */
    POISSON_KERNEL_CHEB_PAIR = 3,       /* two interior Chebyshev steps in one pass */
    POISSON_KERNEL_CHEB_TRIPLE = 4      /* three interior Chebyshev steps in one pass */
};

/* Launch one kernel `reps` times back to back on the context stream over the
   workspace of the last solve (its values are overwritten), for timing with
   events on that stream. precision selects the FP64 or FP32 variant.
   Requires a previous successful poisson_solve with a plan that has the buffers
   (Chebyshev degree >= 3 for CHEB_STEP; a fused plan of degree >= 5 for
   CHEB_PAIR; for CHEB_TRIPLE also three steps per pass, POISSON_OPT_FUSE = 2
   with LDS-staged pairs). Asynchronous. */
int poisson_kernel_bench(poisson_ctx *c, int kernel, int precision, int reps);

/* Algorithmic HBM bytes of one launch of that kernel on this grid. */
double poisson_kernel_bytes(const poisson_ctx *c, int kernel, int precision);

/* ---- synthetic inputs ---------------------------------------------------- */

/* out[i] = 2 u_i - 1, u_i = (splitmix64(splitmix64(seed + G) + (i + 1) G) >> 11) 2^-53,
   G = 0x9E3779B97F4A7C15, i = 0..n-1 (Steele, Lea and Flood, OOPSLA 2014). The
   same bits as the host generator of the test-suite. Asynchronous on stream. */
int poisson_fill_uniform(void *hip_stream, double *out, int64_t n, uint64_t seed);

/* ---- serving: continuous batching of many solves ------------------------ */
/*
 * A server owns one HBM arena of hbm_budget_bytes and up to max_slots running
 * solves. Requests of any grid size are queued first-in first-out and admitted
 * while a slot is free and the request's workspace (its Krylov vectors and
 * reduction partials, poisson_server_footprint) fits in the arena. Running
 * requests keep their vectors resident and are advanced together: every kernel
 * of an iteration runs once per plan (precond, degree, precision) over the
 * tiles of all running requests with that plan. Each request's arithmetic is
 * independent of the others, so its result is bitwise the same alone, in any
 * mix, and through poisson_solve (Block-Jacobi uses 64^3 blocks and the local
 * interval; interval scales are 1).
 */
typedef struct poisson_server poisson_server;

typedef struct {
    size_t struct_size;         /* set by the caller to sizeof(poisson_server_info_t) */
    int queued, active;         /* waiting for admission / running */
    long completed;             /* finished requests (any status) */
    long steps;                 /* poisson_server_step calls that did work */
    size_t bytes_in_use, peak_bytes, budget_bytes; /* arena accounting */
    double busy_ms;             /* device time of all batches (HIP events), summed over
                                   the size classes, whose batches may overlap */
} poisson_server_info_t;

enum {
    POISSON_SERVER_OPT_USE_GRAPH = 1,    /* 1 = replay captured graphs (default), 0 = launch */
    POISSON_SERVER_OPT_SIZE_CLASSES = 2  /* 1..4 size classes by unknowns (default 3: up to
                                            64^3, up to 160^3, larger); each class advances in
                                            its own batches on a stream of its own (default
                                            priority), so small requests are not paced by
                                            large ones; 1 = every request in one batch on the
                                            server's stream. Set before the first step */,
    POISSON_SERVER_OPT_FUSE_UPDATES = 3  /* 1 (default): Chebyshev and Block-Jacobi plans of
                                            degree >= 3 form s = r - alpha w and p = r +
                                            beta (p - omega w) inside the first pass of each
                                            preconditioner apply (Alg. 3's two update passes
                                            folded away, as in poisson_solve from 352^3; two
                                            more FP64 vectors per request); 0: standalone
                                            update passes. Same results either way. Set
                                            before the first submit */,
    POISSON_SERVER_OPT_FOUR_STEPS = 4    /* 1 (default): plans of degree >= 4 (mixed
                                            Chebyshev and Block-Jacobi, FP64 Chebyshev)
                                            run their applies four steps per pass (steps
                                            1-4 first, then fours, then a pair or a single
                                            step); 0: pairs. Same results either way. Set
                                            before the first submit */
};

/* Create a server. hip_stream: the caller's stream (NULL = null stream); the
   inputs of every request are taken to be ready once the work queued on it at
   the step that admits the request has run. With one size class all of the
   server's work runs on it; with several, each class runs on a stream the server
   creates. Host-only: the arena and streams are created by the first
   poisson_server_step.
   ERR_ARG if hbm_budget_bytes < 4096, max_slots outside 1..4096 or out == NULL. */
int poisson_server_create(size_t hbm_budget_bytes, int max_slots, void *hip_stream,
                          poisson_server **out);

/* Set a server option (POISSON_SERVER_OPT_*). */
int poisson_server_set_option(poisson_server *s, int key, double value);

/* Arena bytes a request of this plan needs with the default options (host-only);
   with POISSON_SERVER_OPT_FUSE_UPDATES = 0 a Chebyshev or Block-Jacobi plan of
   degree >= 3 needs 16 bytes per unknown less. */
int poisson_server_footprint(int nx, int ny, int nz, int precond, int degree, int precision,
                             size_t *bytes);

/* Queue one solve of A x = rhs (arguments as poisson_solve, plus the precision;
   rhs and x are caller-owned device FP64 vectors that must stay valid until
   poll reports a final status). Does no device work. *ticket identifies the
   request. ERR_NOMEM if the request alone exceeds the arena; ERR_ARG /
   ERR_UNSUPPORTED / ERR_DEVICE as poisson_solve. */
int poisson_server_submit(poisson_server *s, int nx, int ny, int nz, double h, unsigned bc,
                          const double *rhs, double *x, int precond, int degree, int precision,
                          double tol, int maxit, uint64_t *ticket);

/* One scheduling round. If every size class that has work still has a batch in
   flight, first wait until one finishes. Then every class whose last batch has
   finished retires the requests that batch finished (true residual, stats, free
   the arena block and slot), admits queued requests of its size class in
   arrival order (a request that does not fit in the arena stops admission, so no
   later request passes it), computes their initial residuals, and starts its next
   batch: `iters` iterations (1..4096) of all its running requests, on the class's
   stream, after the work already on the server's stream (the inputs). Returns
   without waiting for the new batches, with the number of queued + running
   requests (>= 0); a request's final status is visible to poll after the step
   that sees its batch finished. */
int poisson_server_step(poisson_server *s, int iters);

/* POISSON_PENDING while queued or running; otherwise the final status
   (OK, NOT_CONVERGED, ERR_BREAKDOWN, ERR_NONFINITE) and, if out != NULL, the
   request's statistics (solve_ms = submit to completion, loop_ms = admission to
   completion, both host wall time; no history). ERR_ARG for an unknown ticket. */
int poisson_server_poll(poisson_server *s, uint64_t ticket, poisson_stats_t *out);

/* Queue, arena and timing counters. */
int poisson_server_info(const poisson_server *s, poisson_server_info_t *out);

/* Release the server (waits for its stream). NULL-safe. */
void poisson_server_destroy(poisson_server *s);

#ifdef __cplusplus
}
#endif
#endif /* POISSON_H */
