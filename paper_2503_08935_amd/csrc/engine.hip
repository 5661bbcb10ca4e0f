// engine.hip -- host engine and C ABI of libpoisson (single solves).
//
// A solve keeps every Krylov vector resident in HBM and never returns control
// to the host inside an iteration: the scalars alpha, omega, rho, beta and the
// stopping tests are computed on the device by the finalize kernel that follows
// each fused reduction kernel (the paper computes them on the host after each
// MPI_Allreduce, Alg. 3 and the alpaka implementation section). The host replays a captured HIP graph of
// several iterations and reads the convergence flag once per graph.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "plan.h"

using namespace pz;

namespace {

struct GraphKey {
    int pc, deg, mixed, iters, fuse, order, pair_lds, upd;
    bool operator<(const GraphKey &o) const
    {
        return std::tie(pc, deg, mixed, iters, fuse, order, pair_lds, upd) <
               std::tie(o.pc, o.deg, o.mixed, o.iters, o.fuse, o.order, o.pair_lds, o.upd);
    }
};

constexpr int MAX_HIST_ITERS = 1 << 16; // per-iteration scalars kept on the device

} // namespace

struct poisson_ctx {
    int nx = 0, ny = 0, nz = 0;
    double h = 0;
    unsigned bc = 0;
    size_t N = 0;
    hipStream_t stream = nullptr;
    // options
    int precision = POISSON_FP64, graph_iters = 8, use_graph = 1, tile_order = 0;
    int pair_lds = 1;
    int fuse_updates = 2;       // fold the s and p updates into the applies' first passes:
                                // 0 never, 1 always, 2 when the grid is large enough
    PlanOpts opt;
    // tiling
    int ntiles = 1;
    int nparts = 1;             // reduction partial slots per problem (every tiling)
    // device state
    bool dev = false;
    hipStream_t cap_stream = nullptr;
    Prob *d_prob = nullptr;     // [0] solve, [1] single operations
    Prob *h_prob = nullptr;     // pinned staging, 2 entries
    Scalars *d_sc = nullptr;    // [0] solve, [1] single operations
    Scalars *h_sc = nullptr;    // pinned
    double *d_partials = nullptr; // 2 * nparts * PARTIAL_STRIDE
    double *d_hist = nullptr;
    int hist_cap = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    std::map<GraphKey, hipGraphExec_t> graphs;
    std::vector<hipGraph_t> graph_src;
    // plan of the last solve
    bool plan_ok = false;
    int plan_pc = -1, plan_deg = 0, plan_mixed = 0, plan_fuse = 0, plan_upd = 0;
    void *vec[V_COUNT] = {};
    int s_slot = V_R;
    double plan_lo = 0, plan_hi = 0;
    // results
    bool have_stats = false;
    poisson_stats_t st{};
    std::vector<double> hist_rel, trace;
};

namespace {

int ensure_device(poisson_ctx *c)
{
    if (c->dev) return POISSON_OK;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipMalloc(&c->d_prob, 2 * sizeof(Prob)));
    HIPCHK(hipHostMalloc(&c->h_prob, 2 * sizeof(Prob), hipHostMallocDefault));
    HIPCHK(hipMalloc(&c->d_sc, 2 * sizeof(Scalars)));
    HIPCHK(hipMemset(c->d_sc, 0, 2 * sizeof(Scalars)));
    HIPCHK(hipHostMalloc(&c->h_sc, 2 * sizeof(Scalars), hipHostMallocDefault));
    HIPCHK(hipMalloc(&c->d_partials, 2 * (size_t)c->nparts * PARTIAL_STRIDE * sizeof(double)));
    HIPCHK(hipEventCreate(&c->ev_a));
    HIPCHK(hipEventCreate(&c->ev_b));
    memset(c->h_prob, 0, 2 * sizeof(Prob));
    c->dev = true;
    return POISSON_OK;
}

// Unknowns from which the default keeps three steps per pass at degree 8 and
// above where four were not faster: FP64 Chebyshev (four-step passes over 64 x 16
// tiles cost per step what the triples do; 512^3 degree 8: 2.051 against
// 2.045 s) and mixed Block-Jacobi (the masked bodies' selects; 512^3 degree 8:
// 2.537 against 2.317 s). Below, and at degrees 4-7 everywhere, four were
// measured faster: FP64 Chebyshev 7-17% (256^3 degrees 4, 6, 8; 512^3 degrees 4,
// 6, 7), mixed Block-Jacobi 5-6% (256^3 degree 8, 512^3 degree 4).
constexpr size_t FOURS_MAX_UNKNOWNS = (size_t)448 * 448 * 448;

// steps per pass a solve runs: POISSON_OPT_FUSE, except where the default (3)
// was measured faster otherwise. FP64 Block-Jacobi keeps the triples: its
// four-step passes were slower (the paper's problem at 255^3, degree 24: BJ(CI)
// 0.79 -> 0.86 s, GNoComm(CI) 0.59 -> 0.64 s; 512^3 degree 8: +25%).
int solve_fuse(const poisson_ctx *c, int pc, int deg, bool mixed)
{
    if (c->opt.fuse != 3) return c->opt.fuse;
    const bool small = deg <= 7 || c->N < FOURS_MAX_UNKNOWNS;
    if (mixed) return (pc == POISSON_PC_BLOCK_JACOBI && !small) ? 2 : 3;
    return (pc == POISSON_PC_CHEBYSHEV && deg >= 4 && small) ? 4 : 3;
}

// size the workspace for a plan; grows (never shrinks) the allocation
int plan_workspace(poisson_ctx *c, int pc, int deg, bool mixed, int upd)
{
    const size_t need = workspace_bytes(c->N, pc, deg, mixed, solve_fuse(c, pc, deg, mixed), upd);
    if (need > c->ws_bytes) {
        if (c->ws) HIPCHK(hipFree(c->ws));
        c->ws = nullptr;
        c->ws_bytes = 0;
        if (hipMalloc(&c->ws, need) != hipSuccess) {
            (void)hipGetLastError();
            c->ws = nullptr;
            return POISSON_ERR_NOMEM;
        }
        c->ws_bytes = need;
    }
    Prob tmp;
    memset(&tmp, 0, sizeof(tmp));
    carve_workspace(tmp, c->ws, c->N, pc, deg, mixed, solve_fuse(c, pc, deg, mixed), upd);
    for (int v = 0; v < V_COUNT; ++v) c->vec[v] = tmp.vec[v];
    c->s_slot = tmp.s_slot;
    return POISSON_OK;
}

// the work list of a single problem (prob = d_prob or d_prob + 1): all tiles in
// the chosen order; the Chebyshev pairs LDS-staged unless that is switched off
Work single_work(const poisson_ctx *c, const Prob *prob)
{
    Work w{prob, nullptr, nullptr, nullptr, c->ntiles, c->tile_order, {0, 0}, c->bc != 0};
    if (c->pair_lds && c->opt.fuse >= 2)
        for (int f = 0; f < 2; ++f) w.triple_tiles[f] = make_triple_tiling(c->nx, c->ny, c->nz, f).ntiles;
    if (c->pair_lds && c->opt.fuse >= 3)
        for (int f = 0; f < 2; ++f) w.quad_tiles[f] = make_quad_tiling(c->nx, c->ny, c->nz, f).ntiles;
    if (c->pair_lds)
        for (int f = 0; f < 2; ++f) w.pair_tiles[f] = make_pair_tiling(c->nx, c->ny, c->nz, f).ntiles;
    return w;
}

// steps per pass the plan runs: three or four only with the LDS-staged tiles
int plan_fuse_level(const poisson_ctx *c, int pc, int deg, bool mixed)
{
    const int f = solve_fuse(c, pc, deg, mixed);
    return (f >= 2 && !c->pair_lds) ? 1 : f;
}

// Unknowns from which the folds pay by default when the first pass of an apply
// runs two or three steps. Below, the vectors partly fit the 256 MB Infinity
// Cache, the standalone update passes run from it, and the folded first passes'
// extra halo reads cost more than the passes they replace (measured per
// iteration, Chebyshev 4 and 8, FP64 and mixed: 0.7-3.8% slower at 256^3-320^3,
// 1.5-2.5% faster at 384^3, 3.6-5.5% faster at 512^3). With a first pass of
// four steps the folds pay from 128^3 (measured in the mixed mode, Chebyshev 4
// and 8: 1-3% faster at 128^3-192^3 but for +0.7% at 192^3 degree 8, 3-14% at
// 256^3-512^3; FP64 follows the same rule); at 64^3 and 96^3, where launches
// dominate, they cost 2-5%.
constexpr size_t FOLD_MIN_UNKNOWNS = (size_t)352 * 352 * 352;
constexpr size_t FOLD_MIN_UNKNOWNS_FOURS = (size_t)128 * 128 * 128;

// the vector updates a solve of this plan folds into the applies' first passes
int plan_updates(const poisson_ctx *c, int pc, int deg, bool mixed)
{
    if (!c->fuse_updates) return 0;
    const Work w = single_work(c, nullptr);
    const int fuse = solve_fuse(c, pc, deg, mixed);
    const bool first4 = starts_with_four(fuse, mixed, deg, w.quad_tiles[mixed ? 1 : 0] > 0,
                                         fuse >= 2 && w.triple_tiles[mixed ? 1 : 0] > 0);
    if (c->fuse_updates == 2 && c->N < (first4 ? FOLD_MIN_UNKNOWNS_FOURS : FOLD_MIN_UNKNOWNS))
        return 0;
    return upd_fusion(pc, deg, mixed, fuse, w);
}

int fill(poisson_ctx *c, Prob &p, int pc, int deg, double tol, int maxit)
{
    return fill_prob(p, c->nx, c->ny, c->nz, c->h, c->bc, pc, deg, c->opt, tol, maxit,
                     &c->plan_lo, &c->plan_hi);
}

int get_graph(poisson_ctx *c, int pc, int m, bool mixed, int iters, hipGraphExec_t *out)
{
    const Work w = single_work(c, c->d_prob);
    const int upd = plan_updates(c, pc, m, mixed);
    GraphKey k{pc, m, mixed ? 1 : 0, iters, c->opt.fuse, c->tile_order, w.pair_tiles[0] > 0, upd};
    auto it = c->graphs.find(k);
    if (it != c->graphs.end()) {
        *out = it->second;
        return POISSON_OK;
    }
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < iters; ++i)
        enqueue_iteration(w, c->ntiles, c->cap_stream, pc, m, mixed, solve_fuse(c, pc, m, mixed), upd);
    HIPCHK(hipStreamEndCapture(c->cap_stream, &g));
    hipGraphExec_t e = nullptr;
    HIPCHK(hipGraphInstantiate(&e, g, nullptr, nullptr, 0));
    c->graph_src.push_back(g);
    c->graphs[k] = e;
    *out = e;
    return POISSON_OK;
}

int upload_prob(poisson_ctx *c, int slot)
{
    // staging is reused by the next call: wait for the copy
    HIPCHK(hipMemcpyAsync(c->d_prob + slot, c->h_prob + slot, sizeof(Prob), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return POISSON_OK;
}

int read_scalars(poisson_ctx *c, int slot)
{
    HIPCHK(hipMemcpyAsync(c->h_sc + slot, c->d_sc + slot, sizeof(Scalars), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return POISSON_OK;
}

// statistics of a finished solve, without the history
void put_stats(poisson_ctx *c, const Scalars &sc, double rr_true, int pc, int deg, double loop_ms)
{
    const bool mixed = c->precision == POISSON_MIXED;
    const double bb = sc.bb;
    poisson_stats_t &st = c->st;
    memset(&st, 0, sizeof(st));
    st.struct_size = sizeof(st);
    st.status = sc.status;
    st.iterations = sc.iter;
    st.half_step_exit = sc.half;
    st.precond = pc;
    st.degree = deg;
    st.precision = c->precision;
    st.relres_recursive = bb > 0 ? std::sqrt(sc.rr / bb) : 0.0;
    st.relres_true = bb > 0 ? std::sqrt(rr_true / bb) : 0.0;
    st.lambda_min = c->plan_lo;
    st.lambda_max = c->plan_hi;
    st.loop_ms = loop_ms;
    st.model_bytes = iteration_bytes(pc, deg, mixed, plan_fuse_level(c, pc, deg, mixed),
                                     plan_updates(c, pc, deg, mixed)) *
                     (double)c->N * sc.iter;
    st.model_gbps = loop_ms > 0 ? st.model_bytes / (loop_ms * 1e6) : 0.0;
}

int solve_impl(poisson_ctx *c, const double *rhs, double *x, int pc, int deg, double tol,
               int maxit)
{
    const double t0 = now_ms();
    const bool mixed = c->precision == POISSON_MIXED;
    int rc;
    if ((rc = validate_ptr(rhs)) != POISSON_OK) return rc;
    if ((rc = validate_ptr(x)) != POISSON_OK) return rc;
    if ((rc = ensure_device(c)) != POISSON_OK) return rc;
    const int upd = plan_updates(c, pc, deg, mixed);
    if ((rc = plan_workspace(c, pc, deg, mixed, upd)) != POISSON_OK) return rc;
    const int hist_iters = std::min(maxit, MAX_HIST_ITERS);
    if (c->hist_cap < 1 + 4 * hist_iters) {
        if (c->d_hist) HIPCHK(hipFree(c->d_hist));
        c->d_hist = nullptr;
        c->hist_cap = 0;
        HIPCHK(hipMalloc(&c->d_hist, (size_t)(1 + 4 * hist_iters) * sizeof(double)));
        c->hist_cap = 1 + 4 * hist_iters;
    }
    Prob &p = c->h_prob[0];
    if ((rc = fill(c, p, pc, deg, tol, maxit)) != POISSON_OK) return rc;
    for (int v = 0; v < V_COUNT; ++v) p.vec[v] = c->vec[v];
    p.s_slot = c->s_slot;
    p.vec[V_X] = x;
    p.vec[V_B] = (void *)rhs;
    p.sc = c->d_sc;
    p.partials = c->d_partials;
    p.hist = c->d_hist;
    p.hist_iters = hist_iters;
    c->plan_ok = true;
    c->plan_pc = pc;
    c->plan_deg = deg;
    c->plan_mixed = mixed;
    c->plan_fuse = fused(pc, deg, mixed, solve_fuse(c, pc, deg, mixed));
    c->plan_upd = upd;
    if ((rc = upload_prob(c, 0)) != POISSON_OK) return rc;

    const Work w = single_work(c, c->d_prob);
    launch_stencil(S_INIT, false, false, w, c->ntiles, c->stream, KArgs{V_X, 0, 0, 0, 0, 0, 0, 0});
    HIPCHK(hipGetLastError());
    if ((rc = read_scalars(c, 0)) != POISSON_OK) return rc;

    double loop_ms = 0;
    if (!c->h_sc[0].done) {
        HIPCHK(hipEventRecord(c->ev_a, c->stream));
        const int K = c->graph_iters;
        hipGraphExec_t g = nullptr;
        if (c->use_graph && (rc = get_graph(c, pc, deg, mixed, K, &g)) != POISSON_OK) return rc;
        const long max_rounds = (long)maxit / K + 2;
        for (long round = 0; round < max_rounds; ++round) {
            if (c->use_graph) {
                HIPCHK(hipGraphLaunch(g, c->stream));
            } else {
                for (int i = 0; i < K; ++i)
                    enqueue_iteration(w, c->ntiles, c->stream, pc, deg, mixed,
                                      solve_fuse(c, pc, deg, mixed), upd);
                HIPCHK(hipGetLastError());
            }
            if ((rc = read_scalars(c, 0)) != POISSON_OK) return rc;
            if (c->h_sc[0].done) break;
        }
        HIPCHK(hipEventRecord(c->ev_b, c->stream));
        HIPCHK(hipEventSynchronize(c->ev_b));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, c->ev_a, c->ev_b));
        loop_ms = ms;
    }
    const Scalars sc = c->h_sc[0];
    if (!sc.done) return POISSON_ERR_INTERNAL;
    if (sc.zero_x) HIPCHK(hipMemsetAsync(x, 0, c->N * sizeof(double), c->stream));
    launch_stencil(S_TRUE, false, false, w, c->ntiles, c->stream, KArgs{V_X, 0, 0, 0, 0, 0, 0, 0});
    HIPCHK(hipGetLastError());
    if ((rc = read_scalars(c, 0)) != POISSON_OK) return rc;
    const double rr_true = c->h_sc[0].rr_true;

    // statistics
    const int iters = std::min(sc.iter, hist_iters);
    c->trace.assign((size_t)4 * iters, 0.0);
    double rr0 = 0;
    {
        std::vector<double> hbuf((size_t)1 + 4 * iters);
        HIPCHK(hipMemcpy(hbuf.data(), c->d_hist, hbuf.size() * sizeof(double),
                         hipMemcpyDeviceToHost));
        rr0 = hbuf[0];
        std::copy(hbuf.begin() + 1, hbuf.end(), c->trace.begin());
    }
    c->hist_rel.assign((size_t)iters + 1, 0.0);
    const double bb = sc.bb;
    if (bb > 0) {
        c->hist_rel[0] = std::sqrt(rr0 / bb);
        for (int i = 1; i <= iters; ++i) c->hist_rel[i] = std::sqrt(c->trace[4 * (i - 1) + 3] / bb);
    }
    put_stats(c, sc, rr_true, pc, deg, loop_ms);
    poisson_stats_t &st = c->st;
    st.history_len = (int)c->hist_rel.size();
    st.history = c->hist_rel.data();
    st.solve_ms = now_ms() - t0;
    c->have_stats = true;
    return sc.status;
}

// ---- the allocation-free solve ----------------------------------------------
// Its device state lives in one static array of POISSON_NOALLOC_SCRATCH_BYTES per
// GPU: the problem descriptor, the scalar block, the tile partials and the
// workspace vectors. On the host the array's name is not a device address; the
// address is taken once per device with hipGetSymbolAddress and only that
// address is handed to the kernels and copies. Every call on a GPU uses the same
// array, so calls that overlap on one GPU race.
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch[NOALLOC_MAX_DEVICES] = {};

} // namespace

static __device__ __align__(256) unsigned char scratch[POISSON_NOALLOC_SCRATCH_BYTES];

namespace {

// the current device's address of `scratch`, taken at its first use there
int scratch_base(char **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return POISSON_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return POISSON_ERR_DEVICE;
        g_scratch[dev] = (char *)p;
    }
    *out = g_scratch[dev];
    return POISSON_OK;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// bytes of the scratch a solve of this plan takes: descriptor, scalars, the
// partials of one problem and the workspace
size_t noalloc_bytes(const poisson_ctx *c, int pc, int deg, bool mixed, int upd)
{
    return round256(sizeof(Prob)) + round256(sizeof(Scalars)) +
           round256((size_t)c->nparts * PARTIAL_STRIDE * sizeof(double)) +
           workspace_bytes(c->N, pc, deg, mixed, solve_fuse(c, pc, deg, mixed), upd);
}

// the solve of solve_impl with every device buffer carved from the scratch,
// launched without graphs, with pageable host copies of the descriptor and the
// scalar block and no history: no device or pinned memory is allocated
int solve_noalloc_impl(poisson_ctx *c, const double *rhs, double *x, int pc, int deg, double tol,
                       int maxit)
{
    const double t0 = now_ms();
    const bool mixed = c->precision == POISSON_MIXED;
    int rc;
    if ((rc = validate_ptr(rhs)) != POISSON_OK) return rc;
    if ((rc = validate_ptr(x)) != POISSON_OK) return rc;
    const int upd = plan_updates(c, pc, deg, mixed);
    if (noalloc_bytes(c, pc, deg, mixed, upd) > POISSON_NOALLOC_SCRATCH_BYTES)
        return POISSON_ERR_NOMEM;
    char *base = nullptr;
    if ((rc = scratch_base(&base)) != POISSON_OK) return rc;
    Prob *d_prob = (Prob *)base;
    Scalars *d_sc = (Scalars *)(base + round256(sizeof(Prob)));
    double *d_part = (double *)((char *)d_sc + round256(sizeof(Scalars)));
    char *ws = (char *)d_part + round256((size_t)c->nparts * PARTIAL_STRIDE * sizeof(double));

    Prob p;
    memset(&p, 0, sizeof(p));
    if ((rc = fill(c, p, pc, deg, tol, maxit)) != POISSON_OK) return rc;
    carve_workspace(p, ws, c->N, pc, deg, mixed, solve_fuse(c, pc, deg, mixed), upd);
    p.vec[V_X] = x;
    p.vec[V_B] = (void *)rhs;
    p.sc = d_sc;
    p.partials = d_part;
    p.hist = nullptr;
    p.hist_iters = 0;
    HIPCHK(hipMemcpyAsync(d_prob, &p, sizeof(Prob), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));

    Scalars sc;
    auto read_sc = [&]() -> int {
        HIPCHK(hipMemcpyAsync(&sc, d_sc, sizeof(Scalars), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        return POISSON_OK;
    };
    const Work w = single_work(c, d_prob);
    // the initial residual's finalize rewrites every flag and scalar the loop
    // reads, so nothing left in the scratch by an earlier call is used
    launch_stencil(S_INIT, false, false, w, c->ntiles, c->stream, KArgs{V_X, 0, 0, 0, 0, 0, 0, 0});
    HIPCHK(hipGetLastError());
    if ((rc = read_sc()) != POISSON_OK) return rc;
    double loop_ms = 0;
    if (!sc.done) {
        const double l0 = now_ms();
        const int K = c->graph_iters;
        const long max_rounds = (long)maxit / K + 2;
        for (long round = 0; round < max_rounds; ++round) {
            for (int i = 0; i < K; ++i)
                enqueue_iteration(w, c->ntiles, c->stream, pc, deg, mixed,
                                  solve_fuse(c, pc, deg, mixed), upd);
            HIPCHK(hipGetLastError());
            if ((rc = read_sc()) != POISSON_OK) return rc;
            if (sc.done) break;
        }
        loop_ms = now_ms() - l0;
    }
    if (!sc.done) return POISSON_ERR_INTERNAL;
    const Scalars fin = sc;
    if (fin.zero_x) HIPCHK(hipMemsetAsync(x, 0, c->N * sizeof(double), c->stream));
    launch_stencil(S_TRUE, false, false, w, c->ntiles, c->stream, KArgs{V_X, 0, 0, 0, 0, 0, 0, 0});
    HIPCHK(hipGetLastError());
    if ((rc = read_sc()) != POISSON_OK) return rc;
    put_stats(c, fin, sc.rr_true, pc, deg, loop_ms);
    c->trace.clear();
    c->hist_rel.clear();
    c->st.history_len = 0;
    c->st.history = nullptr;
    c->st.solve_ms = now_ms() - t0;
    c->have_stats = true;
    return fin.status;
}

// argument checks shared by the solve entry points; a degenerate Chebyshev
// interval is rejected before the device is touched
int check_solve_args(const poisson_ctx *c, const double *rhs, const double *x, int precond,
                     int degree, double tol, int maxit)
{
    if (!c || !rhs || !x) return POISSON_ERR_ARG;
    if (precond < POISSON_PC_NONE || precond > POISSON_PC_BLOCK_JACOBI) return POISSON_ERR_ARG;
    if (is_cheb(precond) && (degree < 0 || degree > MAXDEG)) return POISSON_ERR_ARG;
    if (!(tol > 0) || !(tol < 1)) return POISSON_ERR_ARG;
    if (maxit < 1 || maxit > 10000000) return POISSON_ERR_ARG;
    if (is_cheb(precond)) {
        double lo, hi;
        if (!cheb_interval(c->nx, c->ny, c->nz, c->h, c->bc, precond, c->opt, lo, hi))
            return POISSON_ERR_ARG;
    }
    return POISSON_OK;
}

} // namespace

// ========================================================================
// C ABI
// ========================================================================
extern "C" {

int poisson_create(int nx, int ny, int nz, double h, unsigned bc, poisson_ctx **out)
{
    if (!out) return POISSON_ERR_ARG;
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return POISSON_ERR_ARG;
    if ((double)nx * ny * nz > 17179869184.0) return POISSON_ERR_ARG;
    if ((double)nx * ny >= 268435456.0) return POISSON_ERR_ARG; // plane offsets are 32-bit
    if (!(h > 0) || !std::isfinite(h)) return POISSON_ERR_ARG;
    const int rcb = check_bc(nx, ny, nz, bc);
    if (rcb != POISSON_OK) return rcb;
    poisson_ctx *c = new (std::nothrow) poisson_ctx;
    if (!c) return POISSON_ERR_NOMEM;
    c->nx = nx; c->ny = ny; c->nz = nz; c->h = h; c->bc = bc;
    c->N = (size_t)nx * ny * nz;
    c->ntiles = make_tiling(nx, ny, nz).ntiles;
    c->nparts = partial_slots(nx, ny, nz);
    *out = c;
    return POISSON_OK;
}

int poisson_set_option(poisson_ctx *c, int key, double v)
{
    if (!c || !std::isfinite(v)) return POISSON_ERR_ARG;
    switch (key) {
    case POISSON_OPT_PRECISION:
        if (v != POISSON_FP64 && v != POISSON_MIXED) return POISSON_ERR_ARG;
        c->precision = (int)v;
        return POISSON_OK;
    case POISSON_OPT_BLOCK:
        if (v < 2 || v > 4096 || v != std::floor(v)) return POISSON_ERR_ARG;
        c->opt.block = (int)v;
        return POISSON_OK;
    case POISSON_OPT_LMIN_SCALE:
        if (!(v > 0)) return POISSON_ERR_ARG;
        c->opt.lmin_scale = v;
        return POISSON_OK;
    case POISSON_OPT_LMAX_SCALE:
        if (!(v > 0)) return POISSON_ERR_ARG;
        c->opt.lmax_scale = v;
        return POISSON_OK;
    case POISSON_OPT_BJ_GLOBAL_INTERVAL:
        if (v != 0 && v != 1) return POISSON_ERR_ARG;
        c->opt.bj_global = (int)v;
        return POISSON_OK;
    case POISSON_OPT_GRAPH_ITERS:
        if (v < 1 || v > 256 || v != std::floor(v)) return POISSON_ERR_ARG;
        c->graph_iters = (int)v;
        return POISSON_OK;
    case POISSON_OPT_USE_GRAPH:
        if (v != 0 && v != 1) return POISSON_ERR_ARG;
        c->use_graph = (int)v;
        return POISSON_OK;
    case POISSON_OPT_DEBUG_BREAKDOWN_AT:
        if (v != std::floor(v)) return POISSON_ERR_ARG;
        c->opt.debug_bd = (int)v;
        return POISSON_OK;
    case POISSON_OPT_FUSE:
        if (v != 0 && v != 1 && v != 2 && v != 3 && v != 4) return POISSON_ERR_ARG;
        c->opt.fuse = (int)v;
        return POISSON_OK;
    case POISSON_OPT_TILE_ORDER:
        if (v != 0 && v != 1 && v != 2) return POISSON_ERR_ARG;
        c->tile_order = (int)v;
        return POISSON_OK;
    case POISSON_OPT_PAIR_LDS:
        if (v != 0 && v != 1) return POISSON_ERR_ARG;
        c->pair_lds = (int)v;
        return POISSON_OK;
    case POISSON_OPT_FUSE_UPDATES:
        if (v != 0 && v != 1 && v != 2) return POISSON_ERR_ARG;
        c->fuse_updates = (int)v;
        return POISSON_OK;
    default:
        return POISSON_ERR_ARG;
    }
}

int poisson_set_stream(poisson_ctx *c, void *s)
{
    if (!c) return POISSON_ERR_ARG;
    c->stream = (hipStream_t)s;
    return POISSON_OK;
}

int poisson_solve(poisson_ctx *c, const double *rhs, double *x, int precond, int degree,
                  double tol, int maxit)
{
    int rc;
    if ((rc = check_solve_args(c, rhs, x, precond, degree, tol, maxit)) != POISSON_OK) return rc;
    if (!is_cheb(precond)) degree = 0;
    try {
        c->have_stats = false;
        return solve_impl(c, rhs, x, precond, degree, tol, maxit);
    } catch (...) {
        return POISSON_ERR_INTERNAL;
    }
}

int poisson_solve_noalloc(poisson_ctx *c, const double *rhs, double *x, int precond, int degree,
                          double tol, int maxit)
{
    int rc;
    if ((rc = check_solve_args(c, rhs, x, precond, degree, tol, maxit)) != POISSON_OK) return rc;
    if (!is_cheb(precond)) degree = 0;
    try {
        c->have_stats = false;
        return solve_noalloc_impl(c, rhs, x, precond, degree, tol, maxit);
    } catch (...) {
        return POISSON_ERR_INTERNAL;
    }
}

int poisson_stats(const poisson_ctx *c, poisson_stats_t *out)
{
    if (!c || !out || out->struct_size < sizeof(poisson_stats_t) || !c->have_stats)
        return POISSON_ERR_ARG;
    *out = c->st;
    return POISSON_OK;
}

int poisson_trace(const poisson_ctx *c, double *out, int cap)
{
    if (!c || !out || cap < 0 || !c->have_stats) return POISSON_ERR_ARG;
    const int n = std::min(cap, (int)(c->trace.size() / 4));
    std::copy(c->trace.begin(), c->trace.begin() + 4 * (size_t)n, out);
    return n;
}

int poisson_cheb_interval(const poisson_ctx *c, int precond, double *lambda_min,
                          double *lambda_max)
{
    if (!c || !lambda_min || !lambda_max || !is_cheb(precond)) return POISSON_ERR_ARG;
    double lo, hi;
    if (!cheb_interval(c->nx, c->ny, c->nz, c->h, c->bc, precond, c->opt, lo, hi))
        return POISSON_ERR_ARG;
    *lambda_min = lo;
    *lambda_max = hi;
    return POISSON_OK;
}

void poisson_destroy(poisson_ctx *c)
{
    if (!c) return;
    if (c->dev) {
        (void)hipDeviceSynchronize();
        for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
        for (auto g : c->graph_src) (void)hipGraphDestroy(g);
        if (c->ws) (void)hipFree(c->ws);
        if (c->d_hist) (void)hipFree(c->d_hist);
        (void)hipFree(c->d_partials);
        (void)hipFree(c->d_prob);
        (void)hipFree(c->d_sc);
        (void)hipHostFree(c->h_prob);
        (void)hipHostFree(c->h_sc);
        (void)hipEventDestroy(c->ev_a);
        (void)hipEventDestroy(c->ev_b);
        (void)hipStreamDestroy(c->cap_stream);
    }
    delete c;
}

const char *poisson_strerror(int code)
{
    switch (code) {
    case POISSON_OK: return "ok";
    case POISSON_NOT_CONVERGED: return "not converged within maxit";
    case POISSON_PENDING: return "pending";
    case POISSON_ERR_ARG: return "invalid argument";
    case POISSON_ERR_NOMEM: return "out of device memory or over budget";
    case POISSON_ERR_DEVICE: return "HIP device error";
    case POISSON_ERR_UNSUPPORTED: return "unsupported option";
    case POISSON_ERR_BREAKDOWN: return "Bi-CGSTAB breakdown";
    case POISSON_ERR_NONFINITE: return "non-finite value in a reduction";
    case POISSON_ERR_INTERNAL: return "internal error";
    default: return "unknown status";
    }
}

// ---- single operations ----------------------------------------------------

static int prim_begin(poisson_ctx *c, int pc, int deg, bool mixed)
{
    int rc;
    if ((rc = ensure_device(c)) != POISSON_OK) return rc;
    Prob &p = c->h_prob[1];
    if ((rc = fill(c, p, pc, deg, 0.5, 1)) != POISSON_OK) return rc;
    p.sc = c->d_sc + 1;
    p.partials = c->d_partials + (size_t)c->nparts * PARTIAL_STRIDE;
    p.hist = nullptr;
    (void)mixed;
    return POISSON_OK;
}

int poisson_apply_operator(poisson_ctx *c, const double *u, double *out)
{
    if (!c || !u || !out) return POISSON_ERR_ARG;
    int rc;
    if ((rc = validate_ptr(u)) || (rc = validate_ptr(out))) return rc;
    try {
        if ((rc = prim_begin(c, POISSON_PC_NONE, 0, false)) != POISSON_OK) return rc;
        c->h_prob[1].vec[V_B] = (void *)u;
        c->h_prob[1].vec[V_X] = out;
        if ((rc = upload_prob(c, 1)) != POISSON_OK) return rc;
        const Work w = single_work(c, c->d_prob + 1);
        launch_stencil(S_APPLY, false, false, w, c->ntiles, c->stream, KArgs{V_B, V_X, 0, 0, 0, 0, 0, 0});
        HIPCHK(hipGetLastError());
        return POISSON_OK;
    } catch (...) {
        return POISSON_ERR_INTERNAL;
    }
}

int poisson_apply_precond(poisson_ctx *c, int precond, int degree, const double *v, void *out)
{
    if (!c || !v || !out) return POISSON_ERR_ARG;
    if (precond < POISSON_PC_JACOBI || precond > POISSON_PC_BLOCK_JACOBI) return POISSON_ERR_ARG;
    if (degree < 0 || degree > MAXDEG) return POISSON_ERR_ARG;
    int rc;
    if ((rc = validate_ptr(v)) || (rc = validate_ptr(out))) return rc;
    try {
        const bool mixed = c->precision == POISSON_MIXED;
        if ((rc = ensure_device(c)) != POISSON_OK) return rc;
        if ((rc = plan_workspace(c, precond, degree, mixed, 0)) != POISSON_OK) return rc;
        c->plan_ok = false; // the workspace no longer matches the last solve's plan
        if ((rc = prim_begin(c, precond, degree, mixed)) != POISSON_OK) return rc;
        Prob &p = c->h_prob[1];
        for (int k = 0; k < V_COUNT; ++k) p.vec[k] = c->vec[k];
        p.vec[V_B] = (void *)v;
        p.vec[V_X] = out;
        if ((rc = upload_prob(c, 1)) != POISSON_OK) return rc;
        const Work w = single_work(c, c->d_prob + 1);
        enqueue_pc(w, c->ntiles, c->stream, precond, degree, mixed,
                   solve_fuse(c, precond, degree, mixed), V_B, V_X, 0);
        HIPCHK(hipGetLastError());
        return POISSON_OK;
    } catch (...) {
        return POISSON_ERR_INTERNAL;
    }
}

int poisson_dot(poisson_ctx *c, const double *x, const double *y, double *result)
{
    if (!c || !x || !y || !result) return POISSON_ERR_ARG;
    int rc;
    if ((rc = validate_ptr(x)) || (rc = validate_ptr(y))) return rc;
    try {
        if ((rc = prim_begin(c, POISSON_PC_NONE, 0, false)) != POISSON_OK) return rc;
        c->h_prob[1].vec[V_X] = (void *)x;
        c->h_prob[1].vec[V_B] = (void *)y;
        if ((rc = upload_prob(c, 1)) != POISSON_OK) return rc;
        const Work w = single_work(c, c->d_prob + 1);
        launch_elem(E_DOT, false, w, c->ntiles, c->stream, KArgs{V_X, 0, 0, 0, 0, 0, 0, V_B});
        HIPCHK(hipGetLastError());
        if ((rc = read_scalars(c, 1)) != POISSON_OK) return rc;
        *result = c->h_sc[1].dot;
        return POISSON_OK;
    } catch (...) {
        return POISSON_ERR_INTERNAL;
    }
}

double poisson_kernel_bytes(const poisson_ctx *c, int kernel, int precision)
{
    if (!c) return 0.0;
    const double N = (double)c->N;
    const double tc = precision == POISSON_MIXED ? 4 : 8;
    switch (kernel) {
    case POISSON_KERNEL_CHEB_STEP: return 4 * tc * N;          // y, v, z in; w out
    case POISSON_KERNEL_STENCIL_DOT: return (tc + 16) * N;     // p^, r~ in; w out
    case POISSON_KERNEL_UPDATE_XR: return (48 + 2 * tc) * N;   // x, p^, s^, r, t, r~ in; x, r out
    case POISSON_KERNEL_CHEB_PAIR: return 5 * tc * N;          // y, z, v in; w_i, w_{i+1} out
    case POISSON_KERNEL_CHEB_TRIPLE: return 5 * tc * N;        // y, z, v in; w_{i+1}, w_{i+2} out
    default: return 0.0;
    }
}

int poisson_kernel_bench(poisson_ctx *c, int kernel, int precision, int reps)
{
    if (!c || reps < 1 || !c->dev || !c->plan_ok) return POISSON_ERR_ARG;
    if (precision != POISSON_FP64 && precision != POISSON_MIXED) return POISSON_ERR_ARG;
    const bool mixed = precision == POISSON_MIXED;
    if (mixed != (bool)c->plan_mixed) return POISSON_ERR_ARG;
    const bool cheb = is_cheb(c->plan_pc);
    if (kernel == POISSON_KERNEL_CHEB_STEP && !(cheb && c->plan_deg >= 3)) return POISSON_ERR_ARG;
    if ((kernel == POISSON_KERNEL_STENCIL_DOT || kernel == POISSON_KERNEL_UPDATE_XR) &&
        c->plan_pc == POISSON_PC_NONE)
        return POISSON_ERR_ARG;
    if (kernel == POISSON_KERNEL_CHEB_PAIR && !(c->plan_fuse && c->plan_deg >= 5))
        return POISSON_ERR_ARG;
    if (kernel == POISSON_KERNEL_CHEB_TRIPLE &&
        !(c->plan_fuse && c->plan_deg >= 5 && plan_fuse_level(c, c->plan_pc, c->plan_deg, c->plan_mixed) >= 2))
        return POISSON_ERR_ARG;
    if (kernel < POISSON_KERNEL_CHEB_STEP || kernel > POISSON_KERNEL_CHEB_TRIPLE)
        return POISSON_ERR_ARG;
    try {
        int rc;
        // same descriptor as the solve, but private scalars (never 'done') and
        // the solution slot redirected to scratch so the caller's x is untouched
        Prob &p = c->h_prob[1];
        p = c->h_prob[0];
        p.sc = c->d_sc + 1;
        p.partials = c->d_partials + (size_t)c->nparts * PARTIAL_STRIDE;
        p.hist = nullptr;
        p.vec[V_X] = c->vec[V_W];
        p.vec[V_B] = c->vec[V_T];
        p.maxit = 0x7fffffff;
        // scalars that keep every repetition running: no convergence, no breakdown
        Scalars s0;
        memset(&s0, 0, sizeof(s0));
        s0.rho = s0.alpha = s0.omega = s0.beta = 1.0;
        s0.bb = 1.0;
        s0.tol2bb = -1.0;
        c->h_sc[1] = s0;
        HIPCHK(hipMemcpyAsync(c->d_sc + 1, c->h_sc + 1, sizeof(Scalars), hipMemcpyHostToDevice,
                              c->stream));
        if ((rc = upload_prob(c, 1)) != POISSON_OK) return rc;
        const Work w = single_work(c, c->d_prob + 1);
        for (int r = 0; r < reps; ++r) {
            if (kernel == POISSON_KERNEL_CHEB_STEP)
                launch_stencil(S_CHEBK, mixed, c->plan_pc == POISSON_PC_BLOCK_JACOBI, w, c->ntiles,
                               c->stream, KArgs{V_RA, V_RB, mixed ? (int)V_V32 : (int)V_P, V_RB, 3, 0, 0, 0});
            else if (kernel == POISSON_KERNEL_CHEB_PAIR)
                launch_cheb_pair(mixed, c->plan_pc == POISSON_PC_BLOCK_JACOBI, w, c->ntiles, c->stream,
                                 KArgs{V_RA, V_RC, mixed ? (int)V_V32 : (int)V_P, V_RB, 3, 0, 0, V_RD});
            else if (kernel == POISSON_KERNEL_CHEB_TRIPLE)
                launch_cheb_triple(mixed, c->plan_pc == POISSON_PC_BLOCK_JACOBI, w, c->stream,
                                   KArgs{V_RA, V_RC, mixed ? (int)V_V32 : (int)V_P, V_RB, 3, 0, 0, V_RD});
            else if (kernel == POISSON_KERNEL_STENCIL_DOT)
                launch_stencil(S_SDOT, mixed, false, w, c->ntiles, c->stream,
                               KArgs{V_PH, V_W, 0, 0, 0, 0, 0, 0});
            else
                launch_elem(E_UPD, mixed, w, c->ntiles, c->stream, KArgs{V_PH, 0, 0, 0, 0, 0, 0, V_SH});
        }
        HIPCHK(hipGetLastError());
        return POISSON_OK;
    } catch (...) {
        return POISSON_ERR_INTERNAL;
    }
}

int poisson_fill_uniform(void *stream, double *out, int64_t n, uint64_t seed)
{
    if (!out || n < 0) return POISSON_ERR_ARG;
    if (n == 0) return POISSON_OK;
    int rc;
    if ((rc = validate_ptr(out)) != POISSON_OK) return rc;
    launch_fill_uniform(out, n, seed, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    return POISSON_OK;
}

} // extern "C"
