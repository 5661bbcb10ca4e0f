// engine.hip -- host engine and C ABI of libpoisson (single solves).
//
// A solve keeps every Krylov vector resident in HBM and never returns control
// to the host inside an iteration: the scalars alpha, omega, rho, beta and the
// stopping tests are computed by the last tile of each fused reduction kernel
// (the paper computes them on the host after each MPI_Allreduce, Alg. 3 and the
// alpaka implementation section). The host replays a captured HIP graph of
// several iterations and reads the convergence flag once per graph.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "common.h"
#include "poisson.h"

using namespace pz;

namespace {

bool debug_on()
{
    static int v = -1;
    if (v < 0) v = getenv("POISSON_DEBUG") ? 1 : 0;
    return v == 1;
}

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            if (debug_on())                                                            \
                fprintf(stderr, "poisson: %s failed: %s (%s:%d)\n", #expr,            \
                        hipGetErrorString(e_), __FILE__, __LINE__);                    \
            return POISSON_ERR_DEVICE;                                                 \
        }                                                                              \
    } while (0)

// ---- spectrum: eq. eigenvaluesPoissonDirichletMatrix, eqs. lambdaMin/lambdaMax ----
double dirichlet_eig(int i, int n)
{
    const double s = sin((double)i * M_PI / (2.0 * (double)(n + 1)));
    return 4.0 * s * s;
}

void grid_interval(int nx, int ny, int nz, double h, int block, double &lo, double &hi)
{
    int n[3] = {nx, ny, nz};
    if (block > 0)
        for (int &v : n) v = std::min(v, block);
    const double h2 = h * h;
    lo = dirichlet_eig(1, n[0]) / h2 + dirichlet_eig(1, n[1]) / h2 + dirichlet_eig(1, n[2]) / h2;
    hi = dirichlet_eig(n[0], n[0]) / h2 + dirichlet_eig(n[1], n[1]) / h2 +
         dirichlet_eig(n[2], n[2]) / h2;
}

int choose_kz(int tx, int ty, int nz)
{
    // z-chunk per tile: long chunks amortise the two halo planes, but keep at
    // least ~2048 tiles so 256 CUs have several workgroups each
    int kz = 64;
    const long base = (long)tx * ty;
    while (kz > 8 && base * ((nz + kz - 1) / kz) < 2048) kz /= 2;
    return std::min(kz, std::max(nz, 1));
}

struct GraphKey {
    int pc, deg, mixed, iters;
    bool operator<(const GraphKey &o) const
    {
        return std::tie(pc, deg, mixed, iters) < std::tie(o.pc, o.deg, o.mixed, o.iters);
    }
};

constexpr int MAX_HIST_ITERS = 1 << 16; // per-iteration scalars kept on the device

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

} // namespace

struct poisson_ctx {
    int nx = 0, ny = 0, nz = 0;
    double h = 0;
    unsigned bc = 0;
    size_t N = 0;
    hipStream_t stream = nullptr;
    // options
    int precision = POISSON_FP64, block = 64, bj_global = 0, graph_iters = 8, use_graph = 1;
    int debug_bd = -1;
    double lmin_scale = 1.0, lmax_scale = 1.0;
    // tiling
    int kz = 8, tx = 1, ty = 1, tz = 1, ntiles = 1;
    // device state
    bool dev = false;
    hipStream_t cap_stream = nullptr;
    Prob *d_prob = nullptr;     // [0] solve, [1] single operations
    Prob *h_prob = nullptr;     // pinned staging, 2 entries
    Scalars *d_sc = nullptr;    // [0] solve, [1] single operations
    Scalars *h_sc = nullptr;    // pinned
    double *d_partials = nullptr; // 2 * ntiles * PARTIAL_STRIDE
    double *d_hist = nullptr;
    int hist_cap = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    std::map<GraphKey, hipGraphExec_t> graphs;
    std::vector<hipGraph_t> graph_src;
    // plan of the last solve
    bool plan_ok = false;
    int plan_pc = -1, plan_deg = 0, plan_mixed = 0;
    void *vec[V_COUNT] = {};
    double plan_lo = 0, plan_hi = 0;
    // results
    bool have_stats = false;
    poisson_stats_t st{};
    std::vector<double> hist_rel, trace;
};

namespace {

size_t vec_bytes(const poisson_ctx *c, int v, int pc, int deg, bool mixed)
{
    const size_t N = c->N;
    const bool cheb = pc == POISSON_PC_CHEBYSHEV || pc == POISSON_PC_BLOCK_JACOBI;
    const size_t tp = (mixed && pc != POISSON_PC_NONE) ? 4 : 8;
    switch (v) {
    case V_R: case V_RT: case V_P: case V_W: case V_T: return 8 * N;
    case V_PH: case V_SH: return pc != POISSON_PC_NONE ? tp * N : 0;
    case V_RA: return cheb && deg >= 2 ? tp * N : 0;
    case V_RB: return cheb && deg >= 3 ? tp * N : 0;
    case V_V32: return cheb && mixed && deg >= 1 ? 4 * N : 0;
    default: return 0;
    }
}

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
    HIPCHK(hipMalloc(&c->d_partials, 2 * (size_t)c->ntiles * PARTIAL_STRIDE * sizeof(double)));
    HIPCHK(hipEventCreate(&c->ev_a));
    HIPCHK(hipEventCreate(&c->ev_b));
    memset(c->h_prob, 0, 2 * sizeof(Prob));
    c->dev = true;
    return POISSON_OK;
}

// carve the workspace for a plan; grows (never shrinks) the allocation
int plan_workspace(poisson_ctx *c, int pc, int deg, bool mixed)
{
    size_t need = 0;
    for (int v = 0; v < V_COUNT; ++v) need += (vec_bytes(c, v, pc, deg, mixed) + 255) & ~(size_t)255;
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
    size_t off = 0;
    for (int v = 0; v < V_COUNT; ++v) {
        const size_t b = vec_bytes(c, v, pc, deg, mixed);
        c->vec[v] = b ? c->ws + off : nullptr;
        off += (b + 255) & ~(size_t)255;
    }
    return POISSON_OK;
}

// fill a descriptor: geometry, tolerance, Chebyshev coefficients (Alg. 2 scalars)
int fill_prob(poisson_ctx *c, Prob &p, int pc, int deg, double tol, int maxit)
{
    memset(&p, 0, sizeof(Prob));
    p.nx = c->nx; p.ny = c->ny; p.nz = c->nz; p.kz = c->kz;
    p.tx = c->tx; p.ty = c->ty; p.tz = c->tz; p.ntiles = c->ntiles;
    p.block = pc == POISSON_PC_BLOCK_JACOBI ? c->block : 0;
    p.maxit = maxit;
    p.debug_breakdown_at = c->debug_bd;
    p.degree = deg;
    p.ih2 = 1.0 / (c->h * c->h);
    p.ih2f = (float)p.ih2;
    p.tol2 = tol * tol;
    p.jac_d = 6.0 * p.ih2;
    p.jac_df = (float)p.jac_d;
    c->plan_lo = c->plan_hi = 0;
    if (pc == POISSON_PC_CHEBYSHEV || pc == POISSON_PC_BLOCK_JACOBI) {
        const int local = (pc == POISSON_PC_BLOCK_JACOBI && !c->bj_global) ? c->block : 0;
        double lo, hi;
        grid_interval(c->nx, c->ny, c->nz, c->h, local, lo, hi);
        lo = lo * c->lmin_scale;
        hi = hi * c->lmax_scale;
        if (!(lo > 0) || !(hi > lo) || !std::isfinite(hi)) return POISSON_ERR_ARG;
        c->plan_lo = lo;
        c->plan_hi = hi;
        const double theta = (hi + lo) / 2.0, delta = (hi - lo) / 2.0, sigma = theta / delta;
        double rho_old = 1.0 / sigma;
        double rho_cur = 1.0 / (2.0 * sigma - rho_old);
        p.theta = theta;
        p.c1 = 2.0 * rho_cur / delta;
        p.two_sigma = 2.0 * sigma;
        p.two_over_delta = 2.0 / delta;
        for (int i = 2; i <= deg; ++i) {
            rho_old = rho_cur;
            rho_cur = 1.0 / (2.0 * sigma - rho_old);
            p.rc[i] = rho_cur;
            p.ro[i] = rho_old;
        }
        p.thetaf = (float)p.theta;
        p.c1f = (float)p.c1;
        p.two_sigmaf = (float)p.two_sigma;
        p.two_over_deltaf = (float)p.two_over_delta;
        for (int i = 0; i <= MAXDEG; ++i) {
            p.rcf[i] = (float)p.rc[i];
            p.rof[i] = (float)p.ro[i];
        }
    }
    return POISSON_OK;
}

// preconditioner apply vout = M^-1 vin (Alg. 2; BJ(CI) with the masked operator)
void enqueue_pc(const poisson_ctx *c, const Work &w, hipStream_t s, int pc, int m, bool mixed,
                int vin, int vout, int second)
{
    if (pc == POISSON_PC_NONE) return;
    const int grid = c->ntiles;
    if (pc == POISSON_PC_JACOBI || m == 0) {
        KArgs a{vin, vout, 0, 0, 0, second, pc == POISSON_PC_JACOBI ? 0 : 1, 0};
        launch_elem(E_DIV, mixed, w, grid, s, a);
        return;
    }
    const bool mask = pc == POISSON_PC_BLOCK_JACOBI;
    KArgs a1{vin, m == 1 ? vout : (int)V_RA, 0, 0, 1, second, 0, 0};
    launch_stencil(S_CHEB1, mixed, mask, w, grid, s, a1);
    const int vsrc = mixed ? (int)V_V32 : vin;
    for (int i = 2; i <= m; ++i) {
        // step i reads y = buf(i-1), z = buf(i-2), writes buf(i) (in place over z)
        // where buf(odd) = RA, buf(even) = RB, and the last step writes vout
        const int y = ((i - 1) & 1) ? V_RA : V_RB;
        const int z = ((i - 2) & 1) ? V_RA : V_RB;
        const int out = i == m ? vout : ((i & 1) ? V_RA : V_RB);
        KArgs a{y, out, vsrc, z, i, second, 0, 0};
        launch_stencil(i == 2 ? S_CHEB2 : S_CHEBK, mixed, mask, w, grid, s, a);
    }
}

// one Bi-CGSTAB iteration in the kernel order of Alg. 3
void enqueue_iteration(const poisson_ctx *c, const Work &w, hipStream_t s, int pc, int m,
                       bool mixed)
{
    const int grid = c->ntiles;
    const bool pm = mixed && pc != POISSON_PC_NONE;
    const int ph = pc == POISSON_PC_NONE ? V_P : V_PH;
    const int sh = pc == POISSON_PC_NONE ? V_R : V_SH;
    enqueue_pc(c, w, s, pc, m, mixed, V_P, V_PH, 0);                     // M p^ = p
    launch_stencil(S_SDOT, pm, false, w, grid, s, KArgs{ph, V_W, 0, 0, 0, 0, 0, 0}); // w, alpha
    launch_elem(E_AXPY, false, w, grid, s, KArgs{0, 0, 0, 0, 0, 0, 0, 0});         // s, half step
    enqueue_pc(c, w, s, pc, m, mixed, V_R, V_SH, 1);                     // M s^ = s
    launch_stencil(S_SDOT2, pm, false, w, grid, s, KArgs{sh, V_T, 0, 0, 0, 1, 0, 0}); // t, omega
    launch_elem(E_UPD, pm, w, grid, s, KArgs{ph, 0, 0, 0, 0, 0, 0, sh});           // x, r, beta
    launch_elem(E_PUPD, false, w, grid, s, KArgs{0, 0, 0, 0, 0, 0, 0, 0});         // p
}

// algorithmic bytes per unknown of one iteration of a plan
double iteration_bytes(int pc, int m, bool mixed)
{
    const bool pm = mixed && pc != POISSON_PC_NONE;
    const double tp = pm ? 4 : 8;
    double pcb = 0;
    if (pc == POISSON_PC_JACOBI || ((pc == POISSON_PC_CHEBYSHEV || pc == POISSON_PC_BLOCK_JACOBI) && m == 0))
        pcb = 8 + tp;
    else if (pc == POISSON_PC_CHEBYSHEV || pc == POISSON_PC_BLOCK_JACOBI) {
        const double tc = mixed ? 4 : 8;
        pcb = 8 + tc + (mixed ? 4 : 0);                 // first step: v, y (+ v32)
        if (m >= 2) pcb += 3 * tc;                      // step 2: y, v, w
        if (m >= 3) pcb += (m - 2) * 4 * tc;            // steps 3..m: y, v, z, w
    }
    double b = 2 * pcb;
    b += tp + 16;                                        // w = A p^, r~.w
    b += 24;                                             // s = r - alpha w
    b += tp + 16;                                        // t = A s^, t.s, t.t
    b += pc == POISSON_PC_NONE ? 56 : 48 + 2 * tp;       // x, r updates
    b += 32;                                             // p update
    return b;
}

int validate_ptr(const void *p)
{
    if (!p) return POISSON_ERR_ARG;
    if (((uintptr_t)p) & 15) return POISSON_ERR_ARG;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return POISSON_ERR_DEVICE;
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return POISSON_ERR_ARG;
    return POISSON_OK;
}

int get_graph(poisson_ctx *c, int pc, int m, bool mixed, int iters, hipGraphExec_t *out)
{
    GraphKey k{pc, m, mixed ? 1 : 0, iters};
    auto it = c->graphs.find(k);
    if (it != c->graphs.end()) {
        *out = it->second;
        return POISSON_OK;
    }
    Work w{c->d_prob, nullptr, nullptr, nullptr, c->ntiles};
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < iters; ++i) enqueue_iteration(c, w, c->cap_stream, pc, m, mixed);
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

int solve_impl(poisson_ctx *c, const double *rhs, double *x, int pc, int deg, double tol,
               int maxit)
{
    const double t0 = now_ms();
    const bool mixed = c->precision == POISSON_MIXED;
    int rc;
    if ((rc = validate_ptr(rhs)) != POISSON_OK) return rc;
    if ((rc = validate_ptr(x)) != POISSON_OK) return rc;
    if ((rc = ensure_device(c)) != POISSON_OK) return rc;
    if ((rc = plan_workspace(c, pc, deg, mixed)) != POISSON_OK) return rc;
    const int hist_iters = std::min(maxit, MAX_HIST_ITERS);
    if (c->hist_cap < 1 + 4 * hist_iters) {
        if (c->d_hist) HIPCHK(hipFree(c->d_hist));
        c->d_hist = nullptr;
        c->hist_cap = 0;
        HIPCHK(hipMalloc(&c->d_hist, (size_t)(1 + 4 * hist_iters) * sizeof(double)));
        c->hist_cap = 1 + 4 * hist_iters;
    }
    Prob &p = c->h_prob[0];
    if ((rc = fill_prob(c, p, pc, deg, tol, maxit)) != POISSON_OK) return rc;
    for (int v = 0; v < V_COUNT; ++v) p.vec[v] = c->vec[v];
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
    if ((rc = upload_prob(c, 0)) != POISSON_OK) return rc;

    const Work w{c->d_prob, nullptr, nullptr, nullptr, c->ntiles};
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
                for (int i = 0; i < K; ++i) enqueue_iteration(c, w, c->stream, pc, deg, mixed);
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
    st.model_bytes = iteration_bytes(pc, deg, mixed) * (double)c->N * sc.iter;
    st.model_gbps = loop_ms > 0 ? st.model_bytes / (loop_ms * 1e6) : 0.0;
    st.history_len = (int)c->hist_rel.size();
    st.history = c->hist_rel.data();
    st.solve_ms = now_ms() - t0;
    c->have_stats = true;
    return sc.status;
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
    if (!(h > 0) || !std::isfinite(h)) return POISSON_ERR_ARG;
    if (bc != 0) return POISSON_ERR_UNSUPPORTED;
    poisson_ctx *c = new (std::nothrow) poisson_ctx;
    if (!c) return POISSON_ERR_NOMEM;
    c->nx = nx; c->ny = ny; c->nz = nz; c->h = h; c->bc = bc;
    c->N = (size_t)nx * ny * nz;
    c->tx = (nx + TX - 1) / TX;
    c->ty = (ny + TY - 1) / TY;
    c->kz = choose_kz(c->tx, c->ty, nz);
    c->tz = (nz + c->kz - 1) / c->kz;
    c->ntiles = c->tx * c->ty * c->tz;
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
        c->block = (int)v;
        return POISSON_OK;
    case POISSON_OPT_LMIN_SCALE:
        if (!(v > 0)) return POISSON_ERR_ARG;
        c->lmin_scale = v;
        return POISSON_OK;
    case POISSON_OPT_LMAX_SCALE:
        if (!(v > 0)) return POISSON_ERR_ARG;
        c->lmax_scale = v;
        return POISSON_OK;
    case POISSON_OPT_BJ_GLOBAL_INTERVAL:
        if (v != 0 && v != 1) return POISSON_ERR_ARG;
        c->bj_global = (int)v;
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
        c->debug_bd = (int)v;
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
    if (!c || !rhs || !x) return POISSON_ERR_ARG;
    if (precond < POISSON_PC_NONE || precond > POISSON_PC_BLOCK_JACOBI) return POISSON_ERR_ARG;
    if ((precond == POISSON_PC_CHEBYSHEV || precond == POISSON_PC_BLOCK_JACOBI) &&
        (degree < 0 || degree > MAXDEG))
        return POISSON_ERR_ARG;
    if (precond != POISSON_PC_CHEBYSHEV && precond != POISSON_PC_BLOCK_JACOBI) degree = 0;
    if (!(tol > 0) || !(tol < 1)) return POISSON_ERR_ARG;
    if (maxit < 1 || maxit > 10000000) return POISSON_ERR_ARG;
    if (precond == POISSON_PC_CHEBYSHEV || precond == POISSON_PC_BLOCK_JACOBI) {
        // reject a degenerate interval before touching the device
        const int local = (precond == POISSON_PC_BLOCK_JACOBI && !c->bj_global) ? c->block : 0;
        double lo, hi;
        grid_interval(c->nx, c->ny, c->nz, c->h, local, lo, hi);
        lo *= c->lmin_scale;
        hi *= c->lmax_scale;
        if (!(lo > 0) || !(hi > lo)) return POISSON_ERR_ARG;
    }
    try {
        c->have_stats = false;
        return solve_impl(c, rhs, x, precond, degree, tol, maxit);
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
    if ((rc = fill_prob(c, p, pc, deg, 0.5, 1)) != POISSON_OK) return rc;
    p.sc = c->d_sc + 1;
    p.partials = c->d_partials + (size_t)c->ntiles * PARTIAL_STRIDE;
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
        const Work w{c->d_prob + 1, nullptr, nullptr, nullptr, c->ntiles};
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
        if ((rc = plan_workspace(c, precond, degree, mixed)) != POISSON_OK) return rc;
        c->plan_ok = false; // the workspace no longer matches the last solve's plan
        if ((rc = prim_begin(c, precond, degree, mixed)) != POISSON_OK) return rc;
        Prob &p = c->h_prob[1];
        for (int k = 0; k < V_COUNT; ++k) p.vec[k] = c->vec[k];
        p.vec[V_B] = (void *)v;
        p.vec[V_X] = out;
        if ((rc = upload_prob(c, 1)) != POISSON_OK) return rc;
        const Work w{c->d_prob + 1, nullptr, nullptr, nullptr, c->ntiles};
        enqueue_pc(c, w, c->stream, precond, degree, mixed, V_B, V_X, 0);
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
        const Work w{c->d_prob + 1, nullptr, nullptr, nullptr, c->ntiles};
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
    default: return 0.0;
    }
}

int poisson_kernel_bench(poisson_ctx *c, int kernel, int precision, int reps)
{
    if (!c || reps < 1 || !c->dev || !c->plan_ok) return POISSON_ERR_ARG;
    if (precision != POISSON_FP64 && precision != POISSON_MIXED) return POISSON_ERR_ARG;
    const bool mixed = precision == POISSON_MIXED;
    if (mixed != (bool)c->plan_mixed) return POISSON_ERR_ARG;
    const bool cheb = c->plan_pc == POISSON_PC_CHEBYSHEV || c->plan_pc == POISSON_PC_BLOCK_JACOBI;
    if (kernel == POISSON_KERNEL_CHEB_STEP && !(cheb && c->plan_deg >= 3)) return POISSON_ERR_ARG;
    if ((kernel == POISSON_KERNEL_STENCIL_DOT || kernel == POISSON_KERNEL_UPDATE_XR) &&
        c->plan_pc == POISSON_PC_NONE)
        return POISSON_ERR_ARG;
    if (kernel < POISSON_KERNEL_CHEB_STEP || kernel > POISSON_KERNEL_UPDATE_XR) return POISSON_ERR_ARG;
    try {
        int rc;
        // same descriptor as the solve, but private scalars (never 'done') and
        // the solution slot redirected to scratch so the caller's x is untouched
        Prob &p = c->h_prob[1];
        p = c->h_prob[0];
        p.sc = c->d_sc + 1;
        p.partials = c->d_partials + (size_t)c->ntiles * PARTIAL_STRIDE;
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
        const Work w{c->d_prob + 1, nullptr, nullptr, nullptr, c->ntiles};
        for (int r = 0; r < reps; ++r) {
            if (kernel == POISSON_KERNEL_CHEB_STEP)
                launch_stencil(S_CHEBK, mixed, c->plan_pc == POISSON_PC_BLOCK_JACOBI, w, c->ntiles,
                               c->stream, KArgs{V_RA, V_RB, mixed ? (int)V_V32 : (int)V_P, V_RB, 3, 0, 0, 0});
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
