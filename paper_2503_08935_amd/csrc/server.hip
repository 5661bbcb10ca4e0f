// server.hip -- continuous-batching solve server.
//
// Requests (one Poisson solve each, any grid size) are queued in arrival order
// and admitted while a slot is free and their workspace fits in a fixed HBM
// arena (first-fit allocation, freed on retirement). Every admitted request
// keeps its Krylov vectors resident in its arena block. Requests fall into size
// classes by their unknowns; each class advances on a stream of its own, in
// batches of a few Bi-CGSTAB iterations: each kernel of the iteration is
// launched once per plan group (precond, degree, precision, Neumann faces, size
// class) over the tiles of all the group's requests, from a captured HIP graph
// whose tile list and tile count live in device memory, so the graph does not
// change when the batch does. poisson_server_step() lets every class whose last
// batch has finished retire its finished requests, admit queued requests of its
// size (one batched initial-residual launch) and start its next batch, while
// the other classes' batches keep running: a 32^3 request is not paced by the
// batches of 256^3 ones. Reductions are per request and per tile, so a
// request's result is bitwise the same alone, in any mix, and through
// poisson_solve().
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <thread>
#include <tuple>
#include <vector>

#include "plan.h"

using namespace pz;

namespace {

constexpr int GRID = 2048;   // persistent workgroups of the batched kernels (multiple of 8)

constexpr int MAX_CLASSES = 4; // size classes, each with a stream of its own

struct PlanKey {
    int pc, deg, mixed, neu; // neu: the requests have a Neumann face
    int cls;                 // size class
    bool operator<(const PlanKey &o) const
    {
        return std::tie(pc, deg, mixed, neu, cls) < std::tie(o.pc, o.deg, o.mixed, o.neu, o.cls);
    }
};

struct Request {
    uint64_t ticket;
    int nx, ny, nz;
    double h;
    unsigned bc;
    const double *rhs;
    double *x;
    int pc, deg, prec;
    int upd;                 // vector updates folded into the applies' first passes
    double tol;
    int maxit;
    size_t ws_bytes, footprint;
    double t_submit;
};

struct Result {
    int status;
    poisson_stats_t st;
};

struct Slot {
    bool active = false;
    Request req{};
    size_t off = 0;          // arena offset of the block
    int ntiles = 0;
    int cls = 0;             // size class
    double t_admit = 0;
    double lo = 0, hi = 0;
};

// first-fit allocator over [0, size) with coalescing of free ranges
struct Arena {
    size_t size = 0;
    std::map<size_t, size_t> free_; // offset -> length
    void init(size_t s)
    {
        size = s;
        free_.clear();
        if (s) free_[0] = s;
    }
    bool alloc(size_t n, size_t &off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                off = it->first;
                const size_t rest = it->second - n;
                const size_t noff = it->first + n;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct TileList {
    int *d_prob = nullptr, *d_local = nullptr, *d_count = nullptr;
    int cap = 0;
    int count = 0;
    std::vector<int> h_prob, h_local;
};

struct Group {
    TileList tiles;
    TileList ptiles;          // tiles of the LDS-staged Chebyshev pairs
    TileList qtiles;          // tiles of the four-step passes (mixed, degree >= 4)
    hipGraphExec_t graph = nullptr;
    hipGraph_t graph_src = nullptr;
    int graph_cap = -1;       // capacities the graph was captured with
    int pgraph_cap = -1;
    int qgraph_cap = -1;
    bool dirty = true;        // tile list must be rebuilt
};

// a size class: its stream, its flags after each batch, and the tile lists of
// its initial-residual and true-residual launches
struct ClassState {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipEvent_t ev_a = nullptr, ev_b = nullptr, ev_in = nullptr;
    Scalars *h_sc = nullptr;  // pinned copy of every slot's scalars after a batch
    TileList init_list, true_list;
    bool busy = false;        // a batch is in flight
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// the vector updates folded into the first pass of each preconditioner apply
// (s = r - alpha w and p = r + beta (p - omega w) formed there, as in single
// solves): wherever the applies run as LDS-staged pairs, unless switched off
int server_upd(int pc, int deg, int prec, bool on)
{
    return on && fused(pc, deg, prec == POISSON_MIXED, 1) ? (U_S | U_P) : 0;
}

// bytes of a request's arena block: its workspace (with the folds' two extra
// vectors where they apply), then its reduction partials (one slot per tile
// of the tiling with the most tiles)
size_t block_bytes(int nx, int ny, int nz, int pc, int deg, int prec, int upd, size_t *ws)
{
    const size_t w = workspace_bytes((size_t)nx * ny * nz, pc, deg, prec == POISSON_MIXED, 1, upd);
    if (ws) *ws = w;
    return w + align256((size_t)partial_slots(nx, ny, nz) * PARTIAL_STRIDE * sizeof(double));
}

} // namespace

struct poisson_server {
    size_t budget = 0;
    int max_slots = 0;
    hipStream_t stream = nullptr;   // the caller's stream (inputs are written there)
    hipStream_t cap_stream = nullptr;
    bool dev = false;
    bool use_graph = true;
    int nclasses = 3;               // size classes, each on a stream of its own
    bool fuse_updates = true;       // fold the s and p updates into the first passes
    bool four_steps = true;         // mixed Chebyshev applies of degree >= 4: four steps
                                    // per pass (pairs otherwise)
    char *arena_base = nullptr;
    Arena arena;
    size_t in_use = 0, peak = 0;
    Prob *d_probs = nullptr, *h_probs = nullptr;
    Scalars *d_sc = nullptr;
    std::vector<Slot> slots;
    std::deque<Request> queue;
    std::map<uint64_t, Result> results;
    std::map<PlanKey, Group> groups;
    ClassState cls[MAX_CLASSES];
    uint64_t next_ticket = 1;
    long steps = 0;
    double busy_ms = 0;       // device time of all batches, summed over the classes
};

namespace {

int ensure_dev(poisson_server *s)
{
    if (s->dev) return POISSON_OK;
    HIPCHK(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    if (hipMalloc(&s->arena_base, s->budget) != hipSuccess) {
        (void)hipGetLastError();
        s->arena_base = nullptr;
        return POISSON_ERR_NOMEM;
    }
    s->arena.init(s->budget);
    HIPCHK(hipMalloc(&s->d_probs, s->max_slots * sizeof(Prob)));
    HIPCHK(hipHostMalloc(&s->h_probs, s->max_slots * sizeof(Prob), hipHostMallocDefault));
    HIPCHK(hipMalloc(&s->d_sc, s->max_slots * sizeof(Scalars)));
    HIPCHK(hipMemset(s->d_sc, 0, s->max_slots * sizeof(Scalars)));
    memset(s->h_probs, 0, s->max_slots * sizeof(Prob));
    for (int c = 0; c < s->nclasses; ++c) {
        ClassState &k = s->cls[c];
        // one class runs on the caller's stream; several run on streams of their
        // own, all at the default priority
        if (s->nclasses == 1) k.stream = s->stream;
        else HIPCHK(hipStreamCreateWithFlags(&k.stream, hipStreamNonBlocking));
        k.own_stream = s->nclasses > 1;
        HIPCHK(hipEventCreate(&k.ev_a));
        HIPCHK(hipEventCreate(&k.ev_b));
        HIPCHK(hipEventCreateWithFlags(&k.ev_in, hipEventDisableTiming));
        HIPCHK(hipHostMalloc(&k.h_sc, s->max_slots * sizeof(Scalars), hipHostMallocDefault));
        memset(k.h_sc, 0, s->max_slots * sizeof(Scalars));
    }
    s->dev = true;
    return POISSON_OK;
}

// size class of a request by its unknowns: small grids get classes of their own,
// so that their batches are not paced by the largest grids'
int class_of(const poisson_server *s, const Request &r)
{
    static const double bounds[MAX_CLASSES][MAX_CLASSES - 1] = {
        {0, 0, 0}, {96.0 * 96 * 96, 0, 0}, {64.0 * 64 * 64, 160.0 * 160 * 160, 0},
        {48.0 * 48 * 48, 96.0 * 96 * 96, 192.0 * 192 * 192}};
    const double N = (double)r.nx * r.ny * r.nz;
    int c = 0;
    while (c < s->nclasses - 1 && N > bounds[s->nclasses - 1][c]) ++c;
    return c;
}

// upload a tile list on stream st, growing its device arrays if needed; returns
// whether the device arrays moved (graphs that captured them must be re-captured)
int upload_tiles(hipStream_t st, TileList &t, bool &moved)
{
    moved = false;
    const int n = (int)t.h_prob.size();
    if (n > t.cap || !t.d_count) {
        const int cap = std::max(n, std::max(2 * t.cap, 4096));
        if (t.d_prob) HIPCHK(hipFree(t.d_prob));
        if (t.d_local) HIPCHK(hipFree(t.d_local));
        t.d_prob = t.d_local = nullptr;
        HIPCHK(hipMalloc(&t.d_prob, cap * sizeof(int)));
        HIPCHK(hipMalloc(&t.d_local, cap * sizeof(int)));
        if (!t.d_count) HIPCHK(hipMalloc(&t.d_count, sizeof(int)));
        t.cap = cap;
        moved = true;
    }
    t.count = n;
    if (n) {
        HIPCHK(hipMemcpyAsync(t.d_prob, t.h_prob.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(t.d_local, t.h_local.data(), n * sizeof(int), hipMemcpyHostToDevice,
                              st));
    }
    HIPCHK(hipMemcpyAsync(t.d_count, &t.count, sizeof(int), hipMemcpyHostToDevice, st));
    // the host vectors are the source of async copies: keep them until the copy ran
    HIPCHK(hipStreamSynchronize(st));
    return POISSON_OK;
}

void list_tiles(poisson_server *s, TileList &t, const std::vector<int> &slot_ids)
{
    t.h_prob.clear();
    t.h_local.clear();
    for (int id : slot_ids)
        for (int l = 0; l < s->slots[id].ntiles; ++l) {
            t.h_prob.push_back(id);
            t.h_local.push_back(l);
        }
}

// whether a plan group's applies run four Chebyshev steps per pass: degree >= 4,
// mixed Chebyshev or Block-Jacobi and FP64 Chebyshev, as single solves of the
// server's grid sizes do (FP64 Block-Jacobi keeps the pairs)
bool server_four(const poisson_server *s, int pc, int deg, int prec)
{
    return s->four_steps && is_cheb(pc) && deg >= 4 &&
           (prec == POISSON_MIXED || pc == POISSON_PC_CHEBYSHEV);
}

// the LDS-staged pairs' (make_pair_tiling) or four-step passes' (make_quad_tiling)
// tiles of the requests in ids
void list_pair_tiles(poisson_server *s, TileList &t, const std::vector<int> &slot_ids, bool fp32,
                     bool four = false)
{
    t.h_prob.clear();
    t.h_local.clear();
    for (int id : slot_ids) {
        const Request &rq = s->slots[id].req;
        const int n = four ? make_quad_tiling(rq.nx, rq.ny, rq.nz, fp32).ntiles
                           : make_pair_tiling(rq.nx, rq.ny, rq.nz, fp32).ntiles;
        for (int l = 0; l < n; ++l) {
            t.h_prob.push_back(id);
            t.h_local.push_back(l);
        }
    }
}

Work work_of(const poisson_server *s, const TileList &t)
{
    return Work{s->d_probs, t.d_prob, t.d_local, t.d_count, t.count, 0};
}

// the work of a plan group: its tile list, the pair tile list for the LDS-staged
// Chebyshev pairs, and the four-step passes' tile list where they run
Work group_work(const poisson_server *s, const PlanKey &k, const Group &g, int count)
{
    Work w{s->d_probs, g.tiles.d_prob, g.tiles.d_local, g.tiles.d_count, count, 0};
    w.neumann = k.neu;
    w.pair_prob = g.ptiles.d_prob;
    w.pair_local = g.ptiles.d_local;
    w.pair_count_dev = g.ptiles.d_count;
    if (server_four(s, k.pc, k.deg, k.mixed)) {
        w.quad_prob = g.qtiles.d_prob;
        w.quad_local = g.qtiles.d_local;
        w.quad_count_dev = g.qtiles.d_count;
    }
    return w;
}

// steps per pass of a plan group's applies (enqueue_iteration's fuse)
int group_fuse(const poisson_server *s, const PlanKey &k)
{
    return server_four(s, k.pc, k.deg, k.mixed) ? 4 : 1;
}

// retire finished requests of class c (its stream is idle): true residuals in one
// launch, statistics, arena block and slot freed
int finish_requests(poisson_server *s, int c, const std::vector<int> &ids)
{
    if (ids.empty()) return POISSON_OK;
    ClassState &k = s->cls[c];
    for (int id : ids) {
        const Slot &sl = s->slots[id];
        if (k.h_sc[id].zero_x)
            HIPCHK(hipMemsetAsync(sl.req.x, 0, (size_t)sl.req.nx * sl.req.ny * sl.req.nz * 8,
                                  k.stream));
    }
    list_tiles(s, k.true_list, ids);
    bool moved;
    int rc;
    if ((rc = upload_tiles(k.stream, k.true_list, moved)) != POISSON_OK) return rc;
    launch_stencil(S_TRUE, false, false, work_of(s, k.true_list),
                   std::min(GRID, std::max(8, k.true_list.count)), k.stream,
                   KArgs{V_X, 0, 0, 0, 0, 0, 0, 0});
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(k.h_sc, s->d_sc, s->max_slots * sizeof(Scalars), hipMemcpyDeviceToHost,
                          k.stream));
    HIPCHK(hipStreamSynchronize(k.stream));
    const double t = now_ms();
    for (int id : ids) {
        Slot &sl = s->slots[id];
        const Scalars &sc = k.h_sc[id];
        Result r;
        memset(&r.st, 0, sizeof(r.st));
        r.status = sc.status;
        poisson_stats_t &st = r.st;
        st.struct_size = sizeof(st);
        st.status = sc.status;
        st.iterations = sc.iter;
        st.half_step_exit = sc.half;
        st.precond = sl.req.pc;
        st.degree = sl.req.deg;
        st.precision = sl.req.prec;
        st.relres_recursive = sc.bb > 0 ? std::sqrt(sc.rr / sc.bb) : 0.0;
        st.relres_true = sc.bb > 0 ? std::sqrt(sc.rr_true / sc.bb) : 0.0;
        st.lambda_min = sl.lo;
        st.lambda_max = sl.hi;
        st.solve_ms = t - sl.req.t_submit;   // arrival to completion
        st.loop_ms = t - sl.t_admit;         // admission to completion
        const double N = (double)sl.req.nx * sl.req.ny * sl.req.nz;
        st.model_bytes = iteration_bytes(sl.req.pc, sl.req.deg, sl.req.prec == POISSON_MIXED,
                                         server_four(s, sl.req.pc, sl.req.deg, sl.req.prec) ? 4 : 1,
                                         sl.req.upd, false) * N * sc.iter;
        st.model_gbps = 0;
        s->results[sl.req.ticket] = r;
        s->arena.release(sl.off, sl.req.footprint);
        s->in_use -= sl.req.footprint;
        sl.active = false;
        for (auto &g : s->groups)
            if (g.first.cls == c) g.second.dirty = true;
    }
    return POISSON_OK;
}

int capture_group(poisson_server *s, const PlanKey &k, Group &g)
{
    if (g.graph) {
        (void)hipGraphExecDestroy(g.graph);
        (void)hipGraphDestroy(g.graph_src);
        g.graph = nullptr;
        g.graph_src = nullptr;
    }
    const Work w = group_work(s, k, g, 0);
    HIPCHK(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    enqueue_iteration(w, GRID, s->cap_stream, k.pc, k.deg, k.mixed != 0, group_fuse(s, k),
                      server_upd(k.pc, k.deg, k.mixed, s->fuse_updates));
    HIPCHK(hipStreamEndCapture(s->cap_stream, &g.graph_src));
    HIPCHK(hipGraphInstantiate(&g.graph, g.graph_src, nullptr, nullptr, 0));
    g.graph_cap = g.tiles.cap;
    g.pgraph_cap = g.ptiles.cap;
    g.qgraph_cap = g.qtiles.cap;
    return POISSON_OK;
}

bool has_work(const poisson_server *s, int c)
{
    for (const Slot &sl : s->slots)
        if (sl.active && sl.cls == c) return true;
    for (const Request &r : s->queue)
        if (class_of(s, r) == c) return true;
    return false;
}

int round_impl(poisson_server *s, int iters, int &progress);

// Mark the classes whose batch has finished as idle; with `wait`, first wait
// until at least one busy class has finished.
int poll_classes(poisson_server *s, bool wait)
{
    for (;;) {
        bool any_busy = false, finished = false;
        for (int c = 0; c < s->nclasses; ++c) {
            ClassState &k = s->cls[c];
            if (!k.busy) continue;
            const hipError_t q = hipEventQuery(k.ev_b);
            if (q == hipSuccess) {
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, k.ev_a, k.ev_b));
                s->busy_ms += ms;
                k.busy = false;
                finished = true;
            } else if (q != hipErrorNotReady) {
                HIPCHK(q);
            } else {
                any_busy = true;
            }
        }
        if (!wait || finished || !any_busy) return POISSON_OK;
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

// One scheduling round. Each size class runs its batches on its own stream: a
// class whose last batch has finished retires its finished requests, admits
// queued requests of its class and starts its next batch of `iters` iterations,
// while the other classes' batches keep running. If every class that has work
// is still running, or nothing could be done (a queued request waits for arena
// space or a slot that a running class holds), wait for the first batch to
// finish and try again.
int step_impl(poisson_server *s, int iters)
{
    int rc;
    if ((rc = ensure_dev(s)) != POISSON_OK) return rc;
    for (bool wait = false;; wait = true) {
        if ((rc = poll_classes(s, wait)) != POISSON_OK) return rc;
        bool ready = false, any_busy = false;
        for (int c = 0; c < s->nclasses; ++c) {
            if (s->cls[c].busy) any_busy = true;
            else if (has_work(s, c)) ready = true;
        }
        if (!ready) {
            if (any_busy) continue;              // wait for a batch
            break;                               // nothing running, nothing queued
        }
        int progress = 0;
        if ((rc = round_impl(s, iters, progress)) != POISSON_OK) return rc;
        if (progress || !any_busy) break;
    }
    int active = 0;
    for (const Slot &sl : s->slots) active += sl.active;
    return active + (int)s->queue.size();
}

// retire, admit and launch for every idle class; progress counts what happened
int round_impl(poisson_server *s, int iters, int &progress)
{
    int rc;
    // 2. retire what the idle classes' last batches finished
    for (int c = 0; c < s->nclasses; ++c) {
        ClassState &k = s->cls[c];
        if (k.busy) continue;
        std::vector<int> done;
        for (int i = 0; i < s->max_slots; ++i)
            if (s->slots[i].active && s->slots[i].cls == c && k.h_sc[i].done) done.push_back(i);
        if ((rc = finish_requests(s, c, done)) != POISSON_OK) return rc;
        progress += (int)done.size();
    }
    // 3. admit in arrival order into idle classes while a slot is free and the
    // block fits; a request that does not fit stops admission (no later request
    // passes it), a request whose class is busy waits for that class
    std::vector<int> admitted[MAX_CLASSES];
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        const int c = class_of(s, *it);
        if (s->cls[c].busy) {
            ++it;
            continue;
        }
        int id = -1;
        for (int i = 0; i < s->max_slots; ++i)
            if (!s->slots[i].active) { id = i; break; }
        if (id < 0) break;
        size_t off;
        if (!s->arena.alloc(it->footprint, off)) break;
        Slot &sl = s->slots[id];
        sl.active = true;
        sl.req = *it;
        sl.off = off;
        sl.cls = c;
        sl.t_admit = now_ms();
        s->in_use += it->footprint;
        s->peak = std::max(s->peak, s->in_use);
        it = s->queue.erase(it);
        // descriptor: workspace, partials, scalars in the arena block
        PlanOpts o;
        Prob &p = s->h_probs[id];
        if ((rc = fill_prob(p, sl.req.nx, sl.req.ny, sl.req.nz, sl.req.h, sl.req.bc, sl.req.pc,
                            sl.req.deg, o, sl.req.tol, sl.req.maxit, &sl.lo, &sl.hi)) != POISSON_OK)
            return rc;
        sl.ntiles = p.ntiles;
        char *blk = s->arena_base + off;
        const size_t N = (size_t)sl.req.nx * sl.req.ny * sl.req.nz;
        carve_workspace(p, blk, N, sl.req.pc, sl.req.deg, sl.req.prec == POISSON_MIXED, 1,
                        sl.req.upd);
        // with s formed in the first pass, its s.s is in that pass's tile partials
        if (sl.req.upd & U_S)
            p.nparts_first =
                server_four(s, sl.req.pc, sl.req.deg, sl.req.prec)
                    ? make_quad_tiling(sl.req.nx, sl.req.ny, sl.req.nz, sl.req.prec == POISSON_MIXED).ntiles
                    : make_pair_tiling(sl.req.nx, sl.req.ny, sl.req.nz, sl.req.prec == POISSON_MIXED).ntiles;
        p.vec[V_X] = sl.req.x;
        p.vec[V_B] = (void *)sl.req.rhs;
        p.partials = (double *)(blk + sl.req.ws_bytes);
        p.sc = s->d_sc + id;
        p.hist = nullptr;
        p.hist_iters = 0;
        HIPCHK(hipMemcpyAsync(s->d_probs + id, s->h_probs + id, sizeof(Prob), hipMemcpyHostToDevice,
                              s->cls[c].stream));
        admitted[c].push_back(id);
        s->groups[PlanKey{sl.req.pc, sl.req.deg, sl.req.prec, sl.req.bc != 0, c}].dirty = true;
    }
    // 4. every idle class with running requests starts its next batch
    bool launched = false;
    for (int c = 0; c < s->nclasses; ++c) {
        ClassState &k = s->cls[c];
        if (k.busy) continue;
        bool any = false;
        for (const Slot &sl : s->slots) any = any || (sl.active && sl.cls == c);
        if (!any) continue;
        if (!admitted[c].empty() && k.own_stream) {
            // the new requests' rhs and x were written on the caller's stream
            HIPCHK(hipEventRecord(k.ev_in, s->stream));
            HIPCHK(hipStreamWaitEvent(k.stream, k.ev_in, 0));
        }
        HIPCHK(hipEventRecord(k.ev_a, k.stream));
        if (!admitted[c].empty()) {
            // initial residuals of the new requests, one launch
            list_tiles(s, k.init_list, admitted[c]);
            bool moved;
            if ((rc = upload_tiles(k.stream, k.init_list, moved)) != POISSON_OK) return rc;
            launch_stencil(S_INIT, false, false, work_of(s, k.init_list),
                           std::min(GRID, std::max(8, k.init_list.count)), k.stream,
                           KArgs{V_X, 0, 0, 0, 0, 0, 0, 0});
            HIPCHK(hipGetLastError());
        }
        for (auto &kv : s->groups) {
            if (kv.first.cls != c) continue;
            Group &g = kv.second;
            if (g.dirty) {
                std::vector<int> ids;
                for (int i = 0; i < s->max_slots; ++i) {
                    const Slot &sl = s->slots[i];
                    const PlanKey key{sl.req.pc, sl.req.deg, sl.req.prec, sl.req.bc != 0, sl.cls};
                    if (sl.active && !(key < kv.first) && !(kv.first < key)) ids.push_back(i);
                }
                list_tiles(s, g.tiles, ids);
                list_pair_tiles(s, g.ptiles, ids, kv.first.mixed == POISSON_MIXED);
                const bool four = server_four(s, kv.first.pc, kv.first.deg, kv.first.mixed);
                bool moved, pmoved, qmoved = false;
                if ((rc = upload_tiles(k.stream, g.tiles, moved)) != POISSON_OK) return rc;
                if ((rc = upload_tiles(k.stream, g.ptiles, pmoved)) != POISSON_OK) return rc;
                if (four) {
                    list_pair_tiles(s, g.qtiles, ids, kv.first.mixed == POISSON_MIXED, true);
                    if ((rc = upload_tiles(k.stream, g.qtiles, qmoved)) != POISSON_OK) return rc;
                }
                if ((moved || pmoved || qmoved) && g.graph) g.graph_cap = -1;
                g.dirty = false;
            }
            if (g.tiles.count == 0) continue;
            if (s->use_graph) {
                if ((g.graph_cap != g.tiles.cap || g.pgraph_cap != g.ptiles.cap ||
                     g.qgraph_cap != g.qtiles.cap) &&
                    (rc = capture_group(s, kv.first, g)) != POISSON_OK)
                    return rc;
                for (int i = 0; i < iters; ++i) HIPCHK(hipGraphLaunch(g.graph, k.stream));
            } else {
                const Work w = group_work(s, kv.first, g, g.tiles.count);
                for (int i = 0; i < iters; ++i)
                    enqueue_iteration(w, GRID, k.stream, kv.first.pc, kv.first.deg,
                                      kv.first.mixed != 0, group_fuse(s, kv.first),
                                      server_upd(kv.first.pc, kv.first.deg, kv.first.mixed,
                                                 s->fuse_updates));
                HIPCHK(hipGetLastError());
            }
        }
        // the class's flags after the batch, read when the batch is seen finished
        HIPCHK(hipMemcpyAsync(k.h_sc, s->d_sc, s->max_slots * sizeof(Scalars),
                              hipMemcpyDeviceToHost, k.stream));
        HIPCHK(hipEventRecord(k.ev_b, k.stream));
        k.busy = true;
        launched = true;
        ++progress;
    }
    if (launched) ++s->steps;
    return POISSON_OK;
}

} // namespace

extern "C" {

int poisson_server_create(size_t hbm_budget_bytes, int max_slots, void *hip_stream,
                          poisson_server **out)
{
    if (!out) return POISSON_ERR_ARG;
    *out = nullptr;
    if (hbm_budget_bytes < 4096 || max_slots < 1 || max_slots > 4096) return POISSON_ERR_ARG;
    poisson_server *s = new (std::nothrow) poisson_server;
    if (!s) return POISSON_ERR_NOMEM;
    s->budget = hbm_budget_bytes & ~(size_t)255;
    s->max_slots = max_slots;
    s->stream = (hipStream_t)hip_stream;
    s->slots.resize(max_slots);
    *out = s;
    return POISSON_OK;
}

int poisson_server_set_option(poisson_server *s, int key, double value)
{
    if (!s || !std::isfinite(value)) return POISSON_ERR_ARG;
    if (key == POISSON_SERVER_OPT_USE_GRAPH) {
        if (value != 0 && value != 1) return POISSON_ERR_ARG;
        s->use_graph = value != 0;
        return POISSON_OK;
    }
    if (key == POISSON_SERVER_OPT_FUSE_UPDATES) {
        // fixed once a request was submitted (its workspace is sized by it)
        if (s->next_ticket != 1 || (value != 0 && value != 1)) return POISSON_ERR_ARG;
        s->fuse_updates = value != 0;
        return POISSON_OK;
    }
    if (key == POISSON_SERVER_OPT_FOUR_STEPS) {
        // fixed once a request was submitted (its partials follow the tiling)
        if (s->next_ticket != 1 || (value != 0 && value != 1)) return POISSON_ERR_ARG;
        s->four_steps = value != 0;
        return POISSON_OK;
    }
    if (key == POISSON_SERVER_OPT_SIZE_CLASSES) {
        // fixed once the server has started (its streams exist)
        if (s->dev || value < 1 || value > MAX_CLASSES || value != std::floor(value))
            return POISSON_ERR_ARG;
        s->nclasses = (int)value;
        return POISSON_OK;
    }
    return POISSON_ERR_ARG;
}

int poisson_server_footprint(int nx, int ny, int nz, int precond, int degree, int precision,
                             size_t *bytes)
{
    if (!bytes || nx < 1 || ny < 1 || nz < 1) return POISSON_ERR_ARG;
    if (precond < POISSON_PC_NONE || precond > POISSON_PC_BLOCK_JACOBI) return POISSON_ERR_ARG;
    if (precision != POISSON_FP64 && precision != POISSON_MIXED) return POISSON_ERR_ARG;
    *bytes = block_bytes(nx, ny, nz, precond, is_cheb(precond) ? degree : 0, precision,
                         server_upd(precond, is_cheb(precond) ? degree : 0, precision, true), nullptr);
    return POISSON_OK;
}

int poisson_server_submit(poisson_server *s, int nx, int ny, int nz, double h, unsigned bc,
                          const double *rhs, double *x, int precond, int degree, int precision,
                          double tol, int maxit, uint64_t *ticket)
{
    if (!s || !ticket || !rhs || !x) return POISSON_ERR_ARG;
    if (nx < 1 || ny < 1 || nz < 1 || (double)nx * ny * nz > 17179869184.0) return POISSON_ERR_ARG;
    if ((double)nx * ny >= 268435456.0) return POISSON_ERR_ARG; // plane offsets are 32-bit
    if (!(h > 0) || !std::isfinite(h)) return POISSON_ERR_ARG;
    const int rcb = check_bc(nx, ny, nz, bc);
    if (rcb != POISSON_OK) return rcb;
    if (precond < POISSON_PC_NONE || precond > POISSON_PC_BLOCK_JACOBI) return POISSON_ERR_ARG;
    if (is_cheb(precond) && (degree < 0 || degree > MAXDEG)) return POISSON_ERR_ARG;
    if (!is_cheb(precond)) degree = 0;
    if (precision != POISSON_FP64 && precision != POISSON_MIXED) return POISSON_ERR_ARG;
    if (!(tol > 0) || !(tol < 1) || maxit < 1 || maxit > 10000000) return POISSON_ERR_ARG;
    if (is_cheb(precond)) {
        PlanOpts o;
        double lo, hi;
        if (!cheb_interval(nx, ny, nz, h, bc, precond, o, lo, hi)) return POISSON_ERR_ARG;
    }
    const int upd = server_upd(precond, degree, precision, s->fuse_updates);
    size_t ws;
    const size_t fp = block_bytes(nx, ny, nz, precond, degree, precision, upd, &ws);
    if (fp > s->budget) return POISSON_ERR_NOMEM;
    int rc;
    if ((rc = validate_ptr(rhs)) != POISSON_OK) return rc;
    if ((rc = validate_ptr(x)) != POISSON_OK) return rc;
    Request r;
    r.ticket = s->next_ticket++;
    r.nx = nx; r.ny = ny; r.nz = nz; r.h = h; r.bc = bc;
    r.rhs = rhs; r.x = x;
    r.pc = precond; r.deg = degree; r.prec = precision;
    r.upd = upd;
    r.tol = tol; r.maxit = maxit;
    r.ws_bytes = ws;
    r.footprint = fp;
    r.t_submit = now_ms();
    s->queue.push_back(r);
    *ticket = r.ticket;
    return POISSON_OK;
}

int poisson_server_step(poisson_server *s, int iters)
{
    if (!s || iters < 1 || iters > 4096) return POISSON_ERR_ARG;
    try {
        return step_impl(s, iters);
    } catch (...) {
        return POISSON_ERR_INTERNAL;
    }
}

int poisson_server_poll(poisson_server *s, uint64_t ticket, poisson_stats_t *out)
{
    if (!s || ticket == 0 || ticket >= s->next_ticket) return POISSON_ERR_ARG;
    auto it = s->results.find(ticket);
    if (it == s->results.end()) return POISSON_PENDING;
    if (out) {
        if (out->struct_size < sizeof(poisson_stats_t)) return POISSON_ERR_ARG;
        *out = it->second.st;
    }
    return it->second.status;
}

int poisson_server_info(const poisson_server *s, poisson_server_info_t *out)
{
    if (!s || !out || out->struct_size < sizeof(poisson_server_info_t)) return POISSON_ERR_ARG;
    int active = 0;
    for (const Slot &sl : s->slots) active += sl.active;
    out->queued = (int)s->queue.size();
    out->active = active;
    out->completed = (long)s->results.size();
    out->steps = s->steps;
    out->bytes_in_use = s->in_use;
    out->peak_bytes = s->peak;
    out->budget_bytes = s->budget;
    out->busy_ms = s->busy_ms;
    return POISSON_OK;
}

void poisson_server_destroy(poisson_server *s)
{
    if (!s) return;
    if (s->dev) {
        (void)hipStreamSynchronize(s->stream);
        for (int c = 0; c < s->nclasses; ++c)
            if (s->cls[c].stream) (void)hipStreamSynchronize(s->cls[c].stream);
        for (auto &kv : s->groups) {
            if (kv.second.graph) (void)hipGraphExecDestroy(kv.second.graph);
            if (kv.second.graph_src) (void)hipGraphDestroy(kv.second.graph_src);
            for (TileList *t : {&kv.second.tiles, &kv.second.ptiles, &kv.second.qtiles})
                for (int *p : {t->d_prob, t->d_local, t->d_count})
                    if (p) (void)hipFree(p);
        }
        for (int c = 0; c < s->nclasses; ++c) {
            ClassState &k = s->cls[c];
            for (TileList *t : {&k.init_list, &k.true_list})
                for (int *p : {t->d_prob, t->d_local, t->d_count})
                    if (p) (void)hipFree(p);
            if (k.h_sc) (void)hipHostFree(k.h_sc);
            if (k.ev_a) (void)hipEventDestroy(k.ev_a);
            if (k.ev_b) (void)hipEventDestroy(k.ev_b);
            if (k.ev_in) (void)hipEventDestroy(k.ev_in);
            if (k.own_stream && k.stream) (void)hipStreamDestroy(k.stream);
        }
        (void)hipFree(s->arena_base);
        (void)hipFree(s->d_probs);
        (void)hipFree(s->d_sc);
        (void)hipHostFree(s->h_probs);
        (void)hipStreamDestroy(s->cap_stream);
    }
    delete s;
}

} // extern "C"
