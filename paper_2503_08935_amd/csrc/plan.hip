// plan.hip -- host-side planning shared by single solves and the server.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "plan.h"

namespace pz {

bool debug_on()
{
    static int v = -1;
    if (v < 0) v = getenv("POISSON_DEBUG") ? 1 : 0;
    return v == 1;
}

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ---- Chebyshev interval ----------------------------------------------------
// Every 1D operator on a run of L points (matrix D of eq. matrix_dirichlet, or
// the matrix N of eq. matrix_neuman with a mirror ghost at one or both ends) has
// the eigenvalues 4 sin^2(phi), with phi on an evenly spaced ladder a * pi / q:
//   no Neumann end   a = 1, 2, ..., L          q = 2 (L + 1)   (sine modes)
//   one Neumann end  a = 1, 3, ..., 2L - 1     q = 4 L         (quarter-wave cosines)
//   two Neumann ends a = 0, 1, ..., L - 1      q = 2 (L - 1)   (cosine modes)
// Every rung lies in [0, pi/2], where sin^2 increases, so the bottom rung gives
// the smallest eigenvalue and the top rung the largest.
struct Ladder {
    double bottom, top, q;
};

static Ladder ladder_of(int L, bool neu_lo, bool neu_hi)
{
    const int neumann_ends = (neu_lo ? 1 : 0) + (neu_hi ? 1 : 0);
    if (neumann_ends == 0) return {1.0, (double)L, 2.0 * (double)(L + 1)};
    if (neumann_ends == 1) return {1.0, (double)(2 * L - 1), 4.0 * (double)L};
    return {0.0, (double)(L - 1), 2.0 * (double)(L - 1)};   // L >= 2 (check_bc)
}

static double rung_eigenvalue(double a, double q)
{
    const double s = sin(a * M_PI / q);
    return 4.0 * s * s;
}

// One axis, seen by the operator the Chebyshev iteration runs on: the whole
// axis, or (Block-Jacobi, eq. blockJacobiPreconditioner) the runs of `block`
// points cut out by R_s, whose cut ends act as Dirichlet ends because the
// coupling across them is dropped. A run keeps a Neumann face only if it
// touches that face. A clipped last run lies inside the full-length run of the
// same kind (interlacing), so full-length runs bound every block.
struct AxisRange {
    double mu_lo, mu_hi;
};

static AxisRange axis_range(int n, int block, bool face_lo_neumann, bool face_hi_neumann)
{
    struct Run { int len; bool lo, hi; };
    Run runs[3];
    int nruns = 0;
    if (block <= 0 || n <= block) {
        runs[nruns++] = {n, face_lo_neumann, face_hi_neumann};
    } else {
        runs[nruns++] = {block, face_lo_neumann, false};        // touches the low face
        runs[nruns++] = {block, false, face_hi_neumann};        // touches the high face
        if (n > 2 * block) runs[nruns++] = {block, false, false};  // strictly inside
    }
    AxisRange r{INFINITY, -INFINITY};
    for (int k = 0; k < nruns; ++k) {
        const Ladder l = ladder_of(runs[k].len, runs[k].lo, runs[k].hi);
        r.mu_lo = std::min(r.mu_lo, rung_eigenvalue(l.bottom, l.q));
        r.mu_hi = std::max(r.mu_hi, rung_eigenvalue(l.top, l.q));
    }
    return r;
}

int check_bc(int nx, int ny, int nz, unsigned bc)
{
    if (bc > 63) return POISSON_ERR_ARG;
    const int n[3] = {nx, ny, nz};
    for (int d = 0; d < 3; ++d)
        if (((bc >> (2 * d)) & 3) && n[d] < 2) return POISSON_ERR_ARG;
    if (bc == 63) return POISSON_ERR_UNSUPPORTED;
    return POISSON_OK;
}

Tiling make_tiling(int nx, int ny, int nz)
{
    Tiling t;
    t.tx = (nx + TX - 1) / TX;
    t.ty = (ny + TY * RY - 1) / (TY * RY);
    // z-chunk per tile: long chunks amortise the halo planes (one on each side for
    // a stencil pass, three for the fused Chebyshev pair), but keep at least 1024
    // tiles (4096 waves) so that 256 CUs are busy; at 256^3 kz = 16 measured
    // 11-21% faster solves than kz = 8 with 2048 tiles
    int kz = 64;
    const long base = (long)t.tx * t.ty;
    while (kz > 8 && base * ((nz + kz - 1) / kz) < 1024) kz /= 2;
    t.kz = std::min(kz, std::max(nz, 1));
    t.tz = (nz + t.kz - 1) / t.kz;
    t.ntiles = t.tx * t.ty * t.tz;
    return t;
}

Tiling make_pair_tiling(int nx, int ny, int nz, bool fp32)
{
    Tiling t;
    const int lx = 64 * pair_nxw(fp32), ly = pair_nyw(fp32) * pair_pr(fp32);
    t.tx = (nx + lx - 1) / lx;
    t.ty = (ny + ly - 1) / ly;
    // the longest chunk that leaves a tile for each workgroup slot (FP64: one per
    // CU, FP32: two): 128-plane chunks measured slightly faster than 64-plane
    // ones with 1024 tiles, mostly in the mixed mode
    int kz = 128;
    const long min_tiles = fp32 ? 512 : 256;
    const long base = (long)t.tx * t.ty;
    while (kz > 8 && base * ((nz + kz - 1) / kz) < min_tiles) kz /= 2;
    t.kz = std::min(kz, std::max(nz, 1));
    t.tz = (nz + t.kz - 1) / t.kz;
    t.ntiles = t.tx * t.ty * t.tz;
    return t;
}

Tiling make_triple_tiling(int nx, int ny, int nz, bool fp32)
{
    Tiling t;
    const int lx = 64 * triple_nxw(fp32), ly = triple_nyw(fp32) * triple_pr(fp32);
    t.tx = (nx + lx - 1) / lx;
    t.ty = (ny + ly - 1) / ly;
    // A workgroup fills a CU: take the chunk (8 to 512 planes) that minimises the
    // rounds of 256 tiles times the planes a tile marches (its chunk plus two
    // recomputed planes at each end), the longer one on a tie. At 512^3 that is
    // 256 planes in FP64 and 128 in FP32, one round each (1-2% faster solves than
    // 64-plane chunks, 4% at 256^3); at 640^3 FP64 128 planes in 4 rounds instead
    // of the longest chunk leaving a tile for every CU (256 planes, 600 tiles in 3
    // rounds of which the last is a third full): the solve 5.437 -> 4.713 s
    const long base = (long)t.tx * t.ty;
    const int nzc = std::max(nz, 1);
    long best = -1;
    t.kz = nzc;
    for (int kz = 512; kz >= 8; kz /= 2) {
        const int k = std::min(kz, nzc);
        const long rounds = (base * ((nzc + k - 1) / k) + 255) / 256;
        const long cost = rounds * (k + 4);
        if (best < 0 || cost < best) {
            best = cost;
            t.kz = k;
        }
    }
    t.tz = (nz + t.kz - 1) / t.kz;
    t.ntiles = t.tx * t.ty * t.tz;
    return t;
}

Tiling make_quad_tiling(int nx, int ny, int nz, bool fp32)
{
    Tiling t;
    const int lx = 64 * quad_nxw(fp32), ly = quad_nyw(fp32) * quad_pr(fp32);
    t.tx = (nx + lx - 1) / lx;
    t.ty = (ny + ly - 1) / ly;
    // One workgroup fills a CU, and the pass is bound by issue: its time is about
    // the rounds of 256 tiles times the planes a tile marches (its chunk plus the
    // three recomputed halo planes at each end). Take the chunk (8 to 512 planes)
    // that minimises that product, the longer one on a tie: at 512^3 (FP32) 256
    // planes in one round, measured 1% faster than 128 in two; at 384^3 FP64 32
    // planes in 7 rounds (1728 tiles) where the longest chunk leaving a tile for
    // every CU, 256 planes, gave two rounds of 288 tiles and a 62% slower solve.
    const long base = (long)t.tx * t.ty;
    const int nzc = std::max(nz, 1);
    long best = -1;
    t.kz = nzc;
    for (int kz = 512; kz >= 8; kz /= 2) {
        const int k = std::min(kz, nzc);
        const long rounds = (base * ((nzc + k - 1) / k) + 255) / 256;
        const long cost = rounds * (k + 6);
        if (best < 0 || cost < best) {
            best = cost;
            t.kz = k;
        }
    }
    t.tz = (nz + t.kz - 1) / t.kz;
    t.ntiles = t.tx * t.ty * t.tz;
    return t;
}

bool is_cheb(int pc) { return pc == POISSON_PC_CHEBYSHEV || pc == POISSON_PC_BLOCK_JACOBI; }

bool cheb_interval(int nx, int ny, int nz, double h, unsigned bc, int pc, const PlanOpts &o,
                   double &lo, double &hi)
{
    // The grid operator is a Kronecker sum, so its extreme eigenvalues add over
    // the axes (eqs. lambdaMin, lambdaMax), each axis' divided by h^2. BJ(CI)
    // takes the blocks' interval, GNoComm(CI) the global one (Methodology), and
    // the optional factors rescale the ends (Experimental Setup).
    const bool blocks = pc == POISSON_PC_BLOCK_JACOBI && !o.bj_global;
    const int len[3] = {nx, ny, nz};
    const double h2 = h * h;
    double sum_lo = 0.0, sum_hi = 0.0;
    for (int axis = 0; axis < 3; ++axis) {
        const unsigned faces = bc >> (2 * axis);
        const AxisRange r = axis_range(len[axis], blocks ? o.block : 0, faces & 1u, faces & 2u);
        sum_lo += r.mu_lo / h2;
        sum_hi += r.mu_hi / h2;
    }
    lo = sum_lo * o.lmin_scale;
    hi = sum_hi * o.lmax_scale;
    return lo > 0 && hi > lo && std::isfinite(hi);
}

int fill_prob(Prob &p, int nx, int ny, int nz, double h, unsigned bc, int pc, int deg,
              const PlanOpts &o, double tol, int maxit, double *lo_out, double *hi_out)
{
    memset(&p, 0, sizeof(Prob));
    p.s_slot = V_R;
    const Tiling t = make_tiling(nx, ny, nz);
    p.nx = nx; p.ny = ny; p.nz = nz; p.kz = t.kz;
    p.tx = t.tx; p.ty = t.ty; p.tz = t.tz; p.ntiles = t.ntiles;
    p.pkz[0] = make_pair_tiling(nx, ny, nz, false).kz;
    p.pkz[1] = make_pair_tiling(nx, ny, nz, true).kz;
    p.tkz[0] = make_triple_tiling(nx, ny, nz, false).kz;
    p.tkz[1] = make_triple_tiling(nx, ny, nz, true).kz;
    p.qkz[0] = make_quad_tiling(nx, ny, nz, false).kz;
    p.qkz[1] = make_quad_tiling(nx, ny, nz, true).kz;
    p.block = pc == POISSON_PC_BLOCK_JACOBI ? o.block : 0;
    p.bc = bc;
    p.maxit = maxit;
    p.debug_breakdown_at = o.debug_bd;
    p.degree = deg;
    p.ih2 = 1.0 / (h * h);
    p.ih2f = (float)p.ih2;
    p.tol2 = tol * tol;
    p.jac_d = 6.0 * p.ih2;
    p.jac_df = (float)p.jac_d;
    if (lo_out) *lo_out = 0;
    if (hi_out) *hi_out = 0;
    if (is_cheb(pc)) {
        double lo, hi;
        if (!cheb_interval(nx, ny, nz, h, bc, pc, o, lo, hi)) return POISSON_ERR_ARG;
        if (lo_out) *lo_out = lo;
        if (hi_out) *hi_out = hi;
        // Alg. 2's scalars (eq. chebyshevQuantities) and its rho sequence,
        // rho[0] = 1/sigma and rho[k] = 1/(2 sigma - rho[k-1]); step i >= 2 of
        // an apply takes rho[i] and rho[i-1], the first step rho[1]
        const double theta = (hi + lo) / 2.0, delta = (hi - lo) / 2.0, sigma = theta / delta;
        double rho[MAXDEG + 1];
        rho[0] = 1.0 / sigma;
        for (int k = 1; k <= std::max(deg, 1); ++k) rho[k] = 1.0 / (2.0 * sigma - rho[k - 1]);
        p.theta = theta;
        p.c1 = 2.0 * rho[1] / delta;
        p.two_sigma = 2.0 * sigma;
        p.two_over_delta = 2.0 / delta;
        for (int i = 2; i <= deg; ++i) {
            p.rc[i] = rho[i];
            p.ro[i] = rho[i - 1];
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

bool fused(int pc, int deg, bool mixed, int fuse)
{
    (void)mixed;
    return fuse && is_cheb(pc) && deg >= 3;
}

int upd_fusion(int pc, int deg, bool mixed, int fuse, const Work &w)
{
    if (!fused(pc, deg, mixed, fuse) || w.tile_prob || w.pair_prob) return 0;
    const int f = mixed ? 1 : 0;
    const bool first4 = starts_with_four(fuse, mixed, deg, w.quad_tiles[f] > 0,
                                         fuse >= 2 && w.triple_tiles[f] > 0);
    const bool first3 = fuse >= 2 && w.triple_tiles[f] > 0 && mixed && deg >= 5;
    if (first4 || first3) return U_S | U_P;
    return w.pair_tiles[f] > 0 ? (U_S | U_P) : 0;
}

size_t vec_bytes(size_t N, int v, int pc, int deg, bool mixed, int fuse, int upd)
{
    const bool cheb = is_cheb(pc);
    const size_t tp = (mixed && pc != POISSON_PC_NONE) ? 4 : 8;
    const bool fz = fused(pc, deg, mixed, fuse);
    switch (v) {
    case V_R: case V_RT: case V_P: case V_W: case V_T: return 8 * N;
    case V_PH: case V_SH: return pc != POISSON_PC_NONE ? tp * N : 0;
    case V_RA: return cheb && deg >= 2 ? tp * N : 0;
    case V_RB: return cheb && deg >= 3 ? tp * N : 0;
    // the ring's third and fourth buffers: the pairs after the first one
    case V_RC: return fz && deg >= 4 ? tp * N : 0;
    case V_RD: return fz && deg >= 5 ? tp * N : 0;
    case V_V32: return cheb && mixed && deg >= 1 ? 4 * N : 0;
    case V_S: return (upd & U_S) ? 8 * N : 0;
    case V_P2: return (upd & U_P) ? 8 * N : 0;
    default: return 0;
    }
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t workspace_bytes(size_t N, int pc, int deg, bool mixed, int fuse, int upd)
{
    size_t need = 0;
    for (int v = 0; v < V_COUNT; ++v) need += align256(vec_bytes(N, v, pc, deg, mixed, fuse, upd));
    return need;
}

void carve_workspace(Prob &p, char *ws, size_t N, int pc, int deg, bool mixed, int fuse, int upd)
{
    size_t off = 0;
    for (int v = 0; v < V_COUNT; ++v) {
        const size_t b = vec_bytes(N, v, pc, deg, mixed, fuse, upd);
        if (v != V_X && v != V_B) p.vec[v] = b ? ws + off : nullptr;
        off += align256(b);
    }
    p.s_slot = (upd & U_S) ? V_S : V_R;
}

int partial_slots(int nx, int ny, int nz)
{
    int n = make_tiling(nx, ny, nz).ntiles;
    for (int f = 0; f < 2; ++f) {
        n = std::max(n, make_pair_tiling(nx, ny, nz, f).ntiles);
        n = std::max(n, make_triple_tiling(nx, ny, nz, f).ntiles);
        n = std::max(n, make_quad_tiling(nx, ny, nz, f).ntiles);
    }
    return n;
}

// preconditioner apply vout = M^-1 vin (Alg. 2; BJ(CI) with the masked operator)
void enqueue_pc(const Work &w, int grid, hipStream_t s, int pc, int m, bool mixed, int fuse,
                int vin, int vout, int second, int upd)
{
    if (pc == POISSON_PC_NONE) return;
    if (pc == POISSON_PC_JACOBI || m == 0) {
        KArgs a{vin, vout, 0, 0, 0, second, pc == POISSON_PC_JACOBI ? 0 : 1, 0};
        launch_elem(E_DIV, mixed, w, grid, s, a);
        return;
    }
    const bool mask = pc == POISSON_PC_BLOCK_JACOBI;
    // where later steps read v: the FP32 copy in the mixed mode; with a folded
    // update the vector the first pass formed (s, or this iteration's p)
    int vsrc = vin;
    if (upd == U_S) vsrc = V_S;
    if (upd == U_P) vsrc = V_PCUR;
    if (mixed) vsrc = V_V32;
    if (fused(pc, m, mixed, fuse)) {
        // steps 1 and 2 in one pass: reads v, writes y_1 (RA) and w_2 (RB), and in
        // mixed mode the FP32 copy of v; then steps (i, i+1) in fused pairs, each
        // reading y_{i-1} and z_{i-2} and writing w_i, w_{i+1} to two other buffers
        // of the ring {RA, RB, RC, RD} (nothing is written in place: every input is
        // read by neighbouring tiles); an odd last step runs alone
        // three steps per pass where that is on (LDS-staged single problems):
        // (i, i+1, i+2) read y_{i-1} and z_{i-2} and write w_{i+1}, w_{i+2}; the
        // steps left over run as a pair or alone. The first pass is steps 1-2, or
        // in the mixed mode with degree >= 5 steps 1-3 (in FP64 the two divisions
        // per point of that pass made it slower than a pair: 980 against 605 us)
        const bool tri = fuse >= 2 && w.triple_tiles[mixed ? 1 : 0] > 0;
        // four steps per pass: steps 1-4 first, then fours, then what is left as
        // a triple, pair or single step; a degree 4k+1 with triples starts with
        // steps 1-2 (FP64) or 1-3 (mixed) instead, so that no step is left alone
        const bool quad = quads_on(fuse, mixed) && (w.quad_tiles[mixed ? 1 : 0] > 0 || w.quad_prob);
        const bool first4 = starts_with_four(fuse, mixed, m, quad, tri);
        const bool first3 = !first4 && tri && mixed && m >= 5;
        // a folded update (upd): the first pass forms its input itself; the
        // half-step test of a formed s follows that pass
        const int f = mixed ? 1 : 0;
        const int parts = first4 ? w.quad_tiles[f] : (first3 ? w.triple_tiles[f] : w.pair_tiles[f]);
        // a first pass of four steps that ends the apply writes w_4 alone
        const bool only4 = first4 && m == 4;
        const KArgs a1{vin, V_RA, vin, 0, 1, second, 0, only4 ? vout : V_RB, only4 ? 1 : 0, upd, parts};
        if (first4)
            launch_cheb_first_quad(mixed, mask, w, grid, s, a1);
        else if (first3)
            launch_cheb_first_triple(mask, w, s, a1);
        else
            launch_cheb_first_pair(mixed, mask, w, grid, s, a1);
        if (upd == U_S) launch_finalize_ss(w, grid, s, a1);
        if (only4) return;
        const int ring[4] = {V_RA, V_RB, V_RC, V_RD};
        int y = V_RB, z = V_RA;
        int i = first4 ? 5 : (first3 ? 4 : 3);
        if (quad) {
            for (; i + 3 <= m; i += 4) {
                int o[2], n = 0;
                for (int b : ring)
                    if (b != y && b != z && n < 2) o[n++] = b;
                const bool last = i + 3 == m;
                const int w4 = last ? vout : o[1];
                launch_cheb_quad(mixed, mask, w, grid, s,
                                 KArgs{y, o[0], vsrc, z, i, second, 0, w4, last ? 1 : 0});
                z = o[0];
                y = w4;
            }
        }
        if (tri) {
            for (; i + 2 <= m; i += 3) {
                int o[2], n = 0;
                for (int b : ring)
                    if (b != y && b != z && n < 2) o[n++] = b;
                const bool last = i + 2 == m;
                const int w3 = last ? vout : o[1];
                launch_cheb_triple(mixed, mask, w, s,
                                   KArgs{y, o[0], vsrc, z, i, second, 0, w3, last ? 1 : 0});
                z = o[0];
                y = w3;
            }
        }
        for (; i + 1 <= m; i += 2) {
            int o[2], n = 0;
            for (int b : ring)
                if (b != y && b != z && n < 2) o[n++] = b;
            const bool last = i + 1 == m;
            const int w2 = last ? vout : o[1];
            launch_cheb_pair(mixed, mask, w, grid, s,
                             KArgs{y, o[0], vsrc, z, i, second, 0, w2, last ? 1 : 0});
            z = o[0];
            y = w2;
        }
        if (i == m)
            launch_stencil(S_CHEBK, mixed, mask, w, grid, s, KArgs{y, vout, vsrc, z, m, second, 0, 0});
        return;
    }
    KArgs a1{vin, m == 1 ? vout : (int)V_RA, 0, 0, 1, second, 0, 0};
    launch_stencil(S_CHEB1, mixed, mask, w, grid, s, a1);
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
void enqueue_iteration(const Work &w, int grid, hipStream_t s, int pc, int m, bool mixed,
                       int fuse, int upd)
{
    const bool pm = mixed && pc != POISSON_PC_NONE;
    const int ph = pc == POISSON_PC_NONE ? V_P : V_PH;
    const int sh = pc == POISSON_PC_NONE ? V_R : V_SH;
    // M p^ = p (with U_P the p update of the previous iteration happens here)
    enqueue_pc(w, grid, s, pc, m, mixed, fuse, V_P, V_PH, 0, upd & U_P);
    launch_stencil(S_SDOT, pm, false, w, grid, s, KArgs{ph, V_W, 0, 0, 0, 0, 0, 0});  // w, alpha
    if (!(upd & U_S))
        launch_elem(E_AXPY, false, w, grid, s, KArgs{0, 0, 0, 0, 0, 0, 0, 0});      // s, half step
    enqueue_pc(w, grid, s, pc, m, mixed, fuse, V_R, V_SH, 1, upd & U_S);            // M s^ = s
    launch_stencil(S_SDOT2, pm, false, w, grid, s, KArgs{sh, V_T, 0, 0, 0, 1, 0, 0}); // t, omega
    launch_elem(E_UPD, pm, w, grid, s, KArgs{ph, 0, 0, 0, 0, 0, 0, sh});            // x, r, beta
    if (!(upd & U_P))
        launch_elem(E_PUPD, false, w, grid, s, KArgs{0, 0, 0, 0, 0, 0, 0, 0});      // p
}

// algorithmic bytes per unknown of one iteration of a plan
double iteration_bytes(int pc, int m, bool mixed, int fuse, int upd, bool triples)
{
    const bool pm = mixed && pc != POISSON_PC_NONE;
    const double tp = pm ? 4 : 8;
    double pcb = 0;
    if (pc == POISSON_PC_JACOBI || (is_cheb(pc) && m == 0))
        pcb = 8 + tp;
    else if (is_cheb(pc)) {
        const double tc = mixed ? 4 : 8;
        if (fused(pc, m, mixed, fuse)) {
            // steps 1-2 (or 1-3, mixed with triples; 1-4 mixed with fours): v in;
            // two outputs (+ v32) out, or w_4 alone when that pass ends the apply
            const bool tri = fuse >= 2 && triples, quad = quads_on(fuse, mixed);
            const bool first4 = starts_with_four(fuse, mixed, m, quad, tri);
            if (first4 && m == 4) {
                pcb = 8 + tc;
            } else {
                pcb = 8 + 2 * tc + (mixed ? 4 : 0);
                int steps = m - (first4 ? 4 : ((tri && mixed && m >= 5) ? 3 : 2));
                int passes = 0;                         // passes after the first one
                if (quad) {                             // fours: y, z, v in; two outputs
                    pcb += (steps / 4) * 5 * tc;
                    passes += steps / 4;
                    steps %= 4;
                }
                if (tri) {                              // triples: y, z, v in; w_{i+1}, w_{i+2} out
                    pcb += (steps / 3) * 5 * tc;
                    passes += steps / 3;
                    steps %= 3;
                }
                pcb += (steps / 2) * 5 * tc;            // pairs: y, z, v in; w_i, w_{i+1} out
                passes += steps / 2;
                if (steps & 1) pcb += 4 * tc;           // last step alone: y, v, z, w
                else if (passes > 0) pcb -= tc;         // the last pass stores w_m only
            }
        } else {
            pcb = 8 + tc + (mixed ? 4 : 0);             // first step: v, y (+ v32)
            if (m >= 2) pcb += 3 * tc;                  // step 2: y, v, w
            if (m >= 3) pcb += (m - 2) * 4 * tc;        // steps 3..m: y, v, z, w
        }
    }
    double b = 2 * pcb;
    b += tp + 16;                                        // w = A p^, r~.w
    b += 24;                                             // s = r - alpha w
    b += tp + 16;                                        // t = A s^, t.s, t.t
    b += pc == POISSON_PC_NONE ? 56 : 48 + 2 * tp;       // x, r updates
    b += 32;                                             // p update
    // folded updates: the first pass of the second apply reads r and w instead of
    // s and also writes s (+16) in place of the s update (-24); the first pass of
    // the first apply reads r, w and the previous p instead of p and also writes
    // p (+24) in place of the p update (-32)
    if (upd & U_S) b += 16 - 24;
    if (upd & U_P) b += 24 - 32;
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

} // namespace pz
