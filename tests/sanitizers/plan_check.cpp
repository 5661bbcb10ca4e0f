// Host-side checks of the solver's planning code (plan.hip), built with g++
// under AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_sanitizers.py. The kernel launchers are replaced by recorders, so
// the kernel sequence of one Bi-CGSTAB iteration (Alg. 3 order, Alg. 2 inside
// each preconditioner apply) can be checked without a GPU:
//   * every Chebyshev launch reads and writes workspace slots that the plan
//     allocates, never writes a vector it reads at neighbouring points in the
//     same pass, and each step reads the previous step's output; the last step
//     lands in the apply's output slot;
//   * the algorithmic bytes of the recorded launches, counted launch by launch,
//     equal the closed-form byte model iteration_bytes();
//   * the workspace slots are disjoint, 256-byte aligned and inside the
//     workspace; fill_prob's coefficients are finite.
// Exit status 0 on success; a failed check prints its plan and exits 1.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "plan.h"

using namespace pz;

namespace {

enum Kind { K_STENCIL, K_ELEM, K_PAIR, K_FIRST_PAIR, K_TRIPLE, K_FIRST_TRIPLE, K_QUAD, K_FIRST_QUAD,
            K_FIN_SS };

struct Launch {
    Kind kind;
    int op;
    bool mixed;
    KArgs a;
};

std::vector<Launch> g_log;
int g_fail = 0;

#define CHECK(cond, ...)                                                                 \
    do {                                                                                 \
        if (!(cond)) {                                                                   \
            fprintf(stderr, "check failed: %s: ", #cond);                                \
            fprintf(stderr, __VA_ARGS__);                                                \
            fprintf(stderr, "\n");                                                       \
            ++g_fail;                                                                    \
        }                                                                                \
    } while (0)

} // namespace

namespace pz {
void launch_stencil(int op, bool mixed, bool, const Work &, int, hipStream_t, const KArgs &a)
{
    g_log.push_back({K_STENCIL, op, mixed, a});
}
void launch_elem(int op, bool mixed, const Work &, int, hipStream_t, const KArgs &a)
{
    g_log.push_back({K_ELEM, op, mixed, a});
}
void launch_cheb_pair(bool mixed, bool, const Work &, int, hipStream_t, const KArgs &a)
{
    g_log.push_back({K_PAIR, 0, mixed, a});
}
void launch_cheb_first_pair(bool mixed, bool, const Work &, int, hipStream_t, const KArgs &a)
{
    g_log.push_back({K_FIRST_PAIR, 0, mixed, a});
}
void launch_cheb_triple(bool mixed, bool, const Work &, hipStream_t, const KArgs &a)
{
    g_log.push_back({K_TRIPLE, 0, mixed, a});
}
void launch_cheb_first_triple(bool, const Work &, hipStream_t, const KArgs &a)
{
    g_log.push_back({K_FIRST_TRIPLE, 0, true, a});
}
void launch_cheb_quad(bool mixed, bool, const Work &, int, hipStream_t, const KArgs &a)
{
    g_log.push_back({K_QUAD, 0, mixed, a});
}
void launch_cheb_first_quad(bool mixed, bool, const Work &, int, hipStream_t, const KArgs &a)
{
    g_log.push_back({K_FIRST_QUAD, 0, mixed, a});
}
void launch_finalize_ss(const Work &, int, hipStream_t, const KArgs &a)
{
    g_log.push_back({K_FIN_SS, 0, false, a});
}
void launch_fill_uniform(double *, int64_t, uint64_t, hipStream_t) {}
} // namespace pz

namespace {

// bytes per unknown of one recorded launch: each vector read or written once,
// 8 bytes in FP64, 4 for the preconditioner's vectors in the mixed mode
double launch_bytes(const Launch &l, int pc)
{
    const bool pm = l.mixed && pc != POISSON_PC_NONE;
    const double tp = pm ? 4 : 8;          // p^, s^
    const double tc = l.mixed ? 4 : 8;     // Chebyshev buffers
    // a first pass that forms its v: reads r, w (s) or r, w, p (p) and writes v
    const double vin = l.a.upd == U_S ? 8 + 8 + 8 : l.a.upd == U_P ? 8 + 8 + 8 + 8 : 8;
    switch (l.kind) {
    case K_FIN_SS:
        return 0;
    case K_FIRST_PAIR:
        return vin + 2 * tc + (l.mixed ? 4 : 0);        // v in; y_1, w_2 (+ v32) out
    case K_FIRST_TRIPLE:
        return vin + 2 * tc + 4;                        // v in; y_2, y_3, v32 out
    case K_FIRST_QUAD:                                  // v in; y_3, y_4 (+ v32) out, or y_4
        return l.a.drop1 ? vin + tc : vin + 2 * tc + (l.mixed ? 4 : 0);
    case K_PAIR:
    case K_TRIPLE:
    case K_QUAD:
        return (l.a.drop1 ? 4 : 5) * tc;                // y, z, v in; one or two outputs
    case K_STENCIL:
        switch (l.op) {
        case S_CHEB1: return 8 + tc + (l.mixed ? 4 : 0);
        case S_CHEB2: return 3 * tc;
        case S_CHEBK: return 4 * tc;
        case S_SDOT: return tp + 16;                    // p^ in; r~ in, w out
        case S_SDOT2: return tp + 16;                   // s^ in; s in, t out
        default: return -1e9;
        }
    case K_ELEM:
        switch (l.op) {
        case E_AXPY: return 24;
        case E_UPD: return pc == POISSON_PC_NONE ? 56 : 48 + 2 * tp;
        case E_PUPD: return 32;
        case E_DIV: return 8 + tp;
        default: return -1e9;
        }
    }
    return -1e9;
}

bool is_cheb_launch(const Launch &l)
{
    if (l.kind == K_FIN_SS) return false;
    if (l.kind != K_STENCIL) return l.kind != K_ELEM;
    return l.op == S_CHEB1 || l.op == S_CHEB2 || l.op == S_CHEBK;
}

void check_plan(int pc, int deg, bool mixed, int fuse, bool lds, bool fold)
{
    char tag[160];
    snprintf(tag, sizeof tag, "pc %d degree %d mixed %d fuse %d lds %d fold %d", pc, deg, (int)mixed,
             fuse, (int)lds, (int)fold);
    const size_t N = 1000;
    Work w{};
    w.count = 1;
    if (lds && fuse >= 2) w.triple_tiles[0] = w.triple_tiles[1] = 7;
    if (lds && fuse >= 3) w.quad_tiles[1] = 7;
    if (lds && fuse >= 4) w.quad_tiles[0] = 7;
    if (lds) w.pair_tiles[0] = w.pair_tiles[1] = 7;
    const int upd = fold ? upd_fusion(pc, deg, mixed, fuse, w) : 0;
    if (fold && !upd) return;
    CHECK(!upd || (lds && is_cheb(pc) && deg >= 3 && fuse >= 1), "%s: folds %d", tag, upd);
    g_log.clear();
    enqueue_iteration(w, 8, nullptr, pc, deg, mixed, fuse, upd);
    const int level = (fuse >= 2 && !lds) ? 1 : fuse;
    double sum = 0;
    for (const Launch &l : g_log) sum += launch_bytes(l, pc);
    const double model = iteration_bytes(pc, deg, mixed, level, upd);
    CHECK(sum == model, "%s: launches %g B, model %g B", tag, sum, model);
    // the standalone updates run exactly when they are not folded, and a folded
    // s is followed by its half-step test over the first pass's tiles
    int n_axpy = 0, n_pupd = 0, n_fin = 0;
    for (size_t k = 0; k < g_log.size(); ++k) {
        const Launch &l = g_log[k];
        if (l.kind == K_ELEM && l.op == E_AXPY) ++n_axpy;
        if (l.kind == K_ELEM && l.op == E_PUPD) ++n_pupd;
        if (l.kind == K_FIN_SS) {
            ++n_fin;
            CHECK(k > 0 && g_log[k - 1].a.upd == U_S && l.a.nparts == 7, "%s: finalize", tag);
        }
        if (l.a.upd && l.kind != K_FIN_SS)
            CHECK(l.kind == K_FIRST_PAIR || l.kind == K_FIRST_TRIPLE || l.kind == K_FIRST_QUAD,
                  "%s: upd on kind %d", tag, (int)l.kind);
    }
    CHECK(n_axpy == ((upd & U_S) ? 0 : 1) && n_pupd == ((upd & U_P) ? 0 : 1) &&
              n_fin == ((upd & U_S) ? 1 : 0),
          "%s: %d axpy, %d p updates, %d finalizes", tag, n_axpy, n_pupd, n_fin);

    // the Chebyshev chain of each apply
    const bool cheb = is_cheb(pc) && deg >= 1;
    int applies = 0;
    int expect_in = -1, prev_out = -1, prev_x2 = -1;
    for (size_t k = 0; k < g_log.size(); ++k) {
        const Launch &l = g_log[k];
        if (l.kind == K_FIN_SS) continue;
        if (!is_cheb_launch(l)) {
            prev_out = prev_x2 = -1;
            continue;
        }
        const KArgs &a = l.a;
        const bool first = l.kind == K_FIRST_PAIR || l.kind == K_FIRST_TRIPLE ||
                           l.kind == K_FIRST_QUAD || (l.kind == K_STENCIL && l.op == S_CHEB1);
        if (first) {
            ++applies;
            expect_in = applies == 1 ? (int)V_P : (int)V_R;
            CHECK(a.in == expect_in, "%s: apply %d reads slot %d", tag, applies, a.in);
        } else {
            // y of this pass = the last output of the pass before
            const int y_prev = prev_x2 >= 0 ? prev_x2 : prev_out;
            CHECK(a.in == y_prev, "%s: launch %zu reads y from slot %d, not %d", tag, k, a.in,
                  y_prev);
        }
        const int outs[2] = {a.out, (l.kind == K_STENCIL) ? -1 : a.x2};
        for (int o : outs) {
            if (o < 0) continue;
            CHECK(vec_bytes(N, o, pc, deg, mixed, level, upd) > 0 || o == V_PH || o == V_SH,
                  "%s: launch %zu writes unallocated slot %d", tag, k, o);
            // a fused pass reads y, z and v at neighbouring points: it must not
            // overwrite them; a single step reads z only at its own point
            CHECK(o != a.in, "%s: launch %zu writes its input slot %d", tag, k, o);
            if (l.kind != K_STENCIL && !first) {
                CHECK(o != a.z && o != a.v, "%s: launch %zu overwrites z/v slot %d", tag, k, o);
            }
        }
        // step 2 forms z = v / theta itself; later steps read z
        const bool reads_z = !first && !(l.kind == K_STENCIL && l.op == S_CHEB2);
        if (reads_z)
            CHECK(vec_bytes(N, a.z, pc, deg, mixed, level, upd) > 0 || a.z == V_P || a.z == V_R,
                  "%s: launch %zu reads unallocated z slot %d", tag, k, a.z);
        prev_out = a.out;
        prev_x2 = (l.kind == K_STENCIL) ? -1 : a.x2;
        // the apply's last pass writes p^ or s^
        size_t nk = k + 1;
        while (nk < g_log.size() && g_log[nk].kind == K_FIN_SS) ++nk;
        const bool last = nk == g_log.size() || !is_cheb_launch(g_log[nk]) ||
                          g_log[nk].kind == K_FIRST_PAIR || g_log[nk].kind == K_FIRST_TRIPLE ||
                          g_log[nk].kind == K_FIRST_QUAD;
        if (last) {
            const int fin = prev_x2 >= 0 ? prev_x2 : prev_out;
            CHECK(fin == (applies == 1 ? (int)V_PH : (int)V_SH), "%s: apply %d ends in slot %d",
                  tag, applies, fin);
        }
    }
    if (cheb) CHECK(applies == 2, "%s: %d applies", tag, applies);

    // workspace: disjoint, aligned, inside
    const size_t total = workspace_bytes(N, pc, deg, mixed, level, upd);
    std::vector<char> ws(total + 256);
    char *base = (char *)(((uintptr_t)ws.data() + 255) & ~(uintptr_t)255);
    Prob p;
    memset(&p, 0, sizeof p);
    carve_workspace(p, base, N, pc, deg, mixed, level, upd);
    CHECK(p.s_slot == ((upd & U_S) ? (int)V_S : (int)V_R), "%s: s slot %d", tag, p.s_slot);
    for (int v = 0; v < V_COUNT; ++v) {
        const size_t b = vec_bytes(N, v, pc, deg, mixed, level, upd);
        if (!b || v == V_X || v == V_B) continue;
        const char *s = (const char *)p.vec[v];
        CHECK(s && ((uintptr_t)s & 255) == 0, "%s: slot %d misaligned", tag, v);
        CHECK(s >= base && s + b <= base + total, "%s: slot %d outside the workspace", tag, v);
        for (int u = 0; u < v; ++u) {
            const size_t c = vec_bytes(N, u, pc, deg, mixed, level, upd);
            if (!c || u == V_X || u == V_B) continue;
            const char *t = (const char *)p.vec[u];
            CHECK(s + b <= t || t + c <= s, "%s: slots %d and %d overlap", tag, u, v);
        }
        memset(p.vec[v], 0x5a, b); // touch every byte under AddressSanitizer
    }
}

void check_fill(int n, unsigned bc, int pc, int deg, int block, int bj_global)
{
    PlanOpts o;
    o.block = block;
    o.bj_global = bj_global;
    Prob p;
    memset(&p, 0, sizeof p);
    double lo = 0, hi = 0;
    const int rc = fill_prob(p, n, n + 3, n + 1, 1.0 / (n + 1), bc, pc, deg, o, 1e-8, 100, &lo, &hi);
    CHECK(rc == POISSON_OK, "fill_prob n %d bc %u pc %d: %d", n, bc, pc, rc);
    if (rc != POISSON_OK || !is_cheb(pc)) return;
    CHECK(lo > 0 && hi > lo, "interval n %d bc %u: [%g, %g]", n, bc, lo, hi);
    CHECK(std::isfinite(p.theta) && std::isfinite(p.c1) && std::isfinite(p.two_sigma),
          "coefficients n %d bc %u", n, bc);
    for (int i = 2; i <= deg; ++i)
        CHECK(std::isfinite(p.rc[i]) && std::isfinite(p.ro[i]) && p.rc[i] > 0,
              "rho of step %d, n %d bc %u", i, n, bc);
}

} // namespace

int main()
{
    const int pcs[4] = {POISSON_PC_NONE, POISSON_PC_JACOBI, POISSON_PC_CHEBYSHEV,
                        POISSON_PC_BLOCK_JACOBI};
    for (int pc : pcs)
        for (int deg = 0; deg <= 12; ++deg)
            for (int mixed = 0; mixed < 2; ++mixed)
                for (int fuse = 0; fuse <= 4; ++fuse)
                    for (int lds = 0; lds < 2; ++lds)
                        for (int fold = 0; fold < 2; ++fold) {
                            if (!is_cheb(pc) && deg) continue;
                            check_plan(pc, deg, mixed != 0, fuse, lds != 0, fold != 0);
                        }
    const unsigned bcs[5] = {0u, 1u, 22u, 3u | 12u, 33u};
    for (unsigned bc : bcs)
        for (int n : {2, 5, 17, 64, 100})
            for (int pc : pcs) {
                check_fill(n, bc, pc, 8, 16, 0);
                check_fill(n, bc, pc, 3, 4, 1);
            }
    // tilings cover the grid
    for (int n : {1, 7, 63, 64, 65, 200, 512}) {
        for (int f = 0; f < 2; ++f) {
            const Tiling a = make_tiling(n, n + 1, n + 2);
            const Tiling b = make_pair_tiling(n, n + 1, n + 2, f);
            const Tiling c = make_triple_tiling(n, n + 1, n + 2, f);
            const Tiling d = make_quad_tiling(n, n + 1, n + 2, f);
            for (const Tiling &t : {a, b, c, d})
                CHECK(t.kz >= 1 && (long)t.tz * t.kz >= n + 2 && t.ntiles == t.tx * t.ty * t.tz,
                      "tiling n %d", n);
        }
    }
    // the four-step tiles: the chunk minimises rounds of 256 tiles times the planes
    // a tile marches (chunk + 6), the longer chunk on a tie
    for (int n : {1, 9, 32, 100, 255, 256, 384, 447, 512, 640}) {
        for (int f = 0; f < 2; ++f) {
            const Tiling t = make_quad_tiling(n, n, n, f);
            CHECK(t.tx * 64 * quad_nxw(f) >= n && t.ty * quad_nyw(f) * quad_pr(f) >= n,
                  "quad tiles cover n %d", n);
            const long base = (long)t.tx * t.ty;
            auto cost = [&](int kz) {
                const int k = kz < n ? kz : n;
                return ((base * ((n + k - 1) / k) + 255) / 256) * (k + 6);
            };
            for (int kz = 512; kz >= 8; kz /= 2) {
                const int k = kz < n ? kz : n;
                CHECK(cost(t.kz) < cost(k) || (cost(t.kz) == cost(k) && t.kz >= k),
                      "quad chunk n %d fp32 %d: kz %d against %d", n, f, t.kz, k);
            }
        }
    }
    CHECK(make_quad_tiling(512, 512, 512, true).kz == 256 &&
              make_quad_tiling(512, 512, 512, true).ntiles == 256,
          "512^3 FP32 quad tiling");
    CHECK(make_quad_tiling(512, 512, 512, false).kz == 512 &&
              make_quad_tiling(512, 512, 512, false).ntiles == 256,
          "512^3 FP64 quad tiling");
    // the triples' chunks follow the same rule with two recomputed planes per end
    for (int n : {1, 9, 100, 255, 320, 384, 512, 640}) {
        for (int f = 0; f < 2; ++f) {
            const Tiling t = make_triple_tiling(n, n, n, f);
            const long base = (long)t.tx * t.ty;
            auto cost = [&](int kz) {
                const int k = kz < n ? kz : n;
                return ((base * ((n + k - 1) / k) + 255) / 256) * (k + 4);
            };
            for (int kz = 512; kz >= 8; kz /= 2) {
                const int k = kz < n ? kz : n;
                CHECK(cost(t.kz) < cost(k) || (cost(t.kz) == cost(k) && t.kz >= k),
                      "triple chunk n %d fp32 %d: kz %d against %d", n, f, t.kz, k);
            }
        }
    }
    CHECK(make_triple_tiling(512, 512, 512, false).kz == 256 &&
              make_triple_tiling(512, 512, 512, true).kz == 128 &&
              make_triple_tiling(640, 640, 640, false).kz == 128,
          "512^3 and 640^3 triple tilings");
    CHECK(make_quad_tiling(384, 384, 384, false).kz == 32 &&
              make_quad_tiling(384, 384, 384, true).kz == 128,
          "384^3 quad tilings");
    // a degree 4k+1 with triples starts with a pair (or the mixed first triple)
    for (int m = 4; m <= 13; ++m) {
        CHECK(starts_with_four(3, true, m, true, true) == ((m - 4) % 4 != 1 || m == 4),
              "mixed first pass at degree %d", m);
        CHECK(starts_with_four(3, true, m, true, false), "mixed without triples, degree %d", m);
        CHECK(!starts_with_four(3, false, m, true, true), "FP64 at fuse 3, degree %d", m);
        CHECK(starts_with_four(4, false, m, true, true) == ((m - 4) % 4 != 1),
              "FP64 at fuse 4, degree %d", m);
    }
    if (g_fail) {
        fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    printf("plan checks passed\n");
    return 0;
}
