// Internal types shared by the kernels and the host engine of libpoisson.
//
// A solve (or a batch of solves, for serving) is described to the kernels by
// an array of Prob descriptors in device memory plus a tile list. Every kernel
// walks tiles of TX x TY columns by kz planes; each tile belongs to one
// problem. Reductions are per problem and deterministic: every tile writes a
// double-double partial into its own slot, and a small finalize kernel launched
// right after sums each problem's slots in index order and updates that
// problem's scalars. A problem's arithmetic therefore depends only on the
// problem itself, never on which other problems share the launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pz {

constexpr int TX = 64;          // x extent of a tile = one wave64 row
constexpr int TY = 4;           // waves per workgroup
constexpr int RY = 4;           // y rows per wave (a tile is TY*RY rows)
constexpr int NTHREADS = TX * TY;
constexpr int MAXDEG = 64;      // largest Chebyshev degree
constexpr int PARTIAL_STRIDE = 4; // doubles per tile partial: two double-double sums
// tiles of the LDS-staged Chebyshev pair: pair_nxw x pair_nyw waves, each 64
// columns x pair_pr rows; 128 x 32 in FP64 (eight waves, one workgroup per CU),
// 256 x 16 in FP32 (eight waves in two rows)
constexpr int pair_nxw(bool fp32) { return fp32 ? 4 : 2; }
constexpr int pair_nyw(bool fp32) { return fp32 ? 2 : 4; }
constexpr int pair_pr(bool fp32) { return fp32 ? 8 : 8; }
// tiles of the LDS-staged Chebyshev triple: triple_nxw x triple_nyw waves, each
// 64 columns x triple_pr rows; 64 x 32 in FP64, 128 x 32 in FP32 (eight waves,
// one workgroup per CU, in both)
constexpr int triple_nxw(bool fp32) { return fp32 ? 2 : 1; }
constexpr int triple_nyw(bool fp32) { return fp32 ? 4 : 8; }
constexpr int triple_pr(bool fp32) { return fp32 ? 8 : 4; }
// tiles of the LDS-staged four-step pass (mixed mode only): 64 x 32, eight waves
// of 4 rows (a group of halo-column lanes per held row: at most 8 rows)
constexpr int quad_nxw(bool fp32) { return fp32 ? 1 : 1; }
constexpr int quad_nyw(bool fp32) { return fp32 ? 8 : 8; }
// two rows per wave in FP64: the LDS planes of 64 x 32 tiles would not fit a CU
constexpr int quad_pr(bool fp32) { return fp32 ? 4 : 2; }

// vector slots of a problem. V_S and V_P2 exist only when the vector updates are
// folded into the first pass of the preconditioner applies (upd_fusion): s is
// then written to a vector of its own (neighbouring tiles still read r), and p
// alternates between V_P and V_P2 from one iteration to the next. V_PCUR is not
// a slot: a kernel handed it reads p of the current iteration, (iter & 1) ?
// V_P2 : V_P.
enum Vec {
    V_X = 0, V_B, V_R, V_RT, V_P, V_W, V_T, V_PH, V_SH, V_RA, V_RB, V_V32, V_RC, V_RD, V_S, V_P2,
    V_COUNT, V_PCUR = 31
};

// which vector updates a plan folds into the first pass of an apply
enum Upd {
    U_S = 1,       // s = r - alpha w and s.s in the first pass of the second apply
    U_P = 2        // p = r + beta (p - omega w) in the first pass of the first apply
};

// status codes mirrored from poisson.h
enum {
    ST_OK = 0, ST_NOT_CONVERGED = 1, ST_BREAKDOWN = -5, ST_NONFINITE = -6
};

// Per-problem scalar block (device). Written only by the finalize kernel of a
// reduction, read by every tile at the start of later kernels.
struct Scalars {
    double rho, alpha, omega, beta;
    double bb, tol2bb, rr, ss;
    double rr_true, dot, pad_d[2];
    int iter, done, status, half_pending;
    int half, zero_x, pad_i[2];
    unsigned pad_u[4];
};

struct Prob {
    int nx, ny, nz, kz;          // grid and tile z-chunk
    int tx, ty, tz, ntiles;      // tile counts
    int block;                   // Block-Jacobi block edge (masked operator), 0 = none
    int maxit, debug_breakdown_at, degree;
    int hist_iters;              // iterations recorded in hist
    unsigned bc;                 // bit f (x-, x+, y-, y+, z-, z+) = Neumann on face f
    int pkz[2];                  // z-chunk of the LDS-staged pair's tiles: [0] FP64, [1] FP32
    int tkz[2];                  // and of the LDS-staged triple's tiles
    int qkz[2];                  // and of the LDS-staged four-step pass's tiles
    double ih2;                  // 1/(h*h)
    double tol2;                 // tol*tol
    double jac_d;                // diagonal of A = 6*ih2
    double theta, c1, two_sigma, two_over_delta;
    float ih2f, jac_df, thetaf, c1f, two_sigmaf, two_over_deltaf, padf[2];
    double rc[MAXDEG + 1], ro[MAXDEG + 1];   // rho_cur, rho_old of Chebyshev step i
    float rcf[MAXDEG + 1], rof[MAXDEG + 1];
    void *vec[V_COUNT];
    int s_slot;                  // where the second half of an iteration reads s: V_R, or
                                 // V_S when the first pass of the second apply forms it
    int nparts_first;            // tile partials holding s.s when that pass forms s for
                                 // batched problems (its tiles); 0: given by the launch
    Scalars *sc;
    double *partials;            // ntiles * PARTIAL_STRIDE
    double *hist;                // 1 + 4*hist_iters, or null
};

// Tile work list of one launch.
struct Work {
    const Prob *probs;
    const int *tile_prob;        // null: single problem 0, tile t is local tile t
    const int *tile_local;
    const int *count_dev;        // null: use count
    int count;
    int order;                   // single problem: 0 natural tile order, 1 x-grouped
    int pair_tiles[2];           // single problem: > 0 runs the Chebyshev pairs LDS-staged
                                 // over this many tiles ([0] FP64, [1] FP32); 0 = register tiles
    int neumann;                 // it has (some problem has) a Neumann face: the LDS-staged
                                 // pairs then select neighbours
    int triple_tiles[2];         // single problem: > 0 runs three Chebyshev steps per pass
                                 // (LDS-staged) over this many tiles ([0] FP64, [1] FP32)
    int quad_tiles[2];           // single problem: > 0 runs four Chebyshev steps per pass
                                 // (LDS-staged) over this many tiles ([0] FP64, [1] FP32)
    // batched problems: the LDS-staged pairs' own tile list (null: single problem)
    const int *pair_prob;
    const int *pair_local;
    const int *pair_count_dev;
    // batched problems: the four-step passes' tile list (null: single problem, or
    // no four-step passes)
    const int *quad_prob;
    const int *quad_local;
    const int *quad_count_dev;
};

// operations of the stencil kernel family
enum SOp {
    S_APPLY = 0,  // out = A u
    S_CHEB1,      // y = c1 (2 v - A v / theta)                      (first Chebyshev step)
    S_CHEB2,      // w = rc ((2 sigma y + (2/delta)(v - A y)) - ro v/theta)   (step 2)
    S_CHEBK,      // w = rc ((2 sigma y + (2/delta)(v - A y)) - ro z)         (steps >= 3)
    S_SDOT,       // w = A p^, dot r~.w -> alpha
    S_SDOT2,      // t = A s^, dots t.s, t.t -> omega
    S_INIT,       // r = b - A x0; r~ = p = r; dots r.r, b.b
    S_TRUE        // dot (b - A x).(b - A x)
};

// operations of the elementwise kernel family
enum EOp {
    E_AXPY = 0,   // s = r - alpha w (in place), dot s.s -> half-step test
    E_UPD,        // x = (x + alpha p^) + omega s^, r = s - omega t, dots r~.r, r.r -> beta
    E_PUPD,       // p = r + beta (p - omega w)
    E_DIV,        // out = v / d  (point Jacobi, or Chebyshev degree 0 with d = theta)
    E_DOT         // dot x.y
};

struct KArgs {
    int in, out, v, z;           // vector slots
    int step;                    // Chebyshev step index (S_CHEB2 / S_CHEBK)
    int second;                  // 1: belongs to the second half of the iteration
    int divisor;                 // E_DIV: 0 = jac_d, 1 = theta
    int x2;                      // E_DOT second operand slot / E_UPD s^ slot
    int drop1;                   // fused pair: 1 = w_i is not stored (the last pair of an
                                 // apply, whose w_i no later step reads)
    int upd;                     // first pass of an apply: 0 reads v = in; U_S forms
                                 // v = s = r - alpha w (stored to V_S, s.s reduced); U_P
                                 // forms v = p = r + beta (p - omega w) (stored to the p
                                 // of this iteration)
    int nparts;                  // partial slots the reduction's finalize sums (0: ntiles)
};

// host-side launchers (device.hip)
void launch_stencil(int op, bool mixed, bool mask, const Work &w, int grid, hipStream_t s,
                    const KArgs &a);
void launch_elem(int op, bool mixed, const Work &w, int grid, hipStream_t s, const KArgs &a);
// two fused Chebyshev steps i, i+1 (i >= 3; FP64, or FP32 when mixed): in = y_{i-1},
// z = z_{i-2}, v; out = w_i, x2 = w_{i+1}; step = i
void launch_cheb_pair(bool mixed, bool mask, const Work &w, int grid, hipStream_t s, const KArgs &a);
// Chebyshev steps 1 and 2 in one pass: in = v (FP64), out = y_1, x2 = w_2, step = 1;
// in mixed mode the FP32 copy of v is written to V_V32 as well. a.upd folds a
// vector update into the pass (LDS-staged single problems only)
void launch_cheb_first_pair(bool mixed, bool mask, const Work &w, int grid, hipStream_t s,
                            const KArgs &a);
// the half-step test on the s.s partials of a first pass with a.upd = U_S
void launch_finalize_ss(const Work &w, int grid, hipStream_t s, const KArgs &a);
// four fused Chebyshev steps i..i+3, LDS-staged: in = y_{i-1}, z = y_{i-2},
// v; out = w_{i+2}, x2 = w_{i+3}; drop1: w_{i+2} is not stored. Single problems
// launch one workgroup per tile; batched ones (w.quad_prob) `grid` workgroups
// over the list
void launch_cheb_quad(bool mixed, bool mask, const Work &w, int grid, hipStream_t s, const KArgs &a);
// steps 1-4 in one pass: in = v (FP64), out = y_3, x2 = w_4, in mixed mode also the
// FP32 copy of v (drop1: w_4 alone, the apply's output, when the degree is 4);
// a.upd as for the first pair
void launch_cheb_first_quad(bool mixed, bool mask, const Work &w, int grid, hipStream_t s,
                            const KArgs &a);
// three fused Chebyshev steps i, i+1, i+2 (i >= 3), LDS-staged, single problem:
// in = y_{i-1}, z = y_{i-2}, v; out = w_{i+1}, x2 = w_{i+2}; step = i; drop1:
// w_{i+1} is not stored
void launch_cheb_triple(bool mixed, bool mask, const Work &w, hipStream_t s, const KArgs &a);
// Chebyshev steps 1, 2 and 3 in one pass in the mixed mode (FP32 arithmetic,
// LDS-staged, single problem): in = v (FP64, rounded once), out = y_2,
// x2 = y_3, step = 1; the FP32 copy of v is written to V_V32 as well
void launch_cheb_first_triple(bool mask, const Work &w, hipStream_t s, const KArgs &a);
void launch_fill_uniform(double *out, int64_t n, uint64_t seed, hipStream_t s);

} // namespace pz
