// Host-side planning shared by single solves (engine.hip) and the batched
// server (server.hip): tiling, the Chebyshev interval and coefficients, buffer
// sizes, and the kernel sequence of one Bi-CGSTAB iteration.
#pragma once
#include <cstdio>
#include <cstdlib>

#include "common.h"
#include "poisson.h"

namespace pz {

bool debug_on();

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            if (::pz::debug_on())                                                      \
                fprintf(stderr, "poisson: %s failed: %s (%s:%d)\n", #expr,            \
                        hipGetErrorString(e_), __FILE__, __LINE__);                    \
            return POISSON_ERR_DEVICE;                                                 \
        }                                                                              \
    } while (0)

struct Tiling {
    int tx, ty, kz, tz, ntiles;
};

struct PlanOpts {
    int block = 64;          // Block-Jacobi block edge
    int bj_global = 0;       // 1: GNoComm(CI), global interval on the masked operator
    double lmin_scale = 1.0, lmax_scale = 1.0;
    int debug_bd = -1;
    int fuse = 3;            // Chebyshev steps per pass: 0 one, 1 two, 2 three where possible,
                             // 3 as 2 and four in the mixed mode, 4 four in both modes
};

Tiling make_tiling(int nx, int ny, int nz);
// tiles of the LDS-staged Chebyshev pair (64 * pair_nxw x pair_nyw * pair_pr columns, kz planes)
Tiling make_pair_tiling(int nx, int ny, int nz, bool fp32);
// tiles of the LDS-staged Chebyshev triple (64 * triple_nxw x triple_nyw * triple_pr columns)
Tiling make_triple_tiling(int nx, int ny, int nz, bool fp32);
// tiles of the LDS-staged four-step pass (64 * quad_nxw x quad_nyw * quad_pr columns)
Tiling make_quad_tiling(int nx, int ny, int nz, bool fp32);
bool is_cheb(int pc);
// interval handed to the Chebyshev iteration; false if degenerate
bool cheb_interval(int nx, int ny, int nz, double h, unsigned bc, int pc, const PlanOpts &o,
                   double &lo, double &hi);
// boundary-condition mask checks: Neumann faces need 2 points on their axis, and
// Neumann on all six faces (a singular operator) is not supported
int check_bc(int nx, int ny, int nz, unsigned bc);
// geometry, tolerance and coefficients; vectors, scalars, partials are left null
int fill_prob(Prob &p, int nx, int ny, int nz, double h, unsigned bc, int pc, int deg,
              const PlanOpts &o, double tol, int maxit, double *lo, double *hi);
// whether a plan runs fused Chebyshev step pairs
bool fused(int pc, int deg, bool mixed, int fuse);
// whether the fuse level runs four Chebyshev steps per pass in this precision
inline bool quads_on(int fuse, bool mixed) { return fuse >= 4 || (fuse >= 3 && mixed); }
// whether an apply of degree m starts with steps 1-4 in one pass: four-step
// passes on, and not a degree 4k+1 where triples run (the fours would leave a
// lone last step; such applies start with steps 1-2, or 1-3 in the mixed mode,
// and end on a triple or pair)
inline bool starts_with_four(int fuse, bool mixed, int m, bool quads, bool triples)
{
    return quads && quads_on(fuse, mixed) && m >= 4 && !(triples && m >= 5 && (m - 4) % 4 == 1);
}
// the vector updates (U_S | U_P) a plan can fold into the first passes of its
// applies: fused plans of a single problem with LDS-staged first passes
int upd_fusion(int pc, int deg, bool mixed, int fuse, const Work &w);
// bytes of vector slot v for a plan (0 if unused)
size_t vec_bytes(size_t N, int v, int pc, int deg, bool mixed, int fuse, int upd = 0);
// total workspace of a plan, each slot 256-byte aligned
size_t workspace_bytes(size_t N, int pc, int deg, bool mixed, int fuse, int upd = 0);
// carve a workspace into the vector slots of p (and set p.s_slot)
void carve_workspace(Prob &p, char *ws, size_t N, int pc, int deg, bool mixed, int fuse,
                     int upd = 0);
// reduction partial slots a problem needs: its tiles in every tiling
int partial_slots(int nx, int ny, int nz);
void enqueue_pc(const Work &w, int grid, hipStream_t s, int pc, int m, bool mixed, int fuse,
                int vin, int vout, int second, int upd = 0);
void enqueue_iteration(const Work &w, int grid, hipStream_t s, int pc, int m, bool mixed,
                       int fuse, int upd = 0);
double iteration_bytes(int pc, int m, bool mixed, int fuse, int upd = 0, bool triples = true);
int validate_ptr(const void *p);
double now_ms();

} // namespace pz
