// device.hip -- gfx950 kernels of the preconditioned Bi-CGSTAB Poisson solver.
//
// Two kernel families walk the same tiles (TX x TY columns, kz planes):
//   k_stencil : z-marching 7-point stencil (the matrix-free operator of
//               eq. matrix_p) fused with the consumer of A u: a Chebyshev step
//               (Alg. 2), an outer Bi-CGSTAB matvec with its dot products
//               (Alg. 3: KernelBiCGS1, KernelBiCGS3), the initial residual, or
//               the true residual.
//   k_elem    : streaming vector updates fused with their dot products
//               (Alg. 3: KernelBiCGS2, KernelBiCGS4+5, KernelBiCGS6) and the
//               point-Jacobi / degree-0 scaling.
// Each wave owns RY rows of its tile and marches k upward keeping planes
// k-1, k, k+1 of them in registers; x neighbours move between lanes by DPP
// wave shifts. Streams read or written once bypass the caches' retention
// (non-temporal hint) so the stencil input's halo re-reads stay in L2.
//
// Arithmetic contract (matched by the independent CPU oracle):
//   * no contraction (built with -ffp-contract=off); the only FMA is the
//     explicit error-free product of the dot products;
//   * (A u) = ((((((6u - u_x-) - u_x+) - u_y-) - u_y+) - u_z-) - u_z+) * (1/(h*h))
//     in FP64, and in FP32 (the mixed-precision preconditioner)
//     ((((u - u_x-) + (u - u_x+)) + ((u - u_y-) + (u - u_y+))) + ((u - u_z-) + (u - u_z+))) * (1/(h*h));
//   * vector updates evaluate left to right exactly as written in Alg. 1 / 2;
//   * dot products: per thread Dot2 (TwoProduct + TwoSum, Ogita, Rump and
//     Oishi 2005), then double-double additions (AccurateDWPlusDW, Joldes,
//     Muller and Popescu 2017) in a fixed tree, rounded once. The result equals
//     the correctly rounded dot product except when the exact value lies within
//     about 1e-30 (relative, times the condition number) of a rounding tie.
//   * scalar divisions are IEEE FP64 divisions.
#include <type_traits>

#include "common.h"

namespace pz {

// ------------------------------------------------------------------------
// streaming accesses: vectors read or written once per kernel are accessed
// with the non-temporal hint, so they do not displace the stencil input (whose
// neighbour rows and planes are re-read from L2) from the caches
// ------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T ld_nt(const T *p)
{
    return __builtin_nontemporal_load((const __attribute__((address_space(1))) T *)p);
}
template <typename T> __device__ __forceinline__ void st_nt(T *p, T v)
{
    __builtin_nontemporal_store(v, (__attribute__((address_space(1))) T *)p);
}
// plain loads through the global address space (pointers read from a
// descriptor are generic; these keep the compiler on global, not flat, loads)
template <typename T> __device__ __forceinline__ T ld_g(const T *p)
{
    return *(const __attribute__((address_space(1))) T *)p;
}

// the vector of slot v of a problem; V_PCUR names p of the current iteration,
// which alternates between V_P and V_P2 when the p update is folded into the
// first pass of the first apply
__device__ __forceinline__ void *vec_at(const Prob &P, int v)
{
    if (v == V_PCUR) return P.vec[(P.sc->iter & 1) ? V_P2 : V_P];
    return P.vec[v];
}

// ------------------------------------------------------------------------
// Tile order of a single problem. Workgroup g runs on XCD g % 8 (round-robin
// dispatch). Natural order puts neighbouring x-tiles on different XCDs, so the
// cache lines of their shared x-halo are fetched into two L2s. The x-grouped
// order takes 8 tile rows (a row = the tx tiles of one (y, z)) at a time and
// gives each XCD one whole row: dispatch d of the group runs row d % 8, x-tile
// d / 8. Rows left over at the end keep natural order. The slab order gives
// XCD x the x-th eighth of all tiles, a contiguous range of whole tile rows,
// when the tile count is a multiple of 8: y-neighbouring tiles then run on one
// XCD, at the same time when there is one tile per workgroup slot.
// ------------------------------------------------------------------------
__device__ __forceinline__ int tile_order_tx(int order, int tx, int g, int total)
{
    if (order == 2) {
        // workgroup g runs on XCD g % 8: XCD x takes the x-th eighth of the tiles
        // (whole tile rows and z-slabs), so x and y neighbours share its L2
        if (total % 8) return g;
        return (g % 8) * (total / 8) + g / 8;
    }
    if (order != 1) return g;
    const int grp = 8 * tx;
    const int base = (g / grp) * grp;
    if (base + grp > total) return g;
    const int d = g - base;
    return base + (d & 7) * tx + (d >> 3);
}

__device__ __forceinline__ int tile_order(int order, const Work &W, const Prob &P, int g,
                                          int total)
{
    if (!order || W.tile_prob) return g;
    return tile_order_tx(order, P.tx, g, total);
}

// ------------------------------------------------------------------------
// double-double arithmetic
// ------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void fast_two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    e = b - (s - a);
}

// (hi, lo) += x * y
__device__ __forceinline__ void dd_acc(double &hi, double &lo, double x, double y)
{
    const double p = x * y;
    const double e = __builtin_fma(x, y, -p);
    double s, r;
    two_sum(hi, p, s, r);
    hi = s;
    lo = lo + (r + e);
}

// (zh, zl) = (ah, al) + (bh, bl)
__device__ __forceinline__ void dd_add(double ah, double al, double bh, double bl, double &zh,
                                       double &zl)
{
    double sh, sl, th, tl, vh, vl;
    two_sum(ah, bh, sh, sl);
    two_sum(al, bl, th, tl);
    const double c = sl + th;
    fast_two_sum(sh, c, vh, vl);
    const double w = tl + vl;
    fast_two_sum(vh, w, zh, zl);
}

// Reduce ND double-double values over a workgroup of NW waves; result valid in
// thread 0. lds holds 2 * ND * NW doubles.
template <int ND, int NW = TY>
__device__ __forceinline__ void block_reduce_dd(double (&hi)[ND], double (&lo)[ND], double *lds)
{
    const int lane = threadIdx.x & (TX - 1), wv = threadIdx.x / TX;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        double s, e;
        two_sum(hi[d], lo[d], s, e);
        hi[d] = s;
        lo[d] = e;
    }
#pragma unroll
    for (int off = TX / 2; off >= 1; off >>= 1) {
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            const double oh = __shfl_xor(hi[d], off, TX);
            const double ol = __shfl_xor(lo[d], off, TX);
            dd_add(hi[d], lo[d], oh, ol, hi[d], lo[d]);
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            lds[(wv * ND + d) * 2] = hi[d];
            lds[(wv * ND + d) * 2 + 1] = lo[d];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            double h = lds[d * 2], l = lds[d * 2 + 1];
            for (int w = 1; w < NW; ++w)
                dd_add(h, l, lds[(w * ND + d) * 2], lds[(w * ND + d) * 2 + 1], h, l);
            hi[d] = h;
            lo[d] = l;
        }
    }
    __syncthreads();
}

// Publish this tile's partial sums in its slot. The sums over all tiles are
// formed by k_finalize, launched right after the reduction kernel: the kernel
// boundary makes every slot visible, so no device-scope fence is needed here
// (on this chip such a fence writes back and invalidates the XCD's L2, which at
// one per tile cost ~15% of the reduction kernels' time).
template <int ND>
__device__ void tile_publish(const Prob &P, int local, double (&hi)[ND], double (&lo)[ND],
                             double *lds)
{
    block_reduce_dd<ND>(hi, lo, lds);
    if (threadIdx.x == 0) {
        double *pp = P.partials + (size_t)local * PARTIAL_STRIDE;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            pp[2 * d] = hi[d];
            pp[2 * d + 1] = lo[d];
        }
    }
}

// Sum a problem's tile partials in tile order (res valid in thread 0).
template <int ND>
__device__ void sum_partials(const Prob &P, int nt, double *lds, double (&res)[ND])
{
    const int chunk = (nt + NTHREADS - 1) / NTHREADS;
    const int b0 = threadIdx.x * chunk, b1 = min(b0 + chunk, nt);
    double h2[ND], l2[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) h2[d] = l2[d] = 0.0;
    const double *pp = P.partials;
    for (int b = b0; b < b1; ++b) {
#pragma unroll
        for (int d = 0; d < ND; ++d)
            dd_add(h2[d], l2[d], pp[(size_t)b * PARTIAL_STRIDE + 2 * d],
                   pp[(size_t)b * PARTIAL_STRIDE + 2 * d + 1], h2[d], l2[d]);
    }
    block_reduce_dd<ND>(h2, l2, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int d = 0; d < ND; ++d) res[d] = h2[d] + l2[d];
    }
}

// ------------------------------------------------------------------------
// scalar epilogues of the reductions (finalize kernel, thread 0)
// ------------------------------------------------------------------------
__device__ __forceinline__ void hist_put(const Prob &P, int it, int slot, double v)
{
    if (P.hist && it >= 1 && it <= P.hist_iters) P.hist[1 + 4 * (it - 1) + slot] = v;
}

__device__ __forceinline__ void fail(Scalars *sc, int status, int it)
{
    sc->status = status;
    sc->done = 1;
    sc->iter = it;
}

// r0 = b - A x0: rho0 = r~.r0 = r0.r0, tolerance on b.b
__device__ void fin_init(const Prob &P, double rr, double bb)
{
    Scalars *sc = P.sc;
    sc->bb = bb;
    sc->tol2bb = P.tol2 * bb;
    sc->rr = rr;
    sc->rho = rr;
    sc->ss = 0.0;
    sc->alpha = sc->omega = sc->beta = 0.0;
    sc->iter = 0;
    sc->half = 0;
    sc->half_pending = 0;
    sc->zero_x = 0;
    if (P.hist) P.hist[0] = rr;
    if (!isfinite(bb) || !isfinite(rr)) {
        sc->status = ST_NONFINITE;
        sc->done = 1;
    } else if (bb == 0.0) {
        sc->zero_x = 1;
        sc->status = ST_OK;
        sc->done = 1;
    } else if (rr < sc->tol2bb) {
        sc->status = ST_OK;
        sc->done = 1;
    } else {
        sc->status = ST_NOT_CONVERGED;
        sc->done = 0;
    }
}

// alpha_i = rho_{i-1} / (r~ . A p^_i)
__device__ void fin_sdot(const Prob &P, double d)
{
    Scalars *sc = P.sc;
    const int it = sc->iter + 1;
    if (!isfinite(d)) return fail(sc, ST_NONFINITE, it);
    if (d == 0.0) return fail(sc, ST_BREAKDOWN, it);
    const double alpha = sc->rho / d;
    sc->alpha = alpha;
    hist_put(P, it, 0, alpha);
    hist_put(P, it, 2, sc->rho);
}

// half-step test ||s|| < tol ||b|| of Alg. 1
__device__ void fin_axpy(const Prob &P, double ss)
{
    Scalars *sc = P.sc;
    const int it = sc->iter + 1;
    if (!isfinite(ss)) return fail(sc, ST_NONFINITE, it);
    if (ss < sc->tol2bb) {
        sc->half_pending = 1;
        sc->ss = ss;
        hist_put(P, it, 1, 0.0);
        hist_put(P, it, 3, ss);
    }
}

// omega_i = (t . s) / (t . t)
__device__ void fin_sdot2(const Prob &P, double ts, double tt)
{
    Scalars *sc = P.sc;
    const int it = sc->iter + 1;
    if (!isfinite(ts) || !isfinite(tt)) return fail(sc, ST_NONFINITE, it);
    if (tt == 0.0) return fail(sc, ST_BREAKDOWN, it);
    double omega = ts / tt;
    if (it == P.debug_breakdown_at) omega = 0.0;
    sc->omega = omega;
}

// end of iteration: convergence, rho_i = r~.r_i, beta_i = (rho_i alpha_i)/(rho_{i-1} omega_i)
__device__ void fin_upd(const Prob &P, double rho_new, double rr)
{
    Scalars *sc = P.sc;
    const int it = sc->iter + 1;
    sc->iter = it;
    if (sc->half_pending) {
        sc->half_pending = 0;
        sc->half = 1;
        sc->rr = sc->ss;
        sc->status = ST_OK;
        sc->done = 1;
        return;
    }
    hist_put(P, it, 1, sc->omega);
    hist_put(P, it, 3, rr);
    sc->rr = rr;
    if (!isfinite(rho_new) || !isfinite(rr)) return fail(sc, ST_NONFINITE, it);
    if (rr < sc->tol2bb) {
        sc->status = ST_OK;
        sc->done = 1;
        return;
    }
    if (rho_new == 0.0 || sc->omega == 0.0) return fail(sc, ST_BREAKDOWN, it);
    sc->beta = (rho_new * sc->alpha) / (sc->rho * sc->omega);
    sc->rho = rho_new;
    if (it >= P.maxit) {
        sc->status = ST_NOT_CONVERGED;
        sc->done = 1;
    }
}

template <typename T> struct Coef;
template <> struct Coef<double> {
    static __device__ double ih2(const Prob &P) { return P.ih2; }
    static __device__ double theta(const Prob &P) { return P.theta; }
    static __device__ double c1(const Prob &P) { return P.c1; }
    static __device__ double two_sigma(const Prob &P) { return P.two_sigma; }
    static __device__ double two_over_delta(const Prob &P) { return P.two_over_delta; }
    static __device__ double rc(const Prob &P, int i) { return P.rc[i]; }
    static __device__ double ro(const Prob &P, int i) { return P.ro[i]; }
    static __device__ double jac(const Prob &P) { return P.jac_d; }
};
template <> struct Coef<float> {
    static __device__ float ih2(const Prob &P) { return P.ih2f; }
    static __device__ float theta(const Prob &P) { return P.thetaf; }
    static __device__ float c1(const Prob &P) { return P.c1f; }
    static __device__ float two_sigma(const Prob &P) { return P.two_sigmaf; }
    static __device__ float two_over_delta(const Prob &P) { return P.two_over_deltaf; }
    static __device__ float rc(const Prob &P, int i) { return P.rcf[i]; }
    static __device__ float ro(const Prob &P, int i) { return P.rof[i]; }
    static __device__ float jac(const Prob &P) { return P.jac_df; }
};

// A u at one point from the centre c and its six neighbours, times ih2. FP64
// evaluates 6c minus the neighbours left to right. FP32 sums the second
// differences of the three axes, each as (c - u_minus) + (c - u_plus): where u
// is smooth each difference is exact and so is their sum, so the result keeps
// FP32's relative accuracy; 6c minus the neighbours cancels there and loses up
// to 6 ih2 / lambda_min of it (about 1e5 at 768^3).
template <typename T>
__device__ __forceinline__ T lap7(T c, T xm, T xp, T ym, T yp, T zm, T zp, T ih2)
{
    return (((((((T)6 * c - xm) - xp) - ym) - yp) - zm) - zp) * ih2;
}
template <>
__device__ __forceinline__ float lap7<float>(float c, float xm, float xp, float ym, float yp,
                                             float zm, float zp, float ih2)
{
    const float dx = (c - xm) + (c - xp), dy = (c - ym) + (c - yp), dz = (c - zm) + (c - zp);
    return ((dx + dy) + dz) * ih2;
}

// ------------------------------------------------------------------------
// wave64 lane exchange: DPP wavefront shift by one lane (the lane without a
// source reads 0) and lane broadcast
// ------------------------------------------------------------------------
__device__ __forceinline__ double lane_prev(double v) // lane l gets lane l-1
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_next(double v) // lane l gets lane l+1
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_prev(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_next(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double read_lane(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float read_lane(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// neighbour selection of one point along one axis: 0 zero, 1 neighbour, 2 mirror
__device__ __forceinline__ int sel_lo(int a, int n, bool mask, int B, bool neu)
{
    return a > 0 ? ((!mask || a % B != 0) ? 1 : 0) : ((neu && n >= 2) ? 2 : 0);
}
__device__ __forceinline__ int sel_hi(int a, int n, bool mask, int B, bool neu)
{
    return a + 1 < n ? ((!mask || (a + 1) % B != 0) ? 1 : 0)
                     : ((neu && n >= 2 && (!mask || a % B != 0)) ? 2 : 0);
}

// A selection code as two flags, so that picking a neighbour value is a pair
// of selects (an integer code compared twice tends to become a branch).
struct Sel {
    bool nb, mi; // neighbour, mirror; neither: zero
};
__device__ __forceinline__ Sel to_sel(int code) { return Sel{code == 1, code == 2}; }
__device__ __forceinline__ float pick(Sel s, float nbv, float miv)
{
    const float t = s.mi ? miv : 0.0f;
    return s.nb ? nbv : t;
}
__device__ __forceinline__ double pick(Sel s, double nbv, double miv)
{
    const double t = s.mi ? miv : 0.0;
    return s.nb ? nbv : t;
}

// ------------------------------------------------------------------------
// stencil family
// A tile is TX columns in x (one wave64 row) by TY*RY rows in y (wave w owns
// RY consecutive rows) by kz planes. Each thread marches k upward keeping
// planes k-1, k and k+1 of its RY rows in registers. x neighbours come from
// the adjacent lanes (DPP wave shift); the two x-halo values of every row
// come from one load per wave and plane (lanes 0..RY-1 the left ones, lanes
// 32..32+RY-1 the right ones); y neighbours inside a wave's rows are
// registers and the two halo rows one load each.
// TU: element type of the stencil input; TC: arithmetic type.
// ------------------------------------------------------------------------

// One tile of a stencil pass; its dot products accumulate into hi/lo.
// FULL: the wave's RY rows and the tile's 64 columns are inside the grid, so
// no row or column guard is needed. SIMPLE: no block mask and no Neumann face;
// a neighbour outside the grid then reads as the +0.0 that the zero-filled
// loads already hold, so no neighbour selection is needed either. Loads read
// clamped (valid) addresses and a select keeps or zeroes the value, so the
// loads of a plane issue together instead of each behind its own guard.
template <int OP, typename TU, typename TC, bool MASK, bool FULL, bool SIMPLE>
__device__ __forceinline__ void stencil_tile(const Prob &P, const KArgs &A, int local, int lane,
                                             int wv, double (&hi)[2], double (&lo)[2])
{
    const int nx = P.nx, ny = P.ny, nz = P.nz, tx = P.tx, ty = P.ty;
    const int tix = local % tx, tiy = (local / tx) % ty, tiz = local / (tx * ty);
    const int i0 = tix * TX, i = i0 + lane;
    const int j0 = tiy * (TY * RY) + wv * RY;
    const int k0 = tiz * P.kz, k1 = min(k0 + P.kz, nz);
    if (j0 >= ny) return; // uniform within the wave

    const size_t S = (size_t)nx * (size_t)ny, NXs = (size_t)nx;
    const TU *__restrict__ u = (const TU *)P.vec[A.in];
    const int B = MASK ? P.block : 1;
    const bool xin = FULL || i < nx;
    const int ic = xin ? i : nx - 1;
    // neighbour selection per face: zero (Dirichlet face or another block), the
    // neighbour, or the mirror image across a Neumann face (u_{-1} = u_1, eq.
    // matrix_neuman); mirrors also respect the block mask
    const unsigned bc = P.bc;
    const bool nxl = bc & 1u, nxh = bc & 2u, nyl = bc & 4u, nyh = bc & 8u;
    const bool nzl = bc & 16u, nzh = bc & 32u;
    const Sel sxm = to_sel(xin ? sel_lo(i, nx, MASK, B, nxl) : 0);
    const Sel sxp = to_sel(xin ? sel_hi(i, nx, MASK, B, nxh) : 0);
    bool rin[RY];
    size_t roff[RY]; // in-plane offset of the lane's point in row r (clamped)
    Sel sym[RY], syp[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int j = j0 + r;
        rin[r] = FULL || (xin && j < ny);
        roff[r] = (size_t)ic + NXs * (size_t)(FULL ? j : min(j, ny - 1));
        sym[r] = to_sel(rin[r] ? sel_lo(j, ny, MASK, B, nyl) : 0);
        syp[r] = to_sel(rin[r] ? sel_hi(j, ny, MASK, B, nyh) : 0);
    }
    const bool ymh = xin && j0 > 0;
    const bool yph = xin && j0 + RY < ny;
    const size_t ymoff = (size_t)ic + NXs * (size_t)(j0 > 0 ? j0 - 1 : 0);
    const size_t ypoff = (size_t)ic + NXs * (size_t)min(j0 + RY, ny - 1);
    const int hrow = lane & 31;
    const bool hload = hrow < RY && j0 + hrow < ny && (lane < 32 ? i0 > 0 : i0 + TX < nx);
    const size_t hoff =
        hload ? (size_t)(lane < 32 ? i0 - 1 : i0 + TX) + NXs * (size_t)(j0 + hrow) : 0;
    const TC ih2 = Coef<TC>::ih2(P);
    TC cA = 0, cB = 0, cC = 0, cD = 0, cE = 0;
    if constexpr (OP == S_CHEB1) {
        cA = Coef<TC>::c1(P);
        cB = Coef<TC>::theta(P);
    } else if constexpr (OP == S_CHEB2 || OP == S_CHEBK) {
        cA = Coef<TC>::rc(P, A.step);
        cB = Coef<TC>::ro(P, A.step);
        cC = Coef<TC>::two_sigma(P);
        cD = Coef<TC>::two_over_delta(P);
        cE = Coef<TC>::theta(P);
    }
    TC *out = (TC *)P.vec[A.out];
    const TC *vv = (const TC *)vec_at(P, A.v);
    const TC *zz = (const TC *)P.vec[A.z];
    float *v32 = (float *)P.vec[V_V32];
    const double *__restrict__ rt = (const double *)P.vec[V_RT];
    const double *__restrict__ bv = (const double *)P.vec[V_B];
    const double *sv = (const double *)P.vec[P.s_slot];
    double *rr = (double *)P.vec[V_R];
    double *rtw = (double *)P.vec[V_RT];
    double *pw = (double *)P.vec[V_P];

    // type of the streamed operands: the arithmetic type for the Chebyshev steps
    using TO = typename std::conditional<(OP == S_CHEB2 || OP == S_CHEBK), TC, double>::type;
    const TO *o0p = nullptr;
    if constexpr (OP == S_CHEB2 || OP == S_CHEBK) o0p = vv;
    if constexpr (OP == S_SDOT) o0p = rt;
    if constexpr (OP == S_SDOT2) o0p = sv;
    if constexpr (OP == S_INIT || OP == S_TRUE) o0p = bv;

    TC c[RY], zm[RY]; // planes k and k-1
    {
        const size_t pk = S * (size_t)k0, pm = k0 > 0 ? pk - S : pk;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const TC cv = (TC)ld_g(u + pk + roff[r]);
            const TC mv = (TC)ld_g(u + pm + roff[r]);
            c[r] = rin[r] ? cv : (TC)0;
            zm[r] = (rin[r] && k0 > 0) ? mv : (TC)0;
        }
    }
    for (int k = k0; k < k1; ++k) {
        const size_t pk = S * (size_t)k;
        const bool znext = k + 1 < nz;
        const size_t pn = znext ? pk + S : pk;
        const Sel szm = to_sel(sel_lo(k, nz, MASK, B, nzl));
        const Sel szp = to_sel(sel_hi(k, nz, MASK, B, nzh));
        TC zr[RY];
        TO o0[RY], o1[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const TC nv = (TC)ld_g(u + pn + roff[r]);
            zr[r] = (rin[r] && znext) ? nv : (TC)0;
            o0[r] = o1[r] = (TO)0;
            if constexpr (OP != S_APPLY && OP != S_CHEB1) {
                const TO a0 = ld_nt(o0p + pk + roff[r]);
                o0[r] = rin[r] ? a0 : (TO)0;
            }
            if constexpr (OP == S_CHEBK) {
                const TO a1 = ld_nt(zz + pk + roff[r]);
                o1[r] = rin[r] ? a1 : (TO)0;
            }
        }
        const TC ymr = (TC)ld_g(u + pk + ymoff), ypr = (TC)ld_g(u + pk + ypoff);
        const TC hr = (TC)ld_g(u + pk + hoff);
        const TC ymv = ymh ? ymr : (TC)0, ypv = yph ? ypr : (TC)0, he = hload ? hr : (TC)0;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            // the DPP shifts run in every lane (a shift reads its source lane)
            const TC pv = lane_prev(c[r]), nv = lane_next(c[r]);
            const TC el = read_lane(he, r), er = read_lane(he, 32 + r);
            const TC xl = lane == 0 ? el : pv, xr = lane == TX - 1 ? er : nv;
            const TC yl = r == 0 ? ymv : c[r > 0 ? r - 1 : 0];
            const TC yr = r == RY - 1 ? ypv : c[r < RY - 1 ? r + 1 : 0];
            TC xm, xp, ym, yp, zmv, zpv;
            if constexpr (SIMPLE) {
                xm = xl, xp = xr, ym = yl, yp = yr, zmv = zm[r], zpv = zr[r];
            } else {
                xm = pick(sxm, xl, xr), xp = pick(sxp, xr, xl);
                ym = pick(sym[r], yl, yr), yp = pick(syp[r], yr, yl);
                zmv = pick(szm, zm[r], zr[r]), zpv = pick(szp, zr[r], zm[r]);
            }
            const TC a = lap7<TC>(c[r], xm, xp, ym, yp, zmv, zpv, ih2);
            if (rin[r]) {
                const size_t idx = pk + roff[r];
                if constexpr (OP == S_APPLY) {
                    st_nt(out + idx, a);
                } else if constexpr (OP == S_CHEB1) {
                    st_nt(out + idx, cA * ((TC)2 * c[r] - a / cB));
                    if constexpr (sizeof(TC) == 4) st_nt(v32 + idx, c[r]);
                } else if constexpr (OP == S_CHEB2) {
                    const TC v = (TC)o0[r];
                    const TC z = v / cE;
                    st_nt(out + idx, cA * ((cC * c[r] + cD * (v - a)) - cB * z));
                } else if constexpr (OP == S_CHEBK) {
                    const TC v = (TC)o0[r], z = (TC)o1[r];
                    st_nt(out + idx, cA * ((cC * c[r] + cD * (v - a)) - cB * z));
                } else if constexpr (OP == S_SDOT) {
                    st_nt(out + idx, a);
                    dd_acc(hi[0], lo[0], o0[r], a);
                } else if constexpr (OP == S_SDOT2) {
                    st_nt(out + idx, a);
                    dd_acc(hi[0], lo[0], a, o0[r]);
                    dd_acc(hi[1], lo[1], a, a);
                } else if constexpr (OP == S_INIT) {
                    const double b = o0[r];
                    const double res = b - a;
                    st_nt(rr + idx, res);
                    st_nt(rtw + idx, res);
                    st_nt(pw + idx, res);
                    dd_acc(hi[0], lo[0], res, res);
                    dd_acc(hi[1], lo[1], b, b);
                } else if constexpr (OP == S_TRUE) {
                    const double res = o0[r] - a;
                    dd_acc(hi[0], lo[0], res, res);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            zm[r] = c[r];
            c[r] = zr[r];
        }
    }
}

template <int OP, typename TU, typename TC, bool MASK>
__global__ void __launch_bounds__(NTHREADS) k_stencil(Work W, KArgs A)
{
    constexpr int ND = (OP == S_SDOT2 || OP == S_INIT) ? 2
                       : (OP == S_SDOT || OP == S_TRUE) ? 1 : 0;
    constexpr int NA = ND > 0 ? ND : 1;
    __shared__ double lds[TY * 2 * 2];
    const int total = W.count_dev ? *W.count_dev : W.count;
    const int lane = threadIdx.x & (TX - 1), wv = threadIdx.x / TX;

    for (int g = blockIdx.x; g < total; g += gridDim.x) {
        const int pid = W.tile_prob ? W.tile_prob[g] : 0;
        const Prob &P = W.probs[pid];
        const int local = W.tile_prob ? W.tile_local[g] : tile_order(W.order, W, P, g, total);
        if (OP != S_INIT && OP != S_TRUE && OP != S_APPLY) {
            const Scalars *sc = P.sc;
            if (sc->done || (A.second && sc->half_pending)) continue;
        }
        double hi[2] = {0.0, 0.0}, lo[2] = {0.0, 0.0};
        // one wave-uniform branch per tile
        const int tix = local % P.tx, tiy = (local / P.tx) % P.ty;
        const int j0 = tiy * (TY * RY) + wv * RY;
        const bool full = tix * TX + TX <= P.nx && j0 + RY <= P.ny;
        if constexpr (MASK) {
            if (full) stencil_tile<OP, TU, TC, true, true, false>(P, A, local, lane, wv, hi, lo);
            else stencil_tile<OP, TU, TC, true, false, false>(P, A, local, lane, wv, hi, lo);
        } else {
            if (P.bc == 0) {
                if (full) stencil_tile<OP, TU, TC, false, true, true>(P, A, local, lane, wv, hi, lo);
                else stencil_tile<OP, TU, TC, false, false, true>(P, A, local, lane, wv, hi, lo);
            } else {
                if (full) stencil_tile<OP, TU, TC, false, true, false>(P, A, local, lane, wv, hi, lo);
                else stencil_tile<OP, TU, TC, false, false, false>(P, A, local, lane, wv, hi, lo);
            }
        }
        if constexpr (ND > 0) {
            double h2[NA], l2[NA];
#pragma unroll
            for (int d = 0; d < NA; ++d) h2[d] = hi[d], l2[d] = lo[d];
            tile_publish<NA>(P, local, h2, l2, lds);
        }
    }
}

// ------------------------------------------------------------------------
// FP32 Chebyshev steps (mixed precision) with two consecutive x points per
// lane, so every access moves 8 bytes (4 bytes per lane wastes half of each
// memory transaction slot). Same tiles as k_stencil: the wave's RY rows are
// split between its two half-waves (RY/2 rows each), a half-wave covers the
// tile's 64 x points as 32 lanes x 2. x neighbours inside a lane's pair are
// registers, across lanes DPP wave shifts, at half-wave edges the x-halo
// values. Pair accesses are single 8-/16-byte loads when nx is even (aligned)
// and two scalar accesses otherwise. The arithmetic per point is that of the
// scalar kernel.
// ------------------------------------------------------------------------
template <typename T> struct Pair { T a, b; };
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Pair loads are branch-free: a lane that must not read uses the vector's
// first element (always valid) and discards the value. VEC (nx even, so every
// pair is 8-/16-byte aligned) is a compile-time choice: a run-time test here
// would put every load in its own basic block, each closed by a full wait, and
// serialise a plane's loads.
template <bool VEC, typename TU>
__device__ __forceinline__ Pair<float> load_pair(const TU *p, const TU *base, bool ok0, bool ok1)
{
    Pair<float> r;
    if constexpr (VEC) {
        const TU *q = ok0 ? p : base;
        if constexpr (sizeof(TU) == 8) {
            typedef double d2 __attribute__((ext_vector_type(2)));
            const d2 v = ld_g((const d2 *)q);
            r.a = ok0 ? (float)v.x : 0.0f;
            r.b = ok0 ? (float)v.y : 0.0f;
        } else {
            const f32x2 v = ld_g((const f32x2 *)q);
            r.a = ok0 ? v.x : 0.0f;
            r.b = ok0 ? v.y : 0.0f;
        }
    } else {
        const TU a = ld_g(ok0 ? p : base), b = ld_g(ok1 ? p + 1 : base);
        r.a = ok0 ? (float)a : 0.0f;
        r.b = ok1 ? (float)b : 0.0f;
    }
    return r;
}

template <bool VEC>
__device__ __forceinline__ Pair<float> load_pair_nt(const float *p, const float *base, bool ok0,
                                                    bool ok1)
{
    Pair<float> r;
    if constexpr (VEC) {
        const f32x2 v = ld_nt((const f32x2 *)(ok0 ? p : base));
        r.a = ok0 ? v.x : 0.0f;
        r.b = ok0 ? v.y : 0.0f;
    } else {
        const float a = ld_nt(ok0 ? p : base), b = ld_nt(ok1 ? p + 1 : base);
        r.a = ok0 ? a : 0.0f;
        r.b = ok1 ? b : 0.0f;
    }
    return r;
}

template <bool VEC>
__device__ __forceinline__ void store_pair_nt(float *p, float a, float b, bool ok0, bool ok1)
{
    if constexpr (VEC) {
        if (ok0) {
            const f32x2 v = {a, b};
            st_nt((f32x2 *)p, v);
        }
    } else {
        if (ok0) st_nt(p, a);
        if (ok1) st_nt(p + 1, b);
    }
}

// One tile of an FP32 Chebyshev step. VEC: nx even. FULL: the wave's RY rows
// and the tile's 64 columns are all inside the grid, so no access needs a
// guard (guarded stores let the compiler sink loads into their branches).
template <int OP, typename TU, bool MASK, bool VEC, bool FULL, bool SIMPLE>
__device__ __forceinline__ void cheb_f32x2_tile(const Prob &P, const KArgs &A, int local, int lane,
                                                int wv)
{
    constexpr int RH = RY / 2;
    const int half = lane >> 5, hl = lane & 31;
    const int nx = P.nx, ny = P.ny, nz = P.nz, tx = P.tx, ty = P.ty;
    const int tix = local % tx, tiy = (local / tx) % ty, tiz = local / (tx * ty);
    const int i0 = tix * TX;
    const int x0 = i0 + 2 * hl;
    const int jw = tiy * (TY * RY) + wv * RY; // the wave's first row
    const int jh = jw + half * RH;            // this half-wave's first row
    const int k0 = tiz * P.kz, k1 = min(k0 + P.kz, nz);
    if (jw >= ny) return; // uniform within the wave (no barriers below)

    const size_t S = (size_t)nx * (size_t)ny, NXs = (size_t)nx;
    const bool in0 = FULL || x0 < nx, in1 = FULL || x0 + 1 < nx;
    const int B = MASK ? P.block : 1;
    const unsigned bc = P.bc;
    const bool nxl = bc & 1u, nxh = bc & 2u, nyl = bc & 4u, nyh = bc & 8u;
    const bool nzl = bc & 16u, nzh = bc & 32u;
    // x selections of the two points
    const Sel sxm0 = to_sel(in0 ? sel_lo(x0, nx, MASK, B, nxl) : 0);
    const Sel sxp0 = to_sel(in0 ? sel_hi(x0, nx, MASK, B, nxh) : 0);
    const Sel sxm1 = to_sel(in1 ? sel_lo(x0 + 1, nx, MASK, B, nxl) : 0);
    const Sel sxp1 = to_sel(in1 ? sel_hi(x0 + 1, nx, MASK, B, nxh) : 0);
    bool rin[RH];
    Sel sym[RH], syp[RH];
#pragma unroll
    for (int r = 0; r < RH; ++r) {
        const int j = jh + r;
        rin[r] = FULL || j < ny;
        sym[r] = to_sel(rin[r] ? sel_lo(j, ny, MASK, B, nyl) : 0);
        syp[r] = to_sel(rin[r] ? sel_hi(j, ny, MASK, B, nyh) : 0);
    }
    const bool ymh = in0 && jh > 0 && jh - 1 < ny;
    const bool yph = in0 && jh + RH < ny;
    // x halo: lane q < RY holds the left neighbour of wave row q, lane 32+q the right one
    const int hrow = lane & 31;
    const bool hload = hrow < RY && jw + hrow < ny && (lane < 32 ? i0 > 0 : i0 + TX < nx);
    size_t hidx = (size_t)(lane < 32 ? i0 - 1 : i0 + TX) +
                  NXs * ((size_t)(jw + hrow) + (size_t)ny * (size_t)k0);
    size_t base = (size_t)x0 + NXs * ((size_t)jh + (size_t)ny * (size_t)k0);

    const TU *__restrict__ u = (const TU *)P.vec[A.in];
    float *out = (float *)P.vec[A.out];
    const float *vv = (const float *)vec_at(P, A.v);
    const float *zz = (const float *)P.vec[A.z];
    float *v32 = (float *)P.vec[V_V32];
    const float ih2 = P.ih2f;
    float cA = 0, cB = 0, cC = 0, cD = 0, cE = 0;
    if constexpr (OP == S_CHEB1) {
        cA = P.c1f;
        cB = P.thetaf;
    } else {
        cA = P.rcf[A.step];
        cB = P.rof[A.step];
        cC = P.two_sigmaf;
        cD = P.two_over_deltaf;
        cE = P.thetaf;
    }
    Pair<float> c[RH], zm[RH];
#pragma unroll
    for (int r = 0; r < RH; ++r) {
        const size_t idx = base + r * NXs;
        c[r] = load_pair<VEC>(u + idx, u, in0 && rin[r], in1 && rin[r]);
        zm[r] = load_pair<VEC>(u + idx - (k0 > 0 ? S : 0), u, k0 > 0 && in0 && rin[r],
                               k0 > 0 && in1 && rin[r]);
    }
    for (int k = k0; k < k1; ++k, base += S, hidx += S) {
        const Sel szm = to_sel(sel_lo(k, nz, MASK, B, nzl));
        const Sel szp = to_sel(sel_hi(k, nz, MASK, B, nzh));
        Pair<float> zr[RH], o0[RH], o1[RH];
        const bool zn = k + 1 < nz;
#pragma unroll
        for (int r = 0; r < RH; ++r) {
            const size_t idx = base + r * NXs;
            const bool a0 = in0 && rin[r], a1 = in1 && rin[r];
            zr[r] = load_pair<VEC>(u + idx + (zn ? S : 0), u, zn && a0, zn && a1);
            if constexpr (OP == S_CHEB2) o0[r] = load_pair_nt<VEC>(vv + idx, vv, a0, a1);
            if constexpr (OP == S_CHEBK) {
                o0[r] = load_pair_nt<VEC>(vv + idx, vv, a0, a1);
                o1[r] = load_pair_nt<VEC>(zz + idx, zz, a0, a1);
            }
        }
        const Pair<float> ymv = load_pair<VEC>(u + base - (ymh ? NXs : 0), u, ymh, ymh && in1);
        const Pair<float> ypv = load_pair<VEC>(u + base + (yph ? RH * NXs : 0), u, yph, yph && in1);
        const float hv = (float)ld_g(u + (hload ? hidx : 0));
        const float he = hload ? hv : 0.0f;
#pragma unroll
        for (int r = 0; r < RH; ++r) {
            // neighbours across lanes, fixed up with the halo at half-wave edges
            const float elA = read_lane(he, r), elB = read_lane(he, RH + r);
            const float erA = read_lane(he, 32 + r), erB = read_lane(he, 32 + RH + r);
            const float el = half ? elB : elA, er = half ? erB : erA;
            // the DPP shifts run in every lane (a shift reads its source lane)
            const float pv = lane_prev(c[r].b), nv = lane_next(c[r].a);
            const float xl = hl == 0 ? el : pv;  // x0 - 1
            const float xr = hl == 31 ? er : nv; // x0 + 2
            const Pair<float> yl = r == 0 ? ymv : c[r > 0 ? r - 1 : 0];
            const Pair<float> yr = r == RH - 1 ? ypv : c[r < RH - 1 ? r + 1 : 0];
            // point 0 at x0: left xl, right c.b; point 1 at x0+1: left c.a, right xr
            float xm0, xp0, xm1, xp1, ym0, ym1, yp0, yp1, zm0, zm1, zp0, zp1;
            if constexpr (SIMPLE) {
                xm0 = xl, xp0 = c[r].b, xm1 = c[r].a, xp1 = xr;
                ym0 = yl.a, ym1 = yl.b, yp0 = yr.a, yp1 = yr.b;
                zm0 = zm[r].a, zm1 = zm[r].b, zp0 = zr[r].a, zp1 = zr[r].b;
            } else {
                xm0 = pick(sxm0, xl, c[r].b), xp0 = pick(sxp0, c[r].b, xl);
                xm1 = pick(sxm1, c[r].a, xr), xp1 = pick(sxp1, xr, c[r].a);
                ym0 = pick(sym[r], yl.a, yr.a), ym1 = pick(sym[r], yl.b, yr.b);
                yp0 = pick(syp[r], yr.a, yl.a), yp1 = pick(syp[r], yr.b, yl.b);
                zm0 = pick(szm, zm[r].a, zr[r].a), zm1 = pick(szm, zm[r].b, zr[r].b);
                zp0 = pick(szp, zr[r].a, zm[r].a), zp1 = pick(szp, zr[r].b, zm[r].b);
            }
            const float a0 = lap7<float>(c[r].a, xm0, xp0, ym0, yp0, zm0, zp0, ih2);
            const float a1 = lap7<float>(c[r].b, xm1, xp1, ym1, yp1, zm1, zp1, ih2);
            const size_t idx = base + r * NXs;
            const bool ok0 = in0 && rin[r], ok1 = in1 && rin[r];
            float w0, w1;
            if constexpr (OP == S_CHEB1) {
                w0 = cA * (2.0f * c[r].a - a0 / cB);
                w1 = cA * (2.0f * c[r].b - a1 / cB);
                store_pair_nt<VEC>(v32 + idx, c[r].a, c[r].b, ok0, ok1);
            } else if constexpr (OP == S_CHEB2) {
                const float z0 = o0[r].a / cE, z1 = o0[r].b / cE;
                w0 = cA * ((cC * c[r].a + cD * (o0[r].a - a0)) - cB * z0);
                w1 = cA * ((cC * c[r].b + cD * (o0[r].b - a1)) - cB * z1);
            } else {
                w0 = cA * ((cC * c[r].a + cD * (o0[r].a - a0)) - cB * o1[r].a);
                w1 = cA * ((cC * c[r].b + cD * (o0[r].b - a1)) - cB * o1[r].b);
            }
            store_pair_nt<VEC>(out + idx, w0, w1, ok0, ok1);
        }
#pragma unroll
        for (int r = 0; r < RH; ++r) {
            zm[r] = c[r];
            c[r] = zr[r];
        }
    }
}

template <int OP, typename TU, bool MASK>
__global__ void __launch_bounds__(NTHREADS) k_cheb_f32x2(Work W, KArgs A)
{
    static_assert(OP == S_CHEB1 || OP == S_CHEB2 || OP == S_CHEBK, "Chebyshev steps only");
    const int total = W.count_dev ? *W.count_dev : W.count;
    const int lane = threadIdx.x & (TX - 1), wv = threadIdx.x / TX;
    for (int g = blockIdx.x; g < total; g += gridDim.x) {
        const int pid = W.tile_prob ? W.tile_prob[g] : 0;
        const Prob &P = W.probs[pid];
        const int local = W.tile_prob ? W.tile_local[g] : tile_order(W.order, W, P, g, total);
        {
            const Scalars *sc = P.sc;
            if (sc->done || (A.second && sc->half_pending)) continue;
        }
        // one wave-uniform branch per tile; each body is straight-line in its plane loop
        const int tix = local % P.tx, tiy = (local / P.tx) % P.ty;
        const bool full = tix * TX + TX <= P.nx && tiy * (TY * RY) + wv * RY + RY <= P.ny;
        const bool simple = !MASK && P.bc == 0;
        if (P.nx & 1) cheb_f32x2_tile<OP, TU, MASK, false, false, false>(P, A, local, lane, wv);
        else if (!full) cheb_f32x2_tile<OP, TU, MASK, true, false, false>(P, A, local, lane, wv);
        else if (simple) cheb_f32x2_tile<OP, TU, MASK, true, true, !MASK>(P, A, local, lane, wv);
        else cheb_f32x2_tile<OP, TU, MASK, true, true, false>(P, A, local, lane, wv);
    }
}

// ------------------------------------------------------------------------
// Two consecutive Chebyshev steps in one pass (temporal blocking; FP64, or
// FP32 in the mixed mode), for i >= 3:
//   w_i     = rc_i     ((2 sigma y + (2/delta)(v - A y))   - ro_i     z)
//   w_{i+1} = rc_{i+1} ((2 sigma w_i + (2/delta)(v - A w_i)) - ro_{i+1} y)
// with y = y_{i-1} read with the stencil, z = z_{i-2} and v read pointwise. w_i is computed on the wave's rows plus one halo row
// on each side and one plane ahead of w_{i+1}; at its two halo columns it is
// computed by the halo lanes from the halo values they load anyway plus y one
// column further out, v and z. Reads y, z, v once and writes w_i and w_{i+1}:
// 40 bytes per point instead of 64 for the two separate steps. The arithmetic
// per point is exactly that of two k_stencil steps.
// ------------------------------------------------------------------------
// One tile of the fused pair. FULL: the tile's 64 columns and the wave's rows
// j0-2 .. j0+RY+1 are inside the grid, so the row and column guards are
// compile-time true; plane validity is wave-uniform and every load reads a
// clamped (valid) address whose value a select then keeps or zeroes, so no
// load sits in a branch of its own.
// FIRST: steps 1 and 2 (the first step's own formula, y_0 := v, z = v/theta at
// step 2). The stencil input is then v itself, read as TU (FP64 also when the
// arithmetic is FP32: it is rounded once on load, and the FP32 copy of v that
// the later steps read is written out).
template <typename T, typename TU, bool MASK, bool FULL, bool SIMPLE, bool FIRST>
__device__ __forceinline__ void cheb_pair_tile(const Prob &P, const KArgs &A, int local, int lane,
                                               int wv)
{
    constexpr int RYY = RY + 4; // y rows j0-2 .. j0+RY+1
    constexpr int RW = RY + 2;  // w_i rows j0-1 .. j0+RY
    const int nx = P.nx, ny = P.ny, nz = P.nz, tx = P.tx, ty = P.ty;
    const int tix = local % tx, tiy = (local / tx) % ty, tiz = local / (tx * ty);
    const int i0 = tix * TX, i = i0 + lane;
    const int j0 = tiy * (TY * RY) + wv * RY;
    const int k0 = tiz * P.kz, k1 = min(k0 + P.kz, nz);
    if (j0 >= ny) return; // uniform within the wave; no barriers below

    // Addresses: a wave-uniform plane base plus a per-lane 32-bit byte offset
    // inside the plane (the host uses this kernel only for planes below 2 GiB).
    const size_t PB = (size_t)nx * (size_t)ny * sizeof(T);
    const size_t PBY = (size_t)nx * (size_t)ny * sizeof(TU); // the stencil input's planes
    const int B = MASK ? P.block : 1;
    const unsigned bc = P.bc;
    const bool nxl = bc & 1u, nxh = bc & 2u, nyl = bc & 4u, nyh = bc & 8u;
    const bool nzl = bc & 16u, nzh = bc & 32u;
    const bool xin = FULL || i < nx;
    const int ic = xin ? i : nx - 1; // clamped column
    const Sel sxm = to_sel(xin ? sel_lo(i, nx, MASK, B, nxl) : 0);
    const Sel sxp = to_sel(xin ? sel_hi(i, nx, MASK, B, nxh) : 0);
    const char *Yb = (const char *)P.vec[A.in];
    const char *Vb = (const char *)vec_at(P, A.v);
    const char *Zb = (const char *)P.vec[A.z];
    char *W1b = (char *)P.vec[A.out];
    char *W2b = (char *)P.vec[A.x2];
    char *V32b = (char *)P.vec[V_V32];
    const T ih2 = Coef<T>::ih2(P), theta = Coef<T>::theta(P);
    const T ts = Coef<T>::two_sigma(P), tod = Coef<T>::two_over_delta(P);
    const T rc1 = Coef<T>::rc(P, A.step), ro1 = Coef<T>::ro(P, A.step);
    const T rc2 = Coef<T>::rc(P, A.step + 1), ro2 = Coef<T>::ro(P, A.step + 1);
    const T c1 = Coef<T>::c1(P);
    auto clampi = [](int a, int n) { return a < 0 ? 0 : (a >= n ? n - 1 : a); };
    auto off = [&](int x, int j) { return (unsigned)(x + nx * j) * (unsigned)sizeof(T); };
    auto offy = [&](int x, int j) { return (unsigned)(x + nx * j) * (unsigned)sizeof(TU); };
    auto ld = [](const char *plane, unsigned o) { return ld_g((const T *)(plane + o)); };
    auto ldy = [](const char *plane, unsigned o) { return ld_g((const TU *)(plane + o)); };

    // rows: Y row q is j0-2+q, w row q is j0-1+q
    bool yok[RYY], wok[RW];
    unsigned yoff[RYY], woff[RW];
    Sel wsym[RW], wsyp[RW];
#pragma unroll
    for (int q = 0; q < RYY; ++q) {
        const int j = j0 - 2 + q;
        yok[q] = FULL || (xin && j >= 0 && j < ny);
        yoff[q] = offy(ic, FULL ? j : clampi(j, ny));
    }
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        const int j = j0 - 1 + q;
        wok[q] = FULL || (xin && j >= 0 && j < ny);
        woff[q] = off(ic, FULL ? j : clampi(j, ny));
        wsym[q] = to_sel(wok[q] ? sel_lo(j, ny, MASK, B, nyl) : 0);
        wsyp[q] = to_sel(wok[q] ? sel_hi(j, ny, MASK, B, nyh) : 0);
    }
    // x halo of y for the w_i rows: lane q < RW the left, lane 32+q the right
    const int hq = lane & 31;
    const int hj = j0 - 1 + hq;
    const bool hload = hq < RW && hj >= 0 && hj < ny && (lane < 32 ? i0 > 0 : i0 + TX < nx);
    const unsigned hoff = hload ? offy(lane < 32 ? i0 - 1 : i0 + TX, hj) : 0u;
    // The halo lanes also evaluate w_i at the two halo columns i0-1 and i0+TX:
    // lane q (1..RY) the left point of row j0+q-1, lane 32+q the right one. For
    // that the x-halo load above is joined by three more per plane: y one
    // column further out, v and z, all at the halo column of the lane's row.
    const bool hside = lane >= 32;
    const int hcx = hside ? i0 + TX : i0 - 1;       // halo column
    const int hfx = hside ? i0 + TX + 1 : i0 - 2;   // one further out
    const bool hrow_ok = hq < RW && hj >= 0 && hj < ny;
    const bool fload = hrow_ok && hfx >= 0 && hfx < nx;
    const unsigned foff = fload ? offy(hfx, hj) : 0u;
    const bool cact = hq >= 1 && hq <= RY && hrow_ok && hcx >= 0 && hcx < nx;
    const unsigned coff = cact ? off(hcx, hj) : 0u;
    const Sel csxl = to_sel(cact ? sel_lo(hcx, nx, MASK, B, nxl) : 0);
    const Sel csxh = to_sel(cact ? sel_hi(hcx, nx, MASK, B, nxh) : 0);
    const Sel csyl = to_sel(cact ? sel_lo(hj, ny, MASK, B, nyl) : 0);
    const Sel csyh = to_sel(cact ? sel_hi(hj, ny, MASK, B, nyh) : 0);

    // w_i at one point from its 7 y values, v and z (the k_stencil step)
    auto step1 = [&](T yc, T xm, T xp, T ym, T yp, T zm,
                     T zp, T v, T z) {
        const T a = lap7<T>(yc, xm, xp, ym, yp, zm, zp, ih2);
        if constexpr (FIRST) return c1 * ((T)2 * yc - a / theta);
        else return rc1 * ((ts * yc + tod * (v - a)) - ro1 * z);
    };
    // The plane loop is software-pipelined: iteration k issues the loads of y
    // at plane k+3 and of v, z and the halo values at plane k+2, and consumes
    // what iteration k-1 issued. Raw loaded values are kept until their use;
    // only there are they zeroed outside the grid, so no wait sits between a
    // load and the next iteration.
    struct Raw {
        TU y[RYY], he, hf;
        T v[RW], z[RW], hv, hz;
    };
    auto issueY = [&](int p, TU (&dst)[RYY]) {
        const char *Yp = Yb + (size_t)clampi(p, nz) * PBY;
#pragma unroll
        for (int q = 0; q < RYY; ++q) dst[q] = ldy(Yp, yoff[q]);
    };
    auto issueP = [&](int p, Raw &R) {
        const size_t po = (size_t)clampi(p, nz) * PB;
        // v and z rows are read by three waves (as own and as halo rows), so
        // they are loaded through the caches, not as a read-once stream
        const size_t pyo = (size_t)clampi(p, nz) * PBY;
        if constexpr (!FIRST) {
#pragma unroll
            for (int q = 0; q < RW; ++q) {
                R.v[q] = ld(Vb + po, woff[q]);
                if constexpr (!FIRST) R.z[q] = ld(Zb + po, woff[q]);
            }
            R.hv = ld(Vb + po, coff);
            if constexpr (!FIRST) R.hz = ld(Zb + po, coff);
        }
        R.he = ldy(Yb + pyo, hoff);
        R.hf = ldy(Yb + pyo, foff);
    };
    auto takeY = [&](int p, const TU (&raw)[RYY], T (&dst)[RYY]) {
        const bool pin = p >= 0 && p < nz;
#pragma unroll
        for (int q = 0; q < RYY; ++q) dst[q] = (pin && yok[q]) ? (T)raw[q] : (T)0;
    };

    T ya[RYY], yb[RYY], yc[RYY];
    T wa[RW], wb[RW], wc[RW], vb[RY], vc[RY];
    // halo values: y at the halo column on planes k-1, k, k+1 (ha, hb, hc), and
    // at plane k the further column, v and z (hfb, hvb, hzb)
    T ha = (T)0, hb = (T)0, hc = (T)0, hfb = (T)0, hvb = (T)0, hzb = (T)0;
    // D planes of loads in flight: the first pair issues only y and its halo
    // values, so in FP64 it keeps two planes in flight (measured 769 -> 732 us
    // at 512^3); in FP32 the extra registers would cost a wave per SIMD
    constexpr int D = (FIRST && sizeof(T) == 8) ? 2 : 1;
    Raw R0, R1;
#pragma unroll
    for (int q = 0; q < RW; ++q) R0.v[q] = R0.z[q] = R1.v[q] = R1.z[q] = (T)0;
    R0.hv = R0.hz = R1.hv = R1.hz = (T)0;
    {
        TU t[RYY];
        issueY(k0 - 2, t);
        takeY(k0 - 2, t, ya);
        issueY(k0 - 1, t);
        takeY(k0 - 1, t, yb);
    }
    issueY(k0, R0.y);
    issueP(k0 - 1, R0);
    if constexpr (D == 2) {
        issueY(k0 + 1, R1.y);
        issueP(k0, R1);
    }
#pragma unroll
    for (int q = 0; q < RW; ++q) wa[q] = wb[q] = (T)0;
#pragma unroll
    for (int r = 0; r < RY; ++r) vb[r] = (T)0;
    // iteration k consumes the loads of plane k+2 (y) and k+1 (v, z, halo)
    // held in R and refills R with those of planes k+2+D and k+1+D
    auto iter = [&](int k, Raw &R) {
        const int p = k + 1;
        const bool pin = p >= 0 && p < nz;
        takeY(k + 2, R.y, yc);
        T vv[RW], zz[RW];
#pragma unroll
        for (int q = 0; q < RW; ++q) {
            const bool ok = pin && wok[q];
            vv[q] = FIRST ? yb[q + 1] : (ok ? R.v[q] : (T)0);
            zz[q] = (!FIRST && ok) ? R.z[q] : (T)0;
        }
        const T he = (hload && pin) ? (T)R.he : (T)0;
        const T hfc = (fload && pin) ? (T)R.hf : (T)0;
        const T hvc = (cact && pin) ? R.hv : (T)0;
        const T hzc = (!FIRST && cact && pin) ? R.hz : (T)0;
        hc = he;
        // issue the next plane's loads before computing this one
        issueY(k + 2 + D, R.y);
        issueP(k + 1 + D, R);

        // w_i at plane p = k+1 on the RW rows, from y planes k (ya), k+1 (yb), k+2 (yc)
        {
            const Sel szm = to_sel(pin ? sel_lo(p, nz, MASK, B, nzl) : 0);
            const Sel szp = to_sel(pin ? sel_hi(p, nz, MASK, B, nzh) : 0);
#pragma unroll
            for (int q = 0; q < RW; ++q) {
                // the DPP shifts run in every lane (a shift reads its source lane)
                const T pv = lane_prev(yb[q + 1]), nv = lane_next(yb[q + 1]);
                const T el = read_lane(he, q), er = read_lane(he, 32 + q);
                const T xl = lane == 0 ? el : pv, xr = lane == TX - 1 ? er : nv;
                const T c = yb[q + 1];
                T xm, xp, ym, yp, zm, zp;
                if constexpr (SIMPLE) {
                    xm = xl, xp = xr, ym = yb[q], yp = yb[q + 2], zm = ya[q + 1], zp = yc[q + 1];
                } else {
                    xm = pick(sxm, xl, xr), xp = pick(sxp, xr, xl);
                    ym = pick(wsym[q], yb[q], yb[q + 2]), yp = pick(wsyp[q], yb[q + 2], yb[q]);
                    zm = pick(szm, ya[q + 1], yc[q + 1]), zp = pick(szp, yc[q + 1], ya[q + 1]);
                }
                const T z = zz[q]; // not read by the first pair's step 1
                const T w = step1(c, xm, xp, ym, yp, zm, zp, vv[q], z);
                wc[q] = (pin && wok[q]) ? w : (T)0;
            }
#pragma unroll
            for (int r = 0; r < RY; ++r) vc[r] = vv[r + 1];
        }
        if (k >= k0) {
            // w_i at the halo lanes' points (hcx, hj, k): row neighbours from the
            // adjacent halo lanes, the tile-edge neighbour from lane 0 or TX-1
            T edge = (T)0;
#pragma unroll
            for (int q = 1; q <= RY; ++q) {
                const T eL = read_lane(ya[q + 1], 0), eR = read_lane(ya[q + 1], TX - 1);
                const T e = hside ? eR : eL;
                edge = hq == q ? e : edge;
            }
            T hw;
            {
                const T d = lane_prev(hb), u = lane_next(hb);
                const T l = hside ? edge : hfb, r = hside ? hfb : edge;
                T xm, xp, ym, yp, zm, zp;
                if constexpr (SIMPLE) {
                    xm = l, xp = r, ym = d, yp = u, zm = ha, zp = hc;
                } else {
                    const Sel szl = to_sel(sel_lo(k, nz, MASK, B, nzl));
                    const Sel szh = to_sel(sel_hi(k, nz, MASK, B, nzh));
                    xm = pick(csxl, l, r), xp = pick(csxh, r, l);
                    ym = pick(csyl, d, u), yp = pick(csyh, u, d);
                    zm = pick(szl, ha, hc), zp = pick(szh, hc, ha);
                }
                const T z = hzb;
                const T w = step1(hb, xm, xp, ym, yp, zm, zp, hvb, z);
                hw = cact ? w : (T)0;
            }
            // w_{i+1} at plane k from w_i at planes k-1 (wa), k (wb), k+1 (wc)
            const Sel szm = to_sel(sel_lo(k, nz, MASK, B, nzl));
            const Sel szp = to_sel(sel_hi(k, nz, MASK, B, nzh));
            const size_t po = (size_t)k * PB;
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                const int q = r + 1; // w row of output row j0 + r
                const T pv = lane_prev(wb[q]), nv = lane_next(wb[q]);
                const T el = read_lane(hw, 1 + r), er = read_lane(hw, 33 + r);
                const T xl = lane == 0 ? el : pv, xr = lane == TX - 1 ? er : nv;
                const T c = wb[q];
                T xm, xp, ym, yp, zm, zp;
                if constexpr (SIMPLE) {
                    xm = xl, xp = xr, ym = wb[q - 1], yp = wb[q + 1], zm = wa[q], zp = wc[q];
                } else {
                    xm = pick(sxm, xl, xr), xp = pick(sxp, xr, xl);
                    ym = pick(wsym[q], wb[q - 1], wb[q + 1]), yp = pick(wsyp[q], wb[q + 1], wb[q - 1]);
                    zm = pick(szm, wa[q], wc[q]), zp = pick(szp, wc[q], wa[q]);
                }
                const T a = lap7<T>(c, xm, xp, ym, yp, zm, zp, ih2);
                // step i+1 reads z = y_{i-1}, the pair's stencil input at plane k
                // (for the first pair, z = v/theta with v = that input)
                const T v = FIRST ? ya[q + 1] : vb[r];
                const T z = FIRST ? v / theta : ya[q + 1];
                const T w2 = rc2 * ((ts * c + tod * (v - a)) - ro2 * z);
                if (wok[q]) {
                    if (!A.drop1) st_nt((T *)(W1b + po + woff[q]), c);
                    st_nt((T *)(W2b + po + woff[q]), w2);
                    if constexpr (FIRST && sizeof(T) == 4) st_nt((T *)(V32b + po + woff[q]), v);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < RYY; ++q) {
            ya[q] = yb[q];
            yb[q] = yc[q];
        }
#pragma unroll
        for (int q = 0; q < RW; ++q) {
            wa[q] = wb[q];
            wb[q] = wc[q];
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) vb[r] = vc[r];
        ha = hb, hb = hc, hfb = hfc, hvb = hvc, hzb = hzc;
    };
    if constexpr (D == 1) {
        for (int k = k0 - 2; k < k1; ++k) iter(k, R0);
    } else {
        // two iterations per trip, so each raw buffer stays in registers
        for (int k = k0 - 2; k < k1; k += 2) {
            iter(k, R0);
            if (k + 1 < k1) iter(k + 1, R1);
        }
    }
}

template <typename T, typename TU, bool MASK, bool FIRST>
__global__ void __launch_bounds__(NTHREADS) k_cheb_pair(Work W, KArgs A)
{
    const int total = W.count_dev ? *W.count_dev : W.count;
    const int lane = threadIdx.x & (TX - 1), wv = threadIdx.x / TX;
    for (int g = blockIdx.x; g < total; g += gridDim.x) {
        const int pid = W.tile_prob ? W.tile_prob[g] : 0;
        const Prob &P = W.probs[pid];
        // the default order for this kernel is x-grouped: its x-halo columns (y, v
        // and z) then come from the same L2 as the neighbouring tile's data
        const int local =
            W.tile_prob ? W.tile_local[g] : tile_order(W.order ? W.order : 1, W, P, g, total);
        {
            const Scalars *sc = P.sc;
            if (sc->done || (A.second && sc->half_pending)) continue;
        }
        // one wave-uniform branch per tile
        const int tix = local % P.tx, tiy = (local / P.tx) % P.ty;
        const int j0 = tiy * (TY * RY) + wv * RY;
        const bool full = tix * TX + TX <= P.nx && j0 - 2 >= 0 && j0 + RY + 1 < P.ny;
        if constexpr (MASK) {
            if (full) cheb_pair_tile<T, TU, true, true, false, FIRST>(P, A, local, lane, wv);
            else cheb_pair_tile<T, TU, true, false, false, FIRST>(P, A, local, lane, wv);
        } else if (P.bc == 0) {
            if (full) cheb_pair_tile<T, TU, false, true, true, FIRST>(P, A, local, lane, wv);
            else cheb_pair_tile<T, TU, false, false, true, FIRST>(P, A, local, lane, wv);
        } else {
            if (full) cheb_pair_tile<T, TU, false, true, false, FIRST>(P, A, local, lane, wv);
            else cheb_pair_tile<T, TU, false, false, false, FIRST>(P, A, local, lane, wv);
        }
    }
}

// ------------------------------------------------------------------------
// The fused pair over wide tiles staged in LDS, for grids whose faces are all
// Dirichlet and without a block mask. A workgroup of 2*NXW waves covers
// 64*NXW columns x 2*PR rows x kz planes. Wave (xw, yw) owns 64 columns x PR
// rows; a top wave (yw = 0) also holds the tile's halo row above, a bottom
// wave the halo row below, so w_i is computed on the tile plus its halo ring.
// Per plane every wave writes its rows of y and of w_i to LDS, and the lanes
// at the two halo columns write theirs. A wave then takes the values other
// waves own (the row across the wave boundary, the column beyond its first
// and last lane) from LDS instead of loading them again, and the tile's halo
// lines are fetched once for a perimeter of a 64*NXW x 2*PR tile. Two LDS
// buffers per field, alternating by plane, take one barrier per plane. The
// plane loop is pipelined as in cheb_pair_tile, and the arithmetic per point
// is exactly that of two k_stencil steps.
// ------------------------------------------------------------------------
// the rows a wave of an LDS-staged pair or triple holds: the top and bottom wave
// of a column of waves add the tile's halo rows, the waves between them do not
enum { R_TOP = 0, R_MID = 1, R_BOT = 2 };

template <int NXW, int PR, int NYW> struct LPair {
    static constexpr int X = 64 * NXW, Y = NYW * PR;
    static constexpr int PW = X + 2, PH = Y + 2; // LDS plane: rows -1..Y, columns -1..X
    static constexpr int PLANE = PW * PH;
    static constexpr int NT = 64 * NXW * NYW;
};

// MASK: Block-Jacobi block faces; SIMPLE: no mask and no Neumann face, so every
// neighbour outside the grid is the +0.0 that the zeroed loads already hold and
// no neighbour select is needed. Otherwise each neighbour goes through the same
// selection (neighbour, zero or mirror) as in k_stencil.
// UPD (first pass only): 0 reads v = in; U_S forms v = s = r - alpha w at every
// point it reads, stores s at the tile's points and adds their s.s to (ssh,
// ssl); U_P forms v = p = r + beta (p_prev - omega w) and stores it as this
// iteration's p (in the first iteration v is p itself).
template <typename T, typename TU, bool FIRST, bool DROP, int NXW, int PR, int NYW, int ROLE,
          bool MASK, bool SIMPLE, int UPD>
__device__ __forceinline__ void cheb_pair_lds_tile(const Prob &P, const KArgs &A, int tile,
                                                   int lane, int xw, int yw, T *lds, double &ssh,
                                                   double &ssl)
{
    static_assert(UPD == 0 || FIRST, "a vector update folds only into a first pass");
    constexpr int NU = UPD == U_P ? 2 : (UPD == U_S ? 1 : 0);   // extra operands of v
    constexpr int NUA = NU > 0 ? NU : 1;
    using L = LPair<NXW, PR, NYW>;
    constexpr bool TOP = ROLE == R_TOP, BOT = ROLE == R_BOT, MID = ROLE == R_MID;
    // rows held: PR own rows, and for the top and bottom wave the halo row outside them
    constexpr int E = MID ? PR : PR + 1;
    constexpr int EOWN = TOP ? 1 : 0;   // first own row among the held rows
    constexpr int ERING = TOP ? 0 : (BOT ? PR : -1); // the halo row among them
    constexpr int TRO = TOP ? -2 : L::Y + 1; // tile row of the outer row (y only)
    const int r0 = TOP ? -1 : (BOT ? (NYW - 1) * PR : yw * PR); // tile row of held row 0
    auto trow = [r0](int e) { return r0 + e; };
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int ltx = (nx + L::X - 1) / L::X, lty = (ny + L::Y - 1) / L::Y;
    const int tix = tile % ltx, tiy = (tile / ltx) % lty, tiz = tile / (ltx * lty);
    const int x0 = tix * L::X, y0 = tiy * L::Y;
    const int pkz = P.pkz[sizeof(T) == 4];
    const int k0 = tiz * pkz, k1 = min(k0 + pkz, nz);
    const int cx = xw * 64 + lane; // tile column of the lane
    const int i = x0 + cx;
    const bool xin = i < nx;
    const int ic = xin ? i : nx - 1;
    const size_t PB = (size_t)nx * (size_t)ny * sizeof(T);
    const size_t PBY = (size_t)nx * (size_t)ny * sizeof(TU);
    const char *Yb = (const char *)P.vec[A.in];
    // the folded update's operands: Ub[0] = w, Ub[1] = the previous p
    const char *Ub[2] = {nullptr, nullptr};
    char *Ob = nullptr;
    double ua = 0.0, ub = 0.0, uo = 0.0;
    bool ufirst = false;
    if constexpr (UPD == U_S) {
        Yb = (const char *)P.vec[V_R];
        Ub[0] = (const char *)P.vec[V_W];
        Ob = (char *)P.vec[V_S];
        ua = P.sc->alpha;
    } else if constexpr (UPD == U_P) {
        const int it = P.sc->iter;
        ufirst = it == 0;
        const int pold = ((it - 1) & 1) ? V_P2 : V_P, pnew = (it & 1) ? V_P2 : V_P;
        Yb = (const char *)P.vec[ufirst ? V_P : V_R];
        Ub[0] = (const char *)P.vec[ufirst ? V_P : V_W];
        Ub[1] = (const char *)P.vec[ufirst ? V_P : pold];
        Ob = (char *)P.vec[pnew];
        ub = P.sc->beta;
        uo = P.sc->omega;
    }
    // v from its raw operands, in the rounding order of the standalone updates
    auto comb = [&](TU r, TU w, TU pp) -> TU {
        if constexpr (UPD == U_S) return r - (TU)ua * w;
        else if constexpr (UPD == U_P) return ufirst ? pp : r + (TU)ub * (pp - (TU)uo * w);
        else return r;
    };
    const char *Vb = (const char *)vec_at(P, A.v);
    const char *Zb = (const char *)P.vec[A.z];
    char *W1b = (char *)P.vec[A.out];
    char *W2b = (char *)P.vec[A.x2];
    char *V32b = (char *)P.vec[V_V32];
    const T ih2 = Coef<T>::ih2(P), theta = Coef<T>::theta(P);
    const T ts = Coef<T>::two_sigma(P), tod = Coef<T>::two_over_delta(P);
    const T rc1 = Coef<T>::rc(P, A.step), ro1 = Coef<T>::ro(P, A.step);
    const T rc2 = Coef<T>::rc(P, A.step + 1), ro2 = Coef<T>::ro(P, A.step + 1);
    const T c1 = Coef<T>::c1(P);
    auto clampi = [](int a, int n) { return a < 0 ? 0 : (a >= n ? n - 1 : a); };
    auto off = [&](int x, int j) { return (unsigned)(x + nx * j) * (unsigned)sizeof(T); };
    auto offy = [&](int x, int j) { return (unsigned)(x + nx * j) * (unsigned)sizeof(TU); };
    auto ld = [](const char *plane, unsigned o) { return ld_g((const T *)(plane + o)); };
    auto ldy = [](const char *plane, unsigned o) { return ld_g((const TU *)(plane + o)); };
    // LDS element of tile row r (-1..Y) and tile column c (-1..X)
    auto lidx = [](int r, int c) { return (r + 1) * L::PW + (c + 1); };

    // neighbour selection (used unless SIMPLE): per lane along x, per held row
    // along y, per plane along z
    const int B = MASK ? P.block : 1;
    const unsigned bc = P.bc;
    const bool nxl = bc & 1u, nxh = bc & 2u, nyl = bc & 4u, nyh = bc & 8u;
    const bool nzl = bc & 16u, nzh = bc & 32u;
    const Sel sxm = to_sel(xin ? sel_lo(i, nx, MASK, B, nxl) : 0);
    const Sel sxp = to_sel(xin ? sel_hi(i, nx, MASK, B, nxh) : 0);
    bool rok[E];
    unsigned roff[E], ryoff[E];
    Sel sym[E], syp[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = y0 + trow(e);
        const bool jin = j >= 0 && j < ny;
        rok[e] = xin && jin;
        roff[e] = off(ic, clampi(j, ny));
        ryoff[e] = offy(ic, clampi(j, ny));
        sym[e] = to_sel(jin ? sel_lo(j, ny, MASK, B, nyl) : 0);
        syp[e] = to_sel(jin ? sel_hi(j, ny, MASK, B, nyh) : 0);
    }
    const int jo = y0 + TRO;
    const bool ook = !MID && xin && jo >= 0 && jo < ny;
    const unsigned ooff = offy(ic, clampi(jo, ny));
    // own position in LDS (held row 0); row e adds e*PW
    const int lown = lidx(trow(0), cx);
    // the rows next to the held ones (held by the waves above and below)
    const int linU = lidx(r0 - 1, cx), linD = lidx(r0 + E, cx);

    // Halo lanes: lane e (< E) of the leftmost waves holds tile column -1 of
    // held row e, lane 32+e of the rightmost waves column X. Both write their y
    // value to LDS; on own rows they also compute w_i there, for which they
    // load y one column further out, v and z.
    const bool hside = lane >= 32;
    const int eh = min(lane & 31, E - 1);
    const bool hwave = hside ? xw == NXW - 1 : xw == 0;
    const bool hact = hwave && (lane & 31) < E;
    const int hcol = hside ? L::X : -1;
    const int hi = x0 + hcol, hfi = hside ? hi + 1 : hi - 1;
    const int hj = y0 + trow(eh);
    const bool hrow = hj >= 0 && hj < ny;
    const bool hload = hact && hrow && hi >= 0 && hi < nx;
    const bool hown = hact && eh != ERING;
    const bool cact = hown && hload;
    const bool fload = hown && hrow && hfi >= 0 && hfi < nx;
    const unsigned hoff = offy(clampi(hi, nx), clampi(hj, ny));
    const unsigned foff = offy(clampi(hfi, nx), clampi(hj, ny));
    const unsigned coff = off(clampi(hi, nx), clampi(hj, ny));
    const int lhself = lidx(trow(eh), hcol);
    const int lhin = lidx(trow(eh), hside ? L::X - 1 : 0);
    const int lhup = lidx(max(trow(eh) - 1, -1), hcol), lhdn = lidx(min(trow(eh) + 1, L::Y), hcol);
    const Sel csxl = to_sel(cact ? sel_lo(hi, nx, MASK, B, nxl) : 0);
    const Sel csxh = to_sel(cact ? sel_hi(hi, nx, MASK, B, nxh) : 0);
    const Sel csyl = to_sel(cact ? sel_lo(hj, ny, MASK, B, nyl) : 0);
    const Sel csyh = to_sel(cact ? sel_hi(hj, ny, MASK, B, nyh) : 0);

    auto step1 = [&](T yc, T xm, T xp, T ym, T yp, T zm, T zp, T v, T z) {
        const T a = lap7<T>(yc, xm, xp, ym, yp, zm, zp, ih2);
        if constexpr (FIRST) return c1 * ((T)2 * yc - a / theta);
        else return rc1 * ((ts * yc + tod * (v - a)) - ro1 * z);
    };
    // Loads in flight: y (held rows, outer row, halo column) one plane ahead,
    // issued as soon as the previous plane is taken; v, z (held rows and halo
    // column points) and y one column further out, issued after step i of
    // the plane before their own and consumed straight from these registers.
    struct RawY {
        TU y[E], yo, he;
        TU uy[NUA][E], uyo[NUA], uhe[NUA];
    };
    struct RawV {
        T v[E], z[E], hv, hz;
        TU hf, uhf[NUA];
    };
    // the folded update's extra operands of plane p; in the plane loop they are
    // issued after step i, so fewer loads are in flight across its arithmetic
    auto issueU = [&](int p, RawY &R) {
        const size_t pb = (size_t)clampi(p, nz) * PBY;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const char *Up = Ub[u] + pb;
#pragma unroll
            for (int e = 0; e < E; ++e) R.uy[u][e] = ldy(Up, ryoff[e]);
            if constexpr (!MID) R.uyo[u] = ldy(Up, ooff);
            else R.uyo[u] = (TU)0;
            R.uhe[u] = ldy(Up, hoff);
        }
    };
    auto issueY = [&](int p, RawY &R, bool extra) {
        const size_t pb = (size_t)clampi(p, nz) * PBY;
        const char *Yp = Yb + pb;
#pragma unroll
        for (int e = 0; e < E; ++e) R.y[e] = ldy(Yp, ryoff[e]);
        if constexpr (!MID) R.yo = ldy(Yp, ooff);
        else R.yo = (TU)0;
        R.he = ldy(Yp, hoff);
        if (extra) issueU(p, R);
    };
    // the input v at held row e, the outer row and the halo column
    auto gy = [&](const RawY &R, int e) {
        return comb(R.y[e], R.uy[0][e], R.uy[NUA - 1][e]);
    };
    auto gyo = [&](const RawY &R) { return comb(R.yo, R.uyo[0], R.uyo[NUA - 1]); };
    auto ghe = [&](const RawY &R) { return comb(R.he, R.uhe[0], R.uhe[NUA - 1]); };
    auto issueV = [&](int p, RawV &R) {
        const size_t po = (size_t)clampi(p, nz) * PB;
        if constexpr (!FIRST) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                R.v[e] = ld(Vb + po, roff[e]);
                R.z[e] = ld(Zb + po, roff[e]);
            }
            R.hv = ld(Vb + po, coff);
            R.hz = ld(Zb + po, coff);
        }
        R.hf = ldy(Yb + (size_t)clampi(p, nz) * PBY, foff);
#pragma unroll
        for (int u = 0; u < NU; ++u) R.uhf[u] = ldy(Ub[u] + (size_t)clampi(p, nz) * PBY, foff);
    };
    auto ghf = [&](const RawV &R) { return comb(R.hf, R.uhf[0], R.uhf[NUA - 1]); };
    auto bufy = [&](int k) { return lds + (k & 1) * L::PLANE; };
    auto bufw = [&](int k) { return lds + (2 + (k & 1)) * L::PLANE; };

    // registers across planes: y at plane k-1 (ya), w_i at plane k-2 (wa) and
    // v at plane k-1 (vb) on the held rows; y at plane k and w_i at plane k-1
    // are read back from LDS where they are needed
    T ya[E], wa[E], vb[E];
    T yob, ha;
    RawY RY;
    RawV RV;
#pragma unroll
    for (int e = 0; e < E; ++e) RV.v[e] = RV.z[e] = (T)0;
    RV.hv = RV.hz = (T)0;
    {
        // planes k0-2 and k0-1 of y; plane k0-1 into LDS
        RawY t;
        issueY(k0 - 2, t, true);
        {
            const bool pin = k0 - 2 >= 0;
#pragma unroll
            for (int e = 0; e < E; ++e) ya[e] = (pin && rok[e]) ? (T)gy(t, e) : (T)0;
            ha = (pin && hload) ? (T)ghe(t) : (T)0;
        }
        issueY(k0 - 1, t, true);
        {
            const bool pin = k0 - 1 >= 0;
            T *yd = bufy(k0 - 1);
#pragma unroll
            for (int e = 0; e < E; ++e) yd[lown + e * L::PW] = (pin && rok[e]) ? (T)gy(t, e) : (T)0;
            yob = (pin && ook) ? (T)gyo(t) : (T)0;
            if (hact) yd[lhself] = (pin && hload) ? (T)ghe(t) : (T)0;
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) wa[e] = vb[e] = (T)0;
    issueY(k0, RY, true);
    issueV(k0 - 1, RV);
    __syncthreads();

    for (int k = k0 - 1; k <= k1; ++k) {
        const bool pin1 = k + 1 >= 0 && k + 1 < nz, pin0 = k >= 0 && k < nz;
        // take y at plane k+1, publish it for the next plane, issue plane k+2
        T yc[E];
        TU vn[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            vn[e] = gy(RY, e);
            yc[e] = (pin1 && rok[e]) ? (T)vn[e] : (T)0;
        }
        const T yoc = (pin1 && ook) ? (T)gyo(RY) : (T)0;
        const T hc = (pin1 && hload) ? (T)ghe(RY) : (T)0;
        if constexpr (UPD != 0) {
            // the formed v at the tile's own points of plane k+1: stored, and s.s
            if (k + 1 >= k0 && k + 1 < k1 && !ufirst) {
                const size_t po = (size_t)(k + 1) * PBY;
#pragma unroll
                for (int e = EOWN; e < EOWN + PR; ++e)
                    if (rok[e]) {
                        st_nt((TU *)(Ob + po + ryoff[e]), vn[e]);
                        if constexpr (UPD == U_S) dd_acc(ssh, ssl, (double)vn[e], (double)vn[e]);
                    }
            }
        }
        {
            T *yd = bufy(k + 1);
#pragma unroll
            for (int e = 0; e < E; ++e) yd[lown + e * L::PW] = yc[e];
            if (hact) yd[lhself] = hc;
        }
        issueY(k + 2, RY, false);

        // w_i at plane k on the held rows, from y planes k-1 (ya), k (LDS), k+1 (yc)
        const T *ys = bufy(k);
        T wc[E], vc[E];
        const Sel sz1m = to_sel(pin0 ? sel_lo(k, nz, MASK, B, nzl) : 0);
        const Sel sz1p = to_sel(pin0 ? sel_hi(k, nz, MASK, B, nzh) : 0);
        {
            // the rows across the held rows' edges: the outer row (top, bottom
            // wave) or a row of the neighbouring wave from LDS
            T inU = (T)0, inD = (T)0;
            if constexpr (TOP) inU = yob; else inU = ys[linU];
            if constexpr (BOT) inD = yob; else inD = ys[linD];
            T cen[E];
#pragma unroll
            for (int e = 0; e < E; ++e) cen[e] = ys[lown + e * L::PW];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const T c = cen[e];
                // x neighbours from the LDS plane, which holds every column of the
                // tile and its halo (no lane shifts, no edge patches)
                const T xm = ys[lown - 1 + e * L::PW], xp = ys[lown + 1 + e * L::PW];
                const T ym = e == 0 ? inU : cen[e > 0 ? e - 1 : 0];
                const T yp = e == E - 1 ? inD : cen[e < E - 1 ? e + 1 : e];
                const bool ok = pin0 && rok[e];
                const T v = FIRST ? c : (ok ? RV.v[e] : (T)0);
                const T z = (!FIRST && ok) ? RV.z[e] : (T)0;
                vc[e] = v;
                T w;
                if constexpr (SIMPLE) {
                    w = step1(c, xm, xp, ym, yp, ya[e], yc[e], v, z);
                } else {
                    w = step1(c, pick(sxm, xm, xp), pick(sxp, xp, xm), pick(sym[e], ym, yp),
                              pick(syp[e], yp, ym), pick(sz1m, ya[e], yc[e]),
                              pick(sz1p, yc[e], ya[e]), v, z);
                }
                wc[e] = ok ? w : (T)0;
            }
        }
        // w_i at the halo-column points of the own rows
        T hb, hw;
        {
            hb = ys[lhself];
            const T xn = ys[lhin], d = ys[lhup], u = ys[lhdn];
            const T hf = (fload && pin0) ? (T)ghf(RV) : (T)0;
            const T hv = (!FIRST && cact && pin0) ? RV.hv : (T)0;
            const T hz = (!FIRST && cact && pin0) ? RV.hz : (T)0;
            const T l = hside ? xn : hf, r = hside ? hf : xn;
            T w;
            if constexpr (SIMPLE) {
                w = step1(hb, l, r, d, u, ha, hc, hv, hz);
            } else {
                w = step1(hb, pick(csxl, l, r), pick(csxh, r, l), pick(csyl, d, u), pick(csyh, u, d),
                          pick(sz1m, ha, hc), pick(sz1p, hc, ha), hv, hz);
            }
            hw = (cact && pin0) ? w : (T)0;
        }
        {
            T *wd = bufw(k);
#pragma unroll
            for (int e = 0; e < E; ++e) wd[lown + e * L::PW] = wc[e];
            if (hown) wd[lhself] = hw;
        }
        issueV(k + 1, RV);
        issueU(k + 2, RY);

        // w_{i+1} at plane k-1 from w_i at planes k-2 (wa), k-1 (LDS), k (wc)
        const T *ws = bufw(k - 1);
        T wcen[E];
#pragma unroll
        for (int e = 0; e < E; ++e) wcen[e] = ws[lown + e * L::PW];
        if (k - 1 >= k0) {
            // rows of the neighbouring waves (the top wave's first and the bottom
            // wave's last held row are halo rows, which compute no w_{i+1})
            T inU = (T)0, inD = (T)0;
            if constexpr (!TOP) inU = ws[linU];
            if constexpr (!BOT) inD = ws[linD];
            const size_t po = (size_t)(k - 1) * PB;
            const Sel sz2m = to_sel(sel_lo(k - 1, nz, MASK, B, nzl));
            const Sel sz2p = to_sel(sel_hi(k - 1, nz, MASK, B, nzh));
#pragma unroll
            for (int e = EOWN; e < EOWN + PR; ++e) {
                const T c = wcen[e];
                T xm = ws[lown - 1 + e * L::PW], xp = ws[lown + 1 + e * L::PW];
                T ym = e == 0 ? inU : wcen[e > 0 ? e - 1 : 0];
                T yp = e == E - 1 ? inD : wcen[e < E - 1 ? e + 1 : e];
                T zm = wa[e], zp = wc[e];
                if constexpr (!SIMPLE) {
                    const T xm0 = xm, ym0 = ym, zm0 = zm;
                    xm = pick(sxm, xm0, xp), xp = pick(sxp, xp, xm0);
                    ym = pick(sym[e], ym0, yp), yp = pick(syp[e], yp, ym0);
                    zm = pick(sz2m, zm0, zp), zp = pick(sz2p, zp, zm0);
                }
                const T a = lap7<T>(c, xm, xp, ym, yp, zm, zp, ih2);
                // step i+1 reads z = y_{i-1}, the pair's stencil input at plane k-1
                // (for the first pair, z = v/theta with v = that input)
                const T v = FIRST ? ya[e] : vb[e];
                const T z = FIRST ? v / theta : ya[e];
                const T w2 = rc2 * ((ts * c + tod * (v - a)) - ro2 * z);
                if (rok[e]) {
                    if constexpr (!DROP) st_nt((T *)(W1b + po + roff[e]), c);
                    st_nt((T *)(W2b + po + roff[e]), w2);
                    if constexpr (FIRST && sizeof(T) == 4) st_nt((T *)(V32b + po + roff[e]), v);
                }
            }
        }
        // y at plane k for the next plane's z neighbour
#pragma unroll
        for (int e = 0; e < E; ++e) {
            ya[e] = ys[lown + e * L::PW];
            wa[e] = wcen[e];
            vb[e] = vc[e];
        }
        yob = yoc;
        ha = hb;
        __syncthreads();
    }
}

// DROP: the last pair of an apply, which stores w_{i+1} only (a kernel of its
// own, so that profiles report the two traffic figures apart)
template <typename T, typename TU, bool FIRST, bool DROP, int NXW, int PR, int NYW, bool MASK,
          bool SIMPLE, int UPD = 0>
__global__ void __launch_bounds__(64 * NXW * NYW) k_cheb_pair_lds(Work W, KArgs A)
{
    using L = LPair<NXW, PR, NYW>;
    __shared__ T lds[4 * L::PLANE];
    __shared__ double red[2 * NXW * NYW];
    constexpr int F32 = sizeof(T) == 4;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int xw = wv % NXW, yw = wv / NXW;
    // batched problems walk the pair tile list; a single problem all its tiles
    int total;
    if (W.pair_prob) {
        total = *W.pair_count_dev;
    } else {
        const Prob &P = W.probs[0];
        const int pkz = P.pkz[F32];
        if (pkz < 1) return;
        const int ltx = (P.nx + L::X - 1) / L::X, lty = (P.ny + L::Y - 1) / L::Y;
        total = ltx * lty * ((P.nz + pkz - 1) / pkz);
    }
    // every wave runs the same number of barriers: the tile loop and the plane
    // loop depend only on the workgroup's tiles, and a skipped tile is skipped
    // by the whole workgroup
    for (int g = blockIdx.x; g < total; g += gridDim.x) {
        const int pid = W.pair_prob ? W.pair_prob[g] : 0;
        const Prob &P = W.probs[pid];
        if (P.pkz[F32] < 1) continue;
        {
            const Scalars *sc = P.sc;
            if (sc->done || (A.second && sc->half_pending)) continue;
        }
        // single problem, unless another order is asked for: x-grouped in FP32, so
        // that the tiles of a tile row share the L2 that holds their halo columns;
        // slabs in FP64, whose tiles are all resident at once at 512^3, so that
        // y-neighbouring tiles share it as well
        const int ltx = (P.nx + L::X - 1) / L::X;
        const int t = W.pair_prob ? W.pair_local[g]
                                  : tile_order_tx(W.order ? W.order : (sizeof(T) == 8 ? 2 : 1), ltx, g, total);
        double ssh = 0.0, ssl = 0.0;
        if (yw == 0)
            cheb_pair_lds_tile<T, TU, FIRST, DROP, NXW, PR, NYW, R_TOP, MASK, SIMPLE, UPD>(
                P, A, t, lane, xw, yw, lds, ssh, ssl);
        else if (yw == NYW - 1)
            cheb_pair_lds_tile<T, TU, FIRST, DROP, NXW, PR, NYW, R_BOT, MASK, SIMPLE, UPD>(
                P, A, t, lane, xw, yw, lds, ssh, ssl);
        else if constexpr (NYW > 2)
            cheb_pair_lds_tile<T, TU, FIRST, DROP, NXW, PR, NYW, R_MID, MASK, SIMPLE, UPD>(
                P, A, t, lane, xw, yw, lds, ssh, ssl);
        if constexpr (UPD == U_S) {
            // this tile's s.s in its partial slot (summed by the half-step finalize)
            double hh[1] = {ssh}, ll[1] = {ssl};
            block_reduce_dd<1, NXW * NYW>(hh, ll, red);
            if (threadIdx.x == 0) {
                double *pp = P.partials + (size_t)t * PARTIAL_STRIDE;
                pp[0] = hh[0];
                pp[1] = ll[0];
            }
        }
    }
}

// ------------------------------------------------------------------------
// Three consecutive Chebyshev steps i, i+1, i+2 (i >= 3) in one pass, staged
// in LDS like k_cheb_pair_lds. One pass reads y = y_{i-1}, z = y_{i-2} and v
// and writes w_{i+1}, w_{i+2}: the bytes of one pair for three steps.
//   w_i     = rc_i     ((2 sigma y       + (2/delta)(v - A y))       - ro_i     z)
//   w_{i+1} = rc_{i+1} ((2 sigma w_i     + (2/delta)(v - A w_i))     - ro_{i+1} y)
//   w_{i+2} = rc_{i+2} ((2 sigma w_{i+1} + (2/delta)(v - A w_{i+1})) - ro_{i+2} w_i)
// Plane k of the march computes w_i at plane k, w_{i+1} at k-1 and w_{i+2}
// at k-2. w_i is computed on the tile plus a halo ring of two, w_{i+1} on the
// tile plus one. The workgroup has NXW x NYW waves; a wave owns 64 columns x
// PR rows. The top wave of a column of waves also holds the two halo rows
// above the tile, the bottom wave the two below; waves between them hold only
// their own rows and take the rows across their edges from LDS. At each side
// 2 x 16 halo lanes hold the columns one and two out; they load y, v and z
// there, the lanes two out also y three out, and they compute w_i (and w_{i+1}
// one out) at those points. y, w_i and w_{i+1} each have two LDS planes
// alternating by plane, with one barrier per plane. The arithmetic per point
// is that of k_stencil's step.
// ------------------------------------------------------------------------
template <int NXW, int PR, int NYW> struct LTriple {
    static constexpr int X = 64 * NXW, Y = NYW * PR;
    static constexpr int PW = X + 4, PH = Y + 4; // LDS plane: rows -2..Y+1, columns -2..X+1
    static constexpr int PLANE = PW * PH;
    static constexpr int NT = 64 * NXW * NYW;
};

// FIRST: steps 1, 2 and 3 (the first step's own formula, y_0 := v, z = v/theta
// at step 2; step 3 reads v = the input and z = w_1). The input is then v
// itself, read as TU (FP64 also in the mixed mode, rounded once on load, with
// the FP32 copy of v written out).
// UPD: a vector update folded into the first triple, as in cheb_pair_lds_tile.
template <typename T, typename TU, bool FIRST, bool DROP, int NXW, int PR, int NYW, int ROLE,
          bool MASK, bool SIMPLE, int UPD>
__device__ __forceinline__ void cheb_triple_lds_tile(const Prob &P, const KArgs &A, int tile,
                                                     int lane, int xw, int yw, T *lds, double &ssh,
                                                     double &ssl)
{
    static_assert(UPD == 0 || FIRST, "a vector update folds only into a first pass");
    constexpr int NU = UPD == U_P ? 2 : (UPD == U_S ? 1 : 0);
    constexpr int NUA = NU > 0 ? NU : 1;
    using L = LTriple<NXW, PR, NYW>;
    constexpr bool TOP = ROLE == R_TOP, BOT = ROLE == R_BOT, MID = ROLE == R_MID;
    constexpr int E = MID ? PR : PR + 2;           // held rows: own PR (and two halo rows)
    constexpr int L2LO = TOP ? 1 : 0, L2HI = BOT ? E - 1 : E;   // rows of w_{i+1}
    constexpr int OWNLO = TOP ? 2 : 0, OWNHI = BOT ? PR : E;    // own rows (w_{i+2})
    constexpr int TRO = TOP ? -3 : L::Y + 2;       // tile row of the outer row (y only)
    const int r0 = TOP ? -2 : (BOT ? (NYW - 1) * PR : yw * PR); // tile row of held row 0
    auto trow = [r0](int e) { return r0 + e; };
    auto in2 = [](int e) { return e >= L2LO && e < L2HI; };
    auto own = [](int e) { return e >= OWNLO && e < OWNHI; };
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int ltx = (nx + L::X - 1) / L::X, lty = (ny + L::Y - 1) / L::Y;
    const int tix = tile % ltx, tiy = (tile / ltx) % lty, tiz = tile / (ltx * lty);
    const int x0 = tix * L::X, y0 = tiy * L::Y;
    const int pkz = P.tkz[sizeof(T) == 4];
    const int k0 = tiz * pkz, k1 = min(k0 + pkz, nz);
    const int cx = xw * 64 + lane;
    const int i = x0 + cx;
    const bool xin = i < nx;
    const int ic = xin ? i : nx - 1;
    const size_t PB = (size_t)nx * (size_t)ny * sizeof(T);
    const size_t PBY = (size_t)nx * (size_t)ny * sizeof(TU); // the input's planes
    const char *Yb = (const char *)P.vec[A.in];
    const char *Ub[2] = {nullptr, nullptr};
    char *Ob = nullptr;
    double ua = 0.0, ub = 0.0, uo = 0.0;
    bool ufirst = false;
    if constexpr (UPD == U_S) {
        Yb = (const char *)P.vec[V_R];
        Ub[0] = (const char *)P.vec[V_W];
        Ob = (char *)P.vec[V_S];
        ua = P.sc->alpha;
    } else if constexpr (UPD == U_P) {
        const int it = P.sc->iter;
        ufirst = it == 0;
        const int pold = ((it - 1) & 1) ? V_P2 : V_P, pnew = (it & 1) ? V_P2 : V_P;
        Yb = (const char *)P.vec[ufirst ? V_P : V_R];
        Ub[0] = (const char *)P.vec[ufirst ? V_P : V_W];
        Ub[1] = (const char *)P.vec[ufirst ? V_P : pold];
        Ob = (char *)P.vec[pnew];
        ub = P.sc->beta;
        uo = P.sc->omega;
    }
    auto comb = [&](TU r, TU w, TU pp) -> TU {
        if constexpr (UPD == U_S) return r - (TU)ua * w;
        else if constexpr (UPD == U_P) return ufirst ? pp : r + (TU)ub * (pp - (TU)uo * w);
        else return r;
    };
    const char *Vb = (const char *)vec_at(P, A.v);
    const char *Zb = (const char *)P.vec[A.z];
    char *W1b = (char *)P.vec[A.out];
    char *W2b = (char *)P.vec[A.x2];
    char *V32b = (char *)P.vec[V_V32];
    const T ih2 = Coef<T>::ih2(P), theta = Coef<T>::theta(P), c1 = Coef<T>::c1(P);
    const T ts = Coef<T>::two_sigma(P), tod = Coef<T>::two_over_delta(P);
    const T rc1 = Coef<T>::rc(P, A.step), ro1 = Coef<T>::ro(P, A.step);
    const T rc2 = Coef<T>::rc(P, A.step + 1), ro2 = Coef<T>::ro(P, A.step + 1);
    const T rc3 = Coef<T>::rc(P, A.step + 2), ro3 = Coef<T>::ro(P, A.step + 2);
    auto clampi = [](int a, int n) { return a < 0 ? 0 : (a >= n ? n - 1 : a); };
    auto off = [&](int x, int j) { return (unsigned)(x + nx * j) * (unsigned)sizeof(T); };
    auto offy = [&](int x, int j) { return (unsigned)(x + nx * j) * (unsigned)sizeof(TU); };
    auto ld = [](const char *plane, unsigned o) { return ld_g((const T *)(plane + o)); };
    auto ldy = [](const char *plane, unsigned o) { return ld_g((const TU *)(plane + o)); };
    // LDS element of tile row r (-2..Y+1) and tile column c (-2..X+1)
    auto lidx = [](int r, int c) { return (r + 2) * L::PW + (c + 2); };

    const int B = MASK ? P.block : 1;
    const unsigned bc = P.bc;
    const bool nxl = bc & 1u, nxh = bc & 2u, nyl = bc & 4u, nyh = bc & 8u;
    const bool nzl = bc & 16u, nzh = bc & 32u;
    const Sel sxm = to_sel(xin ? sel_lo(i, nx, MASK, B, nxl) : 0);
    const Sel sxp = to_sel(xin ? sel_hi(i, nx, MASK, B, nxh) : 0);
    bool rok[E];
    unsigned roff[E], ryoff[E];
    Sel sym[E], syp[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = y0 + trow(e);
        const bool jin = j >= 0 && j < ny;
        rok[e] = xin && jin;
        roff[e] = off(ic, clampi(j, ny));
        ryoff[e] = offy(ic, clampi(j, ny));
        sym[e] = to_sel(jin ? sel_lo(j, ny, MASK, B, nyl) : 0);
        syp[e] = to_sel(jin ? sel_hi(j, ny, MASK, B, nyh) : 0);
    }
    const int jo = y0 + TRO;
    const bool ook = !MID && xin && jo >= 0 && jo < ny;
    const unsigned ooff = offy(ic, clampi(jo, ny));
    const int lown = lidx(trow(0), cx);
    // the rows next to the held ones (held by the waves above and below)
    const int linU = lidx(r0 - 1, cx), linD = lidx(r0 + E, cx);

    // Halo lanes. Lanes 0-15 (left) and 32-47 (right) hold the column one out
    // (A), lanes 16-31 and 48-63 the column two out (B); lane e of a group
    // holds held row e. All of them load and publish y there. A computes w_i
    // on the rows of w_{i+1} and w_{i+1} on the own rows; B computes w_i on the
    // own rows and also loads y three columns out.
    const bool hside = lane >= 32, grpb = (lane & 16) != 0;
    const int eh = min(lane & 15, E - 1);
    const bool hwave = hside ? xw == NXW - 1 : xw == 0;
    const bool hact = hwave && (lane & 15) < E;
    const int hcol = hside ? (grpb ? L::X + 1 : L::X) : (grpb ? -2 : -1);
    const int hnear = hside ? hcol - 1 : hcol + 1;      // towards the tile
    const int hfarc = hside ? hcol + 1 : hcol - 1;      // away from it (B: column three out)
    const int hi = x0 + hcol, hfi = x0 + hfarc;
    const int hj = y0 + trow(eh);
    const bool hrow = hj >= 0 && hj < ny;
    const bool hload = hact && hrow && hi >= 0 && hi < nx;
    const bool h1 = hact && (grpb ? own(eh) : in2(eh));  // computes w_i here
    const bool h2 = hact && !grpb && own(eh);            // computes w_{i+1} here
    const bool c1act = h1 && hload, c2act = h2 && hload;
    const bool fload = hact && grpb && hrow && hfi >= 0 && hfi < nx;
    const unsigned hoff = off(clampi(hi, nx), clampi(hj, ny));
    const unsigned hoffy = offy(clampi(hi, nx), clampi(hj, ny));
    const unsigned foff = offy(clampi(hfi, nx), clampi(hj, ny));
    const int lhself = lidx(trow(eh), hcol);
    const int lhnear = lidx(trow(eh), hnear);
    const int lhfar = grpb ? lhself : lidx(trow(eh), hfarc);
    const int lhup = lidx(max(trow(eh) - 1, -2), hcol), lhdn = lidx(min(trow(eh) + 1, L::Y + 1), hcol);
    const Sel csxl = to_sel(hload ? sel_lo(hi, nx, MASK, B, nxl) : 0);
    const Sel csxh = to_sel(hload ? sel_hi(hi, nx, MASK, B, nxh) : 0);
    const Sel csyl = to_sel(hload ? sel_lo(hj, ny, MASK, B, nyl) : 0);
    const Sel csyh = to_sel(hload ? sel_hi(hj, ny, MASK, B, nyh) : 0);

    // one step at one point: A u from the centre and its six neighbours (in
    // the order x-, x+, y-, y+, z-, z+), then the Chebyshev update
    // A u at one point from the centre and its six neighbours (in the order x-,
    // x+, y-, y+, z-, z+), then the Chebyshev update of a step after the first
    auto lap = [&](T c, T xm, T xp, T ym, T yp, T zm, T zp, Sel szl, Sel szh, Sel sxl, Sel sxh,
                   Sel syl, Sel syh) {
        if constexpr (!SIMPLE) {
            const T xm0 = xm, ym0 = ym, zm0 = zm;
            xm = pick(sxl, xm0, xp), xp = pick(sxh, xp, xm0);
            ym = pick(syl, ym0, yp), yp = pick(syh, yp, ym0);
            zm = pick(szl, zm0, zp), zp = pick(szh, zp, zm0);
        }
        return lap7<T>(c, xm, xp, ym, yp, zm, zp, ih2);
    };
    auto step = [&](T rc, T ro, T c, T xm, T xp, T ym, T yp, T zm, T zp, T v, T z, Sel szl,
                    Sel szh, Sel sxl, Sel sxh, Sel syl, Sel syh) {
        const T a = lap(c, xm, xp, ym, yp, zm, zp, szl, szh, sxl, sxh, syl, syh);
        return rc * ((ts * c + tod * (v - a)) - ro * z);
    };
    // step i (the first step's formula when FIRST)
    auto step1 = [&](T c, T xm, T xp, T ym, T yp, T zm, T zp, T v, T z, Sel szl, Sel szh, Sel sxl,
                     Sel sxh, Sel syl, Sel syh) {
        const T a = lap(c, xm, xp, ym, yp, zm, zp, szl, szh, sxl, sxh, syl, syh);
        if constexpr (FIRST) return c1 * ((T)2 * c - a / theta);
        else return rc1 * ((ts * c + tod * (v - a)) - ro1 * z);
    };

    struct RawY {
        TU y[E], yo, he;
        TU uy[NUA][E], uyo[NUA], uhe[NUA];
    };
    struct RawV {
        T v[E], z[E], hv, hz;
        TU hf, uhf[NUA];
    };
    // the folded update's extra operands of plane p; in the plane loop they are
    // issued after step i, so fewer loads are in flight across its arithmetic
    auto issueU = [&](int p, RawY &R) {
        const size_t pb = (size_t)clampi(p, nz) * PBY;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const char *Up = Ub[u] + pb;
#pragma unroll
            for (int e = 0; e < E; ++e) R.uy[u][e] = ldy(Up, ryoff[e]);
            if constexpr (!MID) R.uyo[u] = ldy(Up, ooff);
            else R.uyo[u] = (TU)0;
            R.uhe[u] = ldy(Up, hoffy);
        }
    };
    auto issueY = [&](int p, RawY &R, bool extra) {
        const size_t pb = (size_t)clampi(p, nz) * PBY;
        const char *Yp = Yb + pb;
#pragma unroll
        for (int e = 0; e < E; ++e) R.y[e] = ldy(Yp, ryoff[e]);
        if constexpr (!MID) R.yo = ldy(Yp, ooff);
        else R.yo = (TU)0;
        R.he = ldy(Yp, hoffy);
        if (extra) issueU(p, R);
    };
    auto gy = [&](const RawY &R, int e) {
        return comb(R.y[e], R.uy[0][e], R.uy[NUA - 1][e]);
    };
    auto gyo = [&](const RawY &R) { return comb(R.yo, R.uyo[0], R.uyo[NUA - 1]); };
    auto ghe = [&](const RawY &R) { return comb(R.he, R.uhe[0], R.uhe[NUA - 1]); };
    auto issueV = [&](int p, RawV &R) {
        const size_t po = (size_t)clampi(p, nz) * PB;
        if constexpr (!FIRST) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                R.v[e] = ld(Vb + po, roff[e]);
                R.z[e] = ld(Zb + po, roff[e]);
            }
            R.hv = ld(Vb + po, hoff);
            R.hz = ld(Zb + po, hoff);
        }
        R.hf = ldy(Yb + (size_t)clampi(p, nz) * PBY, foff);
#pragma unroll
        for (int u = 0; u < NU; ++u) R.uhf[u] = ldy(Ub[u] + (size_t)clampi(p, nz) * PBY, foff);
    };
    auto ghf = [&](const RawV &R) { return comb(R.hf, R.uhf[0], R.uhf[NUA - 1]); };
    auto buf = [&](int f, int k) { return lds + (2 * f + (k & 1)) * L::PLANE; }; // f: 0 y, 1 w_i, 2 w_{i+1}

    // registers across planes (k = the plane of w_i): y at k-1 (ya), w_i at
    // k-2 (w1a), w_{i+1} at k-3 (w2a), v at k-1 (vb) and k-2 (vbb); at the halo
    // points y at k-1 (ha), w_i at k-2 (h1a) and v at k-1 (hvb)
    // FIRST: yaa = y (= v) at k-2, the v of step i+2
    T ya[E], w1a[E], w2a[E], vb[E], vbb[E], yaa[E];
    T yob, ha, h1a, hvb;
    RawY RY;
    RawV RV;
#pragma unroll
    for (int e = 0; e < E; ++e) RV.v[e] = RV.z[e] = yaa[e] = (T)0;
    RV.hv = RV.hz = (T)0;
    {
        RawY t;
        issueY(k0 - 3, t, true);
        {
            const bool pin = k0 - 3 >= 0;
#pragma unroll
            for (int e = 0; e < E; ++e) ya[e] = (pin && rok[e]) ? (T)gy(t, e) : (T)0;
            ha = (pin && hload) ? (T)ghe(t) : (T)0;
        }
        issueY(k0 - 2, t, true);
        {
            const bool pin = k0 - 2 >= 0;
            T *yd = buf(0, k0 - 2);
#pragma unroll
            for (int e = 0; e < E; ++e) yd[lown + e * L::PW] = (pin && rok[e]) ? (T)gy(t, e) : (T)0;
            yob = (pin && ook) ? (T)gyo(t) : (T)0;
            if (hact) yd[lhself] = (pin && hload) ? (T)ghe(t) : (T)0;
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) w1a[e] = w2a[e] = vb[e] = vbb[e] = (T)0;
    h1a = hvb = (T)0;
    issueY(k0 - 1, RY, true);
    issueV(k0 - 2, RV);
    __syncthreads();

    for (int k = k0 - 2; k <= k1 + 1; ++k) {
        const bool pin1 = k + 1 >= 0 && k + 1 < nz, pin0 = k >= 0 && k < nz;
        const bool pinm = k - 1 >= 0 && k - 1 < nz;
        // take y at plane k+1, publish it, issue plane k+2
        T yc[E];
        TU vn[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            vn[e] = gy(RY, e);
            yc[e] = (pin1 && rok[e]) ? (T)vn[e] : (T)0;
        }
        const T yoc = (pin1 && ook) ? (T)gyo(RY) : (T)0;
        const T hc = (pin1 && hload) ? (T)ghe(RY) : (T)0;
        if constexpr (UPD != 0) {
            if (k + 1 >= k0 && k + 1 < k1 && !ufirst) {
                const size_t po = (size_t)(k + 1) * PBY;
#pragma unroll
                for (int e = OWNLO; e < OWNHI; ++e)
                    if (rok[e]) {
                        st_nt((TU *)(Ob + po + ryoff[e]), vn[e]);
                        if constexpr (UPD == U_S) dd_acc(ssh, ssl, (double)vn[e], (double)vn[e]);
                    }
            }
        }
        {
            T *yd = buf(0, k + 1);
#pragma unroll
            for (int e = 0; e < E; ++e) yd[lown + e * L::PW] = yc[e];
            if (hact) yd[lhself] = hc;
        }
        issueY(k + 2, RY, false);

        // w_i at plane k on the held rows
        const T *ys = buf(0, k);
        const Sel s1m = to_sel(pin0 ? sel_lo(k, nz, MASK, B, nzl) : 0);
        const Sel s1p = to_sel(pin0 ? sel_hi(k, nz, MASK, B, nzh) : 0);
        T w1c[E], vc[E];
        {
            // the rows across the held rows' edges: the outer row (top, bottom
            // wave) or a row of the neighbouring wave from LDS
            T inU = (T)0, inD = (T)0;
            if constexpr (TOP) inU = yob; else inU = ys[linU];
            if constexpr (BOT) inD = yob; else inD = ys[linD];
            T cen[E];
#pragma unroll
            for (int e = 0; e < E; ++e) cen[e] = ys[lown + e * L::PW];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const T c = cen[e];
                // x neighbours from the LDS plane, which holds every column of the
                // tile and its halo (no lane shifts, no edge patches)
                const T xm = ys[lown - 1 + e * L::PW], xp = ys[lown + 1 + e * L::PW];
                const T ym = e == 0 ? inU : cen[e > 0 ? e - 1 : 0];
                const T yp = e == E - 1 ? inD : cen[e < E - 1 ? e + 1 : e];
                const bool ok = pin0 && rok[e];
                const T v = (!FIRST && ok) ? RV.v[e] : (T)0, z = (!FIRST && ok) ? RV.z[e] : (T)0;
                vc[e] = v;
                const T w = step1(c, xm, xp, ym, yp, ya[e], yc[e], v, z, s1m, s1p, sxm, sxp, sym[e],
                                  syp[e]);
                w1c[e] = ok ? w : (T)0;
            }
        }
        // w_i at the halo points (A: rows of w_{i+1}; B: own rows)
        T hb, h1c, hvc;
        {
            hb = ys[lhself];
            const T xn = ys[lhnear], d = ys[lhup], u = ys[lhdn];
            const T xf = grpb ? ((fload && pin0) ? (T)ghf(RV) : (T)0) : ys[lhfar];
            const bool ok = c1act && pin0;
            hvc = (!FIRST && hload && pin0) ? RV.hv : (T)0;
            const T hz = (!FIRST && ok) ? RV.hz : (T)0;
            const T l = hside ? xn : xf, r = hside ? xf : xn;
            const T w = step1(hb, l, r, d, u, ha, hc, hvc, hz, s1m, s1p, csxl, csxh, csyl, csyh);
            h1c = ok ? w : (T)0;
        }
        {
            T *wd = buf(1, k);
#pragma unroll
            for (int e = 0; e < E; ++e) wd[lown + e * L::PW] = w1c[e];
            if (h1) wd[lhself] = h1c;
        }
        issueV(k + 1, RV);
        issueU(k + 2, RY);

        // w_{i+1} at plane k-1 on its rows, from w_i at k-2 (w1a), k-1 (LDS), k (w1c)
        const T *w1s = buf(1, k - 1);
        const Sel s2m = to_sel(pinm ? sel_lo(k - 1, nz, MASK, B, nzl) : 0);
        const Sel s2p = to_sel(pinm ? sel_hi(k - 1, nz, MASK, B, nzh) : 0);
        T w2c[E], cen1[E];
#pragma unroll
        for (int e = 0; e < E; ++e) cen1[e] = w1s[lown + e * L::PW];
        T h2c = (T)0;
        if (k >= k0) {
            // rows of the neighbouring waves (the top wave's first and the bottom
            // wave's last held row compute no w_{i+1})
            T inU = (T)0, inD = (T)0;
            if constexpr (!TOP) inU = w1s[linU];
            if constexpr (!BOT) inD = w1s[linD];
#pragma unroll
            for (int e = L2LO; e < L2HI; ++e) {
                const T c = cen1[e];
                // x neighbours from the LDS plane, which holds every column of the
                // tile and its halo (no lane shifts, no edge patches)
                const T xm = w1s[lown - 1 + e * L::PW], xp = w1s[lown + 1 + e * L::PW];
                const T ym = e == 0 ? inU : cen1[e > 0 ? e - 1 : 0];
                const T yp = e == E - 1 ? inD : cen1[e < E - 1 ? e + 1 : e];
                // step i+1 reads z = y_{i-1}, the stencil input at plane k-1 (for the
                // first triple v = that input and z = v/theta)
                const T v = FIRST ? ya[e] : vb[e];
                const T z = FIRST ? v / theta : ya[e];
                const T w = step(rc2, ro2, c, xm, xp, ym, yp, w1a[e], w1c[e], v, z, s2m, s2p, sxm, sxp,
                                 sym[e], syp[e]);
                w2c[e] = (pinm && rok[e]) ? w : (T)0;
            }
            // w_{i+1} at the halo points one out, own rows (lanes A)
            {
                const T c = w1s[lhself];
                const T xn = w1s[lhnear], xf = w1s[lhfar], d = w1s[lhup], u = w1s[lhdn];
                const T l = hside ? xn : xf, r = hside ? xf : xn;
                const T v = FIRST ? ha : hvb;
                const T z = FIRST ? v / theta : ha;
                const T w = step(rc2, ro2, c, l, r, d, u, h1a, h1c, v, z, s2m, s2p, csxl, csxh, csyl,
                                 csyh);
                h2c = (c2act && pinm) ? w : (T)0;
            }
            T *wd = buf(2, k - 1);
#pragma unroll
            for (int e = L2LO; e < L2HI; ++e) wd[lown + e * L::PW] = w2c[e];
            if (h2) wd[lhself] = h2c;
        }

        // w_{i+2} at plane k-2 on the own rows, from w_{i+1} at k-3 (w2a), k-2 (LDS), k-1 (w2c)
        const T *w2s = buf(2, k - 2);
        T cen2[E];
#pragma unroll
        for (int e = 0; e < E; ++e) cen2[e] = w2s[lown + e * L::PW];
        if (k >= k0 + 2) {
            T inU = (T)0, inD = (T)0;
            if constexpr (!TOP) inU = w2s[linU];
            if constexpr (!BOT) inD = w2s[linD];
            const Sel s3m = to_sel(sel_lo(k - 2, nz, MASK, B, nzl));
            const Sel s3p = to_sel(sel_hi(k - 2, nz, MASK, B, nzh));
            const size_t po = (size_t)(k - 2) * PB;
#pragma unroll
            for (int e = OWNLO; e < OWNHI; ++e) {
                const T c = cen2[e];
                // x neighbours from the LDS plane, which holds every column of the
                // tile and its halo (no lane shifts, no edge patches)
                const T xm = w2s[lown - 1 + e * L::PW], xp = w2s[lown + 1 + e * L::PW];
                const T ym = e == 0 ? inU : cen2[e > 0 ? e - 1 : 0];
                const T yp = e == E - 1 ? inD : cen2[e < E - 1 ? e + 1 : e];
                // step i+2 reads z = w_i at plane k-2, held in w1a
                const T v = FIRST ? yaa[e] : vbb[e];
                const T w3 = step(rc3, ro3, c, xm, xp, ym, yp, w2a[e], w2c[e], v, w1a[e], s3m, s3p,
                                  sxm, sxp, sym[e], syp[e]);
                if (rok[e]) {
                    if constexpr (!DROP) st_nt((T *)(W1b + po + roff[e]), c);
                    st_nt((T *)(W2b + po + roff[e]), w3);
                    if constexpr (FIRST && sizeof(T) == 4) st_nt((T *)(V32b + po + roff[e]), v);
                }
            }
        }
        // rotate: y at plane k, w_i at k-1, w_{i+1} at k-2 for the next plane
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if constexpr (FIRST) yaa[e] = ya[e];
            ya[e] = ys[lown + e * L::PW];
            w1a[e] = cen1[e];
            w2a[e] = cen2[e];
            vbb[e] = vb[e];
            vb[e] = vc[e];
        }
        yob = yoc;
        h1a = w1s[lhself];
        ha = hb;
        hvb = hvc;
        __syncthreads();
    }
}

// At most 256 VGPRs (two waves per SIMD): the bodies with neighbour selects
// need a few more and spill them (measured faster than one wave per SIMD)
template <typename T, typename TU, bool FIRST, bool DROP, int NXW, int PR, int NYW, bool MASK,
          bool SIMPLE, int UPD = 0>
__global__ void __launch_bounds__(64 * NXW * NYW) __attribute__((amdgpu_waves_per_eu(2)))
k_cheb_triple_lds(Work W, KArgs A)
{
    using L = LTriple<NXW, PR, NYW>;
    __shared__ T lds[6 * L::PLANE];
    __shared__ double red[2 * NXW * NYW];
    constexpr int F32 = sizeof(T) == 4;
    const Prob &P = W.probs[0];
    const int tkz = P.tkz[F32];
    if (tkz < 1) return;
    {
        const Scalars *sc = P.sc;
        if (sc->done || (A.second && sc->half_pending)) return;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int xw = wv % NXW, yw = wv / NXW;
    const int ltx = (P.nx + L::X - 1) / L::X, lty = (P.ny + L::Y - 1) / L::Y;
    const int total = ltx * lty * ((P.nz + tkz - 1) / tkz);
    for (int g = blockIdx.x; g < total; g += gridDim.x) {
        // default order: slabs (512^3: one tile per CU, each XCD running a band
        // of tile rows of all x-tiles, so the y-halo rows between them come from
        // its L2)
        const int t = tile_order_tx(W.order ? W.order : 2, ltx, g, total);
        double ssh = 0.0, ssl = 0.0;
        if (yw == 0)
            cheb_triple_lds_tile<T, TU, FIRST, DROP, NXW, PR, NYW, R_TOP, MASK, SIMPLE, UPD>(
                P, A, t, lane, xw, yw, lds, ssh, ssl);
        else if (yw == NYW - 1)
            cheb_triple_lds_tile<T, TU, FIRST, DROP, NXW, PR, NYW, R_BOT, MASK, SIMPLE, UPD>(
                P, A, t, lane, xw, yw, lds, ssh, ssl);
        else if constexpr (NYW > 2)
            cheb_triple_lds_tile<T, TU, FIRST, DROP, NXW, PR, NYW, R_MID, MASK, SIMPLE, UPD>(
                P, A, t, lane, xw, yw, lds, ssh, ssl);
        if constexpr (UPD == U_S) {
            double hh[1] = {ssh}, ll[1] = {ssl};
            block_reduce_dd<1, NXW * NYW>(hh, ll, red);
            if (threadIdx.x == 0) {
                double *pp = P.partials + (size_t)t * PARTIAL_STRIDE;
                pp[0] = hh[0];
                pp[1] = ll[0];
            }
        }
    }
}

// ------------------------------------------------------------------------
// S consecutive Chebyshev steps i, ..., i+S-1 in one pass, staged in LDS the
// way k_cheb_triple_lds stages three (used with S = 4 in the mixed mode).
// Level l = 0..S-1 of the march computes w_{i+l} at plane k - l. Step i+l
// reads the level before it (the pass input y = y_{i-1} for level 0), v, and
// z = the level two before it (for levels 0 and 1: z_{i-2} and y_{i-1}).
// Level l is needed on the tile plus the points within S-1-l row and column
// steps of it (each step widens the dependence by one point along one axis),
// so the input is read with a halo of S. A wave owns 64 columns x PR rows;
// the top and bottom wave of a column of waves also hold the S-1 halo rows
// above or below the tile (and the input's outer row), the others only their
// own rows. At each side S-1 groups of GS lanes hold the columns 1..S-1 out,
// lane e of a group held row e: group g loads y, v and z there and computes
// the levels up to S-1-g-d, d the row's distance from the tile; group S-1 also
// loads y S columns out. Every level but the last has two LDS planes
// alternating by plane (one barrier per plane), as has y. One pass reads y,
// z, v and writes w_{i+S-2} and w_{i+S-1}: the bytes of a pair for S steps.
// The arithmetic per point is that of k_stencil's step.
// ------------------------------------------------------------------------
template <int NXW, int PR, int NYW, int S> struct LSteps {
    static constexpr int H = S - 1;
    static constexpr int X = 64 * NXW, Y = NYW * PR;
    static constexpr int PW = X + 2 * H, PH = Y + 2 * H; // rows -H..Y+H-1, columns -H..X+H-1
    static constexpr int PLANE = PW * PH;
    static constexpr int NT = 64 * NXW * NYW;
    static constexpr int GS = H == 1 ? 32 : (H == 2 ? 16 : 8); // lanes per halo-column group
};

template <typename T, typename TU, int S, bool FIRST, bool DROP, int NXW, int PR, int NYW, int ROLE,
          bool MASK, bool SIMPLE, int UPD>
__device__ __forceinline__ void cheb_steps_lds_tile(const Prob &P, const KArgs &A, int tile,
                                                    int lane, int xw, int yw, T *lds, double &ssh,
                                                    double &ssl)
{
    static_assert(UPD == 0 || FIRST, "a vector update folds only into a first pass");
    using L = LSteps<NXW, PR, NYW, S>;
    constexpr int H = L::H;
    static_assert(H >= 1 && H * L::GS <= 32, "halo-column groups fit half a wave");
    constexpr int NU = UPD == U_P ? 2 : (UPD == U_S ? 1 : 0);
    constexpr int NUA = NU > 0 ? NU : 1;
    constexpr bool TOP = ROLE == R_TOP, BOT = ROLE == R_BOT, MID = ROLE == R_MID;
    constexpr int E = MID ? PR : PR + H;           // held rows: own PR (and H halo rows)
    static_assert(E <= L::GS, "a halo-column group holds every held row");
    constexpr int EOWN = TOP ? H : 0;              // first own row among the held rows
    constexpr int TRO = TOP ? -(H + 1) : L::Y + H; // tile row of the outer row (y only)
    // distance of held row e from the tile's rows (0: an own row)
    auto ydist = [](int e) { return TOP ? (e < H ? H - e : 0) : (BOT ? (e >= PR ? e - PR + 1 : 0) : 0); };
    const int r0 = TOP ? -H : (BOT ? (NYW - 1) * PR : yw * PR); // tile row of held row 0
    auto trow = [r0](int e) { return r0 + e; };
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int ltx = (nx + L::X - 1) / L::X, lty = (ny + L::Y - 1) / L::Y;
    const int tix = tile % ltx, tiy = (tile / ltx) % lty, tiz = tile / (ltx * lty);
    const int x0 = tix * L::X, y0 = tiy * L::Y;
    const int pkz = P.qkz[sizeof(T) == 4];
    const int k0 = tiz * pkz, k1 = min(k0 + pkz, nz);
    const int cx = xw * 64 + lane;
    const int i = x0 + cx;
    const bool xin = i < nx;
    const int ic = xin ? i : nx - 1;
    const size_t PB = (size_t)nx * (size_t)ny * sizeof(T);
    const size_t PBY = (size_t)nx * (size_t)ny * sizeof(TU); // the input's planes
    const char *Yb = (const char *)P.vec[A.in];
    const char *Ub[2] = {nullptr, nullptr};
    char *Ob = nullptr;
    double ua = 0.0, ub = 0.0, uo = 0.0;
    bool ufirst = false;
    if constexpr (UPD == U_S) {
        Yb = (const char *)P.vec[V_R];
        Ub[0] = (const char *)P.vec[V_W];
        Ob = (char *)P.vec[V_S];
        ua = P.sc->alpha;
    } else if constexpr (UPD == U_P) {
        const int it = P.sc->iter;
        ufirst = it == 0;
        const int pold = ((it - 1) & 1) ? V_P2 : V_P, pnew = (it & 1) ? V_P2 : V_P;
        Yb = (const char *)P.vec[ufirst ? V_P : V_R];
        Ub[0] = (const char *)P.vec[ufirst ? V_P : V_W];
        Ub[1] = (const char *)P.vec[ufirst ? V_P : pold];
        Ob = (char *)P.vec[pnew];
        ub = P.sc->beta;
        uo = P.sc->omega;
    }
    auto comb = [&](TU r, TU w, TU pp) -> TU {
        if constexpr (UPD == U_S) return r - (TU)ua * w;
        else if constexpr (UPD == U_P) return ufirst ? pp : r + (TU)ub * (pp - (TU)uo * w);
        else return r;
    };
    const char *Vb = (const char *)vec_at(P, A.v);
    const char *Zb = (const char *)P.vec[A.z];
    char *W1b = (char *)P.vec[A.out];
    char *W2b = (char *)P.vec[A.x2];
    char *V32b = (char *)P.vec[V_V32];
    const T ih2 = Coef<T>::ih2(P), theta = Coef<T>::theta(P), c1 = Coef<T>::c1(P);
    const T ts = Coef<T>::two_sigma(P), tod = Coef<T>::two_over_delta(P);
    T rcs[S], ros[S]; // the coefficients of step i+l (level 0 of a first pass uses c1)
#pragma unroll
    for (int l = 0; l < S; ++l) {
        rcs[l] = Coef<T>::rc(P, A.step + l);
        ros[l] = Coef<T>::ro(P, A.step + l);
    }
    auto clampi = [](int a, int n) { return a < 0 ? 0 : (a >= n ? n - 1 : a); };
    auto inz = [nz](int p) { return p >= 0 && p < nz; };
    auto off = [&](int x, int j) { return (unsigned)(x + nx * j) * (unsigned)sizeof(T); };
    auto offy = [&](int x, int j) { return (unsigned)(x + nx * j) * (unsigned)sizeof(TU); };
    auto ld = [](const char *plane, unsigned o) { return ld_g((const T *)(plane + o)); };
    auto ldy = [](const char *plane, unsigned o) { return ld_g((const TU *)(plane + o)); };
    // LDS element of tile row r (-H..Y+H-1) and tile column c (-H..X+H-1)
    auto lidx = [](int r, int c) { return (r + H) * L::PW + (c + H); };

    const int B = MASK ? P.block : 1;
    const unsigned bc = P.bc;
    const bool nxl = bc & 1u, nxh = bc & 2u, nyl = bc & 4u, nyh = bc & 8u;
    const bool nzl = bc & 16u, nzh = bc & 32u;
    const Sel sxm = to_sel(xin ? sel_lo(i, nx, MASK, B, nxl) : 0);
    const Sel sxp = to_sel(xin ? sel_hi(i, nx, MASK, B, nxh) : 0);
    bool rok[E];
    unsigned roff[E], ryoff[E];
    Sel sym[E], syp[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = y0 + trow(e);
        const bool jin = j >= 0 && j < ny;
        rok[e] = xin && jin;
        roff[e] = off(ic, clampi(j, ny));
        ryoff[e] = offy(ic, clampi(j, ny));
        sym[e] = to_sel(jin ? sel_lo(j, ny, MASK, B, nyl) : 0);
        syp[e] = to_sel(jin ? sel_hi(j, ny, MASK, B, nyh) : 0);
    }
    const int jo = y0 + TRO;
    const bool ook = !MID && xin && jo >= 0 && jo < ny;
    const unsigned ooff = offy(ic, clampi(jo, ny));
    const int lown = lidx(trow(0), cx);
    // the rows next to the held ones (held by the waves above and below)
    const int linU = lidx(r0 - 1, cx), linD = lidx(r0 + E, cx);

    // Halo lanes: group hg (1..H) of each side holds the column hg out, lane he
    // of the group held row he. hlev: the last level computed at that point.
    const bool hside = lane >= 32;
    const int hsl = lane & 31, hg = hsl / L::GS + 1, he = hsl % L::GS;
    const int eh = min(he, E - 1);
    const bool hwave = hside ? xw == NXW - 1 : xw == 0;
    const bool hact = hwave && hg <= H && he < E;
    const int hcol = hside ? L::X - 1 + hg : -hg;
    const int hnear = hside ? hcol - 1 : hcol + 1;      // towards the tile
    const int hfarc = hside ? hcol + 1 : hcol - 1;      // away from it
    const int hi = x0 + hcol, hfi = x0 + hfarc;
    const int hj = y0 + trow(eh);
    const bool hrow = hj >= 0 && hj < ny;
    const bool hload = hact && hrow && hi >= 0 && hi < nx;
    const int hyd = TOP ? (eh < H ? H - eh : 0) : (BOT ? (eh >= PR ? eh - PR + 1 : 0) : 0);
    const int hlev = hact ? H - hg - hyd : -1;
    const bool fload = hact && hg == H && hrow && hfi >= 0 && hfi < nx; // y one column further out
    const unsigned hoff = off(clampi(hi, nx), clampi(hj, ny));
    const unsigned hoffy = offy(clampi(hi, nx), clampi(hj, ny));
    const unsigned foff = offy(clampi(hfi, nx), clampi(hj, ny));
    const int lhself = lidx(trow(eh), hcol);
    const int lhnear = lidx(trow(eh), hnear);
    const int lhfar = hg < H ? lidx(trow(eh), hfarc) : lhself;
    const int lhup = lidx(max(trow(eh) - 1, -H), hcol);
    const int lhdn = lidx(min(trow(eh) + 1, L::Y + H - 1), hcol);
    const Sel csxl = to_sel(hload ? sel_lo(hi, nx, MASK, B, nxl) : 0);
    const Sel csxh = to_sel(hload ? sel_hi(hi, nx, MASK, B, nxh) : 0);
    const Sel csyl = to_sel(hload ? sel_lo(hj, ny, MASK, B, nyl) : 0);
    const Sel csyh = to_sel(hload ? sel_hi(hj, ny, MASK, B, nyh) : 0);

    // A u at one point from the centre and its six neighbours (in the order x-,
    // x+, y-, y+, z-, z+), then the Chebyshev update
    auto lap = [&](T c, T xm, T xp, T ym, T yp, T zm, T zp, Sel szl, Sel szh, Sel sxl, Sel sxh,
                   Sel syl, Sel syh) {
        if constexpr (!SIMPLE) {
            const T xm0 = xm, ym0 = ym, zm0 = zm;
            xm = pick(sxl, xm0, xp), xp = pick(sxh, xp, xm0);
            ym = pick(syl, ym0, yp), yp = pick(syh, yp, ym0);
            zm = pick(szl, zm0, zp), zp = pick(szh, zp, zm0);
        }
        return lap7<T>(c, xm, xp, ym, yp, zm, zp, ih2);
    };
    auto step = [&](T rc, T ro, T c, T xm, T xp, T ym, T yp, T zm, T zp, T v, T z, Sel szl,
                    Sel szh, Sel sxl, Sel sxh, Sel syl, Sel syh) {
        const T a = lap(c, xm, xp, ym, yp, zm, zp, szl, szh, sxl, sxh, syl, syh);
        return rc * ((ts * c + tod * (v - a)) - ro * z);
    };
    // level 0: step i (the first step's formula when FIRST)
    auto step0 = [&](T c, T xm, T xp, T ym, T yp, T zm, T zp, T v, T z, Sel szl, Sel szh, Sel sxl,
                     Sel sxh, Sel syl, Sel syh) {
        const T a = lap(c, xm, xp, ym, yp, zm, zp, szl, szh, sxl, sxh, syl, syh);
        if constexpr (FIRST) return c1 * ((T)2 * c - a / theta);
        else return rcs[0] * ((ts * c + tod * (v - a)) - ros[0] * z);
    };

    struct RawY {
        TU y[E], yo, he;
        TU uy[NUA][E], uyo[NUA], uhe[NUA];
    };
    struct RawV {
        T v[E], z[E], hv, hz;
        TU hf, uhf[NUA];
    };
    // the folded update's extra operands of plane p; in the plane loop they are
    // issued after level 0, so fewer loads are in flight across its arithmetic
    auto issueU = [&](int p, RawY &R) {
        const size_t pb = (size_t)clampi(p, nz) * PBY;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const char *Up = Ub[u] + pb;
#pragma unroll
            for (int e = 0; e < E; ++e) R.uy[u][e] = ldy(Up, ryoff[e]);
            if constexpr (!MID) R.uyo[u] = ldy(Up, ooff);
            else R.uyo[u] = (TU)0;
            R.uhe[u] = ldy(Up, hoffy);
        }
    };
    auto issueY = [&](int p, RawY &R, bool extra) {
        const size_t pb = (size_t)clampi(p, nz) * PBY;
        const char *Yp = Yb + pb;
#pragma unroll
        for (int e = 0; e < E; ++e) R.y[e] = ldy(Yp, ryoff[e]);
        if constexpr (!MID) R.yo = ldy(Yp, ooff);
        else R.yo = (TU)0;
        R.he = ldy(Yp, hoffy);
        if (extra) issueU(p, R);
    };
    auto gy = [&](const RawY &R, int e) { return comb(R.y[e], R.uy[0][e], R.uy[NUA - 1][e]); };
    auto gyo = [&](const RawY &R) { return comb(R.yo, R.uyo[0], R.uyo[NUA - 1]); };
    auto ghe = [&](const RawY &R) { return comb(R.he, R.uhe[0], R.uhe[NUA - 1]); };
    auto issueV = [&](int p, RawV &R) {
        const size_t po = (size_t)clampi(p, nz) * PB;
        if constexpr (!FIRST) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                R.v[e] = ld(Vb + po, roff[e]);
                R.z[e] = ld(Zb + po, roff[e]);
            }
            R.hv = ld(Vb + po, hoff);
            R.hz = ld(Zb + po, hoff);
        }
        R.hf = ldy(Yb + (size_t)clampi(p, nz) * PBY, foff);
#pragma unroll
        for (int u = 0; u < NU; ++u) R.uhf[u] = ldy(Ub[u] + (size_t)clampi(p, nz) * PBY, foff);
    };
    auto ghf = [&](const RawV &R) { return comb(R.hf, R.uhf[0], R.uhf[NUA - 1]); };
    // f = 0: y; f = l + 1: the output of level l (l < H)
    auto buf = [&](int f, int k) { return lds + (2 * f + (k & 1)) * L::PLANE; };

    // registers across planes (k = the plane of level 0): y at k-1 (ya); the
    // output of level l at plane k-l-2 (pv[l], for l < H), which the level
    // after it reads below its centre and level l+2 reads as its z; v at planes
    // k-1 .. k-H (vl[l-1] is the v of level l; a first pass carries its input
    // there); the same at the halo point (ha, hpv, hvl); the outer row (yob)
    T ya[E], pv[H][E], vl[H][E];
    T yob, ha, hpv[H], hvl[H];
    RawY RY;
    RawV RV;
#pragma unroll
    for (int e = 0; e < E; ++e) RV.v[e] = RV.z[e] = (T)0;
    RV.hv = RV.hz = (T)0;
    {
        RawY t;
        issueY(k0 - H - 1, t, true);
        {
            const bool pin = k0 - H - 1 >= 0;
#pragma unroll
            for (int e = 0; e < E; ++e) ya[e] = (pin && rok[e]) ? (T)gy(t, e) : (T)0;
            ha = (pin && hload) ? (T)ghe(t) : (T)0;
        }
        issueY(k0 - H, t, true);
        {
            const bool pin = k0 - H >= 0;
            T *yd = buf(0, k0 - H);
#pragma unroll
            for (int e = 0; e < E; ++e) yd[lown + e * L::PW] = (pin && rok[e]) ? (T)gy(t, e) : (T)0;
            yob = (pin && ook) ? (T)gyo(t) : (T)0;
            if (hact) yd[lhself] = (pin && hload) ? (T)ghe(t) : (T)0;
        }
    }
#pragma unroll
    for (int l = 0; l < H; ++l) {
#pragma unroll
        for (int e = 0; e < E; ++e) pv[l][e] = vl[l][e] = (T)0;
        hpv[l] = hvl[l] = (T)0;
    }
    issueY(k0 - H + 1, RY, true);
    issueV(k0 - H, RV);
    __syncthreads();

    for (int k = k0 - H; k <= k1 + H - 1; ++k) {
        const bool pin1 = inz(k + 1), pin0 = inz(k);
        // take y at plane k+1, publish it, issue plane k+2
        T yc[E];
        TU vn[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            vn[e] = gy(RY, e);
            yc[e] = (pin1 && rok[e]) ? (T)vn[e] : (T)0;
        }
        const T yoc = (pin1 && ook) ? (T)gyo(RY) : (T)0;
        const T hc = (pin1 && hload) ? (T)ghe(RY) : (T)0;
        if constexpr (UPD != 0) {
            if (k + 1 >= k0 && k + 1 < k1 && !ufirst) {
                const size_t po = (size_t)(k + 1) * PBY;
#pragma unroll
                for (int e = EOWN; e < EOWN + PR; ++e)
                    if (rok[e]) {
                        st_nt((TU *)(Ob + po + ryoff[e]), vn[e]);
                        if constexpr (UPD == U_S) dd_acc(ssh, ssl, (double)vn[e], (double)vn[e]);
                    }
            }
        }
        {
            T *yd = buf(0, k + 1);
#pragma unroll
            for (int e = 0; e < E; ++e) yd[lown + e * L::PW] = yc[e];
            if (hact) yd[lhself] = hc;
        }
        issueY(k + 2, RY, false);

        // level 0 at plane k on every held row
        const T *ys = buf(0, k);
        T cur[H][E], hcur[H];
        T vc[E], ycen[E];
        T hb, hv;
        {
            const Sel s0m = to_sel(pin0 ? sel_lo(k, nz, MASK, B, nzl) : 0);
            const Sel s0p = to_sel(pin0 ? sel_hi(k, nz, MASK, B, nzh) : 0);
            T inU = (T)0, inD = (T)0;
            if constexpr (TOP) inU = yob; else inU = ys[linU];
            if constexpr (BOT) inD = yob; else inD = ys[linD];
#pragma unroll
            for (int e = 0; e < E; ++e) ycen[e] = ys[lown + e * L::PW];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const T c = ycen[e];
                // x neighbours from the LDS plane, which holds every column of the
                // tile and its halo
                const T xm = ys[lown - 1 + e * L::PW], xp = ys[lown + 1 + e * L::PW];
                const T ym = e == 0 ? inU : ycen[e > 0 ? e - 1 : 0];
                const T yp = e == E - 1 ? inD : ycen[e < E - 1 ? e + 1 : e];
                const bool ok = pin0 && rok[e];
                const T v = FIRST ? c : (ok ? RV.v[e] : (T)0);
                const T z = (!FIRST && ok) ? RV.z[e] : (T)0;
                vc[e] = v;
                const T w = step0(c, xm, xp, ym, yp, ya[e], yc[e], v, z, s0m, s0p, sxm, sxp, sym[e],
                                  syp[e]);
                cur[0][e] = ok ? w : (T)0;
            }
            // level 0 at the halo point
            hb = ys[lhself];
            const T xn = ys[lhnear], d = ys[lhup], u = ys[lhdn];
            const T xf = hg == H ? ((fload && pin0) ? (T)ghf(RV) : (T)0) : ys[lhfar];
            const bool ok = hload && pin0 && hlev >= 0;
            hv = FIRST ? hb : ((hload && pin0) ? RV.hv : (T)0);
            const T hz = (!FIRST && ok) ? RV.hz : (T)0;
            const T lft = hside ? xn : xf, rgt = hside ? xf : xn;
            const T w = step0(hb, lft, rgt, d, u, ha, hc, hv, hz, s0m, s0p, csxl, csxh, csyl, csyh);
            hcur[0] = ok ? w : (T)0;
        }
        {
            T *wd = buf(1, k);
#pragma unroll
            for (int e = 0; e < E; ++e) wd[lown + e * L::PW] = cur[0][e];
            if (hact && hlev >= 0) wd[lhself] = hcur[0];
        }
        issueV(k + 1, RV);
        issueU(k + 2, RY);

        // levels 1..H: level l at plane k-l from the output of level l-1 at
        // planes k-l-1 (pv), k-l (LDS, written in the iteration before) and
        // k-l+1 (this iteration)
        T cen[H][E], hcen[H];
#pragma unroll
        for (int l = 1; l <= H; ++l) {
            const int lc = l < H ? l : 0;          // index of this level's output (l < H)
            const int p = k - l;
            const T *ws = buf(l, p);
#pragma unroll
            for (int e = 0; e < E; ++e) cen[l - 1][e] = ws[lown + e * L::PW];
            hcen[l - 1] = ws[lhself];
            if (l < H) {
#pragma unroll
                for (int e = 0; e < E; ++e) cur[lc][e] = (T)0;
                hcur[lc] = (T)0;
            }
            if (k < k0 - H + 2 * l) continue;     // level l runs on planes k0-(H-l) .. k1-1+(H-l)
            const bool pinp = inz(p);
            const Sel slm = to_sel(pinp ? sel_lo(p, nz, MASK, B, nzl) : 0);
            const Sel slp = to_sel(pinp ? sel_hi(p, nz, MASK, B, nzh) : 0);
            T inU = (T)0, inD = (T)0;
            if constexpr (!TOP) inU = ws[linU];
            if constexpr (!BOT) inD = ws[linD];
            const size_t po = (size_t)p * PB;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (ydist(e) > H - l) continue;
                const T c = cen[l - 1][e];
                const T xm = ws[lown - 1 + e * L::PW], xp = ws[lown + 1 + e * L::PW];
                const T ym = e == 0 ? inU : cen[l - 1][e > 0 ? e - 1 : 0];
                const T yp = e == E - 1 ? inD : cen[l - 1][e < E - 1 ? e + 1 : e];
                const T v = vl[l - 1][e];
                // z: y_{i-1} at plane k-1 for level 1 (v / theta in a first pass),
                // else the output of level l-2 at plane k-l
                const T z = l == 1 ? (FIRST ? v / theta : ya[e]) : pv[l >= 2 ? l - 2 : 0][e];
                const T w = step(rcs[l], ros[l], c, xm, xp, ym, yp, pv[l - 1][e], cur[l - 1][e], v, z,
                                 slm, slp, sxm, sxp, sym[e], syp[e]);
                if (l < H) {
                    cur[lc][e] = (pinp && rok[e]) ? w : (T)0;
                } else if (rok[e]) {
                    if constexpr (!DROP) st_nt((T *)(W1b + po + roff[e]), c);
                    st_nt((T *)(W2b + po + roff[e]), w);
                    // the FP32 copy of v for later passes (there are none after a
                    // first pass that ends the apply)
                    if constexpr (FIRST && !DROP && sizeof(T) == 4)
                        st_nt((T *)(V32b + po + roff[e]), v);
                }
            }
            if (l < H) {
                // level l at the halo point, where hlev >= l
                const T c = hcen[l - 1];
                const T xn = ws[lhnear], xf = ws[lhfar], d = ws[lhup], u = ws[lhdn];
                const T lft = hside ? xn : xf, rgt = hside ? xf : xn;
                const T v = hvl[l - 1];
                const T z = l == 1 ? (FIRST ? v / theta : ha) : hpv[l >= 2 ? l - 2 : 0];
                const T w = step(rcs[l], ros[l], c, lft, rgt, d, u, hpv[l - 1], hcur[l - 1], v, z, slm,
                                 slp, csxl, csxh, csyl, csyh);
                hcur[lc] = (hload && pinp && hlev >= l) ? w : (T)0;
                T *wd = buf(l + 1, p);
#pragma unroll
                for (int e = 0; e < E; ++e)
                    if (ydist(e) <= H - l) wd[lown + e * L::PW] = cur[lc][e];
                if (hact && hlev >= l) wd[lhself] = hcur[lc];
            }
        }
        // rotate: y at plane k, the levels' outputs read as centres, v
#pragma unroll
        for (int e = 0; e < E; ++e) {
            ya[e] = ycen[e];
#pragma unroll
            for (int l = 0; l < H; ++l) pv[l][e] = cen[l][e];
#pragma unroll
            for (int l = H - 1; l > 0; --l) vl[l][e] = vl[l - 1][e];
            vl[0][e] = vc[e];
        }
        yob = yoc;
        ha = hb;
#pragma unroll
        for (int l = 0; l < H; ++l) hpv[l] = hcen[l];
#pragma unroll
        for (int l = H - 1; l > 0; --l) hvl[l] = hvl[l - 1];
        hvl[0] = hv;
        __syncthreads();
    }
}

// At most 256 VGPRs (two waves per SIMD)
template <typename T, typename TU, int S, bool FIRST, bool DROP, int NXW, int PR, int NYW, bool MASK,
          bool SIMPLE, int UPD = 0>
__global__ void __launch_bounds__(64 * NXW * NYW) __attribute__((amdgpu_waves_per_eu(2)))
k_cheb_steps_lds(Work W, KArgs A)
{
    using L = LSteps<NXW, PR, NYW, S>;
    __shared__ T lds[2 * S * L::PLANE];
    __shared__ double red[2 * NXW * NYW];
    constexpr int F32 = sizeof(T) == 4;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int xw = wv % NXW, yw = wv / NXW;
    // batched problems walk the four-step tile list; a single problem all its
    // tiles. A skipped tile is skipped by the whole workgroup, so every wave runs
    // the same barriers
    int total;
    if (W.quad_prob) {
        total = *W.quad_count_dev;
    } else {
        const Prob &P = W.probs[0];
        const int qkz = P.qkz[F32];
        if (qkz < 1) return;
        const int ltx = (P.nx + L::X - 1) / L::X, lty = (P.ny + L::Y - 1) / L::Y;
        total = ltx * lty * ((P.nz + qkz - 1) / qkz);
    }
    for (int g = blockIdx.x; g < total; g += gridDim.x) {
        const Prob &P = W.probs[W.quad_prob ? W.quad_prob[g] : 0];
        if (P.qkz[F32] < 1) continue;
        {
            const Scalars *sc = P.sc;
            if (sc->done || (A.second && sc->half_pending)) continue;
        }
        // a single problem's tiles in slabs by default, as for the triples
        const int ltx = (P.nx + L::X - 1) / L::X;
        const int t = W.quad_prob ? W.quad_local[g] : tile_order_tx(W.order ? W.order : 2, ltx, g, total);
        double ssh = 0.0, ssl = 0.0;
        if (yw == 0)
            cheb_steps_lds_tile<T, TU, S, FIRST, DROP, NXW, PR, NYW, R_TOP, MASK, SIMPLE, UPD>(
                P, A, t, lane, xw, yw, lds, ssh, ssl);
        else if (yw == NYW - 1)
            cheb_steps_lds_tile<T, TU, S, FIRST, DROP, NXW, PR, NYW, R_BOT, MASK, SIMPLE, UPD>(
                P, A, t, lane, xw, yw, lds, ssh, ssl);
        else if constexpr (NYW > 2)
            cheb_steps_lds_tile<T, TU, S, FIRST, DROP, NXW, PR, NYW, R_MID, MASK, SIMPLE, UPD>(
                P, A, t, lane, xw, yw, lds, ssh, ssl);
        if constexpr (UPD == U_S) {
            double hh[1] = {ssh}, ll[1] = {ssl};
            block_reduce_dd<1, NXW * NYW>(hh, ll, red);
            if (threadIdx.x == 0) {
                double *pp = P.partials + (size_t)t * PARTIAL_STRIDE;
                pp[0] = hh[0];
                pp[1] = ll[0];
            }
        }
    }
}

// One tile of an elementwise pass for the lanes inside the grid (i < nx);
// FULL: all RY rows of the wave are inside, so no row guard remains and the
// loads of a plane issue together.
template <int OP, typename TP, bool FULL>
__device__ __forceinline__ void elem_tile(const Prob &P, const KArgs &A, const Scalars *sc,
                                          bool half, int i, int j0, int k0, int k1,
                                          double (&hi)[2], double (&lo)[2])
{
    const int nx = P.nx, ny = P.ny;
    const size_t S = (size_t)nx * (size_t)ny, NXs = (size_t)nx;
    size_t base = (size_t)i + NXs * ((size_t)j0 + (size_t)ny * (size_t)k0);
    bool rin[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) rin[r] = FULL || j0 + r < ny;
    const double alpha = sc->alpha, omega = sc->omega, beta = sc->beta;
    for (int k = k0; k < k1; ++k, base += S) {
        if constexpr (OP == E_AXPY) {
            double *r_ = (double *)P.vec[V_R];
            const double *__restrict__ w = (const double *)P.vec[V_W];
            double a[RY], b[RY];
#pragma unroll
            for (int r = 0; r < RY; ++r)
                if (rin[r]) { a[r] = ld_nt(r_ + base + r * NXs); b[r] = ld_nt(w + base + r * NXs); }
#pragma unroll
            for (int r = 0; r < RY; ++r)
                if (rin[r]) {
                    const double s = a[r] - alpha * b[r];
                    st_nt(r_ + base + r * NXs, s);
                    dd_acc(hi[0], lo[0], s, s);
                }
        } else if constexpr (OP == E_UPD) {
            double *x = (double *)P.vec[V_X];
            const TP *ph = (const TP *)P.vec[A.in];
            const TP *sh = (const TP *)P.vec[A.x2];
            double *r_ = (double *)P.vec[V_R];
            const double *s_ = (const double *)P.vec[P.s_slot];
            const double *__restrict__ tv = (const double *)P.vec[V_T];
            const double *__restrict__ rt = (const double *)P.vec[V_RT];
            double xv[RY], pv[RY];
#pragma unroll
            for (int r = 0; r < RY; ++r)
                if (rin[r]) { xv[r] = ld_nt(x + base + r * NXs); pv[r] = (double)ld_nt(ph + base + r * NXs); }
            if (half) {
#pragma unroll
                for (int r = 0; r < RY; ++r)
                    if (rin[r]) st_nt(x + base + r * NXs, xv[r] + alpha * pv[r]);
            } else {
                double sv[RY], shv[RY], tt[RY], rtv[RY];
#pragma unroll
                for (int r = 0; r < RY; ++r)
                    if (rin[r]) {
                        const size_t idx = base + r * NXs;
                        sv[r] = ld_nt(s_ + idx);
                        shv[r] = (double)ld_nt(sh + idx);
                        tt[r] = ld_nt(tv + idx);
                        rtv[r] = ld_nt(rt + idx);
                    }
#pragma unroll
                for (int r = 0; r < RY; ++r)
                    if (rin[r]) {
                        const size_t idx = base + r * NXs;
                        st_nt(x + idx, (xv[r] + alpha * pv[r]) + omega * shv[r]);
                        const double rn = sv[r] - omega * tt[r];
                        st_nt(r_ + idx, rn);
                        dd_acc(hi[0], lo[0], rtv[r], rn);
                        dd_acc(hi[1], lo[1], rn, rn);
                    }
            }
        } else if constexpr (OP == E_PUPD) {
            double *p = (double *)P.vec[V_P];
            const double *__restrict__ r_ = (const double *)P.vec[V_R];
            const double *__restrict__ w = (const double *)P.vec[V_W];
            double a[RY], b[RY], c[RY];
#pragma unroll
            for (int r = 0; r < RY; ++r)
                if (rin[r]) {
                    const size_t idx = base + r * NXs;
                    a[r] = ld_nt(r_ + idx);
                    b[r] = ld_nt(p + idx);
                    c[r] = ld_nt(w + idx);
                }
#pragma unroll
            for (int r = 0; r < RY; ++r)
                if (rin[r]) st_nt(p + base + r * NXs, a[r] + beta * (b[r] - omega * c[r]));
        } else if constexpr (OP == E_DIV) {
            const double *__restrict__ v = (const double *)P.vec[A.in];
            TP *out = (TP *)P.vec[A.out];
            const TP d = A.divisor ? Coef<TP>::theta(P) : Coef<TP>::jac(P);
            double a[RY];
#pragma unroll
            for (int r = 0; r < RY; ++r)
                if (rin[r]) a[r] = ld_nt(v + base + r * NXs);
#pragma unroll
            for (int r = 0; r < RY; ++r)
                if (rin[r]) st_nt(out + base + r * NXs, (TP)a[r] / d);
        } else if constexpr (OP == E_DOT) {
            const double *__restrict__ xv = (const double *)P.vec[A.in];
            const double *__restrict__ yv = (const double *)P.vec[A.x2];
            double a[RY], b[RY];
#pragma unroll
            for (int r = 0; r < RY; ++r)
                if (rin[r]) { a[r] = ld_nt(xv + base + r * NXs); b[r] = ld_nt(yv + base + r * NXs); }
#pragma unroll
            for (int r = 0; r < RY; ++r)
                if (rin[r]) dd_acc(hi[0], lo[0], a[r], b[r]);
        }
    }
}

// ------------------------------------------------------------------------
// elementwise family, same tiles; each thread streams its RY rows plane by
// plane with all loads of a plane issued together.
// TP: element type of p^ / s^ (E_UPD) or of the output (E_DIV).
// ------------------------------------------------------------------------
template <int OP, typename TP>
__global__ void __launch_bounds__(NTHREADS) k_elem(Work W, KArgs A)
{
    constexpr int ND = OP == E_UPD ? 2 : (OP == E_AXPY || OP == E_DOT) ? 1 : 0;
    constexpr int NA = ND > 0 ? ND : 1;
    __shared__ double lds[TY * 2 * 2];
    const int total = W.count_dev ? *W.count_dev : W.count;
    const int lane = threadIdx.x & (TX - 1), wv = threadIdx.x / TX;

    for (int g = blockIdx.x; g < total; g += gridDim.x) {
        const int pid = W.tile_prob ? W.tile_prob[g] : 0;
        const Prob &P = W.probs[pid];
        const int local = W.tile_prob ? W.tile_local[g] : tile_order(W.order, W, P, g, total);
        const Scalars *sc = P.sc;
        if (OP != E_DOT) {
            if (sc->done || (A.second && sc->half_pending)) continue;
        }
        const bool half = OP == E_UPD && sc->half_pending;
        const int nx = P.nx, ny = P.ny, nz = P.nz, tx = P.tx, ty = P.ty;
        const int tix = local % tx, tiy = (local / tx) % ty, tiz = local / (tx * ty);
        const int i = tix * TX + lane;
        const int j0 = tiy * (TY * RY) + wv * RY;
        const int k0 = tiz * P.kz, k1 = min(k0 + P.kz, nz);
        double hi[NA], lo[NA];
#pragma unroll
        for (int d = 0; d < NA; ++d) hi[d] = lo[d] = 0.0;

        if (j0 < ny && i < nx) {
            double h2[2] = {0.0, 0.0}, l2[2] = {0.0, 0.0};
            if (j0 + RY <= ny) elem_tile<OP, TP, true>(P, A, sc, half, i, j0, k0, k1, h2, l2);
            else elem_tile<OP, TP, false>(P, A, sc, half, i, j0, k0, k1, h2, l2);
#pragma unroll
            for (int d = 0; d < NA; ++d) hi[d] = h2[d], lo[d] = l2[d];
        }
        if constexpr (ND > 0) tile_publish<NA>(P, local, hi, lo, lds);
    }
}
// ------------------------------------------------------------------------
// synthetic right-hand sides: counter-based splitmix64
// ------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__global__ void k_fill_uniform(double *out, int64_t n, uint64_t key)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t v = mix64(key + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ULL);
        const double u = (double)(v >> 11) * 0x1.0p-53;
        out[i] = 2.0 * u - 1.0;
    }
}

// ------------------------------------------------------------------------
// Scalar epilogue of a reduction: one workgroup per problem sums the problem's
// tile partials in tile order and updates its scalars (alpha, omega, beta, rho,
// the stopping tests). Launched right after the reduction kernel, with the same
// arguments, so it sees the same flags and skips the same problems.
// ------------------------------------------------------------------------
enum Fin { F_SDOT, F_SDOT2, F_INIT, F_TRUE, F_AXPY, F_UPD, F_DOT };

template <int F>
__global__ void __launch_bounds__(NTHREADS) k_finalize(Work W, KArgs A)
{
    constexpr int ND = (F == F_SDOT2 || F == F_INIT || F == F_UPD) ? 2 : 1;
    constexpr bool SKIPS = F == F_SDOT || F == F_SDOT2 || F == F_AXPY || F == F_UPD;
    __shared__ double lds[TY * 2 * 2];
    const bool single = W.tile_prob == nullptr;
    const int total = single ? 1 : (W.count_dev ? *W.count_dev : W.count);
    for (int g = blockIdx.x; g < total; g += gridDim.x) {
        int pid = 0;
        if (!single) {
            if (W.tile_local[g] != 0) continue; // one entry per problem: its first tile
            pid = W.tile_prob[g];
        }
        const Prob &P = W.probs[pid];
        if constexpr (SKIPS) {
            const Scalars *sc = P.sc;
            if (sc->done || (A.second && sc->half_pending)) continue;
        }
        double res[ND];
        // s.s of a formed s sits in the partials of the first pass's tiles
        const int np = A.nparts > 0 ? A.nparts
                                    : ((F == F_AXPY && P.nparts_first > 0) ? P.nparts_first : P.ntiles);
        sum_partials<ND>(P, np, lds, res);
        if (threadIdx.x == 0) {
            if constexpr (F == F_SDOT) fin_sdot(P, res[0]);
            else if constexpr (F == F_SDOT2) fin_sdot2(P, res[0], res[1]);
            else if constexpr (F == F_INIT) fin_init(P, res[0], res[1]);
            else if constexpr (F == F_TRUE) P.sc->rr_true = res[0];
            else if constexpr (F == F_AXPY) fin_axpy(P, res[0]);
            else if constexpr (F == F_UPD) fin_upd(P, res[0], res[1]);
            else if constexpr (F == F_DOT) P.sc->dot = res[0];
        }
        __syncthreads(); // lds is reused by the next problem
    }
}

template <int F>
static void lfin(const Work &w, int grid, hipStream_t s, const KArgs &a)
{
    const int g = w.tile_prob ? grid : 1;
    hipLaunchKernelGGL((k_finalize<F>), dim3(g), dim3(NTHREADS), 0, s, w, a);
}

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
template <int OP, typename TU, typename TC, bool M>
static void ls(const Work &w, int grid, hipStream_t s, const KArgs &a)
{
    hipLaunchKernelGGL((k_stencil<OP, TU, TC, M>), dim3(grid), dim3(NTHREADS), 0, s, w, a);
}

template <int OP, typename TU, typename TC>
static void ls_mask(bool mask, const Work &w, int grid, hipStream_t s, const KArgs &a)
{
    if (mask) ls<OP, TU, TC, true>(w, grid, s, a);
    else ls<OP, TU, TC, false>(w, grid, s, a);
}

template <int OP, typename TU>
static void lf2_mask(bool mask, const Work &w, int grid, hipStream_t s, const KArgs &a)
{
    if (mask)
        hipLaunchKernelGGL((k_cheb_f32x2<OP, TU, true>), dim3(grid), dim3(NTHREADS), 0, s, w, a);
    else
        hipLaunchKernelGGL((k_cheb_f32x2<OP, TU, false>), dim3(grid), dim3(NTHREADS), 0, s, w, a);
}

// the LDS-staged pair: the last pair of an apply (drop1) and the block mask are
// kernels of their own, and so is the select-free body of all-Dirichlet grids
template <typename T, typename TU, bool FIRST, bool DROP, int NXW, bool MASK, bool SIMPLE>
static void lpl_launch(const Work &w, int grid, hipStream_t s, const KArgs &a)
{
    constexpr int PPR = pair_pr(sizeof(T) == 4), PNYW = pair_nyw(sizeof(T) == 4);
    if constexpr (FIRST) {
        // a folded vector update: single problems only (the server keeps the
        // standalone update kernels)
        if (a.upd == U_S) {
            hipLaunchKernelGGL((k_cheb_pair_lds<T, TU, true, DROP, NXW, PPR, PNYW, MASK, SIMPLE, U_S>),
                               dim3(grid), dim3(LPair<NXW, PPR, PNYW>::NT), 0, s, w, a);
            return;
        }
        if (a.upd == U_P) {
            hipLaunchKernelGGL((k_cheb_pair_lds<T, TU, true, DROP, NXW, PPR, PNYW, MASK, SIMPLE, U_P>),
                               dim3(grid), dim3(LPair<NXW, PPR, PNYW>::NT), 0, s, w, a);
            return;
        }
    }
    hipLaunchKernelGGL((k_cheb_pair_lds<T, TU, FIRST, DROP, NXW, PPR, PNYW, MASK, SIMPLE>), dim3(grid),
                       dim3(LPair<NXW, PPR, PNYW>::NT), 0, s, w, a);
}

template <typename T, typename TU, bool FIRST, bool DROP, int NXW>
static void lpl_drop(bool mask, const Work &w, int grid, hipStream_t s, const KArgs &a)
{
    if (mask) lpl_launch<T, TU, FIRST, DROP, NXW, true, false>(w, grid, s, a);
    else if (w.neumann) lpl_launch<T, TU, FIRST, DROP, NXW, false, false>(w, grid, s, a);
    else lpl_launch<T, TU, FIRST, DROP, NXW, false, true>(w, grid, s, a);
}

// grid: one workgroup per tile for a single problem; for batched problems the
// caller's persistent grid over the pair tile list
template <typename T, typename TU, bool FIRST, int NXW>
static void lpl(bool mask, const Work &w, int grid, hipStream_t s, const KArgs &a)
{
    if constexpr (!FIRST) {
        if (a.drop1) {
            lpl_drop<T, TU, false, true, NXW>(mask, w, grid, s, a);
            return;
        }
    }
    lpl_drop<T, TU, FIRST, false, NXW>(mask, w, grid, s, a);
}

template <typename T, typename TU, bool FIRST>
static void lp(bool mask, const Work &w, int grid, hipStream_t s, const KArgs &a)
{
    constexpr bool F32 = sizeof(T) == 4;
    constexpr int NXW = pair_nxw(F32);
    if (w.pair_prob) {
        lpl<T, TU, FIRST, NXW>(mask, w, grid, s, a);
        return;
    }
    if (!w.tile_prob && w.pair_tiles[F32] > 0) {
        lpl<T, TU, FIRST, NXW>(mask, w, w.pair_tiles[F32], s, a);
        return;
    }
    if (mask) hipLaunchKernelGGL((k_cheb_pair<T, TU, true, FIRST>), dim3(grid), dim3(NTHREADS), 0, s, w, a);
    else hipLaunchKernelGGL((k_cheb_pair<T, TU, false, FIRST>), dim3(grid), dim3(NTHREADS), 0, s, w, a);
}

void launch_cheb_pair(bool mixed, bool mask, const Work &w, int grid, hipStream_t s, const KArgs &a)
{
    if (mixed) lp<float, float, false>(mask, w, grid, s, a);
    else lp<double, double, false>(mask, w, grid, s, a);
}

template <typename T, typename TU, bool FIRST, bool DROP, bool MASK, bool SIMPLE>
static void ltr_launch(const Work &w, hipStream_t s, const KArgs &a)
{
    constexpr bool F32 = sizeof(T) == 4;
    constexpr int NXW = triple_nxw(F32), PR = triple_pr(F32), NYW = triple_nyw(F32);
    if constexpr (FIRST) {
        if (a.upd == U_S) {
            hipLaunchKernelGGL((k_cheb_triple_lds<T, TU, true, DROP, NXW, PR, NYW, MASK, SIMPLE, U_S>),
                               dim3(w.triple_tiles[F32]), dim3(LTriple<NXW, PR, NYW>::NT), 0, s, w, a);
            return;
        }
        if (a.upd == U_P) {
            hipLaunchKernelGGL((k_cheb_triple_lds<T, TU, true, DROP, NXW, PR, NYW, MASK, SIMPLE, U_P>),
                               dim3(w.triple_tiles[F32]), dim3(LTriple<NXW, PR, NYW>::NT), 0, s, w, a);
            return;
        }
    }
    hipLaunchKernelGGL((k_cheb_triple_lds<T, TU, FIRST, DROP, NXW, PR, NYW, MASK, SIMPLE>),
                       dim3(w.triple_tiles[F32]), dim3(LTriple<NXW, PR, NYW>::NT), 0, s, w, a);
}

template <typename T, typename TU, bool FIRST, bool DROP>
static void ltr_drop(bool mask, const Work &w, hipStream_t s, const KArgs &a)
{
    if (mask) ltr_launch<T, TU, FIRST, DROP, true, false>(w, s, a);
    else if (w.neumann) ltr_launch<T, TU, FIRST, DROP, false, false>(w, s, a);
    else ltr_launch<T, TU, FIRST, DROP, false, true>(w, s, a);
}

template <typename T>
static void ltr(bool mask, const Work &w, hipStream_t s, const KArgs &a)
{
    if (a.drop1) ltr_drop<T, T, false, true>(mask, w, s, a);
    else ltr_drop<T, T, false, false>(mask, w, s, a);
}

void launch_cheb_triple(bool mixed, bool mask, const Work &w, hipStream_t s, const KArgs &a)
{
    if (mixed) ltr<float>(mask, w, s, a);
    else ltr<double>(mask, w, s, a);
}

void launch_cheb_first_triple(bool mask, const Work &w, hipStream_t s, const KArgs &a)
{
    ltr_drop<float, double, true, false>(mask, w, s, a);
}

// the four-step pass (mixed mode): its own tiles, one workgroup per tile
template <typename T, typename TU, bool FIRST, bool DROP, bool MASK, bool SIMPLE>
static void lq_launch(const Work &w, int grid, hipStream_t s, const KArgs &a)
{
    constexpr bool F32 = sizeof(T) == 4;
    constexpr int NXW = quad_nxw(F32), PR = quad_pr(F32), NYW = quad_nyw(F32);
    const dim3 g(w.quad_prob ? grid : w.quad_tiles[F32]), b(LSteps<NXW, PR, NYW, 4>::NT);
    if constexpr (FIRST) {
        if (a.upd == U_S) {
            hipLaunchKernelGGL((k_cheb_steps_lds<T, TU, 4, true, DROP, NXW, PR, NYW, MASK, SIMPLE, U_S>),
                               g, b, 0, s, w, a);
            return;
        }
        if (a.upd == U_P) {
            hipLaunchKernelGGL((k_cheb_steps_lds<T, TU, 4, true, DROP, NXW, PR, NYW, MASK, SIMPLE, U_P>),
                               g, b, 0, s, w, a);
            return;
        }
    }
    hipLaunchKernelGGL((k_cheb_steps_lds<T, TU, 4, FIRST, DROP, NXW, PR, NYW, MASK, SIMPLE>), g, b, 0, s,
                       w, a);
}

template <typename T, typename TU, bool FIRST, bool DROP>
static void lq_drop(bool mask, const Work &w, int grid, hipStream_t s, const KArgs &a)
{
    if (mask) lq_launch<T, TU, FIRST, DROP, true, false>(w, grid, s, a);
    else if (w.neumann) lq_launch<T, TU, FIRST, DROP, false, false>(w, grid, s, a);
    else lq_launch<T, TU, FIRST, DROP, false, true>(w, grid, s, a);
}

void launch_cheb_quad(bool mixed, bool mask, const Work &w, int grid, hipStream_t s, const KArgs &a)
{
    if (mixed) {
        if (a.drop1) lq_drop<float, float, false, true>(mask, w, grid, s, a);
        else lq_drop<float, float, false, false>(mask, w, grid, s, a);
    } else {
        if (a.drop1) lq_drop<double, double, false, true>(mask, w, grid, s, a);
        else lq_drop<double, double, false, false>(mask, w, grid, s, a);
    }
}

void launch_cheb_first_quad(bool mixed, bool mask, const Work &w, int grid, hipStream_t s,
                            const KArgs &a)
{
    if (mixed) {
        if (a.drop1) lq_drop<float, double, true, true>(mask, w, grid, s, a);
        else lq_drop<float, double, true, false>(mask, w, grid, s, a);
    } else {
        if (a.drop1) lq_drop<double, double, true, true>(mask, w, grid, s, a);
        else lq_drop<double, double, true, false>(mask, w, grid, s, a);
    }
}

void launch_finalize_ss(const Work &w, int grid, hipStream_t s, const KArgs &a)
{
    lfin<F_AXPY>(w, grid, s, a);
}

void launch_cheb_first_pair(bool mixed, bool mask, const Work &w, int grid, hipStream_t s,
                            const KArgs &a)
{
    if (mixed) lp<float, double, true>(mask, w, grid, s, a);
    else lp<double, double, true>(mask, w, grid, s, a);
}

void launch_stencil(int op, bool mixed, bool mask, const Work &w, int grid, hipStream_t s,
                    const KArgs &a)
{
    switch (op) {
    case S_APPLY: ls<S_APPLY, double, double, false>(w, grid, s, a); break;
    case S_CHEB1:
        if (mixed) lf2_mask<S_CHEB1, double>(mask, w, grid, s, a);
        else ls_mask<S_CHEB1, double, double>(mask, w, grid, s, a);
        break;
    case S_CHEB2:
        if (mixed) lf2_mask<S_CHEB2, float>(mask, w, grid, s, a);
        else ls_mask<S_CHEB2, double, double>(mask, w, grid, s, a);
        break;
    case S_CHEBK:
        if (mixed) lf2_mask<S_CHEBK, float>(mask, w, grid, s, a);
        else ls_mask<S_CHEBK, double, double>(mask, w, grid, s, a);
        break;
    case S_SDOT:
        if (mixed) ls<S_SDOT, float, double, false>(w, grid, s, a);
        else ls<S_SDOT, double, double, false>(w, grid, s, a);
        lfin<F_SDOT>(w, grid, s, a);
        break;
    case S_SDOT2:
        if (mixed) ls<S_SDOT2, float, double, false>(w, grid, s, a);
        else ls<S_SDOT2, double, double, false>(w, grid, s, a);
        lfin<F_SDOT2>(w, grid, s, a);
        break;
    case S_INIT:
        ls<S_INIT, double, double, false>(w, grid, s, a);
        lfin<F_INIT>(w, grid, s, a);
        break;
    case S_TRUE:
        ls<S_TRUE, double, double, false>(w, grid, s, a);
        lfin<F_TRUE>(w, grid, s, a);
        break;
    default: break;
    }
}

template <int OP, typename TP>
static void le(const Work &w, int grid, hipStream_t s, const KArgs &a)
{
    hipLaunchKernelGGL((k_elem<OP, TP>), dim3(grid), dim3(NTHREADS), 0, s, w, a);
}

void launch_elem(int op, bool mixed, const Work &w, int grid, hipStream_t s, const KArgs &a)
{
    switch (op) {
    case E_AXPY:
        le<E_AXPY, double>(w, grid, s, a);
        lfin<F_AXPY>(w, grid, s, a);
        break;
    case E_UPD:
        if (mixed) le<E_UPD, float>(w, grid, s, a);
        else le<E_UPD, double>(w, grid, s, a);
        lfin<F_UPD>(w, grid, s, a);
        break;
    case E_PUPD: le<E_PUPD, double>(w, grid, s, a); break;
    case E_DIV:
        if (mixed) le<E_DIV, float>(w, grid, s, a);
        else le<E_DIV, double>(w, grid, s, a);
        break;
    case E_DOT:
        le<E_DOT, double>(w, grid, s, a);
        lfin<F_DOT>(w, grid, s, a);
        break;
    default: break;
    }
}

void launch_fill_uniform(double *out, int64_t n, uint64_t seed, hipStream_t s)
{
    uint64_t key = seed + 0x9E3779B97F4A7C15ULL;
    key = (key ^ (key >> 30)) * 0xBF58476D1CE4E5B9ULL;
    key = (key ^ (key >> 27)) * 0x94D049BB133111EBULL;
    key = key ^ (key >> 31);
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill_uniform, dim3((unsigned)blocks), dim3(256), 0, s, out, n, key);
}

} // namespace pz
