/*
 * oracle.c -- plain, slow, literal FP64 CPU oracle for the preconditioned
 * Bi-CGSTAB Poisson solver of Pennati et al., "A Parallel and Highly-Portable
 * HPC Poisson Solver: Preconditioned Bi-CGSTAB with alpaka" (arXiv 2503.08935).
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load this file's library. The GPU library neither links
 * nor calls it, and this file includes nothing from the GPU library.
 *
 * Conventions (shared by specification, not by code, with the GPU library):
 *   - unknowns are the interior nodes of an nx*ny*nz grid with one spacing h,
 *     stored x-fastest: idx = i + nx*(j + ny*k); zero Dirichlet boundary, so a
 *     neighbour outside the grid reads as +0.0;
 *   - no floating-point contraction (built with -ffp-contract=off, no fast-math);
 *   - every dot product is the exact sum of the exact products, rounded once to
 *     the nearest double (ties to even).
 *
 * What pins each function (tests/test_oracle_*.py):
 *   orc_dot          exact rational arithmetic on random and adversarial vectors
 *   orc_interval     dense eigenvalues of the Kronecker-sum matrix, n <= 8
 *   orc_apply_A      discrete sine modes (closed-form eigenvalues), dense
 *                    Kronecker assembly, exactness on tensor quadratics
 *   orc_chebyshev    closed-form Chebyshev residual polynomial on sine modes,
 *                    minimax spectral bound of A*M^-1 on dense matrices
 *   orc_chebyshev_f32  the same closed forms to FP32 accuracy
 *   orc_bicgstab     dense direct solves, finite termination on k eigenmodes,
 *                    manufactured solution and its O(h^2) error, power-of-two
 *                    Jacobi scaling identity
 *   *_bc variants    (Neumann faces, eq. matrix_neuman) dense assembly of the
 *                    one-sided matrices, dense non-symmetric eigenvalues,
 *                    cosine eigenmodes, dense solves with mixed faces
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_ERR_ARG (-1)
#define ORC_ERR_BREAKDOWN (-5)
#define ORC_ERR_NONFINITE (-6)

#define PC_NONE 0
#define PC_JACOBI 1
#define PC_CHEBYSHEV 2
#define PC_BLOCK_JACOBI 3

void orc_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int orc_get_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------- */
/* Exact dot product.                                                         */
/* A Kulisch-style long accumulator: value = sum_c cell[c] * 2^(32c - OFF).   */
/* Each product x*y of doubles is formed exactly as a 106-bit integer times a */
/* power of two and added digit by digit, so the sum is exact whatever the    */
/* order, and it is rounded to double once at the end.                        */
/* ------------------------------------------------------------------------- */
#define ACC_OFF 2176   /* 2^-2176 < smallest product 2^-2148 */
#define ACC_CELLS 140  /* top weight 2^(32*140-2176) = 2^2304 > largest sum */

typedef struct {
    int64_t c[ACC_CELLS];
    int64_t nadd;
    int nan, pinf, ninf;
} acc_t;

static void acc_init(acc_t *a) { memset(a, 0, sizeof(*a)); }

/* carry-propagate so every cell but the top one lies in [0, 2^32) */
static void acc_normalize(acc_t *a)
{
    int64_t carry = 0;
    for (int c = 0; c < ACC_CELLS - 1; ++c) {
        int64_t v = a->c[c] + carry;
        int64_t low = v & 0xffffffffLL;
        carry = (v - low) / 4294967296LL; /* exact: v - low is a multiple of 2^32 */
        a->c[c] = low;
    }
    a->c[ACC_CELLS - 1] += carry;
    a->nadd = 0;
}

/* split a finite double into sign, 53-bit integer significand and exponent */
static void split_double(double v, int *neg, uint64_t *m, int *e)
{
    uint64_t bits;
    memcpy(&bits, &v, 8);
    *neg = (int)(bits >> 63);
    int ef = (int)((bits >> 52) & 0x7ff);
    uint64_t frac = bits & ((1ULL << 52) - 1);
    if (ef == 0) { *m = frac; *e = -1074; }
    else { *m = frac | (1ULL << 52); *e = ef - 1075; }
}

static void acc_add_product(acc_t *a, double x, double y)
{
    if (!isfinite(x) || !isfinite(y)) {
        double p = x * y;
        if (isnan(p)) a->nan = 1;
        else if (p > 0) a->pinf = 1;
        else if (p < 0) a->ninf = 1;
        return;
    }
    if (x == 0.0 || y == 0.0) return;
    int nx_, ny_, ex, ey;
    uint64_t mx, my;
    split_double(x, &nx_, &mx, &ex);
    split_double(y, &ny_, &my, &ey);
    unsigned __int128 M = (unsigned __int128)mx * (unsigned __int128)my;
    int neg = nx_ ^ ny_;
    int P = ex + ey + ACC_OFF; /* bit position of M's least significant bit */
    int cell = P >> 5, sh = P & 31;
    for (int q = 0; q < 4; ++q) {
        uint64_t ch = (uint64_t)(M >> (32 * q)) & 0xffffffffULL;
        if (!ch) continue;
        uint64_t v = ch << sh; /* < 2^63 */
        int64_t lo = (int64_t)(v & 0xffffffffULL), hi = (int64_t)(v >> 32);
        if (neg) { a->c[cell + q] -= lo; a->c[cell + q + 1] -= hi; }
        else { a->c[cell + q] += lo; a->c[cell + q + 1] += hi; }
    }
    /* each cell gains < 2^33 per product: normalise long before 2^63 */
    if (++a->nadd >= (1LL << 28)) acc_normalize(a);
}

static void acc_merge(acc_t *dst, const acc_t *src)
{
    for (int c = 0; c < ACC_CELLS; ++c) dst->c[c] += src->c[c];
    dst->nan |= src->nan; dst->pinf |= src->pinf; dst->ninf |= src->ninf;
    acc_normalize(dst);
}

static int acc_bit(const acc_t *a, int b) { return (int)((a->c[b >> 5] >> (b & 31)) & 1); }

/* round the exact accumulated value to the nearest double, ties to even */
static double acc_round(acc_t *a)
{
    if (a->nan || (a->pinf && a->ninf)) return NAN;
    if (a->pinf) return INFINITY;
    if (a->ninf) return -INFINITY;
    acc_normalize(a);
    int neg = a->c[ACC_CELLS - 1] < 0;
    if (neg) {
        for (int c = 0; c < ACC_CELLS; ++c) a->c[c] = -a->c[c];
        acc_normalize(a);
    }
    int top = -1;
    for (int c = ACC_CELLS - 1; c >= 0; --c)
        if (a->c[c]) { top = c; break; }
    if (top < 0) return 0.0;
    int T = 32 * top + 31;
    while (!acc_bit(a, T)) --T;                   /* most significant set bit */
    int lsb = T - 52;                               /* keep 53 bits ... */
    if (lsb < ACC_OFF - 1074) lsb = ACC_OFF - 1074; /* ... or fewer if subnormal */
    uint64_t mant = 0;
    for (int b = T; b >= lsb; --b) mant = (mant << 1) | (uint64_t)acc_bit(a, b);
    int rbit = lsb >= 1 ? acc_bit(a, lsb - 1) : 0;
    int sticky = 0;
    for (int b = lsb - 2; b >= 0 && !sticky; --b) {
        if ((b & 31) == 31 && a->c[b >> 5] == 0) { b -= 31; continue; }
        sticky = acc_bit(a, b);
    }
    if (rbit && (sticky || (mant & 1))) mant += 1;
    double r = ldexp((double)mant, lsb - ACC_OFF);
    return neg ? -r : r;
}

/* sum_i x_i*y_i, exact then rounded once; independent of thread count */
double orc_dot(const double *x, const double *y, int64_t n)
{
    acc_t total;
    acc_init(&total);
#pragma omp parallel
    {
        acc_t a;
        acc_init(&a);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) acc_add_product(&a, x[i], y[i]);
        acc_normalize(&a);
#pragma omp critical
        acc_merge(&total, &a);
    }
    return acc_round(&total);
}

/* ------------------------------------------------------------------------- */
/* Spectrum (Background section: eigenvalues of the Dirichlet matrix D,      */
/* eq. eigenvaluesPoissonDirichletMatrix; Kronecker-sum eigenvalues,          */
/* eqs. lambdaMin and lambdaMax).                                             */
/* ------------------------------------------------------------------------- */
/* i-th eigenvalue (i = 1..n) of D = tridiag(-1, 2, -1) of order n */
double orc_dirichlet_eig(int i, int n)
{
    double s = sin((double)i * M_PI / (2.0 * (double)(n + 1)));
    return 4.0 * s * s;
}

/* Smallest and largest eigenvalue of the 1D operator of one axis of length n:
   D (eq. matrix_dirichlet) when both ends are Dirichlet, N (eq. matrix_neuman)
   when one end is Neumann, and N with both corner entries 2 when both are.
   The paper gives no closed form for N; the eigenvectors of the one-sided case
   are cos((2k-1) pi j / (2n)) (zero just past the Dirichlet end, mirrored at
   the Neumann end), giving 4 sin^2((2k-1) pi / (4n)), k = 1..n; with two
   Neumann ends they are cos(k pi j / (n-1)), giving 4 sin^2(k pi / (2(n-1))),
   k = 0..n-1. These closed forms are pinned against dense eigenvalues. */
static void axis_eigs(int n, int neu_lo, int neu_hi, double *mn, double *mx)
{
    if (!neu_lo && !neu_hi) {
        *mn = orc_dirichlet_eig(1, n);
        *mx = orc_dirichlet_eig(n, n);
    } else if (neu_lo != neu_hi) {
        double a = sin(1.0 * M_PI / (4.0 * (double)n));
        double b = sin((double)(2 * n - 1) * M_PI / (4.0 * (double)n));
        *mn = 4.0 * a * a;
        *mx = 4.0 * b * b;
    } else {
        double b = sin((double)(n - 1) * M_PI / (2.0 * (double)(n - 1)));
        *mn = 0.0;
        *mx = 4.0 * b * b;
    }
}

/* interval containing the spectra of all diagonal blocks of one axis: with
   blocks, the first block keeps the low face's condition, the last the high
   face's, the others are Dirichlet; a block shorter than `block` has its
   spectrum inside that of the full-length block of the same type */
static void axis_interval(int n, int block, int neu_lo, int neu_hi, double *mn, double *mx)
{
    if (block <= 0 || n <= block) {
        axis_eigs(n, neu_lo, neu_hi, mn, mx);
        return;
    }
    double a, b;
    axis_eigs(block, 0, 0, mn, mx);
    axis_eigs(block, neu_lo, 0, &a, &b);
    if (a < *mn) *mn = a;
    if (b > *mx) *mx = b;
    axis_eigs(block, 0, neu_hi, &a, &b);
    if (a < *mn) *mn = a;
    if (b > *mx) *mx = b;
}

/* lambda_min / lambda_max of A = Kronecker sum of O/h^2 over the three axes
   (eqs. lambdaMin, lambdaMax); bc bit f (x-, x+, y-, y+, z-, z+) = Neumann on
   face f. block > 0 gives an interval containing the spectrum of every
   block x block x block diagonal block R_s A R_s^T. */
void orc_interval_bc(int nx, int ny, int nz, double h, int block, unsigned bc, double *lmin,
                     double *lmax)
{
    int n[3] = {nx, ny, nz};
    double mn[3], mx[3];
    for (int d = 0; d < 3; ++d)
        axis_interval(n[d], block, (bc >> (2 * d)) & 1, (bc >> (2 * d + 1)) & 1, &mn[d], &mx[d]);
    double h2 = h * h;
    *lmin = mn[0] / h2 + mn[1] / h2 + mn[2] / h2;
    *lmax = mx[0] / h2 + mx[1] / h2 + mx[2] / h2;
}

void orc_interval(int nx, int ny, int nz, double h, int block, double *lmin, double *lmax)
{
    orc_interval_bc(nx, ny, nz, h, block, 0u, lmin, lmax);
}

/* ------------------------------------------------------------------------- */
/* The operator (eq. matrix_p): for uniform spacing                          */
/* (A u)_ijk = (6 u_ijk - six neighbours) / h^2. Outside a Dirichlet face a   */
/* neighbour reads as zero (matrix D); outside a Neumann face it is the      */
/* mirror image of the interior neighbour, u_{-1} = u_1 (the corner entry 2  */
/* of matrix N, eq. matrix_neuman). With block > 0 a neighbour in another    */
/* block also reads as zero: the block-diagonal part R_s A R_s^T of          */
/* eq. blockJacobiPreconditioner.                                            */
/* ------------------------------------------------------------------------- */
#define IDX(i, j, k) ((size_t)(i) + (size_t)nx * ((size_t)(j) + (size_t)ny * (size_t)(k)))

/* coordinate of the neighbour of a at a + d (d = +-1) along an axis of length n,
   or -1 if it reads as zero */
static int nbr(int a, int d, int n, int block, int neu_lo, int neu_hi)
{
    int b = a + d;
    if (b < 0) {
        if (!neu_lo) return -1;
        b = a + 1; /* mirror ghost */
    } else if (b >= n) {
        if (!neu_hi) return -1;
        b = a - 1;
    }
    if (b < 0 || b >= n) return -1;
    /* the block-diagonal part drops every coupling between blocks, mirrored ones too */
    if (block > 0 && a / block != b / block) return -1;
    return b;
}

void orc_apply_A_bc(int nx, int ny, int nz, double h, int block, unsigned bc, const double *u,
                    double *out)
{
    double ih2 = 1.0 / (h * h);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int im = nbr(i, -1, nx, block, bc & 1, (bc >> 1) & 1);
                int ip = nbr(i, +1, nx, block, bc & 1, (bc >> 1) & 1);
                int jm = nbr(j, -1, ny, block, (bc >> 2) & 1, (bc >> 3) & 1);
                int jp = nbr(j, +1, ny, block, (bc >> 2) & 1, (bc >> 3) & 1);
                int km = nbr(k, -1, nz, block, (bc >> 4) & 1, (bc >> 5) & 1);
                int kp = nbr(k, +1, nz, block, (bc >> 4) & 1, (bc >> 5) & 1);
                double c = u[IDX(i, j, k)];
                double xm = im >= 0 ? u[IDX(im, j, k)] : 0.0;
                double xp = ip >= 0 ? u[IDX(ip, j, k)] : 0.0;
                double ym = jm >= 0 ? u[IDX(i, jm, k)] : 0.0;
                double yp = jp >= 0 ? u[IDX(i, jp, k)] : 0.0;
                double zm = km >= 0 ? u[IDX(i, j, km)] : 0.0;
                double zp = kp >= 0 ? u[IDX(i, j, kp)] : 0.0;
                out[IDX(i, j, k)] = (6.0 * c - xm - xp - ym - yp - zm - zp) * ih2;
            }
}

void orc_apply_A(int nx, int ny, int nz, double h, int block, const double *u, double *out)
{
    orc_apply_A_bc(nx, ny, nz, h, block, 0u, u, out);
}

/* the same operator on FP32 data in FP32 arithmetic (mixed-precision            */
/* preconditioner). The paper fixes no precision; in FP32 the sum is taken as the */
/* three axes' second differences, (c - minus) + (c - plus), added x, y, z, then  */
/* scaled by ih2. On smooth data each difference and each pair sum is exact,     */
/* where 6c minus the six neighbours would cancel most of FP32's digits.          */
static void apply_A_f32(int nx, int ny, int nz, float ih2, int block, unsigned bc, const float *u,
                        float *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int im = nbr(i, -1, nx, block, bc & 1, (bc >> 1) & 1);
                int ip = nbr(i, +1, nx, block, bc & 1, (bc >> 1) & 1);
                int jm = nbr(j, -1, ny, block, (bc >> 2) & 1, (bc >> 3) & 1);
                int jp = nbr(j, +1, ny, block, (bc >> 2) & 1, (bc >> 3) & 1);
                int km = nbr(k, -1, nz, block, (bc >> 4) & 1, (bc >> 5) & 1);
                int kp = nbr(k, +1, nz, block, (bc >> 4) & 1, (bc >> 5) & 1);
                float c = u[IDX(i, j, k)];
                float xm = im >= 0 ? u[IDX(im, j, k)] : 0.0f;
                float xp = ip >= 0 ? u[IDX(ip, j, k)] : 0.0f;
                float ym = jm >= 0 ? u[IDX(i, jm, k)] : 0.0f;
                float yp = jp >= 0 ? u[IDX(i, jp, k)] : 0.0f;
                float zm = km >= 0 ? u[IDX(i, j, km)] : 0.0f;
                float zp = kp >= 0 ? u[IDX(i, j, kp)] : 0.0f;
                float dx = (c - xm) + (c - xp);
                float dy = (c - ym) + (c - yp);
                float dz = (c - zm) + (c - zp);
                out[IDX(i, j, k)] = ((dx + dy) + dz) * ih2;
            }
}

/* ------------------------------------------------------------------------- */
/* Chebyshev iteration (Alg. 2) for A x = b on the interval [lo, hi].        */
/*                                                                           */
/* With theta and delta the centre and half-width of the interval and        */
/* sigma = theta/delta (eq. chebyshevQuantities), the iteration produces     */
/* iterates X_0, X_1, ..., X_m:                                              */
/*   X_0 = b / theta,                                                        */
/*   X_1 = (2 rho_1 / delta) (2 b - (A b) / theta),                          */
/*   X_i = rho_i ((2 sigma X_{i-1} + (2/delta)(b - A X_{i-1}))              */
/*                - rho_{i-1} X_{i-2})                    for i >= 2,        */
/* where rho_0 = 1/sigma and rho_i = 1/(2 sigma - rho_{i-1}) are the ratios  */
/* T_{i-1}(sigma)/T_i(sigma) of Chebyshev polynomials, from their three-term */
/* recurrence. The degree m (the algorithm's iteration count) selects X_m.   */
/* The coefficients are tabulated once; each iterate is one generic step.    */
/* block > 0 uses the block-diagonal operator (BJ(CI) / GNoComm(CI)).         */
/* ------------------------------------------------------------------------- */
#define CHEB_MAXM 64

typedef struct {
    double theta, delta, sigma;
    double g1;                   /* 2 rho_1 / delta, the scale of X_1 */
    double two_sigma, two_over_delta;
    double rho[CHEB_MAXM + 1];   /* rho_0 .. rho_m */
} cheb_coef;

static void cheb_coef_make(double lo, double hi, int m, cheb_coef *c)
{
    c->theta = (hi + lo) / 2.0;
    c->delta = (hi - lo) / 2.0;
    c->sigma = c->theta / c->delta;
    c->rho[0] = 1.0 / c->sigma;
    const int top = m > 1 ? m : 1;
    for (int i = 1; i <= top; ++i) c->rho[i] = 1.0 / (2.0 * c->sigma - c->rho[i - 1]);
    c->g1 = 2.0 * c->rho[1] / c->delta;
    c->two_sigma = 2.0 * c->sigma;
    c->two_over_delta = 2.0 / c->delta;
}

/* X_i from X_{i-1} (prev), A X_{i-1} (aprev) and X_{i-2} (prev2), FP64 */
static void cheb_iterate(size_t N, const cheb_coef *c, int i, const double *b, const double *prev,
                         const double *aprev, const double *prev2, double *out)
{
    const double r = c->rho[i], rm = c->rho[i - 1];
    for (size_t q = 0; q < N; ++q)
        out[q] = r * (c->two_sigma * prev[q] + c->two_over_delta * (b[q] - aprev[q]) - rm * prev2[q]);
}

void orc_chebyshev_bc(int nx, int ny, int nz, double h, int block, unsigned bc, double lo,
                      double hi, int m, const double *b, double *x)
{
    const size_t N = (size_t)nx * ny * nz;
    if (m < 0 || m > CHEB_MAXM) return;
    cheb_coef c;
    cheb_coef_make(lo, hi, m, &c);
    double *X[3], *AX = malloc(N * 8);
    for (int k = 0; k < 3; ++k) X[k] = malloc(N * 8);
    for (size_t q = 0; q < N; ++q) X[0][q] = b[q] / c.theta;
    if (m >= 1) {
        orc_apply_A_bc(nx, ny, nz, h, block, bc, b, AX);
        for (size_t q = 0; q < N; ++q) X[1][q] = c.g1 * (2.0 * b[q] - AX[q] / c.theta);
    }
    for (int i = 2; i <= m; ++i) {
        orc_apply_A_bc(nx, ny, nz, h, block, bc, X[(i - 1) % 3], AX);
        cheb_iterate(N, &c, i, b, X[(i - 1) % 3], AX, X[(i - 2) % 3], X[i % 3]);
    }
    memcpy(x, X[m % 3], N * 8);
    for (int k = 0; k < 3; ++k) free(X[k]);
    free(AX);
}

/* Mixed precision: the same iterates with every coefficient computed in FP64
   and rounded once to FP32, the input rounded once to FP32, and all vector
   arithmetic in FP32. X_m is returned widened (exactly) to FP64. */
static void cheb_iterate_f32(size_t N, float r, float rm, float two_sigma, float two_over_delta,
                             const float *b, const float *prev, const float *aprev,
                             const float *prev2, float *out)
{
    for (size_t q = 0; q < N; ++q)
        out[q] = r * (two_sigma * prev[q] + two_over_delta * (b[q] - aprev[q]) - rm * prev2[q]);
}

void orc_chebyshev_f32_bc(int nx, int ny, int nz, double h, int block, unsigned bc, double lo,
                          double hi, int m, const double *b, double *x)
{
    const size_t N = (size_t)nx * ny * nz;
    if (m < 0 || m > CHEB_MAXM) return;
    cheb_coef c;
    cheb_coef_make(lo, hi, m, &c);
    const float theta = (float)c.theta, g1 = (float)c.g1;
    const float two_sigma = (float)c.two_sigma, two_over_delta = (float)c.two_over_delta;
    const float ih2 = (float)(1.0 / (h * h));
    float *bf = malloc(N * 4), *X[3], *AX = malloc(N * 4);
    for (int k = 0; k < 3; ++k) X[k] = malloc(N * 4);
    for (size_t q = 0; q < N; ++q) bf[q] = (float)b[q];
    for (size_t q = 0; q < N; ++q) X[0][q] = bf[q] / theta;
    if (m >= 1) {
        apply_A_f32(nx, ny, nz, ih2, block, bc, bf, AX);
        for (size_t q = 0; q < N; ++q) X[1][q] = g1 * (2.0f * bf[q] - AX[q] / theta);
    }
    for (int i = 2; i <= m; ++i) {
        apply_A_f32(nx, ny, nz, ih2, block, bc, X[(i - 1) % 3], AX);
        cheb_iterate_f32(N, (float)c.rho[i], (float)c.rho[i - 1], two_sigma, two_over_delta, bf,
                         X[(i - 1) % 3], AX, X[(i - 2) % 3], X[i % 3]);
    }
    for (size_t q = 0; q < N; ++q) x[q] = (double)X[m % 3][q];
    for (int k = 0; k < 3; ++k) free(X[k]);
    free(bf);
    free(AX);
}

void orc_chebyshev(int nx, int ny, int nz, double h, int block, double lo, double hi, int m,
                   const double *b, double *x)
{
    orc_chebyshev_bc(nx, ny, nz, h, block, 0u, lo, hi, m, b, x);
}

void orc_chebyshev_f32(int nx, int ny, int nz, double h, int block, double lo, double hi, int m,
                       const double *b, double *x)
{
    orc_chebyshev_f32_bc(nx, ny, nz, h, block, 0u, lo, hi, m, b, x);
}

/* ------------------------------------------------------------------------- */
/* Preconditioner dispatch M^-1 v (Table 1 and Methodology section).          */
/* ------------------------------------------------------------------------- */
typedef struct {
    int nx, ny, nz;
    double h;
    int precond, degree, mixed, block, bj_global;
    double lmin_scale, lmax_scale, jacobi_diag;
    unsigned bc;
} pc_t;

/* the eigenvalue interval handed to the Chebyshev iteration */
void orc_cheb_interval_bc(int nx, int ny, int nz, double h, unsigned bc, int precond, int block,
                          int bj_global, double lmin_scale, double lmax_scale, double *lo,
                          double *hi)
{
    int local = (precond == PC_BLOCK_JACOBI && !bj_global) ? block : 0;
    double a, b;
    orc_interval_bc(nx, ny, nz, h, local, bc, &a, &b);
    *lo = a * lmin_scale;
    *hi = b * lmax_scale;
}

void orc_cheb_interval(int nx, int ny, int nz, double h, int precond, int block, int bj_global,
                       double lmin_scale, double lmax_scale, double *lo, double *hi)
{
    orc_cheb_interval_bc(nx, ny, nz, h, 0u, precond, block, bj_global, lmin_scale, lmax_scale, lo,
                         hi);
}

static void apply_pc(const pc_t *pc, const double *v, double *out)
{
    size_t N = (size_t)pc->nx * pc->ny * pc->nz;
    if (pc->precond == PC_JACOBI) {
        double d = pc->jacobi_diag > 0 ? pc->jacobi_diag : 6.0 * (1.0 / (pc->h * pc->h));
        if (pc->mixed) {
            float df = (float)d;
            for (size_t q = 0; q < N; ++q) out[q] = (double)((float)v[q] / df);
        } else {
            for (size_t q = 0; q < N; ++q) out[q] = v[q] / d;
        }
        return;
    }
    double lo, hi;
    orc_cheb_interval_bc(pc->nx, pc->ny, pc->nz, pc->h, pc->bc, pc->precond, pc->block,
                         pc->bj_global, pc->lmin_scale, pc->lmax_scale, &lo, &hi);
    int blk = pc->precond == PC_BLOCK_JACOBI ? pc->block : 0;
    if (pc->mixed)
        orc_chebyshev_f32_bc(pc->nx, pc->ny, pc->nz, pc->h, blk, pc->bc, lo, hi, pc->degree, v,
                             out);
    else
        orc_chebyshev_bc(pc->nx, pc->ny, pc->nz, pc->h, blk, pc->bc, lo, hi, pc->degree, v, out);
}

/* one preconditioner application, exported for kernel-level parity tests */
void orc_precond_bc(int nx, int ny, int nz, double h, unsigned bc, int precond, int degree,
                    int mixed, int block, int bj_global, double lmin_scale, double lmax_scale,
                    const double *v, double *out)
{
    pc_t pc = {nx, ny, nz, h, precond, degree, mixed, block, bj_global, lmin_scale, lmax_scale,
               0.0, bc};
    if (precond == PC_NONE) {
        memcpy(out, v, (size_t)nx * ny * nz * 8);
        return;
    }
    apply_pc(&pc, v, out);
}

void orc_precond(int nx, int ny, int nz, double h, int precond, int degree, int mixed, int block,
                 int bj_global, double lmin_scale, double lmax_scale, const double *v, double *out)
{
    orc_precond_bc(nx, ny, nz, h, 0u, precond, degree, mixed, block, bj_global, lmin_scale,
                   lmax_scale, v, out);
}

/* ------------------------------------------------------------------------- */
/* Right-preconditioned Bi-CGSTAB (Alg. 1, with the scalar formulas of        */
/* Alg. 3: beta = (rho_i alpha_i)/(rho_{i-1} omega_i)).                        */
/*                                                                           */
/* An iteration has two halves. The first takes a step along the             */
/* preconditioned direction ph = M^-1 p: alpha makes the new residual        */
/* s = r - alpha A ph orthogonal to the fixed shadow residual rt. If s is     */
/* already small the solve ends there (Alg. 1's half step). The second       */
/* half minimises ||s - omega A sh|| over omega with sh = M^-1 s, moves x    */
/* along ph and sh, and builds the next direction p from the new residual.   */
/* Every test compares squared norms: ||r|| < tol ||b|| is evaluated as      */
/* r.r < (tol*tol)*(b.b).                                                    */
/* trace (optional, 4*maxit doubles): per iteration alpha, omega, rho_{i-1},  */
/* and the squared residual norm tested at exit of that iteration.            */
/* ------------------------------------------------------------------------- */
typedef struct {
    size_t N;
    const pc_t *pc;
    double *r;           /* residual; holds s between the two halves */
    double *rt;          /* shadow residual, r_0 */
    double *p, *ph, *w;  /* direction, M^-1 p, A M^-1 p */
    double *sh, *t;      /* M^-1 s, A M^-1 s */
    double rho;          /* rt . r of the current residual */
} bicg_t;

/* z = M^-1 v (the identity for no preconditioner: z aliases v) */
static const double *bicg_precond(const bicg_t *S, const double *v, double *buf)
{
    if (S->pc->precond == PC_NONE) return v;
    apply_pc(S->pc, v, buf);
    return buf;
}

static void bicg_apply_A(const bicg_t *S, const double *u, double *out)
{
    const pc_t *c = S->pc;
    orc_apply_A_bc(c->nx, c->ny, c->nz, c->h, 0, c->bc, u, out);
}

/* first half: ph, w = A ph, alpha; r becomes s. Status 0 to go on; *stepped is
   set once alpha exists and s is formed (r~.w was usable). */
static int bicg_first_half(bicg_t *S, const double **php, double *alpha, double *ss, int *stepped)
{
    const size_t N = S->N;
    *php = bicg_precond(S, S->p, S->ph);
    bicg_apply_A(S, *php, S->w);
    const double d = orc_dot(S->rt, S->w, (int64_t)N);
    if (!isfinite(d)) return ORC_ERR_NONFINITE;
    if (d == 0.0) return ORC_ERR_BREAKDOWN;
    *alpha = S->rho / d;
    *stepped = 1;
    for (size_t q = 0; q < N; ++q) S->r[q] = S->r[q] - *alpha * S->w[q];
    *ss = orc_dot(S->r, S->r, (int64_t)N);
    return isfinite(*ss) ? 0 : ORC_ERR_NONFINITE;
}

/* second half: sh, t = A sh, omega; x and r move; returns the new rt.r and r.r.
   *moved is set once omega exists and x, r have moved */
static int bicg_second_half(bicg_t *S, double *x, const double *php, double alpha, double *omega,
                            double *rho_new, double *rr, int *moved)
{
    const size_t N = S->N;
    const double *shp = bicg_precond(S, S->r, S->sh);
    bicg_apply_A(S, shp, S->t);
    const double ts = orc_dot(S->t, S->r, (int64_t)N);
    const double tt = orc_dot(S->t, S->t, (int64_t)N);
    if (!isfinite(ts) || !isfinite(tt)) return ORC_ERR_NONFINITE;
    if (tt == 0.0) return ORC_ERR_BREAKDOWN;
    *omega = ts / tt;
    *moved = 1;
    for (size_t q = 0; q < N; ++q) x[q] = x[q] + alpha * php[q] + *omega * shp[q];
    for (size_t q = 0; q < N; ++q) S->r[q] = S->r[q] - *omega * S->t[q];
    *rho_new = orc_dot(S->rt, S->r, (int64_t)N);
    *rr = orc_dot(S->r, S->r, (int64_t)N);
    return (isfinite(*rho_new) && isfinite(*rr)) ? 0 : ORC_ERR_NONFINITE;
}

int orc_bicgstab_bc(int nx, int ny, int nz, double h, unsigned bc, const double *b, double *x,
                    int precond, int degree, int mixed, double tol, int maxit, double lmin_scale,
                    double lmax_scale, int block, int bj_global, double jacobi_diag, double *trace,
                    double *rr0_out, int *iters, int *half)
{
    if (nx < 1 || ny < 1 || nz < 1 || !(h > 0) || maxit < 1) return ORC_ERR_ARG;
    const size_t N = (size_t)nx * ny * nz;
    const pc_t pc = {nx, ny, nz, h, precond, degree, mixed, block, bj_global,
                     lmin_scale, lmax_scale, jacobi_diag, bc};
    bicg_t S = {N, &pc, malloc(N * 8), malloc(N * 8), malloc(N * 8), malloc(N * 8),
                malloc(N * 8), malloc(N * 8), malloc(N * 8), 0.0};
    *iters = 0;
    *half = 0;
    int status = ORC_NOT_CONVERGED;

    /* r_0 = b - A x_0; the shadow residual and the first direction are r_0 */
    bicg_apply_A(&S, x, S.w);
    for (size_t q = 0; q < N; ++q) S.r[q] = b[q] - S.w[q];
    memcpy(S.rt, S.r, N * 8);
    memcpy(S.p, S.r, N * 8);
    const double bb = orc_dot(b, b, (int64_t)N);
    const double tol2bb = (tol * tol) * bb;
    S.rho = orc_dot(S.rt, S.r, (int64_t)N);
    double rr = orc_dot(S.r, S.r, (int64_t)N);
    if (rr0_out) *rr0_out = rr;
    if (!isfinite(bb) || !isfinite(rr)) { status = ORC_ERR_NONFINITE; goto out; }
    if (bb == 0.0) { memset(x, 0, N * 8); status = ORC_OK; goto out; }
    if (rr < tol2bb) { status = ORC_OK; goto out; }

    for (int i = 1; i <= maxit; ++i) {
        double *tr = trace ? trace + 4 * (i - 1) : NULL;
        const double *php;
        double alpha = 0.0, ss = 0.0, omega = 0.0, rho_new = 0.0;
        int stepped = 0, moved = 0;
        *iters = i;
        int st = bicg_first_half(&S, &php, &alpha, &ss, &stepped);
        /* alpha and rho_{i-1} are recorded once alpha exists (also if s.s then fails) */
        if (tr && stepped) { tr[0] = alpha; tr[2] = S.rho; }
        if (st) { status = st; goto out; }
        if (ss < tol2bb) {
            for (size_t q = 0; q < N; ++q) x[q] = x[q] + alpha * php[q];
            if (tr) { tr[1] = 0.0; tr[3] = ss; }
            *half = 1;
            status = ORC_OK;
            goto out;
        }
        st = bicg_second_half(&S, x, php, alpha, &omega, &rho_new, &rr, &moved);
        if (tr && moved) { tr[1] = omega; tr[3] = rr; }
        if (st) { status = st; goto out; }
        if (rr < tol2bb) { status = ORC_OK; goto out; }
        if (rho_new == 0.0 || omega == 0.0) { status = ORC_ERR_BREAKDOWN; goto out; }
        /* next direction p = r + beta (p - omega w) */
        const double beta = (rho_new * alpha) / (S.rho * omega);
        for (size_t q = 0; q < N; ++q) S.p[q] = S.r[q] + beta * (S.p[q] - omega * S.w[q]);
        S.rho = rho_new;
    }
    status = ORC_NOT_CONVERGED;
out:
    free(S.r); free(S.rt); free(S.p); free(S.w); free(S.t); free(S.ph); free(S.sh);
    return status;
}

int orc_bicgstab(int nx, int ny, int nz, double h, const double *b, double *x, int precond,
                 int degree, int mixed, double tol, int maxit, double lmin_scale,
                 double lmax_scale, int block, int bj_global, double jacobi_diag, double *trace,
                 double *rr0_out, int *iters, int *half)
{
    return orc_bicgstab_bc(nx, ny, nz, h, 0u, b, x, precond, degree, mixed, tol, maxit,
                           lmin_scale, lmax_scale, block, bj_global, jacobi_diag, trace, rr0_out,
                           iters, half);
}
