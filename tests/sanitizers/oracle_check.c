/* The oracle (oracle/oracle.c) driven over small grids under AddressSanitizer
 * and UndefinedBehaviorSanitizer, built with gcc by tests/test_sanitizers.py:
 * every exported routine on ragged shapes, every preconditioner and face mask,
 * FP64 and the FP32 emulation, with x0 = 0 and x0 != 0. Checks only that each
 * solve ends with its expected status and that the true residual meets the
 * tolerance (the numerics are pinned by the Python tests); the sanitizers
 * check every access. Exit status 0 on success. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

double orc_dot(const double *x, const double *y, int64_t n);
void orc_interval_bc(int nx, int ny, int nz, double h, int block, unsigned bc, double *lmin,
                     double *lmax);
void orc_apply_A_bc(int nx, int ny, int nz, double h, int block, unsigned bc, const double *u,
                    double *out);
void orc_chebyshev_bc(int nx, int ny, int nz, double h, int block, unsigned bc, double lo,
                      double hi, int m, const double *v, double *out);
void orc_chebyshev_f32_bc(int nx, int ny, int nz, double h, int block, unsigned bc, double lo,
                          double hi, int m, const double *v, double *out);
void orc_cheb_interval_bc(int nx, int ny, int nz, double h, unsigned bc, int precond, int block,
                          int bj_global, double lmin_scale, double lmax_scale, double *lo,
                          double *hi);
void orc_precond_bc(int nx, int ny, int nz, double h, unsigned bc, int precond, int degree,
                    int mixed, int block, int bj_global, double lmin_scale, double lmax_scale,
                    const double *v, double *out);
int orc_bicgstab_bc(int nx, int ny, int nz, double h, unsigned bc, const double *b, double *x,
                    int precond, int degree, int mixed, double tol, int maxit, double lmin_scale,
                    double lmax_scale, int block, int bj_global, double jacobi_diag,
                    double *trace, double *rr0_out, int *iters, int *half);

static int fails = 0;

static double *vec(size_t n, unsigned seed)
{
    double *v = malloc(n * sizeof(double));
    uint64_t s = 0x9E3779B97F4A7C15ull * (seed + 1);
    for (size_t i = 0; i < n; ++i) {
        s ^= s << 13;
        s ^= s >> 7;
        s ^= s << 17;
        v[i] = (double)(s >> 11) * 0x1p-53 * 2.0 - 1.0;
    }
    return v;
}

static void solve(int nx, int ny, int nz, unsigned bc, int pc, int m, int mixed, int block,
                  int nonzero_x0)
{
    const size_t N = (size_t)nx * ny * nz;
    const double h = 1.0 / (nx + 1), tol = 1e-8;
    double *b = vec(N, (unsigned)(nx + 7 * pc + m));
    double *x = nonzero_x0 ? vec(N, 99) : calloc(N, sizeof(double));
    double *r = malloc(N * sizeof(double));
    const int maxit = 4000;
    double *trace = malloc((size_t)4 * maxit * sizeof(double));
    double rr0 = 0;
    int iters = 0, half = 0;
    const int st = orc_bicgstab_bc(nx, ny, nz, h, bc, b, x, pc, m, mixed, tol, maxit, 1.0, 1.0,
                                   block, 0, 0.0, trace, &rr0, &iters, &half);
    orc_apply_A_bc(nx, ny, nz, h, 0, bc, x, r);
    for (size_t i = 0; i < N; ++i) r[i] = b[i] - r[i];
    const double rel = sqrt(orc_dot(r, r, (int64_t)N) / orc_dot(b, b, (int64_t)N));
    if (st != 0 || !(rel < 2 * tol) || iters < 1) {
        fprintf(stderr, "solve %dx%dx%d bc %u pc %d m %d mixed %d: status %d, %d iterations, "
                        "true relres %g\n", nx, ny, nz, bc, pc, m, mixed, st, iters, rel);
        ++fails;
    }
    free(b);
    free(x);
    free(r);
    free(trace);
}

int main(void)
{
    const unsigned bcs[4] = {0u, 22u, 3u | 16u, 9u};
    const int shapes[3][3] = {{9, 7, 5}, {13, 4, 6}, {3, 11, 8}};
    for (int s = 0; s < 3; ++s) {
        const int nx = shapes[s][0], ny = shapes[s][1], nz = shapes[s][2];
        const size_t N = (size_t)nx * ny * nz;
        double *u = vec(N, (unsigned)s), *o = malloc(N * sizeof(double));
        for (int k = 0; k < 4; ++k) {
            const unsigned bc = bcs[k];
            double lo, hi;
            orc_interval_bc(nx, ny, nz, 0.1, 0, bc, &lo, &hi);
            orc_interval_bc(nx, ny, nz, 0.1, 3, bc, &lo, &hi);
            orc_cheb_interval_bc(nx, ny, nz, 0.1, bc, 3, 4, 1, 10.0, 0.999, &lo, &hi);
            for (int blk = 0; blk <= 4; blk += 4) {
                orc_apply_A_bc(nx, ny, nz, 0.1, blk, bc, u, o);
                orc_interval_bc(nx, ny, nz, 0.1, blk, bc, &lo, &hi);
                for (int m = 0; m <= 5; ++m) {
                    orc_chebyshev_bc(nx, ny, nz, 0.1, blk, bc, lo, hi, m, u, o);
                    orc_chebyshev_f32_bc(nx, ny, nz, 0.1, blk, bc, lo, hi, m, u, o);
                }
            }
            for (int pc = 0; pc <= 3; ++pc)
                for (int mixed = 0; mixed < 2; ++mixed)
                    orc_precond_bc(nx, ny, nz, 0.1, bc, pc, 4, mixed, 4, 0, 1.0, 1.0, u, o);
        }
        for (int k = 0; k < 4; ++k)
            for (int pc = 0; pc <= 3; ++pc) {
                solve(nx, ny, nz, bcs[k], pc, pc >= 2 ? 4 : 0, 0, 4, k & 1);
                if (pc >= 2) solve(nx, ny, nz, bcs[k], pc, 5, 1, 4, 0);
            }
        (void)orc_dot(u, o, 0);
        (void)orc_dot(u, o, 1);
        free(u);
        free(o);
    }
    if (fails) {
        fprintf(stderr, "%d oracle checks failed\n", fails);
        return 1;
    }
    printf("oracle checks passed\n");
    return 0;
}
