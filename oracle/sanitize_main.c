/*
 * sanitize_main.c -- driver that runs every entry point of smg_oracle.c on
 * small odd and even bricks, for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer.  TEST INFRASTRUCTURE ONLY (the CPU tests compile
 * and run it; nothing else uses it).  Exit status 0 means every call returned
 * finite results; the sanitizers abort on the first invalid access or
 * undefined operation.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct oracle_smg oracle_smg;
void oracle_matvec(int, int, int, double, double, double, const double *, double *);
void oracle_line_solve(int, double, double, const double *, double *, double *);
oracle_smg *oracle_smg_create(int, int, int, double, double, double, int, int, int, int, int);
void oracle_smg_destroy(oracle_smg *);
void oracle_smg_apply(oracle_smg *, const double *, double *);
void oracle_smg_plane_solve(oracle_smg *, int, int, const double *, double *);
int oracle_smg_nlevels(const oracle_smg *);
int oracle_smg_level_nz(const oracle_smg *, int);
void oracle_smg_plane_coef(const oracle_smg *, int, int, double *);
int oracle_smg_plane_nlevels(const oracle_smg *, int, int);
int oracle_smg_plane_level_ny(const oracle_smg *, int, int, int);
void oracle_smg_line_coef(const oracle_smg *, int, int, int, int, double *);
int oracle_krylov(oracle_smg *, int, int, int, int, double, double, double, const double *, double *, double,
                  int, int, double *, double *, int *, double *, double *);

static int finite_all(const double *v, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

int main(void)
{
    const int shapes[][3] = {{1, 1, 1}, {5, 4, 3}, {13, 9, 7}, {8, 8, 8}, {1, 6, 11}, {17, 2, 1}};
    const int pp[][2] = {{1, 1}, {1, 0}, {0, 1}, {2, 1}};
    int fails = 0;
    for (size_t si = 0; si < sizeof shapes / sizeof shapes[0]; ++si) {
        const int nx = shapes[si][0], ny = shapes[si][1], nz = shapes[si][2];
        const size_t n = (size_t)nx * ny * nz;
        double *b = malloc(n * sizeof(double)), *x = malloc(n * sizeof(double)), *y = malloc(n * sizeof(double));
        double *hist = malloc(201 * sizeof(double)), *histc = malloc(201 * sizeof(double));
        double *u = malloc((size_t)nx * sizeof(double)), *w = malloc((size_t)nx * sizeof(double));
        double *pb = malloc((size_t)nx * ny * sizeof(double)), *px = malloc((size_t)nx * ny * sizeof(double));
        for (size_t i = 0; i < n; ++i) b[i] = sin(0.7 * (double)i + 0.3);
        oracle_matvec(nx, ny, nz, 1.0, 2.0, 0.5, b, y);
        fails += !finite_all(y, n);
        oracle_line_solve(nx, 1.0, 0.5, b, u, w);
        fails += !finite_all(u, (size_t)nx);
        for (size_t pi = 0; pi < sizeof pp / sizeof pp[0]; ++pi)
            for (int order = 0; order < 2; ++order) {
                oracle_smg *S = oracle_smg_create(nx, ny, nz, 1.0, 2.0, 0.5, pp[pi][0], pp[pi][1], -1, -1, order);
                if (!S) { ++fails; continue; }
                oracle_smg_apply(S, b, y);
                fails += !finite_all(y, n);
                double coef[4];
                for (int l = 0; l < oracle_smg_nlevels(S); ++l)
                    for (int K = 0; K < oracle_smg_level_nz(S, l); ++K) {
                        oracle_smg_plane_coef(S, l, K, coef);
                        for (int l2 = 0; l2 < oracle_smg_plane_nlevels(S, l, K); ++l2)
                            for (int j = 0; j < oracle_smg_plane_level_ny(S, l, K, l2); ++j)
                                oracle_smg_line_coef(S, l, K, l2, j, coef);
                    }
                oracle_smg_plane_solve(S, 0, 0, b, px);
                fails += !finite_all(px, (size_t)nx * ny);
                for (int method = 0; method < 3; ++method)
                    for (int stop_c = 0; stop_c < 2; ++stop_c) {
                        int it = 0;
                        double rel = 0, trel = 0;
                        for (size_t i = 0; i < n; ++i) x[i] = (method == 1) ? 0.1 * cos((double)i) : 0.0;
                        int st = oracle_krylov(S, method, nx, ny, nz, 1.0, 2.0, 0.5, b, x, 1e-8, stop_c, 200, hist,
                                               histc, &it, &rel, &trel);
                        fails += (st < 0) || !finite_all(x, n);
                    }
                oracle_smg_destroy(S);
            }
        free(b); free(x); free(y); free(hist); free(histc); free(u); free(w); free(pb); free(px);
    }
    printf("sanitize driver: %d failures\n", fails);
    return fails ? 1 : 0;
}
