/* Host sanitizer run of the FP64 oracle (test infrastructure): tiny solves
 * through every path of oracle_si_solve, compiled together with the oracle
 * under AddressSanitizer and UndefinedBehaviorSanitizer by the CPU test that
 * builds this file.  Exit status 0 when every solve returns as expected. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_si_solve(int nx, int ny, const uint8_t *solid, int periodic_y, double cells_per_H, const double *dy,
                    int nv, const double *delta, int delta_is_field, double alpha, double drive, double u_bot,
                    double u_top, double tol, long max_iter, double *rho, double *u1, double *u2, double *tau,
                    double *p12, double *info, double *hist, double *h);
int oracle_quadrature(int nv, double *v, double *w1, double *xi, double *eta, double *W, double *consts);

static int run(int nx, int ny, const uint8_t *solid, int periodic_y, const double *dy, int nv,
               const double *delta, int field, double alpha, double drive, double u_top, double tol, int max_iter,
               int want_h)
{
    size_t nc = (size_t)nx * ny;
    double *f[5];
    for (int i = 0; i < 5; ++i)
        f[i] = calloc(nc, sizeof(double));
    double info[3] = {0, 0, 0};
    double *hist = calloc((size_t)max_iter, sizeof(double));
    double *h = want_h ? calloc(nc * (size_t)nv * nv, sizeof(double)) : NULL;
    int rc = oracle_si_solve(nx, ny, solid, periodic_y, (double)ny, dy, nv, delta, field, alpha, drive, 0.0, u_top,
                             tol, max_iter, f[0], f[1], f[2], f[3], f[4], info, hist, h);
    printf("nx %d ny %d nv %d periodic %d alpha %.2f: rc %d Q %.12g iters %g\n", nx, ny, nv, periodic_y, alpha, rc,
           info[0], info[1]);
    for (int i = 0; i < 5; ++i)
        free(f[i]);
    free(hist);
    free(h);
    return rc;
}

int main(void)
{
    int bad = 0;
    /* rough channel, walls on y, nonuniform rows, specular share, sliding top wall */
    enum { NX = 12, NY = 8 };
    uint8_t solid[NX * NY];
    memset(solid, 0, sizeof solid);
    for (int x = 0; x < NX; x += 4)
        solid[x] = solid[x + 1] = 1;                 /* roughness on the bottom row */
    double dy[NY];
    for (int y = 0; y < NY; ++y)
        dy[y] = (y < 3 ? 0.5 : 1.5) / NY;
    double d1 = 1.0;
    bad |= run(NX, NY, solid, 0, NULL, 6, &d1, 0, 1.0, 1.0, 0.0, 1e-10, 20000, 1) != 0;
    bad |= run(NX, NY, solid, 0, dy, 6, &d1, 0, 0.8, 1.0, 0.0, 1e-10, 20000, 0) != 0;
    bad |= run(NX, NY, solid, 0, NULL, 6, &d1, 0, 1.0, 0.0, 1.0, 1e-10, 20000, 0) != 0;
    /* periodic porous cell with a delta field and a fixed iteration count */
    enum { N = 10 };
    uint8_t pm[N * N];
    memset(pm, 0, sizeof pm);
    for (int y = 3; y < 6; ++y)
        for (int x = 4; x < 7; ++x)
            pm[y * N + x] = 1;
    double df[N * N];
    for (int i = 0; i < N * N; ++i)
        df[i] = 0.5 + 0.01 * (i % 13);
    bad |= run(N, N, pm, 1, NULL, 8, df, 1, 1.0, 1.0, 0.0, -1.0, 50, 1) < 0;
    /* a one-column channel (x-invariant) */
    uint8_t col[16] = {0};
    bad |= run(1, 16, col, 0, NULL, 8, &d1, 0, 1.0, 1.0, 0.0, 1e-12, 20000, 0) != 0;
    /* rejected inputs: too few columns, odd velocity count */
    uint8_t full[4] = {1, 1, 1, 1};
    bad |= run(2, 2, full, 0, NULL, 8, &d1, 0, 1.0, 1.0, 0.0, 1e-10, 10, 0) >= 0;
    bad |= run(NX, NY, solid, 0, NULL, 5, &d1, 0, 1.0, 1.0, 0.0, 1e-10, 10, 0) >= 0;
    double v[8], w1[8], xi[64], eta[64], W[64], consts[7];
    bad |= oracle_quadrature(8, v, w1, xi, eta, W, consts) != 0;
    bad |= oracle_quadrature(7, v, w1, xi, eta, W, consts) == 0;
    printf("%s\n", bad ? "FAILED" : "ok");
    return bad;
}
