/* Host sanitizer run of the C ABI's host layer (test infrastructure): the
 * argument checks, geometry preprocessing (stencil codes, percolation,
 * wall faces), row heights, driving and the permeability post-processing,
 * none of which touches the GPU.  The CPU test builds this file with the
 * library's HIP sources, host code under AddressSanitizer and
 * UndefinedBehaviorSanitizer.  Exit status 0 when every call returns what
 * it should. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../include/dvm.h"

static int bad = 0;
#define EXPECT(cond)                                                                 \
    do {                                                                             \
        if (!(cond)) {                                                               \
            fprintf(stderr, "line %d: %s (%s)\n", __LINE__, #cond, dvm_last_error()); \
            bad = 1;                                                                 \
        }                                                                            \
    } while (0)

int main(void)
{
    dvm_config cfg;
    memset(&cfg, 0, sizeof cfg);
    dvm_ctx *c = NULL;
    EXPECT(dvm_create(&c, 7, 1, &cfg, NULL, NULL, NULL, NULL) == DVM_EINVAL);
    EXPECT(dvm_create(&c, 8, 0, &cfg, NULL, NULL, NULL, NULL) == DVM_EINVAL);
    cfg.krylov_deflate = 40;
    EXPECT(dvm_create(&c, 8, 1, &cfg, NULL, NULL, NULL, NULL) == DVM_EINVAL);
    cfg.krylov_deflate = 0;
    EXPECT(dvm_create(&c, 8, 3, &cfg, NULL, NULL, NULL, NULL) == DVM_OK);

    /* a rough channel: walls on y, roughness on the bottom row */
    enum { NX = 24, NY = 12 };
    uint8_t m[NX * NY];
    memset(m, 0, sizeof m);
    for (int x = 0; x < NX; x += 6)
        m[x] = m[x + 1] = m[NX + x] = 1;
    EXPECT(dvm_set_geometry(c, 0, NX, NY, m, 0, (double)NY) == DVM_OK);
    /* a periodic porous cell with a closed pore (a solid ring around a
     * fluid pocket): rejected, the pocket does not percolate */
    enum { N = 16 };
    uint8_t p[N * N];
    memset(p, 0, sizeof p);
    for (int i = 4; i <= 9; ++i)
        p[4 * N + i] = p[9 * N + i] = p[i * N + 4] = p[i * N + 9] = 1;
    EXPECT(dvm_set_geometry(c, 1, N, N, p, 1, (double)N) != DVM_OK);
    /* the same cell with the ring opened: accepted */
    p[9 * N + 6] = 0;
    EXPECT(dvm_set_geometry(c, 1, N, N, p, 1, (double)N) == DVM_OK);
    /* an all-solid mask and bad sizes */
    uint8_t s[16];
    memset(s, 1, sizeof s);
    EXPECT(dvm_set_geometry(c, 2, 4, 4, s, 0, 4.0) != DVM_OK);
    EXPECT(dvm_set_geometry(c, 2, 0, 4, s, 0, 4.0) != DVM_OK);
    EXPECT(dvm_set_geometry(c, 5, NX, NY, m, 0, (double)NY) != DVM_OK);
    EXPECT(dvm_set_geometry(c, 2, NX, NY, m, 0, -1.0) != DVM_OK);
    EXPECT(dvm_set_geometry(c, 2, NX, NY, m, 0, (double)NY) == DVM_OK);

    double dy[NY];
    for (int y = 0; y < NY; ++y)
        dy[y] = (y < 4 ? 0.5 : 1.25) / NY;
    EXPECT(dvm_set_row_heights(c, 0, dy) == DVM_OK);
    dy[3] = -1.0;
    EXPECT(dvm_set_row_heights(c, 0, dy) != DVM_OK);
    EXPECT(dvm_set_driving(c, 0, 0.0, 0.0, 1.0) == DVM_OK);
    EXPECT(dvm_set_driving(c, 0, NAN, 0.0, 1.0) != DVM_OK);

    /* solves validate their arguments on the host before any device work */
    double d = -1.0;
    dvm_info info;
    EXPECT(dvm_solve(c, 0, &d, 0, 1.0, &info) != DVM_OK);
    d = 1.0;
    EXPECT(dvm_solve(c, 0, &d, 0, 1.5, &info) != DVM_OK);
    EXPECT(dvm_solve(c, 7, &d, 0, 1.0, &info) != DVM_OK);
    EXPECT(dvm_solve(c, 0, NULL, 0, 1.0, &info) != DVM_OK);
    double Q, ka;
    EXPECT(dvm_flow_rate(c, 0, &Q, &ka) != DVM_OK);    /* nothing solved yet */

    /* permeability post-processing (host only) */
    double dl[6] = {0.1, 0.3, 1.0, 3.0, 10.0, 30.0}, qv[6];
    for (int i = 0; i < 6; ++i)
        qv[i] = 0.05 * dl[i] + 0.3 + 0.2 / dl[i];
    double kinf, hs, kns[6], kar[6], kn[6], kav[6];
    EXPECT(dvm_permeability(6, dl, qv, 0.6, &kinf, &hs, kns, kar, kn, kav) == DVM_OK);
    EXPECT(kinf > 0.0 && isfinite(hs));
    EXPECT(dvm_permeability(2, dl, qv, 0.6, &kinf, &hs, kns, kar, kn, kav) != DVM_OK);
    EXPECT(dvm_permeability(6, dl, qv, 1.5, &kinf, &hs, kns, kar, kn, kav) != DVM_OK);

    dvm_destroy(c);
    dvm_destroy(NULL);
    printf("%s\n", bad ? "FAILED" : "ok");
    return bad;
}
