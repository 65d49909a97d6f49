/*
 * dvm_oracle.c -- plain, slow, FP64 CPU reference for the discrete velocity
 * method (DVM) solution of the steady linearized BGK equation in 2-D
 * staircase geometries (Lindsay, Su, Liu & Wu, "Comparative study of the
 * discrete velocity and lattice Boltzmann methods for rarefied gas flows
 * through irregular channels", arXiv:1704.03126).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU solver.
 *
 * What it computes (paper section / equation it follows):
 *   - velocity nodes of Eq. (nonuniform_v) (Sec. II.A) on a tensor grid;
 *   - f_eq = exp(-|v|^2)/pi as the quadrature weight (Sec. II.A, linearisation);
 *   - moments rho, u1, u2, tau of Sec. II.A (below Eq. BGK);
 *   - the gain term L(rho,u,tau) of Eq. (BGK);
 *   - the source iteration of Eq. (iteration) with a second-order upwind
 *     difference for v . grad h (Sec. II.A, text after Eq. iteration);
 *   - diffuse walls of Eq. (diffuse2) on the staircase (Sec. II.A);
 *   - periodic inlet/outlet (Sec. II.B and Sec. III);
 *   - the stop rule on the relative change of the horizontal velocity
 *     (Sec. II.A, end);
 *   - the Poiseuille flow rate Q of Sec. III (divided by the cell length L).
 * Readings where the paper is silent (weights, discrete-conservative
 * equilibrium, drive term, wall stencil, seam lag, stop-rule norm) are the
 * ones listed in the design notes; each is marked "reading" below.
 *
 * Layout: h[k * ncell + y * nx + x], k = i * nv + j with (xi, eta) = (v_i, v_j).
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { DIR_W = 0, DIR_E = 1, DIR_S = 2, DIR_N = 3 };
enum { ST_INT = 0, ST_NEAR = 1, ST_WALL = 2, ST_NONE = 3 };

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the next solves (timing on a given number of host cores). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Eq. (nonuniform_v): v_j = 4 s_j^3 with s_j = (2j - Nv + 1)/(Nv - 1).
 * Reading: the 1-D weights are the trapezoid rule in s, w_j = (dv/ds) * ds,
 * halved at both ends.  The 2-D weight of velocity (v_i, v_j) carries the
 * global Maxwellian exp(-|v|^2)/pi of the linearisation.
 * consts = {m0, m2, M2, M4, c2, c4, D}. */
int oracle_quadrature(int nv, double *v, double *w1, double *xi, double *eta,
                      double *W, double *consts)
{
    if (nv < 4 || (nv % 2) != 0)
        return -1;
    const double ds = 2.0 / (double)(nv - 1);
    for (int j = 0; j < nv; ++j) {
        double s = (double)(2 * j - nv + 1) / (double)(nv - 1);
        v[j] = 4.0 * s * s * s;
        w1[j] = 12.0 * s * s * ds;
        if (j == 0 || j == nv - 1)
            w1[j] *= 0.5;
    }
    double m0 = 0, m2 = 0, M2 = 0, M4 = 0, D = 0;
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) {
            int k = i * nv + j;
            xi[k] = v[i];
            eta[k] = v[j];
            W[k] = w1[i] * w1[j] * exp(-v[i] * v[i] - v[j] * v[j]) / M_PI;
            double q = v[i] * v[i] + v[j] * v[j];
            m0 += W[k];
            m2 += W[k] * v[i] * v[i];
            M2 += W[k] * q;
            M4 += W[k] * q * q;
            if (v[i] > 0)
                D += W[k] * v[i];
        }
    consts[0] = m0;
    consts[1] = m2;
    consts[2] = M2;
    consts[3] = M4;
    consts[4] = M2 / m0;
    consts[5] = M4 - M2 * M2 / m0;
    consts[6] = D;
    return 0;
}

static int solid_at(const uint8_t *solid, int nx, int ny, int periodic_y,
                    int x, int y)
{
    x = ((x % nx) + nx) % nx; /* the flow direction is always periodic */
    if (y < 0 || y >= ny) {
        if (!periodic_y)
            return 1; /* walls on the outer y faces */
        y = ((y % ny) + ny) % ny;
    }
    return solid[y * nx + x] != 0;
}

/* Staircase stencil classification (Sec. II.A "stair case"; reading): for each
 * fluid cell and each side d the flow can come from, look at the first and
 * second neighbour on that side: solid first neighbour -> the cell touches a
 * wall face on that side (ST_WALL); solid second neighbour -> the upwind
 * neighbour touches a wall (ST_NEAR); otherwise the plain second-order upwind
 * difference (ST_INT).  nx == 1 means x-invariant (no x transport). */
int oracle_codes(int nx, int ny, const uint8_t *solid, int periodic_y,
                 uint8_t *codes)
{
    if (!(nx == 1 || nx >= 4) || ny < 4)
        return -1;
    static const int ddx[4] = {-1, 1, 0, 0};
    static const int ddy[4] = {0, 0, -1, 1};
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int c = y * nx + x;
            for (int d = 0; d < 4; ++d) {
                uint8_t code;
                if (solid[c] || (d < 2 && nx == 1)) {
                    code = ST_NONE;
                } else if (solid_at(solid, nx, ny, periodic_y, x + ddx[d], y + ddy[d])) {
                    code = ST_WALL;
                } else if (solid_at(solid, nx, ny, periodic_y, x + 2 * ddx[d], y + 2 * ddy[d])) {
                    code = ST_NEAR;
                } else {
                    code = ST_INT;
                }
                codes[4 * c + d] = code;
            }
        }
    return 0;
}

static inline int wrap(int a, int n) { return ((a % n) + n) % n; }

typedef struct {
    int nx, ny, nv, K, nc, periodic_y;
    double dx, alpha;
    double drive;                          /* pressure-gradient source factor */
    double u_wall[2];                      /* x velocity of the outer bottom / top wall */
    const double *xi, *eta, *W;
    const uint8_t *solid, *codes;
    const double *dl;                      /* delta per cell */
    const double *dy;                      /* row heights (units of H), NULL: uniform dx */
    const double *a0, *a1, *a2, *a3;       /* equilibrium coefficients per cell */
    const double *rho_w;                   /* reflected density per cell and side */
    const int *wall_slot;                  /* cell -> wall-cell row or -1 */
    const double *hinc;                    /* incident face values [slot][side][k] */
    double *h;
} si_ctx;

/* Mirror of velocity k across a face whose normal lies along x (d < 2) or y. */
static inline int mirror(int k, int d, int nv)
{
    int i = k / nv, j = k % nv;
    return d < 2 ? (nv - 1 - i) * nv + j : i * nv + (nv - 1 - j);
}

/* x velocity of the wall behind side d of cell c: the outer bottom and top
 * walls of a channel may slide along x (the moving plate of Sec. II); the
 * solid staircase is at rest. */
static inline double wall_speed(const si_ctx *s, int c, int d)
{
    if (s->periodic_y)
        return 0.0;
    int y = c / s->nx;
    if (d == DIR_S && y == 0)
        return s->u_wall[0];
    if (d == DIR_N && y == s->ny - 1)
        return s->u_wall[1];
    return 0.0;
}

/* Value of h on the wall face on side d of cell c for a velocity k leaving
 * that face: Eq. (diffuse2) (full accommodation) -- for a wall sliding at
 * speed U along x, Eq. (diffuse1): the reflected density plus 2 U xi (the
 * linearised Maxwellian of the moving wall) -- plus, as a reading for
 * alpha < 1, Maxwell's specular share 1 - alpha of the mirrored incident
 * face value.  The density and incident values come from the previous
 * iterate. */
static inline double face_out(const si_ctx *s, int c, int d, int k)
{
    double f = s->alpha * (s->rho_w[4 * c + d] + 2.0 * wall_speed(s, c, d) * s->xi[k]);
    if (s->alpha < 1.0)
        f += (1.0 - s->alpha) *
             s->hinc[((size_t)s->wall_slot[c] * 4 + d) * s->K + mirror(k, d, s->nv)];
    return f;
}

/* Upwind part of v.grad h along one axis for cell c, written as
 * diag * h_c - rhs.  Reading of the second-order upwind difference on the
 * staircase, in flux form: |v| (h_out - h_in) / dx, where the value on a cell
 * face is extrapolated linearly from the upwind cell, 1.5 h_u - 0.5 h_uu, when
 * the upwind cell's own upwind neighbour is fluid, and is the upwind cell
 * value h_u when that neighbour is solid; on a wall face the value leaving
 * the wall is the wall value.  In the interior this is exactly the paper's
 * (3 h_c - 4 h_1 + h_2) / (2 dx); every face carries one value for both cells
 * it separates, so the scheme conserves mass.  On rows of unequal height
 * (the nonuniform spacing across the channel of Sec. II.A) the same linear
 * extrapolation reads h_u + r (h_u - h_uu), r = dy_u / (dy_u + dy_uu) the
 * ratio of the distances from the face and from uu's centre to u's centre:
 * rc for the cell's own outgoing face, ru for the incoming one (both 1/2 on
 * a uniform grid), and cv = |v| / dy_c. */
static inline void upwind_axis(const si_ctx *s, const double *hk, int code,
                               int c, int c1, int c2, int d, int k, double cv,
                               double rc, double ru, double *den, double *num)
{
    switch (code) {
    case ST_INT: /* faces: h_c + rc (h_c - h_1) and h_1 + ru (h_1 - h_2) */
        *den += (1.0 + rc) * cv;
        *num += cv * ((1.0 + rc + ru) * hk[c1] - ru * hk[c2]);
        break;
    case ST_NEAR: /* faces: h_c + rc (h_c - h_1) and h_1 */
        *den += (1.0 + rc) * cv;
        *num += (1.0 + rc) * cv * hk[c1];
        break;
    case ST_WALL: /* faces: h_c and the wall value */
        *den += cv;
        *num += cv * face_out(s, c, d, k);
        break;
    default:
        break;
    }
    (void)c2;
}

/* One velocity of Eq. (iteration): march the cells in upwind order, solving
 * delta h + v.grad h = delta E(m^n) + xi for h^{n+1} cell by cell.  Upwind
 * cells across a periodic seam still hold h^n (Gauss-Seidel seam lag). */
static void sweep_velocity(const si_ctx *s, int k)
{
    const int nx = s->nx, ny = s->ny, nc = s->nc;
    const double xi = s->xi[k], eta = s->eta[k];
    const double q = xi * xi + eta * eta;
    const double cx = fabs(xi) / s->dx;
    const int dxs = xi > 0 ? DIR_W : DIR_E;
    const int dys = eta > 0 ? DIR_S : DIR_N;
    const int sx = xi > 0 ? -1 : 1; /* step towards the upwind side */
    const int sy = eta > 0 ? -1 : 1;
    double *hk = s->h + (size_t)k * nc;
    for (int yy = 0; yy < ny; ++yy) {
        int y = eta > 0 ? yy : ny - 1 - yy;
        for (int xx = 0; xx < nx; ++xx) {
            int x = xi > 0 ? xx : nx - 1 - xx;
            int c = y * nx + x;
            if (s->solid[c])
                continue;
            double E = s->a0[c] + s->a1[c] * xi + s->a2[c] * eta + s->a3[c] * q;
            double num = s->dl[c] * E + s->drive * xi; /* pressure-gradient drive */
            double den = s->dl[c];
            upwind_axis(s, hk, s->codes[4 * c + dxs], c,
                        y * nx + wrap(x + sx, nx), y * nx + wrap(x + 2 * sx, nx),
                        dxs, k, cx, 0.5, 0.5, &den, &num);
            const int y1 = wrap(y + sy, ny), y2 = wrap(y + 2 * sy, ny);
            double cy = fabs(eta) / s->dx, rc = 0.5, ru = 0.5;
            if (s->dy) {
                cy = fabs(eta) / s->dy[y];
                rc = s->dy[y] / (s->dy[y] + s->dy[y1]);
                ru = s->dy[y1] / (s->dy[y1] + s->dy[y2]);
            }
            upwind_axis(s, hk, s->codes[4 * c + dys], c,
                        y1 * nx + x, y2 * nx + x, dys, k, cy, rc, ru, &den, &num);
            hk[c] = num / den;
        }
    }
}

/* Source iteration (Eq. iteration) to the stop rule.
 *   delta: 1 value or one per cell (ny*nx); alpha in (0,1].
 *   dy: ny row heights in units of H (nonuniform spacing across the
 *   channel), or NULL for rows of height 1/cells_per_H; cells_per_H always
 *   sets the x spacing.
 *   drive: factor of the pressure-gradient source xi (1: Poiseuille flow of
 *   Sec. III, 0: Couette flow of Sec. II); u_bottom, u_top: x velocities of
 *   the outer walls (walled channels only; Eq. (diffuse1) with U0/v_m = 1
 *   is u_top = 1).
 *   tol < 0 runs exactly max_iter iterations (timing mode).
 *   Outputs (ny*nx, zero in solids): rho (zero fluid mean), u1, u2, tau, p12.
 *   info_out = {Q, iterations, final relative change}.
 *   eps_hist (max_iter, nullable): relative change per iteration.
 *   h_out (K*ny*nx, nullable): converged perturbation h.
 * Returns 0 when the stop rule was met, 1 when max_iter was exhausted,
 * negative on bad input. */
int oracle_si_solve(int nx, int ny, const uint8_t *solid, int periodic_y,
                    double cells_per_H, const double *dy, int nv, const double *delta,
                    int delta_is_field, double alpha, double drive,
                    double u_bottom, double u_top, double tol, long max_iter,
                    double *rho, double *u1, double *u2, double *tau,
                    double *p12, double *info_out, double *eps_hist,
                    double *h_out)
{
    if (!(nx == 1 || nx >= 4) || ny < 4 || nv < 4 || (nv % 2) || cells_per_H <= 0 ||
        !(alpha > 0 && alpha <= 1) || max_iter < 1 || !isfinite(drive) ||
        !isfinite(u_bottom) || !isfinite(u_top) ||
        (periodic_y && (u_bottom != 0.0 || u_top != 0.0)))
        return -2;
    if (dy)
        for (int y = 0; y < ny; ++y)
            if (!(dy[y] > 0 && isfinite(dy[y])))
                return -2;
    const int K = nv * nv, nc = nx * ny;
    double *v = malloc(sizeof(double) * nv), *w1 = malloc(sizeof(double) * nv);
    double *xi = malloc(sizeof(double) * K), *eta = malloc(sizeof(double) * K);
    double *W = malloc(sizeof(double) * K), consts[7];
    uint8_t *codes = malloc((size_t)4 * nc);
    double *dl = malloc(sizeof(double) * nc);
    double *a = calloc((size_t)4 * nc, sizeof(double));
    double *mom = calloc((size_t)4 * nc, sizeof(double)); /* rho, u1, u2, e */
    double *u1old = calloc((size_t)nc, sizeof(double));
    double *rho_w = calloc((size_t)4 * nc, sizeof(double));
    double *rho_w_new = calloc((size_t)4 * nc, sizeof(double));
    int *wall_slot = malloc(sizeof(int) * nc);
    double *h = calloc((size_t)K * nc, sizeof(double));
    if (!v || !w1 || !xi || !eta || !W || !codes || !dl || !a || !mom || !u1old ||
        !rho_w || !rho_w_new || !wall_slot || !h)
        return -3;
    oracle_quadrature(nv, v, w1, xi, eta, W, consts);
    oracle_codes(nx, ny, solid, periodic_y, codes);
    const double m0 = consts[0], m2 = consts[1], c2 = consts[4], c4 = consts[5], D = consts[6];
    int nwall = 0;
    for (int c = 0; c < nc; ++c) {
        dl[c] = delta_is_field ? delta[c] : delta[0];
        int isw = 0;
        for (int d = 0; d < 4; ++d)
            isw |= (codes[4 * c + d] == ST_WALL);
        wall_slot[c] = isw ? nwall++ : -1;
        if (!solid[c] && (!isfinite(dl[c]) || dl[c] < 0))
            return -2;
    }
    double *hinc = calloc((size_t)(nwall > 0 ? nwall : 1) * 4 * K, sizeof(double));
    double *hinc_new = calloc((size_t)(nwall > 0 ? nwall : 1) * 4 * K, sizeof(double));
    if (!hinc || !hinc_new)
        return -3;
    si_ctx s = {nx, ny, nv, K, nc, periodic_y, 1.0 / cells_per_H, alpha, drive,
                {u_bottom, u_top}, xi, eta, W,
                solid, codes, dl, dy, a, a + nc, a + 2 * nc, a + 3 * nc,
                rho_w, wall_slot, hinc, h};

    double eps = INFINITY, eps_prev = -1.0;
    int npass = 0, status = 1;
    long it;
    for (it = 0; it < max_iter; ++it) {
        /* Gain term of Eq. (BGK) from m^n.  Reading: coefficients chosen so
         * that the discrete sums conserve mass, momentum and energy exactly;
         * with exact quadrature this is rho + 2 u.v + tau (|v|^2 - 1). */
        for (int c = 0; c < nc; ++c) {
            double r = mom[c], e = mom[3 * nc + c];
            double t = (e - r * c2) / c4;
            a[c] = r / m0 - t * c2;
            a[nc + c] = mom[nc + c] / m2;
            a[2 * nc + c] = mom[2 * nc + c] / m2;
            a[3 * nc + c] = t;
        }
        /* Eq. (diffuse2): the reflected density of each wall face is the
         * incident flux of h^n through that face (incident face values are the
         * same upwind reconstruction the transport uses, so each face carries
         * zero net mass flux), normalised by the discrete outgoing flux of a
         * unit density. */
        for (int c = 0; c < nc; ++c) {
            if (wall_slot[c] < 0)
                continue;
            int x = c % nx, y = c / nx;
            for (int d = 0; d < 4; ++d) {
                if (codes[4 * c + d] != ST_WALL)
                    continue;
                int od = d ^ 1; /* opposite side */
                int nb = od == DIR_W ? y * nx + wrap(x - 1, nx) :
                         od == DIR_E ? y * nx + wrap(x + 1, nx) :
                         od == DIR_S ? wrap(y - 1, ny) * nx + x : wrap(y + 1, ny) * nx + x;
                double num = 0.0;
                for (int k = 0; k < K; ++k) {
                    double vn = d == DIR_W ? -xi[k] : d == DIR_E ? xi[k] :
                                d == DIR_S ? -eta[k] : eta[k];
                    if (vn <= 0) /* only velocities moving into this wall */
                        continue;
                    double hc = h[(size_t)k * nc + c], hf;
                    if (codes[4 * c + od] == ST_WALL) {
                        hf = hc;
                    } else if (dy && d >= 2) {
                        /* face value extrapolated across a row of height dy[y] */
                        double r = dy[y] / (dy[y] + dy[nb / nx]);
                        hf = (1.0 + r) * hc - r * h[(size_t)k * nc + nb];
                    } else {
                        hf = 1.5 * hc - 0.5 * h[(size_t)k * nc + nb];
                    }
                    hinc_new[((size_t)wall_slot[c] * 4 + d) * K + k] = hf;
                    num += W[k] * vn * hf;
                }
                rho_w_new[4 * c + d] = num / D;
            }
        }
        { double *t = rho_w; rho_w = rho_w_new; rho_w_new = t; }
        { double *t = hinc; hinc = hinc_new; hinc_new = t; }
        s.rho_w = rho_w;
        s.hinc = hinc;
#pragma omp parallel for schedule(dynamic, 1)
        for (int k = 0; k < K; ++k)
            sweep_velocity(&s, k);

        /* Moments of Sec. II.A by quadrature. */
        memcpy(u1old, mom + nc, sizeof(double) * nc);
#pragma omp parallel for schedule(static)
        for (int c = 0; c < nc; ++c) {
            double r = 0, m1 = 0, m2v = 0, e = 0;
            if (!solid[c])
                for (int k = 0; k < K; ++k) {
                    double wh = W[k] * h[(size_t)k * nc + c];
                    r += wh;
                    m1 += wh * xi[k];
                    m2v += wh * eta[k];
                    e += wh * (xi[k] * xi[k] + eta[k] * eta[k]);
                }
            mom[c] = r;
            mom[nc + c] = m1;
            mom[2 * nc + c] = m2v;
            mom[3 * nc + c] = e;
        }
        /* Stop rule (Sec. II.A, end): relative change of u1 between two
         * iterations; reading: max norm, plus an a-posteriori bound from the
         * observed contraction, required on 3 consecutive iterations (a change
         * at the round-off floor passes without the bound). */
        double dmax = 0, umax = 0;
        for (int c = 0; c < nc; ++c) {
            if (solid[c])
                continue;
            double d = fabs(mom[nc + c] - u1old[c]);
            double u = fabs(mom[nc + c]);
            if (d > dmax)
                dmax = d;
            if (u > umax)
                umax = u;
        }
        eps = umax > 0 ? dmax / umax : (dmax == 0 ? 0.0 : INFINITY);
        if (eps_hist)
            eps_hist[it] = eps;
        if (tol >= 0) {
            int pass = 0;
            if (eps <= 16.0 * DBL_EPSILON) {
                pass = 1; /* change at the round-off floor: the ratio is noise */
            } else if (eps <= tol && eps_prev > 0) {
                double rh = eps / eps_prev;
                pass = rh < 1.0 && eps * rh / (1.0 - rh) <= tol;
            }
            npass = pass ? npass + 1 : 0;
            eps_prev = eps;
            if (npass >= 3) {
                status = 0;
                ++it;
                break;
            }
        }
    }

    /* Outputs; density gauge fixed to zero fluid mean (constant h is a null
     * vector of the discrete problem). */
    double rmean = 0, Qs = 0;
    int nf = 0;
    for (int c = 0; c < nc; ++c)
        if (!solid[c]) {
            rmean += mom[c];
            Qs += dy ? mom[nc + c] * dy[c / nx] : mom[nc + c];
            ++nf;
        }
    rmean /= nf;
    for (int c = 0; c < nc; ++c) {
        int f = !solid[c];
        double r = f ? mom[c] - rmean : 0.0;
        double e = f ? mom[3 * nc + c] - rmean * consts[2] / m0 : 0.0;
        if (rho) rho[c] = r;
        if (u1) u1[c] = f ? mom[nc + c] : 0.0;
        if (u2) u2[c] = f ? mom[2 * nc + c] : 0.0;
        if (tau) tau[c] = f ? e - r : 0.0;
        if (p12) {
            double p = 0;
            if (f)
                for (int k = 0; k < K; ++k)
                    p += W[k] * xi[k] * eta[k] * h[(size_t)k * nc + c];
            p12[c] = 2.0 * p;
        }
    }
    if (info_out) {
        /* Q = (1/L) * sum u1 * dA, L = nx * dx, dA = dx * dy */
        info_out[0] = dy ? Qs / nx : Qs / (cells_per_H * nx);
        info_out[1] = (double)it;
        info_out[2] = eps;
    }
    if (h_out)
        memcpy(h_out, h, sizeof(double) * (size_t)K * nc);
    free(v); free(w1); free(xi); free(eta); free(W); free(codes); free(dl); free(a);
    free(mom); free(u1old); free(rho_w); free(rho_w_new); free(wall_slot); free(h);
    free(hinc); free(hinc_new);
    return status;
}
