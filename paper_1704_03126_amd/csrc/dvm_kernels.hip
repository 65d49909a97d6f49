// dvm_kernels.hip -- gfx950 kernels of the linearized-BGK discrete velocity
// solver (source iteration of Eq. (iteration), arXiv:1704.03126 Sec. II.A).
//
// Mapping (one source iteration = k_sweep + k_moments + k_record + k_status):
//
//   k_sweep   One workgroup = one (instance, strip of <= 64 rows, velocity
//             group of G*V velocities of one quadrant).  Lane l of every wave
//             owns grid row l of the strip; the wave marches x on a skewed,
//             wrap-around diagonal (lane l treats x = (t - l) mod nx at step
//             t), so the upwind neighbours of a cell are the lane's own two
//             previous results (x direction) and the results of lanes l-1,
//             l-2 one and two steps earlier (y direction, moved with DPP
//             wave_shr).  Each lane carries V velocities at once; velocity
//             constants are wave-uniform.  Grids narrower than WRAP_MIN
//             use a skewed schedule without wrap-around (lane l treats x at
//             step x + l), which lags only the periodic seam.  The
//             perturbation h is never
//             written to memory: the lane accumulates the quadrature moments
//             of its V velocities, the G waves of the group add theirs in
//             LDS, and the group writes one partial per cell.  Values that
//             cross a strip boundary or the wrap-around diagonal come from
//             the previous iteration (seam and wrap buffers).
//   k_moments sums the partials of all velocity groups per cell (fixed order,
//             deterministic): rho, u1, u2, e and the four half-range fluxes.
//   k_record  builds the next sweep's per-cell record: the collision gain of
//             Eq. (BGK) (discrete-conservative coefficients, times delta, plus
//             the pressure-gradient drive) and the reflected densities of
//             Eq. (diffuse2) on every wall face; folds |du1|, |u1| into the
//             convergence test.
//   k_status  applies the stop rule of Sec. II.A per instance.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dvm_internal.h"

namespace dvm {

// ----------------------------------------------------------------- helpers
__device__ __forceinline__ double dpp_shr1(double old_v, double src)
{
    // wave_shr:1 -- lane l receives lane l-1; lane 0 keeps old_v.
    int2 o = __builtin_bit_cast(int2, old_v);
    int2 s = __builtin_bit_cast(int2, src);
    int2 r;
    r.x = __builtin_amdgcn_update_dpp(o.x, s.x, 0x138, 0xF, 0xF, false);
    r.y = __builtin_amdgcn_update_dpp(o.y, s.y, 0x138, 0xF, 0xF, false);
    return __builtin_bit_cast(double, r);
}

__device__ __forceinline__ float dpp_shr1(float old_v, float src)
{
    int o = __builtin_bit_cast(int, old_v);
    int s = __builtin_bit_cast(int, src);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(o, s, 0x138, 0xF, 0xF, false));
}

__device__ __forceinline__ double rcp_full(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ float rcp_full(float d)
{
    float r = __builtin_amdgcn_rcpf(d);
    float e = fmaf(-d, r, 1.0f);
    return fmaf(r, e, r);
}

__device__ __forceinline__ int wrap_mod(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Cell handled by lane `l` at step `t` of a strip pass.  Returns -1 when the
// lane has no cell at that step (beyond the strip, or x outside the grid when
// the schedule period exceeds nx).
__device__ __forceinline__ int strip_cell(const InstDev &in, int y0, int hs,
                                          bool xpos, bool ypos, int t, int l)
{
    if (l >= hs)
        return -1;
    int xr = wrap_mod(t - l, in.tp);
    if (xr >= in.nx)
        return -1;
    int x = xpos ? xr : in.nx - 1 - xr;
    int row = ypos ? y0 + l : y0 + hs - 1 - l;
    return row * in.nx + x;
}

// ------------------------------------------------------------------- sweep
template <typename T, int V, int G, bool FIELD, bool FINAL>
__global__ void __launch_bounds__(64 * G) k_sweep(SweepArgs<T> a)
{
    constexpr int S = 2;                 // steps per moment flush
    constexpr int NM = FINAL ? 1 : 4;    // moments accumulated
    __shared__ double lds_part[2][S][G][64][NM];
    __shared__ T lds_rinv[G * V][NSTENCIL];
    __shared__ T lds_pq[4][2];

    const WorkItem it = a.items[blockIdx.x];
    const InstDev in = a.inst[it.inst];
    if (!a.force && a.st[it.inst].active == 0)
        return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int q = it.group / a.gq;
    const bool xpos = (q & 1) == 0, ypos = (q & 2) == 0;
    const int dxs = xpos ? SIDE_W : SIDE_E;     // side the flow comes from
    const int dys = ypos ? SIDE_S : SIDE_N;
    const int kq0 = q * a.kq + (it.group % a.gq) * (G * V);   // first velocity
    const int kw = kq0 + wave * V;                              // this wave's
    const T *__restrict__ vt = a.vtab + (size_t)it.inst * a.kp4 * VT_STRIDE;

    const int y0 = it.strip * in.strip_h;
    const int hs = min(in.strip_h, in.ny - y0);
    const long long iter = a.st[it.inst].iter;
    const int par_w = (int)(iter & 1), par_r = par_w ^ 1;

    // per-group tables in LDS: reciprocal diagonals and stencil weights
    if (!FIELD) {
        for (int e = tid; e < G * V * NSTENCIL; e += 64 * G) {
            int v = e / NSTENCIL, ci = e % NSTENCIL;
            const T *c = vt + (size_t)(kq0 + v) * VT_STRIDE;
            T cx = c[VT_CX], cy = c[VT_CY], w = c[VT_W];
            T ax = (ci & 2) ? T(1) : T(1.5), ay = (ci & 1) ? T(1) : T(1.5);
            T den = T(in.delta) + ax * cx + ay * cy;
            lds_rinv[v][ci] = (ci == STENCIL_SOLID || w == T(0) || den == T(0)) ? T(0) : T(1) / den;
        }
    }
    if (tid < 4) {
        lds_pq[tid][0] = tid == CODE_INT ? T(2) : (tid == CODE_NEAR ? T(1.5) : T(0));
        lds_pq[tid][1] = tid == CODE_INT ? T(-0.5) : T(0);
    }
    __syncthreads();

    // the strip upstream of this one (values lagged by one iteration)
    const bool has_up = ypos ? (it.strip > 0 || in.periodic_y)
                             : (it.strip < in.nstrips - 1 || in.periodic_y);
    const int s_up = ypos ? (it.strip + in.nstrips - 1) % in.nstrips
                          : (it.strip + 1) % in.nstrips;
    const bool has_down = ypos ? (it.strip < in.nstrips - 1 || in.periodic_y)
                               : (it.strip > 0 || in.periodic_y);
    const size_t seam_row = (size_t)2 * a.kp4;   // values per x position
    const T *seam_in = a.seam + (size_t)par_r * a.seam_half + in.seam_off +
                       (size_t)s_up * in.nx * seam_row;
    T *seam_out = a.seam + (size_t)par_w * a.seam_half + in.seam_off +
                  (size_t)it.strip * in.nx * seam_row;
    const bool x_coupled = in.nx > 1;

    // wrap-around state: this lane's last two results and the last y-upstream
    T prev1[V], prev2[V], hs1p[V];
    T *wrapp = a.wrap + in.wrap_off +
               (((size_t)it.strip * (a.kp4 / V) + kw / V) * 64 + lane) * (3 * V);
#pragma unroll
    for (int v = 0; v < V; ++v) {
        prev1[v] = x_coupled ? wrapp[v] : T(0);
        prev2[v] = x_coupled ? wrapp[V + v] : T(0);
        hs1p[v] = x_coupled ? wrapp[2 * V + v] : T(0);
    }

    const long long cbase = in.cell_off;
    const int nsteps = in.tp;
    double acc[NM];
    int buf = 0;
    for (int t0 = 0; t0 < nsteps; t0 += S) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int t = t0 + s;
#pragma unroll
            for (int m = 0; m < NM; ++m)
                acc[m] = 0.0;
            if (t < nsteps) {
                const int cl = strip_cell(in, y0, hs, xpos, ypos, t, lane);
                const bool xact = wrap_mod(t - lane, in.tp) < in.nx;
                const long long cg = cbase + (cl < 0 ? 0 : cl);
                const int code = cl < 0 ? 0xFF : a.codes[cg];
                const int cxc = (code >> (2 * dxs)) & 3;
                const int cyc = (code >> (2 * dys)) & 3;
                const T *rec = a.rec + cg * REC_STRIDE;
                T b0 = rec[0], b1 = rec[1], b2 = rec[2], b3 = rec[3];
                T gx = rec[4 + dxs], gy = rec[4 + dys];
                T px = lds_pq[cxc][0], qx = lds_pq[cxc][1];
                T py = lds_pq[cyc][0], qy = lds_pq[cyc][1];
                const int ci = code == 0xFF ? STENCIL_SOLID
                                            : ((cxc == CODE_WALL) ? 2 : 0) + ((cyc == CODE_WALL) ? 1 : 0);
                T dl = T(0), ax = T(0), ay = T(0);
                if (FIELD) {
                    dl = T(a.delta_field[cg]);
                    ax = (cxc == CODE_WALL) ? T(1) : T(1.5);
                    ay = (cyc == CODE_WALL) ? T(1) : T(1.5);
                }
                if (code == 0xFF) {
                    b0 = b1 = b2 = b3 = gx = gy = T(0);
                }
                // lagged rows of the upstream strip for lane 0
                T sm1[V], sm2[V];
                const int x0 = xpos ? wrap_mod(t, in.tp) : in.nx - 1 - wrap_mod(t, in.tp);
                if (has_up && lane == 0 && wrap_mod(t, in.tp) < in.nx) {
                    const T *sp = seam_in + (size_t)x0 * seam_row;
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        sm2[v] = sp[kw + v];
                        sm1[v] = sp[a.kp4 + kw + v];
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        sm1[v] = sm2[v] = T(0);
                }
                T hout[V];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const T *c = vt + (size_t)(kw + v) * VT_STRIDE;
                    const T xi = c[VT_XI], eta = c[VT_ETA], qq = c[VT_Q];
                    const T cx = c[VT_CX], cy = c[VT_CY];
                    const double w = (double)c[VT_W];
                    const T hS1 = dpp_shr1(sm1[v], prev1[v]);
                    const T hS2 = dpp_shr1(sm2[v], hs1p[v]);
                    const T S = fma(b3, qq, fma(b2, eta, fma(b1, xi, b0)));
                    const T ux = fma(px, prev1[v], fma(qx, prev2[v], gx));
                    const T uy = fma(py, hS1, fma(qy, hS2, gy));
                    const T g = fma(cx, ux, fma(cy, uy, S));
                    T rinv;
                    if (FIELD) {
                        const T den = fma(ax, cx, fma(ay, cy, dl));
                        rinv = (ci == STENCIL_SOLID || w == 0.0) ? T(0) : rcp_full(den);
                    } else {
                        rinv = lds_rinv[wave * V + v][ci];
                    }
                    const T h = g * rinv;
                    const double hw = (double)h * w;
                    if (FINAL) {
                        acc[0] = fma((double)xi * (double)eta, hw, acc[0]);
                    } else {
                        acc[0] += hw;
                        acc[1] = fma((double)xi, hw, acc[1]);
                        acc[2] = fma((double)eta, hw, acc[2]);
                        acc[3] = fma((double)qq, hw, acc[3]);
                    }
                    hout[v] = h;
                    if (in.tp == in.nx) {
                        hs1p[v] = hS1;
                        prev2[v] = prev1[v];
                        prev1[v] = h;
                    } else {
                        // skewed schedule: outside its window of the pass a
                        // lane keeps the results it will need next
                        hs1p[v] = xact ? hS1 : hs1p[v];
                        prev2[v] = xact ? prev1[v] : prev2[v];
                        prev1[v] = xact ? h : prev1[v];
                    }
                }
                // the top two rows of the strip feed the next strip next iteration
                if (!FINAL && has_down && cl >= 0 && lane >= hs - 2) {
                    const int slot = lane - (hs - 2);
                    const int xx = cl % in.nx;
                    T *sp = seam_out + (size_t)xx * seam_row + (size_t)slot * a.kp4 + kw;
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        sp[v] = hout[v];
                }
            }
#pragma unroll
            for (int m = 0; m < NM; ++m)
                lds_part[buf][s][wave][lane][m] = acc[m];
        }
        __syncthreads();
        // group-wide sum of the partial moments of the S steps just done
        for (int e = tid; e < S * 64 * NM; e += 64 * G) {
            const int s = e / (64 * NM), l = (e / NM) % 64, m = e % NM;
            const int t = t0 + s;
            if (t >= nsteps)
                continue;
            const int cl = strip_cell(in, y0, hs, xpos, ypos, t, l);
            if (cl < 0)
                continue;
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < G; ++w)
                sum += lds_part[buf][s][w][l][m];
            a.part[((size_t)it.group * a.ncell + cbase + cl) * NM + m] = sum;
        }
        buf ^= 1;
    }
    if (!FINAL && x_coupled) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            wrapp[v] = prev1[v];
            wrapp[V + v] = prev2[v];
            wrapp[2 * V + v] = hs1p[v];
        }
    }
}

// ----------------------------------------------------------------- moments
__global__ void __launch_bounds__(256) k_moments(MomArgs a)
{
    const int inst = blockIdx.y;
    const InstDev in = a.inst[inst];
    if (a.st[inst].active == 0)
        return;
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= in.nx * in.ny)
        return;
    const long long cg = in.cell_off + c;
    double *m = a.mom + cg * MOM_STRIDE;
    if (a.codes[cg] == 0xFF) {
        for (int i = 0; i < MOM_STRIDE; ++i)
            m[i] = 0.0;
        return;
    }
    double r = 0, u1 = 0, u2 = 0, e = 0, fxp = 0, fxm = 0, fyp = 0, fym = 0;
    for (int q = 0; q < 4; ++q) {
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        for (int g = q * a.gq; g < (q + 1) * a.gq; ++g) {
            const double *p = a.part + ((size_t)g * a.ncell + cg) * 4;
            s0 += p[0];
            s1 += p[1];
            s2 += p[2];
            s3 += p[3];
        }
        r += s0;
        u1 += s1;
        u2 += s2;
        e += s3;
        if ((q & 1) == 0) fxp += s1; else fxm += s1;
        if ((q & 2) == 0) fyp += s2; else fym += s2;
    }
    m[MOM_RHO] = r;
    m[MOM_U1] = u1;
    m[MOM_U2] = u2;
    m[MOM_E] = e;
    m[MOM_FXP] = fxp;
    m[MOM_FXM] = fxm;
    m[MOM_FYP] = fyp;
    m[MOM_FYM] = fym;
}

// sum of a single diagnostic moment (shear stress) over velocity groups
__global__ void __launch_bounds__(256) k_sum1(MomArgs a, double *out)
{
    const int inst = blockIdx.y;
    const InstDev in = a.inst[inst];
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= in.nx * in.ny)
        return;
    const long long cg = in.cell_off + c;
    double s = 0.0;
    if (a.codes[cg] != 0xFF)
        for (int g = 0; g < 4 * a.gq; ++g)
            s += a.part[(size_t)g * a.ncell + cg];
    out[cg] = 2.0 * s;
}

// ------------------------------------------------------------------ record
template <typename T>
__global__ void __launch_bounds__(256) k_record(RecArgs<T> a)
{
    const int inst = blockIdx.y;
    const InstDev in = a.inst[inst];
    SolveState *st = a.st + inst;
    if (st->active == 0)
        return;
    const int c = blockIdx.x * 256 + threadIdx.x;
    double diff = 0.0, absu = 0.0;
    if (c < in.nx * in.ny) {
        const long long cg = in.cell_off + c;
        T *rec = a.rec + cg * REC_STRIDE;
        const int code = a.codes[cg];
        if (code == 0xFF) {
            for (int i = 0; i < REC_STRIDE; ++i)
                rec[i] = T(0);
        } else {
            const double *m = a.mom + cg * MOM_STRIDE;
            const double r = m[MOM_RHO], u1 = m[MOM_U1], u2 = m[MOM_U2], e = m[MOM_E];
            const double t = (e - r * a.c2) / a.c4;
            const double dl = in.field ? a.delta_field[cg] : in.delta;
            rec[0] = T(dl * (r / a.m0 - t * a.c2));
            rec[1] = T(dl * (u1 / a.m2) + in.drive);
            rec[2] = T(dl * (u2 / a.m2));
            rec[3] = T(dl * t);
            const int x = c % in.nx, y = c / in.nx;
            for (int d = 0; d < 4; ++d) {
                const int cd = (code >> (2 * d)) & 3;
                double gval = 0.0;
                if (cd == CODE_WALL) {
                    // incident flux through the wall face on side d: the
                    // half-range flux of the cell, extrapolated from the
                    // neighbour on the opposite side unless that side is a
                    // wall as well (first-order face value)
                    const int od = d ^ 1;
                    const int co = (code >> (2 * od)) & 3;
                    const int hf = (d == SIDE_W) ? MOM_FXM : (d == SIDE_E) ? MOM_FXP
                                 : (d == SIDE_S) ? MOM_FYM : MOM_FYP;
                    const double sgn = (d == SIDE_W || d == SIDE_S) ? -1.0 : 1.0;
                    double f = m[hf];
                    if (co != CODE_WALL && co != CODE_NONE) {
                        int nxx = x, nyy = y;
                        if (od == SIDE_W) nxx = (x + in.nx - 1) % in.nx;
                        else if (od == SIDE_E) nxx = (x + 1) % in.nx;
                        else if (od == SIDE_S) nyy = (y + in.ny - 1) % in.ny;
                        else nyy = (y + 1) % in.ny;
                        const double fo = a.mom[(in.cell_off + (long long)nyy * in.nx + nxx) * MOM_STRIDE + hf];
                        f = 1.5 * f - 0.5 * fo;
                    }
                    gval = in.alpha * sgn * f / a.D;
                }
                rec[4 + d] = T(gval);
            }
            const double up = a.u1prev[cg];
            diff = fabs(u1 - up);
            absu = fabs(u1);
            a.u1prev[cg] = u1;
        }
    }
    // block max, then one atomic per block (max is order independent)
    __shared__ double sd[256], sa[256];
    sd[threadIdx.x] = diff;
    sa[threadIdx.x] = absu;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + o]);
            sa[threadIdx.x] = fmax(sa[threadIdx.x], sa[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // a NaN anywhere must reach the status kernel: encode it as +inf
        double dmax = sd[0] != sd[0] ? __builtin_inf() : sd[0];
        double amax = sa[0] != sa[0] ? __builtin_inf() : sa[0];
        atomicMax(&st->maxdiff_bits, (unsigned long long)__builtin_bit_cast(long long, dmax));
        atomicMax(&st->maxabs_bits, (unsigned long long)__builtin_bit_cast(long long, amax));
    }
}

// ------------------------------------------------------------------ status
__global__ void k_status(SolveState *st, int n, double tol, long long max_iter)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    SolveState &s = st[i];
    if (s.active == 0)
        return;
    const double dmax = __builtin_bit_cast(double, (long long)s.maxdiff_bits);
    const double amax = __builtin_bit_cast(double, (long long)s.maxabs_bits);
    s.maxdiff_bits = 0ull;
    s.maxabs_bits = 0ull;
    s.iter += 1;
    double eps = amax > 0.0 ? dmax / amax : (dmax == 0.0 ? 0.0 : __builtin_inf());
    // iterates of this linear problem are O(delta) at most; values beyond
    // 1e30 (or non-finite) mean the lagged iteration is amplifying errors
    if (!(amax < 1e30) || eps != eps) {
        s.status = STATUS_DIVERGED;
        s.active = 0;
        s.eps = eps;
        return;
    }
    // Sec. II.A stop rule on the relative change of u1, with the a-posteriori
    // bound from the observed contraction, on 3 consecutive iterations; a
    // change at the round-off floor passes without the bound.
    int pass = 0;
    double est = eps;
    if (eps <= 16.0 * 2.220446049250313e-16) {
        pass = 1;
    } else if (eps <= tol && s.eps_prev > 0.0) {
        const double rh = eps / s.eps_prev;
        est = rh < 1.0 ? eps * rh / (1.0 - rh) : __builtin_inf();
        pass = rh < 1.0 && est <= tol;
    }
    s.npass = pass ? s.npass + 1 : 0;
    s.eps_prev = eps;
    s.eps = eps;
    s.est = est;
    if (s.npass >= 3) {
        s.status = STATUS_CONVERGED;
        s.active = 0;
    } else if (s.iter - s.iter0 >= max_iter) {
        s.status = STATUS_MAXITER;
        s.active = 0;
    }
}

// ----------------------------------------------------------- misc kernels
__global__ void k_fill_zero(double *p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void k_fill_zero_f(float *p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

__global__ void k_copy(const double *__restrict__ src, double *__restrict__ dst, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// --------------------------------------------------------- host launchers
template <typename T, int V, int G, bool FIELD, bool FINAL>
static hipError_t launch_sweep_t(const SweepArgs<T> &a, int nitems, hipStream_t s)
{
    hipLaunchKernelGGL((k_sweep<T, V, G, FIELD, FINAL>), dim3(nitems), dim3(64 * G), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep(const SweepArgs<T> &a, int nitems, int V, int G, bool field,
                        bool final_pass, hipStream_t s)
{
#define DVM_SW(VV, GG)                                                                  \
    if (V == VV && G == GG) {                                                            \
        if (final_pass)                                                                  \
            return field ? launch_sweep_t<T, VV, GG, true, true>(a, nitems, s)           \
                         : launch_sweep_t<T, VV, GG, false, true>(a, nitems, s);         \
        return field ? launch_sweep_t<T, VV, GG, true, false>(a, nitems, s)              \
                     : launch_sweep_t<T, VV, GG, false, false>(a, nitems, s);            \
    }
    DVM_SW(8, 8)
    DVM_SW(4, 8)
    DVM_SW(8, 4)
    DVM_SW(4, 4)
    DVM_SW(4, 16)
    DVM_SW(2, 16)
#undef DVM_SW
    return hipErrorInvalidValue;
}

template hipError_t launch_sweep<double>(const SweepArgs<double> &, int, int, int, bool, bool, hipStream_t);
template hipError_t launch_sweep<float>(const SweepArgs<float> &, int, int, int, bool, bool, hipStream_t);

hipError_t launch_moments(const MomArgs &a, int max_cells, int n_inst, hipStream_t s)
{
    hipLaunchKernelGGL(k_moments, dim3((max_cells + 255) / 256, n_inst), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sum1(const MomArgs &a, double *out, int max_cells, int n_inst, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum1, dim3((max_cells + 255) / 256, n_inst), dim3(256), 0, s, a, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_record(const RecArgs<T> &a, int max_cells, int n_inst, hipStream_t s)
{
    hipLaunchKernelGGL((k_record<T>), dim3((max_cells + 255) / 256, n_inst), dim3(256), 0, s, a);
    return hipGetLastError();
}
template hipError_t launch_record<double>(const RecArgs<double> &, int, int, hipStream_t);
template hipError_t launch_record<float>(const RecArgs<float> &, int, int, hipStream_t);

hipError_t launch_status(SolveState *st, int n, double tol, long long max_iter, hipStream_t s)
{
    hipLaunchKernelGGL(k_status, dim3((n + 63) / 64), dim3(64), 0, s, st, n, tol, max_iter);
    return hipGetLastError();
}

hipError_t launch_zero(double *p, size_t n, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill_zero, dim3(1024), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_zero_f(float *p, size_t n, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill_zero_f, dim3(1024), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_copy(const double *src, double *dst, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy, dim3(2048), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

} // namespace dvm
