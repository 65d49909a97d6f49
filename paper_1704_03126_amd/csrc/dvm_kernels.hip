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

// ------------------------------------------------------------------- sweep
// Velocity constants are read through the constant address space so that the
// compiler keeps them on the scalar path (they are wave-uniform).
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

template <typename T>
__device__ __forceinline__ T ldc(cptr<T> p, int i)
{
    return p[i];
}

// Steps of a pass staged per chunk: a multiple of 6 so that the 3-register
// rotation of the x-upwind values and the 2-register rotation of the
// y-upwind value are pure renaming inside a chunk.
constexpr int SWEEP_C = 6;

// One velocity of one step for one lane (see k_sweep).  xa: the lane has a
// cell at this step (false keeps the registers, used off the lane's window).
template <typename T, bool FIELD, bool FINAL, bool HOLD>
__device__ __forceinline__ void sweep_update(
    T &p1, T &p2, T &pn, T &hs1p, T &hs1n, T &hout, double *acc,
    T sm1, T sm2, T b0, T b1, T b2, T b3, T gx, T gy, T px, T qx, T py, T qy,
    T rinv_or_dl, T ax, T ay, bool solid, bool xa,
    T xi, T eta, T qq, T cx, T cy, double w, double wxi, double weta, double wq)
{
    const T hS1 = dpp_shr1(sm1, p1);
    const T hS2 = dpp_shr1(sm2, hs1p);
    const T S = fma(b3, qq, fma(b2, eta, fma(b1, xi, b0)));
    const T ux = fma(px, p1, fma(qx, p2, gx));
    const T uy = fma(py, hS1, fma(qy, hS2, gy));
    const T g = fma(cx, ux, fma(cy, uy, S));
    T rinv;
    if (FIELD) {
        const T den = fma(ax, cx, fma(ay, cy, rinv_or_dl));
        rinv = (solid || w == 0.0) ? T(0) : rcp_full(den);
    } else {
        rinv = rinv_or_dl;
    }
    const T h = g * rinv;
    const double hd = (double)h;
    if (FINAL) {
        acc[0] = fma(wxi * (double)eta, hd, acc[0]);
    } else {
        acc[0] = fma(w, hd, acc[0]);
        acc[1] = fma(wxi, hd, acc[1]);
        acc[2] = fma(weta, hd, acc[2]);
        acc[3] = fma(wq, hd, acc[3]);
    }
    hout = h;
    if (HOLD) {
        // keep prev1/prev2/hs1 when the lane has no cell at this step
        pn = xa ? h : p1;
        p1 = xa ? p1 : p2;        // becomes prev2 of the next step
        hs1n = xa ? hS1 : hs1p;
    } else {
        pn = h;
        hs1n = hS1;
    }
}

template <typename T, int V, int G, bool FIELD, bool FINAL>
__global__ void __launch_bounds__(64 * G) k_sweep(SweepArgs<T> a)
{
    constexpr int C = SWEEP_C;                 // steps per chunk
    constexpr int NM = FINAL ? 1 : 4;          // moments accumulated
    constexpr int P = G * V;                   // velocities of the group
    constexpr int UPE = 8 * sizeof(T) / 16;    // 16-byte units per record
    __shared__ __attribute__((aligned(16))) T st_rec[2][C][64][8];
    __shared__ uint8_t st_code[2][C][64];
    __shared__ int st_cell[2][C][64];
    __shared__ __attribute__((aligned(16))) T st_seam[2][C][2][P];
    __shared__ double lds_part[C][G][64][NM];
    __shared__ T lds_rinv[P][NSTENCIL];
    __shared__ __attribute__((aligned(16))) T lds_pq[4][2];

    const WorkItem it = a.items[blockIdx.x];
    const InstDev in = a.inst[it.inst];
    if (!a.force && a.st[it.inst].active == 0)
        return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int q = it.group / a.gq;
    const bool xpos = (q & 1) == 0, ypos = (q & 2) == 0;
    const int kq0 = q * a.kq + (it.group % a.gq) * P;   // first velocity of the group
    const int kw = kq0 + wave * V;                      // first velocity of this wave
    cptr<T> vt = (cptr<T>)(a.vtab + (size_t)it.inst * a.kp4 * VT_STRIDE);

    const int y0 = it.strip * in.strip_h;
    const int hs = min(in.strip_h, in.ny - y0);
    const long long iter = a.st[it.inst].iter;
    const int par_w = (int)(iter & 1), par_r = par_w ^ 1;
    const int tp = in.tp, nx = in.nx;
    const size_t ebase = (size_t)in.sk_off + ((size_t)(q * in.nstrips + it.strip) * tp) * 64;
    const T *__restrict__ srec = a.srec + ebase * 8;
    const uint8_t *__restrict__ scode = a.scode + ebase;
    const int *__restrict__ smap = a.smap + ebase;

    if (!FIELD) {
        for (int e = tid; e < P * NSTENCIL; e += 64 * G) {
            const int v = e / NSTENCIL, ci = e % NSTENCIL;
            const T cx = vt[(kq0 + v) * VT_STRIDE + VT_CX], cy = vt[(kq0 + v) * VT_STRIDE + VT_CY];
            const T w = vt[(kq0 + v) * VT_STRIDE + VT_W];
            const T ax = (ci & 2) ? T(1) : T(1.5), ay = (ci & 1) ? T(1) : T(1.5);
            const T den = T(in.delta) + ax * cx + ay * cy;
            lds_rinv[v][ci] = (ci == STENCIL_SOLID || w == T(0) || den == T(0)) ? T(0) : T(1) / den;
        }
    }
    if (tid < 4) {
        lds_pq[tid][0] = tid == CODE_INT ? T(2) : (tid == CODE_NEAR ? T(1.5) : T(0));
        lds_pq[tid][1] = tid == CODE_INT ? T(-0.5) : T(0);
    }

    const bool has_up = ypos ? (it.strip > 0 || in.periodic_y)
                             : (it.strip < in.nstrips - 1 || in.periodic_y);
    const int s_up = ypos ? (it.strip + in.nstrips - 1) % in.nstrips : (it.strip + 1) % in.nstrips;
    const bool has_down = ypos ? (it.strip < in.nstrips - 1 || in.periodic_y)
                               : (it.strip > 0 || in.periodic_y);
    const size_t seam_row = (size_t)2 * a.kp4;
    const T *seam_in = a.seam + (size_t)par_r * a.seam_half + in.seam_off + (size_t)s_up * nx * seam_row;
    T *seam_out = a.seam + (size_t)par_w * a.seam_half + in.seam_off + (size_t)it.strip * nx * seam_row;
    const bool x_coupled = nx > 1;

    // ---- staging of one chunk of steps into LDS buffer b (global loads are
    //      issued into registers first and stored after the current chunk)
    constexpr int REC_UNITS = C * 64 * UPE;
    constexpr int RU_PER_T = (REC_UNITS + 64 * G - 1) / (64 * G);
    constexpr int SEAM_VALS = C * 2 * P;
    constexpr int SV_PER_T = (SEAM_VALS + 64 * G - 1) / (64 * G);
    constexpr int CC_PER_T = (C * 64 + 64 * G - 1) / (64 * G);
    uint4 ru[RU_PER_T];
    T sv[SV_PER_T];
    int cc[CC_PER_T];
    uint8_t cb[CC_PER_T];
    auto issue = [&](int c) {
        const int t0 = c * C;
#pragma unroll
        for (int r = 0; r < RU_PER_T; ++r) {
            const int u = tid + r * 64 * G;
            ru[r] = make_uint4(0, 0, 0, 0);
            if (u < REC_UNITS && t0 + (u / UPE) / 64 < tp)
                ru[r] = reinterpret_cast<const uint4 *>(srec + ((size_t)t0 * 64) * 8)[u];
        }
#pragma unroll
        for (int r = 0; r < CC_PER_T; ++r) {
            const int e = tid + r * 64 * G;
            cc[r] = -1;
            cb[r] = 0x1F;
            if (e < C * 64 && t0 + e / 64 < tp) {
                cc[r] = smap[(size_t)t0 * 64 + e];
                cb[r] = scode[(size_t)t0 * 64 + e];
            }
        }
#pragma unroll
        for (int r = 0; r < SV_PER_T; ++r) {
            const int e = tid + r * 64 * G;       // (s, slot, j)
            sv[r] = T(0);
            if (e < SEAM_VALS && has_up) {
                const int sidx = e / (2 * P), slot = (e / P) & 1, j = e % P;
                const int xr = t0 + sidx;            // lane 0 treats x_r = t
                if (xr < nx) {
                    const int x0 = xpos ? xr : nx - 1 - xr;
                    sv[r] = seam_in[(size_t)x0 * seam_row + (size_t)slot * a.kp4 + kq0 + j];
                }
            }
        }
    };
    auto commit = [&](int b) {
#pragma unroll
        for (int r = 0; r < RU_PER_T; ++r) {
            const int u = tid + r * 64 * G;
            if (u < REC_UNITS)
                reinterpret_cast<uint4 *>(&st_rec[b][0][0][0])[u] = ru[r];
        }
#pragma unroll
        for (int r = 0; r < CC_PER_T; ++r) {
            const int e = tid + r * 64 * G;
            if (e < C * 64) {
                (&st_cell[b][0][0])[e] = cc[r];
                (&st_code[b][0][0])[e] = cb[r];
            }
        }
#pragma unroll
        for (int r = 0; r < SV_PER_T; ++r) {
            const int e = tid + r * 64 * G;
            if (e < SEAM_VALS)
                (&st_seam[b][0][0][0])[e] = sv[r];
        }
    };

    // velocity constants of this wave, for the whole pass
    T cxi[V], ceta[V], cqq[V], ccx[V], ccy[V];
    double cw[V], cwxi[V], cweta[V], cwq[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int k = (kw + v) * VT_STRIDE;
        cxi[v] = ldc(vt, k + VT_XI);
        ceta[v] = ldc(vt, k + VT_ETA);
        cqq[v] = ldc(vt, k + VT_Q);
        ccx[v] = ldc(vt, k + VT_CX);
        ccy[v] = ldc(vt, k + VT_CY);
        cw[v] = (double)ldc(vt, k + VT_W);
        cwxi[v] = cw[v] * (double)cxi[v];
        cweta[v] = cw[v] * (double)ceta[v];
        cwq[v] = cw[v] * (double)cqq[v];
    }

    // rotating registers: x-upwind values A (prev1), B (prev2), X (free);
    // y-upwind chain H0 (current hs1), H1 (free)
    T rA[V], rB[V], rX[V], rH0[V], rH1[V];
    T *wrapp = a.wrap + in.wrap_off + (((size_t)it.strip * (a.kp4 / V) + kw / V) * 64 + lane) * (3 * V);
#pragma unroll
    for (int v = 0; v < V; ++v) {
        rA[v] = x_coupled ? wrapp[v] : T(0);
        rB[v] = x_coupled ? wrapp[V + v] : T(0);
        rH0[v] = x_coupled ? wrapp[2 * V + v] : T(0);
        rX[v] = T(0);
        rH1[v] = T(0);
    }

    const long long cbase = in.cell_off;
    const int nchunks = (tp + C - 1) / C;
    const bool skew = tp != nx;
    // x position (in sweep order) of this lane's cell at the chunk start
    int xr0 = (tp - (lane % tp)) % tp;

    issue(0);
    commit(0);
    __syncthreads();

    // one step: s-th step of the chunk in buffer b; (PA, PB, PX) and (HA, HB)
    // are the register roles of this step in the rotation
    auto step = [&](int b, int s, int t, T *PA, T *PB, T *PX, T *HA, T *HB, bool hold, bool xa) {
        double acc[NM];
#pragma unroll
        for (int m = 0; m < NM; ++m)
            acc[m] = 0.0;
        const T *rec = &st_rec[b][s][lane][0];
        const int code = st_code[b][s][lane];
        const int cxc = code & 3, cyc = (code >> 2) & 3;
        const bool solid = (code >> 4) != 0;
        const T b0 = rec[0], b1 = rec[1], b2 = rec[2], b3 = rec[3];
        const T gx = rec[4], gy = rec[5];
        const T px = lds_pq[cxc][0], qx = lds_pq[cxc][1];
        const T py = lds_pq[cyc][0], qy = lds_pq[cyc][1];
        const int ci = solid ? STENCIL_SOLID : ((cxc == CODE_WALL) ? 2 : 0) + ((cyc == CODE_WALL) ? 1 : 0);
        T ax = T(0), ay = T(0), rdl[V];
        if (FIELD) {
            ax = (cxc == CODE_WALL) ? T(1) : T(1.5);
            ay = (cyc == CODE_WALL) ? T(1) : T(1.5);
#pragma unroll
            for (int v = 0; v < V; ++v)
                rdl[v] = rec[6];
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v)
                rdl[v] = lds_rinv[wave * V + v][ci];
        }
        T sm1[V], sm2[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            sm1[v] = has_up ? st_seam[b][s][1][wave * V + v] : T(0);
            sm2[v] = has_up ? st_seam[b][s][0][wave * V + v] : T(0);
        }
        T hout[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if (hold)
                sweep_update<T, FIELD, FINAL, true>(PA[v], PB[v], PX[v], HA[v], HB[v], hout[v], acc,
                                                    sm1[v], sm2[v], b0, b1, b2, b3, gx, gy, px, qx, py, qy,
                                                    rdl[v], ax, ay, solid, xa, cxi[v], ceta[v], cqq[v],
                                                    ccx[v], ccy[v], cw[v], cwxi[v], cweta[v], cwq[v]);
            else
                sweep_update<T, FIELD, FINAL, false>(PA[v], PB[v], PX[v], HA[v], HB[v], hout[v], acc,
                                                     sm1[v], sm2[v], b0, b1, b2, b3, gx, gy, px, qx, py, qy,
                                                     rdl[v], ax, ay, solid, xa, cxi[v], ceta[v], cqq[v],
                                                     ccx[v], ccy[v], cw[v], cwxi[v], cweta[v], cwq[v]);
        }
        // the last two rows of the strip feed the next strip next iteration
        if (!FINAL && has_down && t < tp && lane >= hs - 2 && lane < hs) {
            const int cl = st_cell[b][s][lane];
            if (cl >= 0) {
                const int slot = lane - (hs - 2);
                T *sp = seam_out + (size_t)(cl % nx) * seam_row + (size_t)slot * a.kp4 + kw;
#pragma unroll
                for (int v = 0; v < V; ++v)
                    sp[v] = hout[v];
            }
        }
#pragma unroll
        for (int m = 0; m < NM; ++m)
            lds_part[s][wave][lane][m] = acc[m];
    };

    for (int c = 0; c < nchunks; ++c) {
        const int b = c & 1;
        const int t0 = c * C;
        if (c + 1 < nchunks)
            issue(c + 1);
        // register roles cycle with period 6: (A,B,X)(H0,H1) -> (X,A,B)(H1,H0) -> ...
        if (!skew && t0 + C <= tp) {
            step(b, 0, t0 + 0, rA, rB, rX, rH0, rH1, false, true);
            step(b, 1, t0 + 1, rX, rA, rB, rH1, rH0, false, true);
            step(b, 2, t0 + 2, rB, rX, rA, rH0, rH1, false, true);
            step(b, 3, t0 + 3, rA, rB, rX, rH1, rH0, false, true);
            step(b, 4, t0 + 4, rX, rA, rB, rH0, rH1, false, true);
            step(b, 5, t0 + 5, rB, rX, rA, rH1, rH0, false, true);
        } else {
            // skewed schedule or the partial last chunk: lanes keep their
            // registers at steps where they have no cell
            int xr = xr0;
            bool xa[C];
#pragma unroll
            for (int s = 0; s < C; ++s) {
                xa[s] = (t0 + s < tp) && (xr < nx);
                xr = (xr + 1 == tp) ? 0 : xr + 1;
            }
            step(b, 0, t0 + 0, rA, rB, rX, rH0, rH1, true, xa[0]);
            step(b, 1, t0 + 1, rX, rA, rB, rH1, rH0, true, xa[1]);
            step(b, 2, t0 + 2, rB, rX, rA, rH0, rH1, true, xa[2]);
            step(b, 3, t0 + 3, rA, rB, rX, rH1, rH0, true, xa[3]);
            step(b, 4, t0 + 4, rX, rA, rB, rH0, rH1, true, xa[4]);
            step(b, 5, t0 + 5, rB, rX, rA, rH1, rH0, true, xa[5]);
        }
        xr0 = (xr0 + C) % tp;
        if (c + 1 < nchunks)
            commit(b ^ 1);
        __syncthreads();
        // group-wide sum of the partial moments of this chunk
        for (int e = tid; e < C * 64 * NM; e += 64 * G) {
            const int s = e / (64 * NM), l = (e / NM) % 64, m = e % NM;
            const int cl = st_cell[b][s][l];
            if (cl < 0 || (st_code[b][s][l] >> 4))
                continue;
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < G; ++w)
                sum += lds_part[s][w][l][m];
            a.part[((size_t)it.group * a.ncell + cbase + cl) * NM + m] = sum;
        }
        __syncthreads();
    }
    if (!FINAL && x_coupled) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            wrapp[v] = rA[v];
            wrapp[V + v] = rB[v];
            wrapp[2 * V + v] = rH0[v];
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
        const int code = a.codes[cg];
        if (code != 0xFF) {
            const double *m = a.mom + cg * MOM_STRIDE;
            const double r = m[MOM_RHO], u1 = m[MOM_U1], u2 = m[MOM_U2], e = m[MOM_E];
            const double t = (e - r * a.c2) / a.c4;
            const double dl = in.field ? a.delta_field[cg] : in.delta;
            T rec[8];
            rec[0] = T(dl * (r / a.m0 - t * a.c2));
            rec[1] = T(dl * (u1 / a.m2) + in.drive);
            rec[2] = T(dl * (u2 / a.m2));
            rec[3] = T(dl * t);
            rec[6] = T(dl);
            rec[7] = T(0);
            double gside[4];
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
                gside[d] = gval;
            }
            // one copy per quadrant, in that quadrant's sweep order
            for (int qd = 0; qd < 4; ++qd) {
                rec[4] = T(gside[(qd & 1) ? SIDE_E : SIDE_W]);
                rec[5] = T(gside[(qd & 2) ? SIDE_N : SIDE_S]);
                const long long pos = a.spos[cg * 4 + qd];
                T *dst = a.srec + pos * 8;
                for (int i = 0; i < 8; ++i)
                    dst[i] = rec[i];
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
    DVM_SW(4, 8)
    DVM_SW(8, 4)
    DVM_SW(4, 4)
    DVM_SW(2, 8)
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
