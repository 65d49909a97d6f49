// dvm_kernels.hip -- gfx950 kernels of the linearized-BGK discrete velocity
// solver (source iteration of Eq. (iteration), arXiv:1704.03126 Sec. II.A).
//
// Mapping (one source iteration = k_sweep + k_moments + k_record + k_status):
//
//   k_sweep   One workgroup = one (instance, strip of <= 64 rows, velocity
//             group of G*V velocities of one quadrant).  Lane l of every wave
//             owns grid row l of the strip; the wave marches x on a skewed
//             diagonal (lane l treats x = t - l at step t, x counted from the
//             upwind side), so the upwind neighbours of a cell are the lane's
//             own two previous results (x direction) and the results of
//             lanes l-1, l-2 one and two steps earlier (y direction, moved
//             with DPP wave_shr).  Only values that cross the periodic x seam
//             or a strip boundary come from the previous iteration (wrap and
//             seam buffers).  The optional wrap-around schedule (x = (t - l)
//             mod nx) saves the 63 fill steps but also lags the y coupling of
//             every lane's first cell.  Each lane carries V velocities at
//             once; velocity constants are wave-uniform.  The perturbation h
//             is never written to memory (except by the checkpoint pass of
//             the gradient): the lane accumulates the quadrature moments of
//             its V velocities, the G waves of the group add theirs in LDS,
//             and the group writes one partial per cell.
//   k_moments sums the partials of all velocity groups per cell (fixed order,
//             deterministic): rho, u1, u2, e and the four half-range fluxes.
//   k_record  builds the next sweep's per-cell record: the collision gain of
//             Eq. (BGK) (discrete-conservative coefficients, times delta, plus
//             the pressure-gradient drive) and the reflected densities of
//             Eq. (diffuse2) on every wall face; folds |du1|, |u1| into the
//             convergence test.
//   k_status  applies the stop rule of Sec. II.A per instance.
#include <hip/hip_runtime.h>
#include <hip/hip_cooperative_groups.h>
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

// Plain FP32 sweeps in 8-wave workgroups are held to 128 VGPRs (4 waves per
// SIMD): with their half-size LDS staging two workgroups then share a CU,
// twice the waves of the FP64 sweep to hide the LDS and DPP latencies of the
// diagonal (measured on the uneven batch: 3.6 ms per sweep against 5.3 ms at
// the compiler's 144 VGPRs).  The passes with face records (specular walls,
// gradient) keep their registers: 128 would spill inside the step loop.
template <typename T, int G, int MODE>
constexpr int sweep_waves_per_eu()
{
    return (sizeof(T) == 4 && G == 8 && (MODE & (MODE_SPEC | MODE_CKPT | MODE_GRAD)) == 0) ? 4 : 1;
}

// One work item of the sweep (instance, strip, velocity group) by the
// calling workgroup; the body of k_sweep and of the persistent iteration.
template <typename T, int V, int G, int MODE>
__device__ __forceinline__ void sweep_item(SweepArgs<T> a, int item)
{
    constexpr bool FIELD = (MODE & MODE_FIELD) != 0;
    constexpr bool SPEC = (MODE & MODE_SPEC) != 0;
    constexpr bool ADJ = (MODE & MODE_ADJ) != 0;
    constexpr bool P12 = (MODE & MODE_P12) != 0;
    constexpr bool CKPT = (MODE & MODE_CKPT) != 0;
    constexpr bool GRAD = (MODE & MODE_GRAD) != 0;
    // xi (and |xi|/dx) uniform over the wave's velocities: the collision gain's
    // b0 + b1 xi and the u1 partial (xi times the density partial) once per step
    constexpr bool XU = (MODE & MODE_XU) != 0;
    constexpr bool FACES = SPEC || CKPT || GRAD;          // face records needed
    constexpr bool FBWRITE = (SPEC || CKPT || GRAD) && !P12;
    constexpr int C = SWEEP_C;                 // steps per chunk
    // moments gathered: 4 (rho, u1, u2, e) and an extra one (P12 or gradient)
    constexpr int NACC = P12 ? 1 : (GRAD ? 5 : 4);
    // moment partials: an FP64 sweep sums in FP64; an FP32 sweep (the
    // refinement's correction, itself held in FP32) sums the V velocities of
    // a lane in FP32 and the G waves of the group in FP64
    using AccT = typename std::conditional<sizeof(T) == 4, float, double>::type;
    // steps per partial flush: the whole chunk unless LDS is short
    // (4-wave workgroups: half the partial buffer, so two workgroups share
    // a CU)
    constexpr int FL = (FACES || NACC > 4 || G > 8 || G <= 4) ? C / 2 : C;
    constexpr int P = G * V;                   // velocities of the group
    constexpr int UPE = 8 * sizeof(T) / 16;    // 16-byte units per record
    __shared__ __attribute__((aligned(16))) T st_rec[2][C][64][8];
    __shared__ uint8_t st_code[2][C][64];
    __shared__ int st_cell[2][C][64];
    __shared__ __attribute__((aligned(16))) T st_seam[2][C][2][P];
    __shared__ __attribute__((aligned(16))) FaceRec st_face[FACES ? 2 : 1][FACES ? C : 1][64];
    __shared__ AccT lds_part[FL][G][64][NACC];
    __shared__ T lds_rinv[P][NSTENCIL];
    __shared__ T lds_lut[NWPAIR][2];

    const WorkItem it = a.items[item];
    const InstDev in = a.inst[it.inst];
    if (!a.force && a.st[it.inst].active == 0)
        return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int q = it.group / a.gq;
    const bool xpos = (q & 1) == 0, ypos = (q & 2) == 0;
    const int idx0 = (it.group % a.gq) * P + wave * V;  // index in the quadrant
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
    const FaceRec *__restrict__ sface = FACES ? a.sface + ebase : nullptr;

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
    if (tid < NWPAIR) {
        // neighbour weight pairs of the stencil nibbles (bits 0-2)
        const T w1 = tid < 2 ? T(2) : tid < 4 ? T(1.5) : T(0);
        const T w2 = (tid & 1) == 0 && tid < 6 ? T(-0.5) : T(0);
        lds_lut[tid][0] = w1;
        lds_lut[tid][1] = w2;
    }

    const bool has_up = ypos ? (it.strip > 0 || in.periodic_y)
                             : (it.strip < in.nstrips - 1 || in.periodic_y);
    const int s_up = ypos ? (it.strip + in.nstrips - 1) % in.nstrips : (it.strip + 1) % in.nstrips;
    const bool has_down = ypos ? (it.strip < in.nstrips - 1 || in.periodic_y)
                               : (it.strip > 0 || in.periodic_y);
    const size_t seam_row = (size_t)2 * a.kp4;
    const T *seam_in = a.seam + (size_t)par_r * a.seam_half + in.seam_off + (size_t)s_up * nx * seam_row;
    T *seam_out = a.seam + (size_t)par_w * a.seam_half + in.seam_off + (size_t)it.strip * nx * seam_row;
    const T *fb_rd = FACES ? a.fb + (size_t)par_r * a.fb_half : nullptr;
    T *fb_wr = FACES ? a.fb + (size_t)par_w * a.fb_half : nullptr;
    const bool x_coupled = nx > 1;
    const T spec = T(1.0 - in.alpha);
    // mirrored velocities (first of this wave) across x- and y-normal faces
    const int kmx = (q ^ 1) * a.kq + idx0, kmy = (q ^ 2) * a.kq + idx0;
    const int krev = (q ^ 3) * a.kq + idx0;   // reversed velocity (gradient)

    // ---- staging of one chunk of steps into LDS buffer b
    constexpr int REC_UNITS = C * 64 * UPE;
    constexpr int RU_PER_T = (REC_UNITS + 64 * G - 1) / (64 * G);
    constexpr int SEAM_VALS = C * 2 * P;
    constexpr int SV_PER_T = (SEAM_VALS + 64 * G - 1) / (64 * G);
    constexpr int CC_PER_T = (C * 64 + 64 * G - 1) / (64 * G);
    constexpr int FR_UNITS = FACES ? C * 64 * 2 : 0;     // 16-byte units
    constexpr int FR_PER_T = FACES ? (FR_UNITS + 64 * G - 1) / (64 * G) : 1;
    uint4 ru[RU_PER_T];
    uint4 fu[FR_PER_T];
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
        if (FACES) {
#pragma unroll
            for (int r = 0; r < FR_PER_T; ++r) {
                const int u = tid + r * 64 * G;
                fu[r] = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
                if (u < FR_UNITS) {
                    if (t0 + (u / 2) / 64 < tp)
                        fu[r] = reinterpret_cast<const uint4 *>(sface + (size_t)t0 * 64)[u];
                    else if (u & 1)
                        fu[r] = make_uint4(0, 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < CC_PER_T; ++r) {
            const int e = tid + r * 64 * G;
            cc[r] = -1;
            cb[r] = 0xFF;
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
        if (FACES) {
#pragma unroll
            for (int r = 0; r < FR_PER_T; ++r) {
                const int u = tid + r * 64 * G;
                if (u < FR_UNITS)
                    reinterpret_cast<uint4 *>(&st_face[b][0][0])[u] = fu[r];
            }
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
    AccT cw[V], cwxi[V], cweta[V], cwq[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int k = (kw + (XU ? 0 : v)) * VT_STRIDE;
        const int kv = (kw + v) * VT_STRIDE;
        cxi[v] = ldc(vt, k + VT_XI);
        ccx[v] = ldc(vt, k + VT_CX);
        ceta[v] = ldc(vt, kv + VT_ETA);
        cqq[v] = ldc(vt, kv + VT_Q);
        ccy[v] = ldc(vt, kv + VT_CY);
        cw[v] = (AccT)ldc(vt, kv + VT_W);
        cwxi[v] = cw[v] * (AccT)cxi[v];
        cweta[v] = cw[v] * (AccT)ceta[v];
        cwq[v] = cw[v] * (AccT)cqq[v];
    }
    const AccT xi0 = (AccT)cxi[0];

    // per-cell-delta mode also serves rows of unequal height (nonuniform
    // spacing across the channel): along y the face value extrapolated from
    // the upwind cell u through uu is h_u + r (h_u - h_uu), r the ratio of
    // the distances from the face and from uu's centre to u's centre; rc for
    // this lane's row and its upwind neighbour (yrc), for the neighbour and
    // the second one (yru), both 1/2 on a uniform grid; ysc = dx / dy scales
    // |eta|/dx
    // The transposed problem (adjoint) couples the cell to the rows of its
    // two upwind neighbours with their own forward weights, scaled by
    // dy_c / dy_n (the coupling enters row n divided by dy_n): first
    // neighbour (1 + rn + rd) dy_c/dy_1 or (1 + rn) dy_c/dy_1, second
    // -rn dy_c/dy_2, with rn = dy_1/(dy_1 + dy_c), rd = dy_c/(dy_c + dy_d)
    // (d the downstream neighbour); diagonal 1 + rd (2, 1.5, -1/2 and 1.5
    // on a uniform grid).
    T ysc = T(1), yrc = T(0.5), yru = T(0.5);
    T yA1 = T(2), yA15 = T(1.5), yB = T(-0.5), yaD = T(1.5);
    if constexpr (FIELD) {
        if (in.nonuniform && lane < hs) {
            const int row = ypos ? y0 + lane : y0 + hs - 1 - lane;
            const int stp = ypos ? -1 : 1;
            int r1 = row + stp, r2 = row + 2 * stp, rd = row - stp;
            if (in.periodic_y) {
                r1 = wrap_mod(r1, in.ny);
                r2 = wrap_mod(r2, in.ny);
                rd = wrap_mod(rd, in.ny);
            } else {
                // beyond an outer wall the codes use the wall value instead
                r1 = min(max(r1, 0), in.ny - 1);
                r2 = min(max(r2, 0), in.ny - 1);
                rd = min(max(rd, 0), in.ny - 1);
            }
            const double *rw = a.rows + in.row_off;
            const double d0 = rw[row], d1 = rw[r1], d2 = rw[r2], dd = rw[rd];
            ysc = T(1.0 / (d0 * in.inv_dx));
            yrc = T(d0 / (d0 + d1));
            yru = T(d1 / (d1 + d2));
            if (ADJ) {
                const double rn = d1 / (d1 + d0), rdn = d0 / (d0 + dd);
                yA1 = T((1.0 + rn + rdn) * (d0 / d1));
                yA15 = T((1.0 + rn) * (d0 / d1));
                yB = T(-rn * (d0 / d2));
                yaD = T(1.0 + rdn);
            }
        }
    }

    // rotating registers: x-upwind values A (prev1), B (prev2), X (free);
    // y-upwind chain H0 (current hs1), H1 (free)
    T rA[V], rB[V], rX[V], rH0[V], rH1[V];
    // wrap state [strip][slot][velocity][lane]: independent of V and G
    T *wrapp = a.wrap + in.wrap_off + ((size_t)it.strip * 3 * a.kp4 + kw) * 64 + lane;
    const size_t wslot = (size_t)a.kp4 * 64;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        rA[v] = x_coupled ? wrapp[v * 64] : T(0);
        rB[v] = x_coupled ? wrapp[wslot + v * 64] : T(0);
        rH0[v] = x_coupled ? wrapp[2 * wslot + v * 64] : T(0);
        rX[v] = T(0);
        rH1[v] = T(0);
    }

    const long long cbase = in.cell_off;
    const int nchunks = (tp + C - 1) / C;
    const bool skew = tp != nx;
    int xr0 = (tp - (lane % tp)) % tp;

    issue(0);
    commit(0);
    __syncthreads();

    // one step (s-th of the chunk in buffer b); (PA, PB, PX) and (HA, HB) are
    // the register roles of this step in the rotation; hold: keep the
    // registers when the lane has no cell at this step (xa false)
    auto step = [&](int b, int s, int t, T *PA, T *PB, T *PX, T *HA, T *HB, bool hold, bool xa, int xr) {
        const int sl = s % FL;
        AccT acc[NACC];
#pragma unroll
        for (int m = 0; m < NACC; ++m)
            acc[m] = AccT(0);
        const T *rec = &st_rec[b][s][lane][0];
        const int code = st_code[b][s][lane];
        const int craw = st_cell[b][s][lane];
        const int xn = code & 15, yn = code >> 4;
        const bool solid = craw < 0;
        const int cl = craw & SMAP_CELL;
        const T b0 = rec[0], b1 = rec[1], b2 = rec[2], b3 = rec[3];
        // wall values only where the cell has a wall term (LDS bandwidth);
        // mw = 2 alpha U of a sliding wall on the y-upwind side (else 0)
        T gx = T(0), gy = T(0), mw = T(0);
        if (FIELD || (craw & SMAP_WALL) != 0) {
            gx = rec[4];
            gy = rec[5];
            mw = rec[7];
        }
        const T px = lds_lut[xn & 7][0], qx = lds_lut[xn & 7][1];
        T py = lds_lut[yn & 7][0], qy = lds_lut[yn & 7][1];
        if constexpr (FIELD && !ADJ) {
            // forward y weights from the row ratios (2, -1/2 and 3/2 when
            // both are 1/2)
            const int yp = yn & 7;
            py = yp == NIB_INT ? T(1) + yrc + yru : yp == NIB_NEAR ? T(1) + yrc : T(0);
            qy = yp == NIB_INT ? -yru : T(0);
        }
        if constexpr (FIELD && ADJ) {
            // transposed y weights: pair index 2 w1 + w2 of the nibble
            const int yp = yn & 7, w1i = yp >> 1;
            py = w1i == 0 ? yA1 : w1i == 1 ? yA15 : T(0);
            qy = ((yp & 1) == 0 && yp < 6) ? yB : T(0);
        }
        const int aox = xn >> 3, aoy = yn >> 3;
        const int ci = solid ? STENCIL_SOLID : 2 * aox + aoy;
        T ax = T(0), ay = T(0), dl = T(0);
        if (FIELD) {
            ax = aox ? T(1) : T(1.5);
            ay = aoy ? T(1) : (ADJ ? yaD : T(1) + yrc);
            dl = rec[6];
        }
        const T sbase = XU ? fma(b1, cxi[0], b0) : T(0);
        const T gyw = XU ? fma(mw, cxi[0], gy) : T(0);
        FaceRec fr;
        if (FACES)
            fr = st_face[b][s][lane];
        T hout[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const T p1 = PA[v], p2 = PB[v], h1 = HA[v];
            // staged as zero when the strip has no upstream neighbour
            const T sm1 = st_seam[b][s][1][wave * V + v];
            const T sm2 = st_seam[b][s][0][wave * V + v];
            const T hS1 = dpp_shr1(sm1, p1);
            const T hS2 = dpp_shr1(sm2, h1);
            // a sliding wall emits rho_w + 2 U xi (Eq. diffuse1)
            T gxv = gx, gyv = XU ? gyw : fma(mw, cxi[v], gy);
            if (SPEC) {
                // Maxwell's specular share: mirrored value of the previous iterate
                if (fr.rdx >= 0)
                    gxv = fma(T(fr.kx) * spec, fb_rd[(size_t)fr.rdx * a.kp4 + kmx + v], gxv);
                if (fr.rdy >= 0)
                    gyv = fma(T(fr.ky) * spec, fb_rd[(size_t)fr.rdy * a.kp4 + kmy + v], gyv);
            }
            const T S = fma(b3, cqq[v], fma(b2, ceta[v], XU ? sbase : fma(b1, cxi[v], b0)));
            const T ux = fma(px, p1, fma(qx, p2, gxv));
            const T uy = fma(py, hS1, fma(qy, hS2, gyv));
            const T cyv = FIELD ? ccy[v] * ysc : ccy[v];
            const T g = fma(ccx[v], ux, fma(cyv, uy, S));
            T rinv;
            if (FIELD) {
                const T den = fma(ax, ccx[v], fma(ay, cyv, dl));
                rinv = (solid || cw[v] == 0.0) ? T(0) : rcp_full(den);
            } else {
                rinv = lds_rinv[wave * V + v][ci];
            }
            const T h = g * rinv;
            const AccT hd = (AccT)h;
            if (P12) {
                acc[0] = fma(cwxi[v] * (AccT)ceta[v], hd, acc[0]);
            } else {
                acc[0] = fma(cw[v], hd, acc[0]);
                if (!XU)
                    acc[1] = fma(cwxi[v], hd, acc[1]);
                acc[2] = fma(cweta[v], hd, acc[2]);
                acc[3] = fma(cwq[v], hd, acc[3]);
                if (GRAD && !solid)
                    acc[4] = fma(cw[v], hd * a.ckpt[((size_t)cbase + cl) * a.kp4 + krev + v], acc[4]);
            }
            if (FBWRITE && !solid && xa) {
                // values this cell sends through its downstream wall faces:
                // forward -- the reconstructed incident face value;
                // adjoint -- the cell value
                if (fr.wrx >= 0)
                    fb_wr[(size_t)fr.wrx * a.kp4 + kw + v] =
                        ADJ ? h : (aox ? h : T(1.5) * h - T(0.5) * p1);
                if (fr.wry >= 0)
                    fb_wr[(size_t)fr.wry * a.kp4 + kw + v] =
                        ADJ ? h : (aoy ? h : (FIELD ? (T(1) + yrc) * h - yrc * hS1 : T(1.5) * h - T(0.5) * hS1));
            }
            if (CKPT && !solid && xa)
                a.ckpt[((size_t)cbase + cl) * a.kp4 + kw + v] = hd;
            hout[v] = h;
            if (hold) {
                PX[v] = xa ? h : p1;
                PA[v] = xa ? p1 : p2;       // prev2 of the next step
                HB[v] = xa ? hS1 : h1;
            } else {
                PX[v] = h;
                HB[v] = hS1;
            }
        }
        if (XU && !P12)
            acc[1] = xi0 * acc[0];
        // the last two rows of the strip feed the next strip next iteration
        if (!P12 && has_down && t < tp && lane >= hs - 2 && lane < hs && xa) {
            // x of this lane's cell from its running position on the diagonal
            // (the seam of one strip holds < 2^31 values, checked on the host)
            const int xx = xpos ? xr : nx - 1 - xr;
            const int slot = lane - (hs - 2);
            T *sp = seam_out + (xx * (2 * a.kp4) + slot * a.kp4 + kw);
#pragma unroll
            for (int v = 0; v < V; ++v)
                sp[v] = hout[v];
        }
#pragma unroll
        for (int m = 0; m < NACC; ++m)
            lds_part[sl][wave][lane][m] = acc[m];
    };

    // group-wide sum of the partial moments of steps [s0, s0 + FL) of buffer b
    auto flush = [&](int b, int s0) {
        __syncthreads();
        for (int e = tid; e < FL * 64 * NACC; e += 64 * G) {
            const int sl = e / (64 * NACC), l = (e / NACC) % 64, m = e % NACC;
            const int craw = st_cell[b][s0 + sl][l];
            if (craw < 0)
                continue;
            const int cl = craw & SMAP_CELL;
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < G; ++w)
                sum += lds_part[sl][w][l][m];
            const size_t cg = (size_t)it.group * a.ncell + cbase + cl;
            if (P12)
                a.part5[cg] = sum;
            else if (m < 4)
                a.part[cg * 4 + m] = (T)sum;
            else
                a.part5[cg] = sum;
        }
        __syncthreads();
    };

    for (int c = 0; c < nchunks; ++c) {
        const int b = c & 1;
        const int t0 = c * C;
        if (c + 1 < nchunks)
            issue(c + 1);
        bool xa[C];
        int xrs[C];
        {
            int xr = xr0;
#pragma unroll
            for (int s = 0; s < C; ++s) {
                xa[s] = (t0 + s < tp) && (xr < nx);
                xrs[s] = xr;
                xr = (xr + 1 == tp) ? 0 : xr + 1;
            }
        }
        // every lane has a cell at every step of the chunk: no register holds
        const bool fast = skew ? (t0 >= 63 && t0 + C <= nx) : (t0 + C <= tp);
        // register roles cycle with period 6: (A,B,X)(H0,H1) -> (X,A,B)(H1,H0) -> ...
        if (fast) {
            step(b, 0, t0 + 0, rA, rB, rX, rH0, rH1, false, true, xrs[0]);
            step(b, 1, t0 + 1, rX, rA, rB, rH1, rH0, false, true, xrs[1]);
            step(b, 2, t0 + 2, rB, rX, rA, rH0, rH1, false, true, xrs[2]);
            if (FL == 3)
                flush(b, 0);
            step(b, 3, t0 + 3, rA, rB, rX, rH1, rH0, false, true, xrs[3]);
            step(b, 4, t0 + 4, rX, rA, rB, rH0, rH1, false, true, xrs[4]);
            step(b, 5, t0 + 5, rB, rX, rA, rH1, rH0, false, true, xrs[5]);
        } else {
            step(b, 0, t0 + 0, rA, rB, rX, rH0, rH1, true, xa[0], xrs[0]);
            step(b, 1, t0 + 1, rX, rA, rB, rH1, rH0, true, xa[1], xrs[1]);
            step(b, 2, t0 + 2, rB, rX, rA, rH0, rH1, true, xa[2], xrs[2]);
            if (FL == 3)
                flush(b, 0);
            step(b, 3, t0 + 3, rA, rB, rX, rH1, rH0, true, xa[3], xrs[3]);
            step(b, 4, t0 + 4, rX, rA, rB, rH0, rH1, true, xa[4], xrs[4]);
            step(b, 5, t0 + 5, rB, rX, rA, rH1, rH0, true, xa[5], xrs[5]);
        }
        xr0 = (xr0 + C) % tp;
        if (c + 1 < nchunks)
            commit(b ^ 1);
        flush(b, C - FL);
    }
    if (!P12 && x_coupled) {
        if (sizeof(T) == 4 && a.rwrap) {
            // FP32 correction iteration: plus its constant term
            const double *rw = a.rwrap + (wrapp - a.wrap);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                wrapp[v * 64] = (T)((double)rA[v] + rw[v * 64]);
                wrapp[wslot + v * 64] = (T)((double)rB[v] + rw[wslot + v * 64]);
                wrapp[2 * wslot + v * 64] = (T)((double)rH0[v] + rw[2 * wslot + v * 64]);
            }
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                wrapp[v * 64] = rA[v];
                wrapp[wslot + v * 64] = rB[v];
                wrapp[2 * wslot + v * 64] = rH0[v];
            }
        }
    }
}

template <typename T, int V, int G, int MODE>
__global__ void __launch_bounds__(64 * G) __attribute__((amdgpu_waves_per_eu(sweep_waves_per_eu<T, G, MODE>())))
k_sweep(SweepArgs<T> a)
{
    sweep_item<T, V, G, MODE>(a, blockIdx.x);
}

// ----------------------------------------------------------------- moments
// 256 threads = 64 cells x 4 quadrants: each thread sums its quadrant's
// groups in order, the four quadrant sums are combined in a fixed order
// sum of the partials of quadrant q's velocity groups at cell cg (in order,
// in FP64 also for the FP32 partials of an FP32 sweep)
__device__ __forceinline__ double4 moments_quadrant(const MomArgs &a, long long cg, int q)
{
    double4 s = make_double4(0.0, 0.0, 0.0, 0.0);
    if (a.part32) {
        for (int g = q * a.gq; g < (q + 1) * a.gq; ++g) {
            const float4 p = *reinterpret_cast<const float4 *>(a.part32 + ((size_t)g * a.ncell + cg) * 4);
            s.x += (double)p.x;
            s.y += (double)p.y;
            s.z += (double)p.z;
            s.w += (double)p.w;
        }
        return s;
    }
    for (int g = q * a.gq; g < (q + 1) * a.gq; ++g) {
        const double4 p = *reinterpret_cast<const double4 *>(a.part + ((size_t)g * a.ncell + cg) * 4);
        s.x += p.x;
        s.y += p.y;
        s.z += p.z;
        s.w += p.w;
    }
    return s;
}

// the cell's moments from its four quadrant sums, combined in quadrant order
// (plus r, the FP32 correction's constant term, where non-null)
__device__ __forceinline__ void moments_store(double *m, const double4 (&qs)[4], bool fluid, const double *rr)
{
    if (!fluid) {
        for (int i = 0; i < MOM_STRIDE; ++i)
            m[i] = rr ? 0.0 + rr[i] : 0.0;
        return;
    }
    double r = 0, u1 = 0, u2 = 0, e = 0, fxp = 0, fxm = 0, fyp = 0, fym = 0;
    for (int qq = 0; qq < 4; ++qq) {
        r += qs[qq].x;
        u1 += qs[qq].y;
        u2 += qs[qq].z;
        e += qs[qq].w;
        if ((qq & 1) == 0) fxp += qs[qq].y; else fxm += qs[qq].y;
        if ((qq & 2) == 0) fyp += qs[qq].z; else fym += qs[qq].z;
    }
    if (rr) {
        r += rr[MOM_RHO];
        u1 += rr[MOM_U1];
        u2 += rr[MOM_U2];
        e += rr[MOM_E];
        fxp += rr[MOM_FXP];
        fxm += rr[MOM_FXM];
        fyp += rr[MOM_FYP];
        fym += rr[MOM_FYM];
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

__global__ void __launch_bounds__(256) k_moments(MomArgs a)
{
    __shared__ double4 qs[4][64];
    const int inst = blockIdx.y;
    const InstDev in = a.inst[inst];
    if (!a.force && a.st[inst].active == 0)
        return;
    const int q = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int c = blockIdx.x * 64 + l;
    const bool valid = c < in.nx * in.ny;
    const long long cg = in.cell_off + (valid ? c : 0);
    const bool fluid = valid && a.codes[cg] != 0xFF;
    qs[q][l] = fluid ? moments_quadrant(a, cg, q) : make_double4(0.0, 0.0, 0.0, 0.0);
    __syncthreads();
    if (q != 0 || !valid)
        return;
    const double4 mine[4] = {qs[0][l], qs[1][l], qs[2][l], qs[3][l]};
    moments_store(a.mom + cg * MOM_STRIDE, mine, fluid, a.radd ? a.radd + cg * MOM_STRIDE : nullptr);
}

// sum of one extra per-group partial (shear stress, gradient term) over the
// velocity groups, fixed order
__global__ void __launch_bounds__(256) k_sum1(MomArgs a, const double *part5, double *out, double scale)
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
            s += part5[(size_t)g * a.ncell + cg];
    out[cg] = scale * s;
}

// ------------------------------------------------------------- flow rate
// Q of Sec. III per instance: (1/L) sum over fluid cells of u1 dx dy, with
// L = nx dx, i.e. sum u1 dy / nx.  One workgroup per instance: each thread
// adds its cells (stride 256) in order, then a fixed tree over the threads.
__global__ void __launch_bounds__(256) k_flow(const InstDev *inst, const uint8_t *codes, const double *mom,
                                              const double *rows, double *q)
{
    __shared__ double red[256];
    const InstDev in = inst[blockIdx.x];
    const long long n = (long long)in.nx * in.ny;
    const double dy0 = 1.0 / in.inv_dx;
    double s = 0.0;
    for (long long c = threadIdx.x; c < n; c += 256) {
        const long long cg = in.cell_off + c;
        if (codes[cg] == 0xFF)
            continue;
        const double dy = in.nonuniform ? rows[in.row_off + c / in.nx] : dy0;
        s += mom[cg * MOM_STRIDE + MOM_U1] * dy;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        q[blockIdx.x] = red[0] / (double)in.nx;
}

// ------------------------------------------------- moments on the device
// The work items of one instance (every strip x velocity group), in the
// order the context lists them: strip-major, then group.
__global__ void k_items(WorkItem *dst, int inst, int nstrips, int ngroups)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nstrips * ngroups)
        dst[i] = WorkItem{inst, i / ngroups, i % ngroups, 0};
}

// Gauge of the density (constant h is a null vector): the mean of rho over
// the instance's fluid cells, one workgroup, fixed summation order; written
// to *mean (overwritten, nothing accumulates across calls).
__global__ void __launch_bounds__(256) k_gauge(const InstDev *inst, int instance, const uint8_t *codes,
                                               const double *mom, double *mean)
{
    __shared__ double sr[256];
    __shared__ double sn[256];
    const InstDev in = inst[instance];
    const long long n = (long long)in.nx * in.ny;
    double r = 0.0, c = 0.0;
    for (long long k = threadIdx.x; k < n; k += 256) {
        const long long cg = in.cell_off + k;
        if (codes[cg] == 0xFF)
            continue;
        r += mom[cg * MOM_STRIDE + MOM_RHO];
        c += 1.0;
    }
    sr[threadIdx.x] = r;
    sn[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sr[threadIdx.x] += sr[threadIdx.x + o];
            sn[threadIdx.x] += sn[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *mean = sn[0] > 0.0 ? sr[0] / sn[0] : 0.0;
}

// rho (zero fluid mean), u1, u2, tau = e - rho (both shifted by the gauge:
// a constant h adds m0 to rho and M2 to e) and the shear stress from the
// summed diagnostic partial; 0 in solids.  Any output may be null.
__global__ void __launch_bounds__(256) k_moments_out(const InstDev *inst, int instance, const uint8_t *codes,
                                                     const double *mom, const double *shear, const double *mean,
                                                     double e_per_rho, double *rho, double *u1, double *u2,
                                                     double *tau, double *p12)
{
    const InstDev in = inst[instance];
    const long long n = (long long)in.nx * in.ny;
    const long long k = blockIdx.x * 256ll + threadIdx.x;
    if (k >= n)
        return;
    const long long cg = in.cell_off + k;
    const bool f = codes[cg] != 0xFF;
    const double *m = mom + cg * MOM_STRIDE;
    const double rm = *mean;
    const double r = f ? m[MOM_RHO] - rm : 0.0;
    const double e = f ? m[MOM_E] - rm * e_per_rho : 0.0;
    if (rho) rho[k] = r;
    if (u1) u1[k] = f ? m[MOM_U1] : 0.0;
    if (u2) u2[k] = f ? m[MOM_U2] : 0.0;
    if (tau) tau[k] = f ? e - r : 0.0;
    if (p12) p12[k] = f ? shear[cg] : 0.0;
}

// ------------------------------------------------------------------ record
// The record of one cell c of an instance (the body of k_record): the
// collision gain and wall values of the next sweep, for every quadrant; diff
// and absu receive |du1| and |u1| when the stop statistics are monitored.
template <typename T>
__device__ __forceinline__ void record_cell(const RecArgs<T> &a, const InstDev &in, int c, double &diff,
                                            double &absu)
{
    const long long cg = in.cell_off + c;
    const int code = a.codes[cg];
    if (code == 0xFF)
        return;
    const double *m = a.mom + cg * MOM_STRIDE;
    const double r = m[MOM_RHO], u1 = m[MOM_U1], u2 = m[MOM_U2], e = m[MOM_E];
    const double t = (e - r * a.c2) / a.c4;
    const double dl = in.field ? a.delta_field[cg] : in.delta;
    T rec[8];
    rec[0] = T(dl * (r / a.m0 - t * a.c2));
    // drive: the pressure-gradient factor of the instance (forward); the adjoint
    // is driven by -dQ/dh / W = -(dx / nx) xi
    const double *rw = in.nonuniform ? a.rows + in.row_off : nullptr;
    const double dyc = rw ? rw[c / in.nx] : 1.0 / in.inv_dx;
    const double drive = a.homog ? 0.0 : a.adjoint ? -dyc / (double)in.nx : in.drive;
    rec[1] = T(dl * (u1 / a.m2) + drive);
    rec[2] = T(dl * (u2 / a.m2));
    rec[3] = T(dl * t);
    rec[6] = T(dl);
    double gside[4], mside[4];
    const int x = c % in.nx, y = c / in.nx;
    for (int d = 0; d < 4; ++d) {
        const int cd = (code >> (2 * d)) & 3;
        const int od = d ^ 1;
        const int co = (code >> (2 * od)) & 3;
        // half-range flux moment of the velocities that cross side d
        // outwards, and its sign as a flux through that face
        const int hf = (d == SIDE_W) ? MOM_FXM : (d == SIDE_E) ? MOM_FXP
                     : (d == SIDE_S) ? MOM_FYM : MOM_FYP;
        const double sgn = (d == SIDE_W || d == SIDE_S) ? -1.0 : 1.0;
        auto nbr = [&](int side) {
            int nxx = x, nyy = y;
            if (side == SIDE_W) nxx = (x + in.nx - 1) % in.nx;
            else if (side == SIDE_E) nxx = (x + 1) % in.nx;
            else if (side == SIDE_S) nyy = (y + in.ny - 1) % in.ny;
            else nyy = (y + 1) % in.ny;
            return in.cell_off + (long long)nyy * in.nx + nxx;
        };
        double gval = 0.0;
        mside[d] = 0.0;
        if (!a.adjoint) {
            // the outer bottom / top wall of a channel may slide along
            // x: its diffuse emission gains 2 U xi (Eq. diffuse1), a
            // source term (left out of the homogeneous map)
            if (cd == CODE_WALL && !in.periodic_y && !a.homog) {
                if (d == SIDE_S && y == 0)
                    mside[d] = 2.0 * in.alpha * in.u_bot;
                else if (d == SIDE_N && y == in.ny - 1)
                    mside[d] = 2.0 * in.alpha * in.u_top;
            }
            if (cd == CODE_WALL) {
                // incident flux through the wall face on side d: the
                // half-range flux of the cell, extrapolated from the
                // neighbour on the opposite side unless that side is
                // a wall as well (first-order face value)
                double f = m[hf];
                if (co != CODE_WALL && co != CODE_NONE) {
                    // face value extrapolated across the cell through
                    // its neighbour opposite the face
                    double r = 0.5;
                    if (in.nonuniform && d >= SIDE_S) {
                        const double *rw = a.rows + in.row_off;
                        const int yo = (int)((nbr(od) - in.cell_off) / in.nx);
                        r = rw[y] / (rw[y] + rw[yo]);
                    }
                    f = (1.0 + r) * f - r * a.mom[nbr(od) * MOM_STRIDE + hf];
                }
                gval = in.alpha * sgn * f / a.D;
            }
        } else {
            // transposed wall coupling: the diffuse wall of a face
            // gathers the incident flux of the adjoint cell values and
            // returns it to the two cells whose values built the
            // face value (weights 1.5 / -0.5, or 1 next to a second
            // wall on the opposite side)
            // (rows of unequal height: weights 1 + r / -r of the
            // face extrapolation, the neighbour's scaled by
            // dy_c / dy_n as it enters the neighbour's row)
            if (cd == CODE_WALL) {
                double kap = 1.0;
                if (co != CODE_WALL && co != CODE_NONE) {
                    kap = 1.5;
                    if (rw && d >= SIDE_S) {
                        const double dyo = rw[(nbr(od) - in.cell_off) / in.nx];
                        kap = 1.0 + dyc / (dyc + dyo);
                    }
                }
                gval = kap * in.alpha * sgn * m[hf] / a.D;
            } else if (cd == CODE_NEAR) {
                double kn = -0.5;
                if (rw && d >= SIDE_S) {
                    const double dyn = rw[(nbr(d) - in.cell_off) / in.nx];
                    kn = -(dyn / (dyn + dyc)) * (dyc / dyn);
                }
                gval = kn * in.alpha * sgn * a.mom[nbr(d) * MOM_STRIDE + hf] / a.D;
            }
        }
        gside[d] = gval;
    }
    // one copy per quadrant, in that quadrant's sweep order
    for (int qd = 0; qd < 4; ++qd) {
        rec[4] = T(gside[(qd & 1) ? SIDE_E : SIDE_W]);
        rec[5] = T(gside[(qd & 2) ? SIDE_N : SIDE_S]);
        rec[7] = T(mside[(qd & 2) ? SIDE_N : SIDE_S]);
        const long long pos = a.spos[cg * 4 + qd];
        T *dst = a.srec + pos * 8;
        for (int i = 0; i < 8; ++i)
            dst[i] = rec[i];
    }
    if (a.monitor) {
        const double up = a.u1prev[cg];
        diff = fabs(u1 - up);
        absu = fabs(u1);
        a.u1prev[cg] = u1;
    }
}

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
    if (c < in.nx * in.ny)
        record_cell(a, in, c, diff, absu);
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
    if (threadIdx.x == 0 && a.monitor) {
        // a NaN anywhere must reach the status kernel: encode it as +inf
        double dmax = sd[0] != sd[0] ? __builtin_inf() : sd[0];
        double amax = sa[0] != sa[0] ? __builtin_inf() : sa[0];
        atomicMax(&st->maxdiff_bits, (unsigned long long)__builtin_bit_cast(long long, dmax));
        atomicMax(&st->maxabs_bits, (unsigned long long)__builtin_bit_cast(long long, amax));
    }
}

// -------------------------------------------------------------- gradient
// dQ/d delta_c = -sum_k lambda_ck (h_ck - E_k(h_c)) with lambda_ck = W_k nu_c(-k):
// the group partials hold sum_k W_k nu_c,k h_c(-k); the equilibrium part
// follows from the moments of both fields (E is linear in the forward moments
// and the reversal flips the odd moments of nu).
__global__ void __launch_bounds__(256) k_grad_cell(GradArgs a, int instance)
{
    const InstDev in = a.inst[instance];
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= in.nx * in.ny)
        return;
    const long long cg = in.cell_off + c;
    if (a.codes[cg] == 0xFF) {
        a.dqdd[cg] = 0.0;
        return;
    }
    double s5 = 0.0;
    for (int g = 0; g < a.ngroups; ++g)
        s5 += a.part5[(size_t)g * a.ncell + cg];
    const double *m = a.mom_fwd + cg * MOM_STRIDE;
    const double *n = a.mom_adj + cg * MOM_STRIDE;
    const double t = (m[MOM_E] - a.c2 * m[MOM_RHO]) / a.c4;
    const double a0 = m[MOM_RHO] / a.m0 - t * a.c2, a1 = m[MOM_U1] / a.m2, a2 = m[MOM_U2] / a.m2;
    const double eq = a0 * n[MOM_RHO] - a1 * n[MOM_U1] - a2 * n[MOM_U2] + t * n[MOM_E];
    a.dqdd[cg] = -(s5 - eq);
}

// dQ/d alpha, part of wall face phi: sum over the velocities j that cross
// the face towards the wall of
// (|v_n|/dx) W_j nu_j (rho_w + 2 U xi(-j) - h_inc(mirror(-j))),
// rho_w the diffuse density of the face from the forward incident values and
// U the x velocity of a sliding outer wall (0 for the staircase).
__global__ void __launch_bounds__(256) k_grad_face(GradArgs a)
{
    const int f = a.face0 + blockIdx.x;
    const int side = a.face_side[f];
    const InstDev in = a.inst[a.face_inst[f]];
    const double *vt = a.vtab + (size_t)a.face_inst[f] * a.kp4 * VT_STRIDE;
    const double *ff = a.fb_fwd + (size_t)f * a.kp4;
    const double *fa = a.fb_adj + (size_t)f * a.kp4;
    // quadrants whose velocities move into the face; reversing a velocity
    // flips both quadrant bits, mirroring in the face flips the bit of the
    // normal component (bit 0: xi < 0, bit 1: eta < 0)
    const bool xface = side < 2;
    const int qa = side == SIDE_W ? 1 : side == SIDE_E ? 0 : side == SIDE_S ? 2 : 0;
    const int qb = side == SIDE_W ? 3 : side == SIDE_E ? 2 : side == SIDE_S ? 3 : 1;
    const int mflip = xface ? 1 : 2;
    const int fy = (int)((a.face_cell[f] - in.cell_off) / in.nx);
    const double uw = in.periodic_y ? 0.0
                    : (side == SIDE_S && fy == 0) ? in.u_bot
                    : (side == SIDE_N && fy == in.ny - 1) ? in.u_top : 0.0;
    __shared__ double red[256];
    double r = 0.0;
    for (int e = threadIdx.x; e < 2 * a.kq; e += 256) {
        const int q = e < a.kq ? qa : qb;
        const int j = q * a.kq + (e % a.kq);
        const double vn = fabs(vt[(size_t)j * VT_STRIDE + (xface ? VT_XI : VT_ETA)]);
        r += vt[(size_t)j * VT_STRIDE + VT_W] * vn * ff[j];
    }
    red[threadIdx.x] = r;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double rho_w = red[0] / a.D;
    __syncthreads();
    double g = 0.0;
    for (int e = threadIdx.x; e < 2 * a.kq; e += 256) {
        const int q = e < a.kq ? qa : qb;
        const int idx = e % a.kq;
        const int j = q * a.kq + idx;
        const int jm = (q ^ 3 ^ mflip) * a.kq + idx;
        const double vn = fabs(vt[(size_t)j * VT_STRIDE + (xface ? VT_XI : VT_ETA)]);
        const double emit = rho_w - 2.0 * uw * vt[(size_t)j * VT_STRIDE + VT_XI];   // xi(-j) = -xi(j)
        g += vt[(size_t)j * VT_STRIDE + VT_W] * vn * fa[j] * (emit - ff[jm]);
    }
    red[threadIdx.x] = g;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    // the face value enters its cell's row with |v_n| / dx (x faces) or
    // |v_n| / dy of the cell's row (y faces)
    double inv_h = in.inv_dx;
    if (!xface && in.nonuniform)
        inv_h = 1.0 / a.rows[in.row_off + fy];
    if (threadIdx.x == 0)
        a.dqda_face[f] = red[0] * inv_h;
}

// ------------------------------------------------------------------ status
// floor: a relative change at the round-off level of the iterate's storage
// precision passes without the bound (16 ulp of FP64, or of FP32 for the
// refinement's FP32 correction iteration, whose changes cannot drop below
// the rounding of its state)
__device__ __forceinline__ void status_one(SolveState &s, double tol, long long max_iter, double floor)
{
    if (s.active == 0)
        return;
    const double dmax = __builtin_bit_cast(double, (long long)s.maxdiff_bits);
    const double amax = __builtin_bit_cast(double, (long long)s.maxabs_bits);
    s.maxdiff_bits = 0ull;
    s.maxabs_bits = 0ull;
    s.iter += 1;
    s.amax = amax;
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
    // change at the round-off floor passes without the bound.  After an
    // extrapolation of the dominant mode the ratio is held at least at that
    // mode's rate: what is left of the mode still contracts at it, while two
    // successive changes first show the faster modes.
    const double tl = s.tol > 0.0 ? s.tol : tol;
    int pass = 0;
    double est = eps;
    if (eps <= floor) {
        pass = 1;
    } else if (eps <= tl && s.eps_prev > 0.0) {
        const double rh = fmax(eps / s.eps_prev, s.qfloor);
        est = rh < 1.0 ? eps * rh / (1.0 - rh) : __builtin_inf();
        pass = rh < 1.0 && est <= tl;
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

__global__ void k_status(SolveState *st, int n, double tol, long long max_iter, double floor)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        status_one(st[i], tol, max_iter, floor);
}

// ------------------------------------------------------------- persistent
// instance that holds global cell cg (the cells of the instances follow one
// another; an instance without cells holds none)
__device__ __forceinline__ int inst_of_cell(const InstDev *inst, int n, long long cg)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (inst[mid].cell_off <= cg)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// k_moments over the grid: four consecutive lanes per cell, one quadrant
// each, the first of them combines the four sums (the same order)
__device__ __forceinline__ void persist_moments(const MomArgs &a, int n_inst, long long gtid, long long gthr)
{
    const int q = (int)(threadIdx.x & 3);
    const int lead = (int)(threadIdx.x & 63) & ~3;
    for (long long cg = gtid >> 2; cg < a.ncell; cg += gthr >> 2) {
        const int inst = inst_of_cell(a.inst, n_inst, cg);
        if (!a.force && a.st[inst].active == 0)
            continue;
        const bool fluid = a.codes[cg] != 0xFF;
        const double4 s = fluid ? moments_quadrant(a, cg, q) : make_double4(0.0, 0.0, 0.0, 0.0);
        double4 qs[4];
        for (int k = 0; k < 4; ++k) {
            qs[k].x = __shfl(s.x, lead + k, 64);
            qs[k].y = __shfl(s.y, lead + k, 64);
            qs[k].z = __shfl(s.z, lead + k, 64);
            qs[k].w = __shfl(s.w, lead + k, 64);
        }
        if (q == 0)
            moments_store(a.mom + cg * MOM_STRIDE, qs, fluid, a.radd ? a.radd + cg * MOM_STRIDE : nullptr);
    }
}

// k_record over the grid: chunks of NW * 64 consecutive cells; a chunk in one
// instance folds its stop statistics with one atomic pair (max is order
// independent), a chunk across instances with one pair per cell (a NaN there
// is reported as +inf)
template <typename T, int NW>
__device__ __forceinline__ void persist_record(const RecArgs<T> &a, long long ncell, int n_inst,
                                               double (&red)[2][NW])
{
    const int nthr = NW * 64;
    for (long long c0 = (long long)blockIdx.x * nthr; c0 < ncell; c0 += (long long)gridDim.x * nthr) {
        const long long cg = c0 + threadIdx.x;
        const int i0 = inst_of_cell(a.inst, n_inst, c0);
        const int i1 = inst_of_cell(a.inst, n_inst, (c0 + nthr < ncell ? c0 + nthr : ncell) - 1);
        const bool valid = cg < ncell;
        const int inst = (i0 == i1 || !valid) ? i0 : inst_of_cell(a.inst, n_inst, cg);
        const bool act = valid && a.st[inst].active != 0;
        double diff = 0.0, absu = 0.0;
        if (act) {
            const InstDev in = a.inst[inst];
            record_cell(a, in, (int)(cg - in.cell_off), diff, absu);
        }
        if (!a.monitor)
            continue;
        if (i0 == i1) {
            for (int o = 32; o > 0; o >>= 1) {
                diff = fmax(diff, __shfl_xor(diff, o, 64));
                absu = fmax(absu, __shfl_xor(absu, o, 64));
            }
            if ((threadIdx.x & 63) == 0) {
                red[0][threadIdx.x >> 6] = diff;
                red[1][threadIdx.x >> 6] = absu;
            }
            __syncthreads();
            if (threadIdx.x == 0 && a.st[i0].active != 0) {
                double dmax = red[0][0], amax = red[1][0];
                for (int w = 1; w < NW; ++w) {
                    dmax = fmax(dmax, red[0][w]);
                    amax = fmax(amax, red[1][w]);
                }
                dmax = dmax != dmax ? __builtin_inf() : dmax;
                amax = amax != amax ? __builtin_inf() : amax;
                atomicMax(&a.st[i0].maxdiff_bits, (unsigned long long)__builtin_bit_cast(long long, dmax));
                atomicMax(&a.st[i0].maxabs_bits, (unsigned long long)__builtin_bit_cast(long long, amax));
            }
            __syncthreads();
        } else if (act) {
            diff = diff != diff ? __builtin_inf() : diff;
            absu = absu != absu ? __builtin_inf() : absu;
            atomicMax(&a.st[inst].maxdiff_bits, (unsigned long long)__builtin_bit_cast(long long, diff));
            atomicMax(&a.st[inst].maxabs_bits, (unsigned long long)__builtin_bit_cast(long long, absu));
        }
    }
}

// a struct of uniform values read from device memory into scalar registers
template <typename S>
__device__ __forceinline__ S load_uniform(const S *p)
{
    static_assert(sizeof(S) % 4 == 0, "whole words");
    S out;
    const unsigned int *w = reinterpret_cast<const unsigned int *>(p);
    unsigned int *o = reinterpret_cast<unsigned int *>(&out);
    for (int i = 0; i < (int)(sizeof(S) / 4); ++i)
        o[i] = __builtin_amdgcn_readfirstlane(w[i]);
    return out;
}

// The arguments stay in device memory and each phase reads its own after the
// grid barrier before it (kept in registers across the whole loop they would
// crowd out the sweep's).
template <typename T, int V, int G, int MODE>
__global__ void __launch_bounds__(64 * G) __attribute__((amdgpu_waves_per_eu(sweep_waves_per_eu<T, G, MODE>())))
k_persist(const PersistArgs<T> *pa, int iters, double tol)
{
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    __shared__ int s_item;
    __shared__ double red[2][G];
    for (int j = 0; j < iters; ++j) {
        {
            // every workgroup claims until it draws past the end: iteration
            // j's claims are the counter values j (nitems + grid) onwards
            const int nitems = pa->nitems;
            unsigned int *ctr = pa->ctr;
            const unsigned int base = (unsigned int)j * (unsigned int)(nitems + gridDim.x);
            for (;;) {
                if (threadIdx.x == 0)
                    s_item = (int)(atomicAdd(ctr, 1u) - base);
                __syncthreads();
                const int item = s_item;
                __syncthreads();
                if (item < 0 || item >= nitems)
                    break;
                const SweepArgs<T> sw = load_uniform(&pa->sw);
                sweep_item<T, V, G, MODE>(sw, item);
                __syncthreads();
            }
        }
        grid.sync();
        {
            const MomArgs mom = load_uniform(&pa->mom);
            persist_moments(mom, pa->n_inst, (long long)blockIdx.x * (64 * G) + threadIdx.x,
                            (long long)gridDim.x * (64 * G));
        }
        grid.sync();
        if (pa->seg) {
            const VSeg2 *seg = pa->seg;
            const int nseg = pa->nseg;
            const StateBufs32 sb = pa->sb;
            const double *rr = pa->rr;
            const SolveState *st = pa->st;
            for (int k = blockIdx.x; k < nseg; k += gridDim.x) {
                const VSeg2 sg = seg[k];
                if (st[sg.inst].active != 0)
                    state32_add(sg, (int)(st[sg.inst].iter & 1), sb, rr, threadIdx.x, 64 * G);
            }
            grid.sync();
        }
        {
            const RecArgs<T> rec = load_uniform(&pa->rec);
            persist_record<T, G>(rec, pa->mom.ncell, pa->n_inst, red);
        }
        grid.sync();
        if (blockIdx.x == 0) {
            SolveState *st = pa->st;
            const int n = pa->n_inst;
            const long long max_iter = pa->max_iter;
            const double floor = pa->floor;
            for (int i = threadIdx.x; i < n; i += 64 * G)
                status_one(st[i], tol, max_iter, floor);
        }
        grid.sync();
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
template <typename T, int V, int G, int MODE>
static hipError_t launch_sweep_t(const SweepArgs<T> &a, int nitems, hipStream_t s)
{
    hipLaunchKernelGGL((k_sweep<T, V, G, MODE>), dim3(nitems), dim3(64 * G), 0, s, a);
    return hipGetLastError();
}

// plain iterations run in every supported shape
template <typename T, int V, int G>
static hipError_t launch_plain(const SweepArgs<T> &a, int n, int mode, hipStream_t s)
{
    switch (mode) {
    case 0: return launch_sweep_t<T, V, G, 0>(a, n, s);
    case MODE_FIELD: return launch_sweep_t<T, V, G, MODE_FIELD>(a, n, s);
    case MODE_XU: return launch_sweep_t<T, V, G, MODE_XU>(a, n, s);
    case MODE_XU | MODE_FIELD: return launch_sweep_t<T, V, G, MODE_XU | MODE_FIELD>(a, n, s);
    default: return hipErrorInvalidValue;
    }
}

// the other modes run with 4 velocities per lane, in the wave count that
// keeps the velocity group (and so the partial and seam layout) unchanged
template <int G>
static hipError_t launch_special(const SweepArgs<double> &a, int n, int mode, hipStream_t s)
{
    constexpr int F = MODE_FIELD, S = MODE_SPEC;
#define DVM_SP(M)                                                                         \
    case (M): return launch_sweep_t<double, 4, G, (M)>(a, n, s);                          \
    case (M) | F: return launch_sweep_t<double, 4, G, (M) | F>(a, n, s);                  \
    case (M) | S: return launch_sweep_t<double, 4, G, (M) | S>(a, n, s);                  \
    case (M) | F | S: return launch_sweep_t<double, 4, G, (M) | F | S>(a, n, s);
    switch (mode) {
    case S: return launch_sweep_t<double, 4, G, S>(a, n, s);
    case F | S: return launch_sweep_t<double, 4, G, F | S>(a, n, s);
    DVM_SP(MODE_P12)
    DVM_SP(MODE_CKPT)
    DVM_SP(MODE_ADJ)
    DVM_SP(MODE_ADJ | MODE_GRAD)
    default: return hipErrorInvalidValue;
    }
#undef DVM_SP
}

// FP32 sweeps (refinement): specular walls only
template <int G>
static hipError_t launch_special_f(const SweepArgs<float> &a, int n, int mode, hipStream_t s)
{
    if (mode == MODE_SPEC)
        return launch_sweep_t<float, 4, G, MODE_SPEC>(a, n, s);
    if (mode == (MODE_SPEC | MODE_FIELD))
        return launch_sweep_t<float, 4, G, MODE_SPEC | MODE_FIELD>(a, n, s);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_sweep(const SweepArgs<T> &a, int nitems, int V, int G, int mode, hipStream_t s)
{
    if ((mode & ~(MODE_FIELD | MODE_XU)) != 0) {
        mode &= ~MODE_XU;
        if constexpr (sizeof(T) == 8) {
            if (V * G == 32)
                return launch_special<8>(a, nitems, mode, s);
            if (V * G == 16)
                return launch_special<4>(a, nitems, mode, s);
        } else {
            if (V * G == 32)
                return launch_special_f<8>(a, nitems, mode, s);
            if (V * G == 16)
                return launch_special_f<4>(a, nitems, mode, s);
        }
        return hipErrorInvalidValue;
    }
#define DVM_SW(VV, GG)                                                                    \
    if (V == VV && G == GG)                                                                \
        return launch_plain<T, VV, GG>(a, nitems, mode, s);
    DVM_SW(4, 8)
    DVM_SW(8, 4)
    DVM_SW(4, 4)
    DVM_SW(2, 8)
#undef DVM_SW
    return hipErrorInvalidValue;
}

template hipError_t launch_sweep<double>(const SweepArgs<double> &, int, int, int, int, hipStream_t);
template hipError_t launch_sweep<float>(const SweepArgs<float> &, int, int, int, int, hipStream_t);

hipError_t launch_moments(const MomArgs &a, int max_cells, int n_inst, hipStream_t s)
{
    hipLaunchKernelGGL(k_moments, dim3((max_cells + 63) / 64, n_inst), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sum1(const MomArgs &a, const double *part5, double *out, double scale, int max_cells,
                       int n_inst, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum1, dim3((max_cells + 255) / 256, n_inst), dim3(256), 0, s, a, part5, out, scale);
    return hipGetLastError();
}

hipError_t launch_items(WorkItem *dst, int inst, int nstrips, int ngroups, hipStream_t s)
{
    const int n = nstrips * ngroups;
    hipLaunchKernelGGL(k_items, dim3((n + 255) / 256), dim3(256), 0, s, dst, inst, nstrips, ngroups);
    return hipGetLastError();
}

hipError_t launch_moments_out(const InstDev *inst, int instance, int ncells, const uint8_t *codes,
                              const double *mom, const double *shear, double *mean, double e_per_rho,
                              double *rho, double *u1, double *u2, double *tau, double *p12, hipStream_t s)
{
    hipLaunchKernelGGL(k_gauge, dim3(1), dim3(256), 0, s, inst, instance, codes, mom, mean);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_moments_out, dim3((ncells + 255) / 256), dim3(256), 0, s, inst, instance, codes, mom,
                       shear, (const double *)mean, e_per_rho, rho, u1, u2, tau, p12);
    return hipGetLastError();
}

hipError_t launch_flow(const InstDev *inst, const uint8_t *codes, const double *mom, const double *rows,
                       double *q, int n_inst, hipStream_t s)
{
    hipLaunchKernelGGL(k_flow, dim3(n_inst), dim3(256), 0, s, inst, codes, mom, rows, q);
    return hipGetLastError();
}

hipError_t launch_grad(const GradArgs &a, int instance, int ncells, hipStream_t s)
{
    hipLaunchKernelGGL(k_grad_cell, dim3((ncells + 255) / 256), dim3(256), 0, s, a, instance);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.nfaces == 0)
        return e;
    hipLaunchKernelGGL(k_grad_face, dim3(a.nfaces), dim3(256), 0, s, a);
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

hipError_t launch_status(SolveState *st, int n, double tol, long long max_iter, double floor, hipStream_t s)
{
    hipLaunchKernelGGL(k_status, dim3((n + 63) / 64), dim3(64), 0, s, st, n, tol, max_iter, floor);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_persist(const PersistArgs<T> *dev_args, int nitems, int iters, double tol, int mode,
                          hipStream_t s)
{
    const void *fn = nullptr;
    switch (mode) {
    case 0: fn = reinterpret_cast<const void *>(&k_persist<T, 4, 8, 0>); break;
    case MODE_FIELD: fn = reinterpret_cast<const void *>(&k_persist<T, 4, 8, MODE_FIELD>); break;
    case MODE_XU: fn = reinterpret_cast<const void *>(&k_persist<T, 4, 8, MODE_XU>); break;
    case MODE_FIELD | MODE_XU:
        fn = reinterpret_cast<const void *>(&k_persist<T, 4, 8, MODE_FIELD | MODE_XU>);
        break;
    default: return hipErrorNotSupported;
    }
    int dev = 0, coop = 0, ncu = 0, nb = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 64 * 8, 0);
    if (e != hipSuccess)
        return e;
    if (!coop || ncu < 1 || nb < 1)
        return hipErrorNotSupported;
    // the counter's values stay below 2^31
    if ((long long)iters * ((long long)nitems + (long long)nb * ncu) >= (1ll << 31))
        return hipErrorNotSupported;
    // every workgroup of the grid is resident at once (the cooperative
    // launch refuses a grid that is not)
    const PersistArgs<T> *pa = dev_args;
    void *args[] = {&pa, &iters, &tol};
    return hipLaunchCooperativeKernel(fn, dim3(nb * ncu), dim3(64 * 8), args, 0, s);
}

template hipError_t launch_persist<double>(const PersistArgs<double> *, int, int, double, int, hipStream_t);
template hipError_t launch_persist<float>(const PersistArgs<float> *, int, int, double, int, hipStream_t);

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
