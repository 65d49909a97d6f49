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
// calling workgroup: work item blockIdx.x in k_sweep, drawn from a counter
// in the persistent iteration.  The body is the text of dvm_sweep_body.inc
// in both: the kernel reads its arguments in place from the kernel argument
// segment (a by-value copy handed to an inlined function stays live in
// registers across the pass and spilled the specular per-cell passes).
template <typename T, int V, int G, int MODE>
__global__ void __launch_bounds__(64 * G) __attribute__((amdgpu_waves_per_eu(sweep_waves_per_eu<T, G, MODE>())))
k_sweep(SweepArgs<T> a)
{
    const int item = blockIdx.x;
#include "dvm_sweep_body.inc"
}

template <typename T, int V, int G, int MODE>
__device__ __forceinline__ void sweep_item(const SweepArgs<T> &a, int item)
{
#include "dvm_sweep_body.inc"
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
            const float *rr32 = pa->rr32;
            const SolveState *st = pa->st;
            for (int k = blockIdx.x; k < nseg; k += gridDim.x) {
                const VSeg2 sg = seg[k];
                if (st[sg.inst].active != 0) {
                    if (rr32)
                        state32_add(sg, (int)(st[sg.inst].iter & 1), sb, rr32, threadIdx.x, 64 * G);
                    else
                        state32_add(sg, (int)(st[sg.inst].iter & 1), sb, rr, threadIdx.x, 64 * G);
                }
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
