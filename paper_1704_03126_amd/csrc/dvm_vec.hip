// dvm_vec.hip -- kernels on compact state vectors of the source iteration:
// gather / scatter between the solver buffers (moments, strip seams, wrap
// state, wall-face values) and one vector per instance slot, and the
// deterministic inner products and updates of the Krylov (GMRES) driver.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dvm_internal.h"
#include "dvm_krylov.h"

namespace dvm {

template <typename TS>
__global__ void __launch_bounds__(256) k_gather(const VSeg *seg, StateBufs b, double *vec, const TS *sub)
{
    const VSeg sg = seg[blockIdx.x];
    const double *src = b.b[sg.buf] + sg.buf_off;
    double *dst = vec + sg.vec_off;
    if (sub) {
        const TS *sb = sub + sg.vec_off;
        for (int i = threadIdx.x; i < sg.len; i += 256)
            dst[i] = (double)sb[i] - src[i];
    } else {
        for (int i = threadIdx.x; i < sg.len; i += 256)
            dst[i] = src[i];
    }
}

template <typename TS>
__global__ void __launch_bounds__(256) k_scatter(const VSeg *seg, StateBufs b, const TS *vec)
{
    const VSeg sg = seg[blockIdx.x];
    double *dst = b.b[sg.buf] + sg.buf_off;
    const TS *src = vec + sg.vec_off;
    for (int i = threadIdx.x; i < sg.len; i += 256)
        dst[i] = (double)src[i];
}

__device__ __forceinline__ double block_sum256(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    return red[0];
}

// Grid (chunks, row groups of VROWS): a block holds its chunk of w in
// registers and forms the dots of up to VROWS rows at once (w against
// V_0..V_{nvec-1}, then |w|^2 if asked in row nvec), so w is read once per
// row group and the rows' loads overlap.  With skipc (the slot's
// coefficients of a first projection pass, |w|^2 before it in row nvec) a
// slot whose first pass removed at most half of |w|^2 needs no second pass
// (the Kahan-Parlett "twice is enough" test): its dot rows are written as
// zero without reading V.  Fixed-order reductions: wave butterflies, then the
// four waves in order.
constexpr int VROWS = 8;
constexpr int VPER = VCHUNK / 256;

template <typename TV>
__global__ void __launch_bounds__(256) k_vdots(const VChunk *ch, const double *w, const TV *V, long long ldv,
                                               int nvec, int with_norm, double *part, int nch,
                                               const double *skipc, int cst)
{
    __shared__ double red[4][VROWS];
    const VChunk c = ch[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int r0 = blockIdx.y * VROWS;
    const int nrows = nvec + (with_norm ? 1 : 0);
    bool skip = false;
    if (skipc) {
        const double *cf = skipc + (size_t)c.slot * cst;
        double s = 0.0;
        for (int j = 0; j < nvec; ++j)
            s = fma(cf[j], cf[j], s);
        skip = s <= 0.5 * cf[nvec];
    }
    double acc[VROWS];
#pragma unroll
    for (int rr = 0; rr < VROWS; ++rr)
        acc[rr] = 0.0;
#pragma unroll 4
    for (int e = 0; e < VPER; ++e) {
        const int i = tid + 256 * e;
        if (i >= c.len)
            break;
        const double wi = w[c.start + i];
#pragma unroll
        for (int rr = 0; rr < VROWS; ++rr) {
            const int r = r0 + rr;
            if (r < nvec) {
                if (!skip)
                    acc[rr] = fma(wi, (double)V[(size_t)r * ldv + c.start + i], acc[rr]);
            } else if (r < nrows) {
                acc[rr] = fma(wi, wi, acc[rr]);
            }
        }
    }
#pragma unroll
    for (int rr = 0; rr < VROWS; ++rr) {
        double s = acc[rr];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            s += __shfl_xor(s, o);
        if (lane == 0)
            red[wv][rr] = s;
    }
    __syncthreads();
    if (tid < VROWS && r0 + tid < nrows)
        part[(size_t)(r0 + tid) * nch + blockIdx.x] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
}

// grid (slots, rows): 256 threads sum the slot's chunk partials of one row
// (strided, then a fixed-order tree)
__global__ void __launch_bounds__(256) k_vsum(const int *slot_chunk0, const int *slot_nchunk, const double *part,
                                              int nch, double *out, int ostride)
{
    __shared__ double red[256];
    const int slot = blockIdx.x, j = blockIdx.y;
    const double *p = part + (size_t)j * nch + slot_chunk0[slot];
    const int nc = slot_nchunk[slot];
    double s = 0.0;
    for (int c = threadIdx.x; c < nc; c += 256)
        s += p[c];
    s = block_sum256(s, red);
    if (threadIdx.x == 0)
        out[(size_t)slot * ostride + j] = s;
}

template <typename TV>
__global__ void __launch_bounds__(256) k_vupdate(const VChunk *ch, double *w, const TV *V, long long ldv,
                                                 int nvec, const double *coef, int cstride, TV *vout)
{
    const VChunk c = ch[blockIdx.x];
    const double *cf = coef + (size_t)c.slot * cstride;
    double inv = 0.0;
    if (vout) {
        double n2 = cf[nvec];
        for (int j = 0; j < nvec; ++j)
            n2 -= cf[j] * cf[j];
        inv = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
    }
    for (int i = threadIdx.x; i < c.len; i += 256) {
        const size_t e = c.start + i;
        double acc = w[e];
        // groups of 8 rows: the loads of a group are issued together (the
        // sum keeps the row order); a group whose coefficients are all zero
        // (rows a skipped second pass left at zero) is not read
        int j = 0;
        for (; j + 8 <= nvec; j += 8) {
            double cj[8], vj[8];
            bool any = false;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                cj[u] = cf[j + u];
                any = any || cj[u] != 0.0;
            }
            if (!any)
                continue;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                vj[u] = (double)V[(size_t)(j + u) * ldv + e];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                acc = fma(-cj[u], vj[u], acc);
        }
        for (; j < nvec; ++j) {
            const double cj = cf[j];
            if (cj != 0.0)
                acc = fma(-cj, (double)V[(size_t)j * ldv + e], acc);
        }
        w[e] = acc;
        if (vout)
            vout[e] = (TV)(acc * inv);
    }
}

// FP32-basis variants for chunks that start on a multiple of 4 elements with
// a leading dimension that is one too (the GMRES driver lays its vectors out
// so): each thread takes groups of 4 consecutive elements with 16-byte loads
// of the basis (float4) and of w (two double2); the last len % 4 elements of
// a chunk go one by one.
__global__ void __launch_bounds__(256) k_vdots4(const VChunk *ch, const double *w, const float *V, long long ldv,
                                                int nvec, int with_norm, double *part, int nch,
                                                const double *skipc, int cst)
{
    __shared__ double red[4][VROWS];
    const VChunk c = ch[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int r0 = blockIdx.y * VROWS;
    const int nrows = nvec + (with_norm ? 1 : 0);
    bool skip = false;
    if (skipc) {
        const double *cf = skipc + (size_t)c.slot * cst;
        double s = 0.0;
        for (int j = 0; j < nvec; ++j)
            s = fma(cf[j], cf[j], s);
        skip = s <= 0.5 * cf[nvec];
    }
    double acc[VROWS];
#pragma unroll
    for (int rr = 0; rr < VROWS; ++rr)
        acc[rr] = 0.0;
    const int ng = c.len >> 2;
    for (int g = tid; g < ng; g += 256) {
        const size_t e = (size_t)c.start + 4 * (size_t)g;
        const double2 wa = *reinterpret_cast<const double2 *>(w + e);
        const double2 wb = *reinterpret_cast<const double2 *>(w + e + 2);
#pragma unroll
        for (int rr = 0; rr < VROWS; ++rr) {
            const int r = r0 + rr;
            if (r < nvec) {
                if (!skip) {
                    const float4 v = *reinterpret_cast<const float4 *>(V + (size_t)r * ldv + e);
                    acc[rr] = fma(wa.x, (double)v.x, acc[rr]);
                    acc[rr] = fma(wa.y, (double)v.y, acc[rr]);
                    acc[rr] = fma(wb.x, (double)v.z, acc[rr]);
                    acc[rr] = fma(wb.y, (double)v.w, acc[rr]);
                }
            } else if (r < nrows) {
                acc[rr] = fma(wa.x, wa.x, acc[rr]);
                acc[rr] = fma(wa.y, wa.y, acc[rr]);
                acc[rr] = fma(wb.x, wb.x, acc[rr]);
                acc[rr] = fma(wb.y, wb.y, acc[rr]);
            }
        }
    }
    for (int i = 4 * ng + tid; i < c.len; i += 256) {
        const double wi = w[c.start + i];
#pragma unroll
        for (int rr = 0; rr < VROWS; ++rr) {
            const int r = r0 + rr;
            if (r < nvec) {
                if (!skip)
                    acc[rr] = fma(wi, (double)V[(size_t)r * ldv + c.start + i], acc[rr]);
            } else if (r < nrows) {
                acc[rr] = fma(wi, wi, acc[rr]);
            }
        }
    }
#pragma unroll
    for (int rr = 0; rr < VROWS; ++rr) {
        double s = acc[rr];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            s += __shfl_xor(s, o);
        if (lane == 0)
            red[wv][rr] = s;
    }
    __syncthreads();
    if (tid < VROWS && r0 + tid < nrows)
        part[(size_t)(r0 + tid) * nch + blockIdx.x] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
}

__global__ void __launch_bounds__(256) k_vupdate4(const VChunk *ch, double *w, const float *V, long long ldv,
                                                  int nvec, const double *coef, int cstride, float *vout_all,
                                                  const int *vwrite)
{
    const VChunk c = ch[blockIdx.x];
    // vwrite (optional): per slot, whether vout is written (an instance whose
    // Arnoldi process is not at this column keeps its basis vector)
    float *vout = vout_all && (!vwrite || vwrite[c.slot]) ? vout_all : nullptr;
    const double *cf = coef + (size_t)c.slot * cstride;
    double inv = 0.0;
    if (vout) {
        double n2 = cf[nvec];
        for (int j = 0; j < nvec; ++j)
            n2 -= cf[j] * cf[j];
        inv = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
    }
    const int ng = c.len >> 2;
    for (int g = threadIdx.x; g < ng; g += 256) {
        const size_t e = (size_t)c.start + 4 * (size_t)g;
        const double2 wa = *reinterpret_cast<const double2 *>(w + e);
        const double2 wb = *reinterpret_cast<const double2 *>(w + e + 2);
        double a0 = wa.x, a1 = wa.y, a2 = wb.x, a3 = wb.y;
        int j = 0;
        for (; j + 8 <= nvec; j += 8) {
            double cj[8];
            bool any = false;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                cj[u] = cf[j + u];
                any = any || cj[u] != 0.0;
            }
            if (!any)
                continue;
            float4 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] = *reinterpret_cast<const float4 *>(V + (size_t)(j + u) * ldv + e);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                a0 = fma(-cj[u], (double)v[u].x, a0);
                a1 = fma(-cj[u], (double)v[u].y, a1);
                a2 = fma(-cj[u], (double)v[u].z, a2);
                a3 = fma(-cj[u], (double)v[u].w, a3);
            }
        }
        for (; j < nvec; ++j) {
            const double cj = cf[j];
            if (cj != 0.0) {
                const float4 v = *reinterpret_cast<const float4 *>(V + (size_t)j * ldv + e);
                a0 = fma(-cj, (double)v.x, a0);
                a1 = fma(-cj, (double)v.y, a1);
                a2 = fma(-cj, (double)v.z, a2);
                a3 = fma(-cj, (double)v.w, a3);
            }
        }
        *reinterpret_cast<double2 *>(w + e) = make_double2(a0, a1);
        *reinterpret_cast<double2 *>(w + e + 2) = make_double2(a2, a3);
        if (vout)
            *reinterpret_cast<float4 *>(vout + e) =
                make_float4((float)(a0 * inv), (float)(a1 * inv), (float)(a2 * inv), (float)(a3 * inv));
    }
    for (int i = 4 * ng + threadIdx.x; i < c.len; i += 256) {
        const size_t e = c.start + i;
        double acc = w[e];
        for (int j = 0; j < nvec; ++j) {
            const double cj = cf[j];
            if (cj != 0.0)
                acc = fma(-cj, (double)V[(size_t)j * ldv + e], acc);
        }
        w[e] = acc;
        if (vout)
            vout[e] = (float)(acc * inv);
    }
}

// Deflated GMRES restart: out_o = sum_j P[slot][j][o] V_j for o < nout, j <
// nin (the slot's combination coefficients staged in LDS; FP64 sums of the
// FP32 basis, stored in FP32).
__global__ void __launch_bounds__(256) k_vcombine(const VChunk *ch, const float *V, long long ldv, int nin,
                                                  int nout, const double *P, int pstride, float *out)
{
    __shared__ double sp[VCOMB_IN * VCOMB_OUT];
    const VChunk c = ch[blockIdx.x];
    const double *pp = P + (size_t)c.slot * pstride;
    for (int i = threadIdx.x; i < nin * nout; i += 256)
        sp[i] = pp[i];
    __syncthreads();
    for (int e = threadIdx.x; e < c.len; e += 256) {
        const size_t g = (size_t)c.start + e;
        double acc[VCOMB_OUT];
#pragma unroll
        for (int o = 0; o < VCOMB_OUT; ++o)
            acc[o] = 0.0;
        for (int j = 0; j < nin; ++j) {
            const double v = (double)V[(size_t)j * ldv + g];
            const double *pj = sp + j * nout;
#pragma unroll
            for (int o = 0; o < VCOMB_OUT; ++o)
                if (o < nout)
                    acc[o] = fma(pj[o], v, acc[o]);
        }
#pragma unroll
        for (int o = 0; o < VCOMB_OUT; ++o)
            if (o < nout)
                out[(size_t)o * ldv + g] = (float)acc[o];
    }
}

__global__ void __launch_bounds__(256) k_state32(const VSeg2 *seg, const SolveState *st, StateBufs32 b,
                                                 double *vec, int what)
{
    const VSeg2 sg = seg[blockIdx.x];
    // the add runs inside captured blocks of iterations: an instance that
    // has stopped iterating keeps its state
    if (what == 0 && st[sg.inst].active == 0)
        return;
    const int par = (int)(st[sg.inst].iter & 1);
    if (what == 0) {
        state32_add(sg, par, b, vec, threadIdx.x, 256);
        return;
    }
    const long long off = sg.off[what == 3 ? par : par ^ 1];
    double *v = vec + sg.vec_off;
    if (sg.buf == 0) {
        double *m = b.mom + off;
        for (int i = threadIdx.x; i < sg.len; i += 256) {
            if (what == 1)
                m[i] = v[i];
            else
                v[i] = m[i];
        }
    } else {
        float *f = b.b[sg.buf - 1] + off;
        for (int i = threadIdx.x; i < sg.len; i += 256) {
            if (what == 1)
                f[i] = (float)v[i];
            else
                v[i] = (double)f[i];
        }
    }
}

hipError_t launch_state32(const VSeg2 *seg, int nseg, const SolveState *st, StateBufs32 b, double *vec, int what,
                          hipStream_t s)
{
    if (nseg == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_state32, dim3(nseg), dim3(256), 0, s, seg, st, b, vec, what);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_rscatter(const VSeg2 *seg, const double *vec, double *rmom, double *rwrap,
                                                  float *rseam32)
{
    const VSeg2 sg = seg[blockIdx.x];
    const double *v = vec + sg.vec_off;
    if (sg.buf == 1) {
        float *r = rseam32 + sg.vec_off;
        for (int i = threadIdx.x; i < sg.len; i += 256)
            r[i] = (float)v[i];
        return;
    }
    double *dst = sg.buf == 0 ? rmom : sg.buf == 2 ? rwrap : nullptr;
    if (!dst)
        return;
    // moments and wrap state: one offset for both parities
    dst += sg.off[0];
    for (int i = threadIdx.x; i < sg.len; i += 256)
        dst[i] = v[i];
}

hipError_t launch_rscatter(const VSeg2 *seg, int nseg, const double *vec, double *rmom, double *rwrap,
                           float *rseam32, hipStream_t s)
{
    if (nseg == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_rscatter, dim3(nseg), dim3(256), 0, s, seg, vec, rmom, rwrap, rseam32);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_state32_add32(const VSeg2 *seg, const SolveState *st, StateBufs32 b,
                                                       const float *vec32)
{
    const VSeg2 sg = seg[blockIdx.x];
    // the add runs inside captured blocks of iterations: an instance that
    // has stopped iterating keeps its state
    if (sg.buf == 0 || st[sg.inst].active == 0)
        return;
    state32_add(sg, (int)(st[sg.inst].iter & 1), b, vec32, threadIdx.x, 256);
}

hipError_t launch_state32_add32(const VSeg2 *seg, int nseg, const SolveState *st, StateBufs32 b,
                                const float *vec32, hipStream_t s)
{
    if (nseg == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_state32_add32, dim3(nseg), dim3(256), 0, s, seg, st, b, vec32);
    return hipGetLastError();
}

// Krylov basis vector <-> FP32 correction state (mixed-precision GMRES):
// what 0 -- state inputs of the next sweep (parity st.iter & 1 ^ 1) = v;
// what 1 -- w = v - state outputs of the sweep just run (parity st.iter & 1).
__global__ void __launch_bounds__(256) k_state32_basis(const VSeg2 *seg, const SolveState *st, StateBufs32 b,
                                                       double *w, const float *v, int what)
{
    const VSeg2 sg = seg[blockIdx.x];
    const int par = (int)(st[sg.inst].iter & 1);
    const long long off = sg.off[what == 1 ? par : par ^ 1];
    const float *vv = v + sg.vec_off;
    double *ww = w ? w + sg.vec_off : nullptr;
    if (sg.buf == 0) {
        double *m = b.mom + off;
        for (int i = threadIdx.x; i < sg.len; i += 256) {
            if (what == 0)
                m[i] = (double)vv[i];
            else
                ww[i] = (double)vv[i] - m[i];
        }
    } else {
        float *f = b.b[sg.buf - 1] + off;
        for (int i = threadIdx.x; i < sg.len; i += 256) {
            if (what == 0)
                f[i] = vv[i];
            else
                ww[i] = (double)vv[i] - (double)f[i];
        }
    }
}

hipError_t launch_state32_basis(const VSeg2 *seg, int nseg, const SolveState *st, StateBufs32 b, double *w,
                                const float *v, int what, hipStream_t s)
{
    if (nseg == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_state32_basis, dim3(nseg), dim3(256), 0, s, seg, st, b, w, v, what);
    return hipGetLastError();
}

__global__ void k_axpy(double *y, const double *x, double a, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = fma(a, x[i], y[i]);
}

hipError_t launch_axpy(double *y, const double *x, double a, size_t n, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_axpy, dim3(1024), dim3(256), 0, s, y, x, a, n);
    return hipGetLastError();
}

template <typename TS>
static hipError_t gather_t(const VSeg *seg, int nseg, StateBufs b, double *vec, const TS *sub, hipStream_t s)
{
    if (nseg == 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_gather<TS>), dim3(nseg), dim3(256), 0, s, seg, b, vec, sub);
    return hipGetLastError();
}
hipError_t launch_gather(const VSeg *seg, int nseg, StateBufs b, double *vec, const double *sub, hipStream_t s)
{
    return gather_t(seg, nseg, b, vec, sub, s);
}
hipError_t launch_gather_sub32(const VSeg *seg, int nseg, StateBufs b, double *vec, const float *sub, hipStream_t s)
{
    return gather_t(seg, nseg, b, vec, sub, s);
}

template <typename TS>
static hipError_t scatter_t(const VSeg *seg, int nseg, StateBufs b, const TS *vec, hipStream_t s)
{
    if (nseg == 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_scatter<TS>), dim3(nseg), dim3(256), 0, s, seg, b, vec);
    return hipGetLastError();
}
hipError_t launch_scatter(const VSeg *seg, int nseg, StateBufs b, const double *vec, hipStream_t s)
{
    return scatter_t(seg, nseg, b, vec, s);
}
hipError_t launch_scatter(const VSeg *seg, int nseg, StateBufs b, const float *vec, hipStream_t s)
{
    return scatter_t(seg, nseg, b, vec, s);
}

template <typename TV>
static hipError_t vdots_t(const VChunk *ch, int nch, const double *w, const TV *V, long long ldv, int nvec,
                          int with_norm, double *part, const double *skipc, int cst, hipStream_t s)
{
    const int nrows = nvec + (with_norm ? 1 : 0);
    if (nrows == 0 || nch == 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_vdots<TV>), dim3(nch, (nrows + VROWS - 1) / VROWS), dim3(256), 0, s, ch, w, V, ldv,
                       nvec, with_norm, part, nch, skipc, cst);
    return hipGetLastError();
}
hipError_t launch_vdots(const VChunk *ch, int nch, const double *w, const double *V, long long ldv, int nvec,
                        int with_norm, double *part, const double *skipc, int cst, hipStream_t s)
{
    return vdots_t(ch, nch, w, V, ldv, nvec, with_norm, part, skipc, cst, s);
}
hipError_t launch_vdots(const VChunk *ch, int nch, const double *w, const float *V, long long ldv, int nvec,
                        int with_norm, double *part, const double *skipc, int cst, hipStream_t s)
{
    return vdots_t(ch, nch, w, V, ldv, nvec, with_norm, part, skipc, cst, s);
}

hipError_t launch_vsum(const int *slot_chunk0, const int *slot_nchunk, int nslots, const double *part, int nch,
                       int nrows, double *out, int ostride, hipStream_t s)
{
    if (nslots == 0 || nrows == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_vsum, dim3(nslots, nrows), dim3(256), 0, s, slot_chunk0, slot_nchunk, part, nch, out,
                       ostride);
    return hipGetLastError();
}

hipError_t launch_vupdate(const VChunk *ch, int nch, double *w, const double *V, long long ldv, int nvec,
                          const double *coef, int cstride, double *vout, hipStream_t s)
{
    hipLaunchKernelGGL((k_vupdate<double>), dim3(nch), dim3(256), 0, s, ch, w, V, ldv, nvec, coef, cstride, vout);
    return hipGetLastError();
}
hipError_t launch_vdots4(const VChunk *ch, int nch, const double *w, const float *V, long long ldv, int nvec,
                         int with_norm, double *part, const double *skipc, int cst, hipStream_t s)
{
    const int nrows = nvec + (with_norm ? 1 : 0);
    if (nrows == 0 || nch == 0)
        return hipSuccess;
    if (ldv % 4 != 0 || reinterpret_cast<uintptr_t>(V) % 16 != 0 || reinterpret_cast<uintptr_t>(w) % 16 != 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_vdots4, dim3(nch, (nrows + VROWS - 1) / VROWS), dim3(256), 0, s, ch, w, V, ldv, nvec,
                       with_norm, part, nch, skipc, cst);
    return hipGetLastError();
}
hipError_t launch_vupdate4(const VChunk *ch, int nch, double *w, const float *V, long long ldv, int nvec,
                           const double *coef, int cstride, float *vout, hipStream_t s)
{
    if (nch == 0)
        return hipSuccess;
    if (ldv % 4 != 0 || reinterpret_cast<uintptr_t>(V) % 16 != 0 || reinterpret_cast<uintptr_t>(w) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(vout) % 16 != 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_vupdate4, dim3(nch), dim3(256), 0, s, ch, w, V, ldv, nvec, coef, cstride, vout,
                       static_cast<const int *>(nullptr));
    return hipGetLastError();
}
hipError_t launch_vupdate4_masked(const VChunk *ch, int nch, double *w, const float *V, long long ldv, int nvec,
                                  const double *coef, int cstride, float *vout, const int *vwrite, hipStream_t s)
{
    if (nch == 0)
        return hipSuccess;
    if (ldv % 4 != 0 || reinterpret_cast<uintptr_t>(V) % 16 != 0 || reinterpret_cast<uintptr_t>(w) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(vout) % 16 != 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_vupdate4, dim3(nch), dim3(256), 0, s, ch, w, V, ldv, nvec, coef, cstride, vout, vwrite);
    return hipGetLastError();
}
hipError_t launch_vupdate(const VChunk *ch, int nch, double *w, const float *V, long long ldv, int nvec,
                          const double *coef, int cstride, float *vout, hipStream_t s)
{
    hipLaunchKernelGGL((k_vupdate<float>), dim3(nch), dim3(256), 0, s, ch, w, V, ldv, nvec, coef, cstride, vout);
    return hipGetLastError();
}

hipError_t launch_vcombine(const VChunk *ch, int nch, const float *V, long long ldv, int nin, int nout,
                           const double *P, int pstride, float *out, hipStream_t s)
{
    if (nch == 0)
        return hipSuccess;
    if (nin < 1 || nin > VCOMB_IN || nout < 1 || nout > VCOMB_OUT || pstride < nin * nout)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_vcombine, dim3(nch), dim3(256), 0, s, ch, V, ldv, nin, nout, P, pstride, out);
    return hipGetLastError();
}

} // namespace dvm
