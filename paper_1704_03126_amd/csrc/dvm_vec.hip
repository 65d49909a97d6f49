// dvm_vec.hip -- kernels on compact state vectors of the source iteration:
// gather / scatter between the solver buffers (moments, strip seams, wrap
// state, wall-face values) and one vector per instance slot, and the
// deterministic inner products and updates of the Krylov (GMRES) driver.
#include <hip/hip_runtime.h>

#include "dvm_internal.h"

namespace dvm {

__global__ void __launch_bounds__(256) k_gather(const VSeg *seg, StateBufs b, double *vec, const double *sub)
{
    const VSeg sg = seg[blockIdx.x];
    const double *src = b.b[sg.buf] + sg.buf_off;
    double *dst = vec + sg.vec_off;
    if (sub) {
        const double *sb = sub + sg.vec_off;
        for (int i = threadIdx.x; i < sg.len; i += 256)
            dst[i] = sb[i] - src[i];
    } else {
        for (int i = threadIdx.x; i < sg.len; i += 256)
            dst[i] = src[i];
    }
}

__global__ void __launch_bounds__(256) k_scatter(const VSeg *seg, StateBufs b, const double *vec)
{
    const VSeg sg = seg[blockIdx.x];
    double *dst = b.b[sg.buf] + sg.buf_off;
    const double *src = vec + sg.vec_off;
    for (int i = threadIdx.x; i < sg.len; i += 256)
        dst[i] = src[i];
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

// grid (chunks, nvec + with_norm)
__global__ void __launch_bounds__(256) k_vdots(const VChunk *ch, const double *w, const double *V, long long ldv,
                                               int nvec, double *part, int nch)
{
    __shared__ double red[256];
    const VChunk c = ch[blockIdx.x];
    const int j = blockIdx.y;
    const double *v = j < nvec ? V + (size_t)j * ldv : w;
    double s = 0.0;
    for (int i = threadIdx.x; i < c.len; i += 256)
        s = fma(w[c.start + i], v[c.start + i], s);
    s = block_sum256(s, red);
    if (threadIdx.x == 0)
        part[(size_t)j * nch + blockIdx.x] = s;
}

// one block per slot, one thread per row
__global__ void k_vsum(const int *slot_chunk0, const int *slot_nchunk, const double *part, int nch, int nrows,
                       double *out, int ostride)
{
    const int slot = blockIdx.x;
    for (int j = threadIdx.x; j < nrows; j += blockDim.x) {
        const double *p = part + (size_t)j * nch + slot_chunk0[slot];
        double s = 0.0;
        for (int c = 0; c < slot_nchunk[slot]; ++c)
            s += p[c];
        out[(size_t)slot * ostride + j] = s;
    }
}

__global__ void __launch_bounds__(256) k_vupdate(const VChunk *ch, double *w, const double *V, long long ldv,
                                                 int nvec, const double *coef, int cstride, double *vout)
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
        for (int j = 0; j < nvec; ++j)
            acc = fma(-cf[j], V[(size_t)j * ldv + e], acc);
        w[e] = acc;
        if (vout)
            vout[e] = acc * inv;
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
    const long long off = sg.off[(what == 0 || what == 3) ? par : par ^ 1];
    double *v = vec + sg.vec_off;
    if (sg.buf == 0) {
        double *m = b.mom + off;
        for (int i = threadIdx.x; i < sg.len; i += 256) {
            if (what == 0)
                m[i] += v[i];
            else if (what == 1)
                m[i] = v[i];
            else
                v[i] = m[i];
        }
    } else {
        float *f = b.b[sg.buf - 1] + off;
        for (int i = threadIdx.x; i < sg.len; i += 256) {
            if (what == 0)
                f[i] = (float)((double)f[i] + v[i]);
            else if (what == 1)
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

hipError_t launch_gather(const VSeg *seg, int nseg, StateBufs b, double *vec, const double *sub, hipStream_t s)
{
    if (nseg == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(nseg), dim3(256), 0, s, seg, b, vec, sub);
    return hipGetLastError();
}

hipError_t launch_scatter(const VSeg *seg, int nseg, StateBufs b, const double *vec, hipStream_t s)
{
    if (nseg == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3(nseg), dim3(256), 0, s, seg, b, vec);
    return hipGetLastError();
}

hipError_t launch_vdots(const VChunk *ch, int nch, const double *w, const double *V, long long ldv, int nvec,
                        int with_norm, double *part, hipStream_t s)
{
    hipLaunchKernelGGL(k_vdots, dim3(nch, nvec + (with_norm ? 1 : 0)), dim3(256), 0, s, ch, w, V, ldv, nvec,
                       part, nch);
    return hipGetLastError();
}

hipError_t launch_vsum(const int *slot_chunk0, const int *slot_nchunk, int nslots, const double *part, int nch,
                       int nrows, double *out, int ostride, hipStream_t s)
{
    hipLaunchKernelGGL(k_vsum, dim3(nslots), dim3(64), 0, s, slot_chunk0, slot_nchunk, part, nch, nrows, out,
                       ostride);
    return hipGetLastError();
}

hipError_t launch_vupdate(const VChunk *ch, int nch, double *w, const double *V, long long ldv, int nvec,
                          const double *coef, int cstride, double *vout, hipStream_t s)
{
    hipLaunchKernelGGL(k_vupdate, dim3(nch), dim3(256), 0, s, ch, w, V, ldv, nvec, coef, cstride, vout);
    return hipGetLastError();
}

} // namespace dvm
