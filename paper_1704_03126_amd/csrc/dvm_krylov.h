// dvm_krylov.h -- Krylov-vector kernels of the deflated GMRES restart (device
// kernels in dvm_vec.hip, called from the solver in dvm_api.hip).
#pragma once

#include "dvm_internal.h"

namespace dvm {

// out_o = sum_{j < nin} P[slot][j * nout + o] V_j for o < nout: the next
// cycle's first nout basis vectors from this cycle's nin ones (out holds nout
// vectors of stride ldv, in FP32 like V; P holds pstride doubles per slot).
// nin <= VCOMB_IN, nout <= VCOMB_OUT, pstride >= nin * nout, else
// hipErrorInvalidValue.
enum { VCOMB_IN = 65, VCOMB_OUT = 33 };
hipError_t launch_vcombine(const VChunk *ch, int nch, const float *V, long long ldv, int nin, int nout,
                           const double *P, int pstride, float *out, hipStream_t s);

// launch_vupdate4 with a per-slot switch for vout: vwrite[slot] == 0 leaves
// that slot's part of vout as it is (its own Arnoldi process is not at this
// column)
hipError_t launch_vupdate4_masked(const VChunk *ch, int nch, double *w, const float *V, long long ldv, int nvec,
                                  const double *coef, int cstride, float *vout, const int *vwrite, hipStream_t s);

} // namespace dvm
