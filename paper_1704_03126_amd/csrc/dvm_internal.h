// dvm_internal.h -- structures shared by the host driver and the gfx950
// kernels of the discrete velocity solver (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dvm {

// sides of a cell, and the per-side stencil code of the forward problem
// (2 bits each in a byte: bits 2d..2d+1 for side d).  A solid cell has code
// byte 0xFF.
enum { SIDE_W = 0, SIDE_E = 1, SIDE_S = 2, SIDE_N = 3 };
enum { CODE_INT = 0, CODE_NEAR = 1, CODE_WALL = 2, CODE_NONE = 3 };
// reciprocal-diagonal variants: bit 1 = x diagonal weight 1 (else 1.5),
// bit 0 = same for y; 4 = no cell
enum { NSTENCIL = 5, STENCIL_SOLID = 4 };

// Per-axis stencil nibble of a sweep entry (low nibble x, high nibble y):
// bit 3 = the diagonal weight is 1 (a wall face on the relevant side), else
// 1.5; bits 0-2 select the neighbour weights (w1, w2) so that the sweep
// evaluates  diag * h = ... + c (w1 h_1 + w2 h_2 + face term):
//   0 (2, -0.5)   1 (2, 0)   2 (1.5, -0.5)   3 (1.5, 0)   4 (0, -0.5)   5 (0, 0)
// Forward codes: INT -> 0, NEAR -> 3, WALL -> 8 + 5, NONE -> 5.  Adjoint
// (transposed) stencils use every pair (see adjoint_nibble on the host).
enum { NIB_ONE = 8, NIB_INT = 0, NIB_NEAR = 3, NIB_ZERO = 5, NWPAIR = 8 };

// sweep modes (template bit flags)
enum {
    MODE_FIELD = 1,   // delta per cell (one reciprocal per update)
    MODE_SPEC = 2,    // alpha < 1: Maxwell specular share through face buffers
    MODE_ADJ = 4,     // adjoint sweep (face buffers receive cell values)
    MODE_P12 = 8,     // diagnostic pass: shear stress only, no state written
    MODE_CKPT = 16,   // forward pass that also stores h and the face values
    MODE_GRAD = 32,   // adjoint pass that also accumulates sum W nu h(-v)
    MODE_XU = 64,     // plain passes: the V velocities of a wave share one xi
};

// per-velocity constants, VT_STRIDE values per velocity, velocities ordered
// by quadrant (q = 0: xi>0,eta>0; 1: xi<0,eta>0; 2: xi>0,eta<0; 3: both <0)
enum { VT_XI = 0, VT_ETA = 1, VT_Q = 2, VT_W = 3, VT_CX = 4, VT_CY = 5, VT_STRIDE = 8 };

// record read by the sweep, one per (quadrant, strip, step, lane) entry in
// that quadrant's sweep order: b0..b3 (delta times the collision gain
// coefficients, drive included in b1), the values leaving the wall faces on
// the x and y upwind sides, delta, pad.  The per-entry code byte holds the x
// and y stencil codes (bits 0-1, 2-3) and a no-cell flag (bit 4).
enum { REC_STRIDE = 8 };

// per-cell moments written by k_moments
enum {
    MOM_RHO = 0, MOM_U1 = 1, MOM_U2 = 2, MOM_E = 3,
    MOM_FXP = 4, MOM_FXM = 5, MOM_FYP = 6, MOM_FYM = 7, MOM_STRIDE = 8
};

enum { STATUS_RUNNING = 0, STATUS_CONVERGED = 1, STATUS_MAXITER = 2, STATUS_DIVERGED = 3 };

struct InstDev {
    int nx, ny;
    int tp;          // steps of a strip pass: nx (wrap-around) or nx + 63 (skewed)
    int nstrips;
    int strip_h;     // rows per strip (last strip may be shorter, >= 2)
    int periodic_y;
    int field;       // delta given per cell
    int nonuniform;  // rows of unequal height (row heights at rows + row_off)
    long long cell_off;   // first cell of this instance in the cell arrays
    long long seam_off;   // offset in one parity half of the seam buffer
    long long wrap_off;   // offset in the wrap-state buffer
    long long sk_off;     // first skewed entry: 4 quadrants x nstrips x tp x 64
    long long row_off;    // first row height of this instance
    double delta;         // uniform delta (field == 0)
    double alpha;         // accommodation coefficient
    double drive;         // coefficient of the pressure-gradient source
    double inv_dx;
    double u_bot, u_top;  // x velocities of the outer bottom / top walls
    long long wl_off;     // first entry of this instance's wall-read lists
};

// Steps of a pass staged per chunk: a multiple of 6 so that the 3-register
// rotation of the x-upwind values and the 2-register rotation of the
// y-upwind value are pure renaming inside a chunk.
enum { SWEEP_C = 6 };

// Maxwell's specular share reads the previous iterate's values on the
// upwind wall faces.  Per chunk of a strip pass the wall faces read are
// listed (up to SPEC_SLOTS, as 2 face + axis, -1 unused) so that the sweep
// fetches their mirrored values into LDS one chunk ahead; a face record's
// rdx / rdy carry the face in bits 0-24 and the slot in bits 25-30
// (SPEC_SLOT_NONE: read directly).
enum { SPEC_SLOTS = 48, SPEC_SLOT_SHIFT = 25, SPEC_SLOT_NONE = 63, SPEC_FACE_MASK = (1 << 25) - 1 };

struct WorkItem {
    int inst, strip, group, pad;
};

// skewed cell map entries: fluid cell index, with SMAP_WALL set when the
// cell has a wall term on an upwind side (the record's wall values are read
// only then) and SMAP_FACE when its face record (forward or adjoint) names a
// wall face (the record is read only then); -1 for no cell
enum { SMAP_WALL = 1 << 30, SMAP_FACE = 1 << 29, SMAP_CELL = (1 << 29) - 1 };

// grids at least this wide use the wrap-around diagonal schedule
enum { WRAP_MIN = 8 };

struct SolveState {
    long long iter;       // completed iterations
    long long iter0;      // iterations completed before the current solve
    int status;
    int npass;
    int active;
    int pad0;
    double eps, eps_prev, est;
    unsigned long long maxdiff_bits, maxabs_bits;
    double tol;           // stop tolerance of this instance (0: the launch's)
    double amax;          // max |u1| of the last iteration
    double qfloor;        // lower bound on the contraction ratio of the stop
                          // rule's error estimate (0: the observed ratio)
};

// face record of a sweep entry (alpha < 1 and the gradient): faces whose
// buffer is read on the x / y upwind side, and the cell's own faces on the
// x / y downstream side that receive values (-1: none)
struct FaceRec {
    int rdx, rdy, wrx, wry;
};
// weights of the faces read by the adjoint sweep's entries (the forward
// sweep reads its faces with weight 1)
struct FaceK {
    double kx, ky;
};

template <typename T>
struct SweepArgs {
    const InstDev *inst;
    const WorkItem *items;
    const T *srec;            // skewed records [entry][REC_STRIDE]
    const uint8_t *scode;     // skewed stencil nibbles [entry]
    const int *smap;          // skewed entry -> fluid cell of the instance, -1 none
    const FaceRec *sface;     // skewed face records [entry] (MODE_SPEC/CKPT/GRAD)
    const FaceK *sfacek;      // their read weights [entry] (adjoint with MODE_SPEC)
    const int *wl;            // wall-read lists [wl_off + (pass * chunks + chunk) * SPEC_SLOTS + slot]
    T *fb;                    // wall-face values [2][fb_half]: [parity][face][kp4]
    double *ckpt;             // checkpoint h [cell][kp4] (MODE_CKPT writes, MODE_GRAD reads)
    double *part5;            // extra partial [group][ncell] (P12 / gradient)
    const T *vtab;            // [inst][kp4][VT_STRIDE]
    const double *delta_field;
    T *part;                  // [group][ncell][4] moment partials (FP32 for the FP32 sweep)
    T *seam;                  // [2][seam_half]
    T *wrap;                  // [strip][3][kp4][64] per instance
    SolveState *st;
    long long ncell;          // total cells over all instances
    long long seam_half;
    long long fb_half;
    int gq;                   // velocity groups per quadrant
    int kq;                   // padded velocities per quadrant (= gq * G * V)
    int kp4;                  // 4 * kq
    int force;                // run even for converged instances
    const double *rows;       // row heights in units of H, [row_off + row]
    // FP32 correction iteration: its constant term in the layout of the wrap
    // buffer, added to the wrap values the sweep writes (at the end of a work
    // item); null otherwise (FP32 sweeps only).  The seam values get theirs
    // in a separate pass: read inside the step loop it stalled the sweep.
    const double *rwrap;
};

struct MomArgs {
    const InstDev *inst;
    const uint8_t *codes;
    const double *part;
    const float *part32;      // non-null: the partials of an FP32 sweep instead
    const double *radd;       // non-null: added to every moment (FP32 correction's constant term)
    double *mom;
    SolveState *st;
    long long ncell;
    int gq;
    int force;                // also for instances that are not iterating
};

template <typename T>
struct RecArgs {
    int adjoint;              // wall terms of the transposed problem
    int homog;                // leave the drive out (linear part of the iteration map)
    int monitor;              // fold |du1|, |u1| into the stop statistics
    const InstDev *inst;
    const uint8_t *codes;
    const double *mom;
    const double *delta_field;
    double *u1prev;
    T *srec;
    const long long *spos;    // [cell][quadrant] -> skewed entry
    SolveState *st;
    double m0, m2, c2, c4, D;
    const double *rows;       // row heights in units of H, [row_off + row]
};

template <typename T>
hipError_t launch_sweep(const SweepArgs<T> &a, int nitems, int V, int G, int mode, hipStream_t s);
hipError_t launch_moments(const MomArgs &a, int max_cells, int n_inst, hipStream_t s);
// out[cell] = scale * sum over velocity groups of part5[group][cell]
hipError_t launch_sum1(const MomArgs &a, const double *part5, double *out, double scale, int max_cells,
                       int n_inst, hipStream_t s);

// gradient assembly at one instance: per cell dQ/d delta, per wall face
// the part of dQ/d alpha
struct GradArgs {
    const InstDev *inst;
    const uint8_t *codes;
    const double *mom_fwd;    // forward moments [cell][MOM_STRIDE]
    const double *mom_adj;    // adjoint moments [cell][MOM_STRIDE]
    const double *part5;      // [group][ncell] sum W nu h(-v) per group
    double *dqdd;             // [cell]
    const int *face_cell;     // [face] cell (global index)
    const int *face_side;     // [face]
    const int *face_inst;     // [face]
    const double *fb_fwd;     // forward incident face values [face][kp4]
    const double *fb_adj;     // adjoint cell values at incident velocities [face][kp4]
    const double *vtab;       // [inst][kp4][VT_STRIDE]
    double *dqda_face;        // [face]
    long long ncell;
    int ngroups, kq, kp4, face0, nfaces;
    double m0, m2, c2, c4, D;
    const double *rows;       // row heights in units of H, [row_off + row]
};
hipError_t launch_grad(const GradArgs &a, int instance, int ncells, hipStream_t s);
// the work items of one instance (strip-major, then velocity group) into dst
hipError_t launch_items(WorkItem *dst, int inst, int nstrips, int ngroups, hipStream_t s);
// moments of one instance on the device: *mean = fluid mean of rho (one
// workgroup, fixed order), then rho - mean, u1, u2, tau = (e - mean e_per_rho)
// - (rho - mean), p12 = shear[cell]; 0 in solids; null outputs are skipped
hipError_t launch_moments_out(const InstDev *inst, int instance, int ncells, const uint8_t *codes,
                              const double *mom, const double *shear, double *mean, double e_per_rho,
                              double *rho, double *u1, double *u2, double *tau, double *p12, hipStream_t s);
// q[i] = flow rate of instance i (Sec. III): sum over fluid cells of u1 dy / nx
hipError_t launch_flow(const InstDev *inst, const uint8_t *codes, const double *mom, const double *rows,
                       double *q, int n_inst, hipStream_t s);
template <typename T>
hipError_t launch_record(const RecArgs<T> &a, int max_cells, int n_inst, hipStream_t s);
// stop rule per instance; a relative change <= floor passes without the
// a-posteriori bound (round-off level of the iterate's precision)
constexpr double STOP_FLOOR64 = 16.0 * 2.220446049250313e-16;
constexpr double STOP_FLOOR32 = 16.0 * 1.1920928955078125e-07;
hipError_t launch_status(SolveState *st, int n, double tol, long long max_iter, double floor, hipStream_t s);

hipError_t launch_zero(double *p, size_t n, hipStream_t s);
hipError_t launch_zero_f(float *p, size_t n, hipStream_t s);
hipError_t launch_copy(const double *src, double *dst, size_t n, hipStream_t s);

// ---- state vectors of the iteration (Krylov acceleration, refinement)
// A run of consecutive elements of one solver buffer and its place in a
// compact state vector.
struct VSeg {
    long long buf_off;   // element offset in the solver buffer
    long long vec_off;   // element offset in the state vector
    int len;
    int buf;             // 0 moments, 1 seams, 2 wrap state, 3 wall faces
};
// A chunk of a state vector that belongs to one instance slot.
struct VChunk {
    long long start;
    int len;
    int slot;
};
struct StateBufs {
    double *b[4];
};
enum { VCHUNK = 4096 };
// vec[vec_off..] = buf[buf_off..]        (sub == nullptr)
// vec[vec_off..] = sub[..] - buf[..]     (sub != nullptr)
hipError_t launch_gather(const VSeg *seg, int nseg, StateBufs b, double *vec, const double *sub, hipStream_t s);
// the same with sub in FP32 (a Krylov basis vector)
hipError_t launch_gather_sub32(const VSeg *seg, int nseg, StateBufs b, double *vec, const float *sub,
                               hipStream_t s);
// buf[buf_off..] = vec[vec_off..]
hipError_t launch_scatter(const VSeg *seg, int nseg, StateBufs b, const double *vec, hipStream_t s);
hipError_t launch_scatter(const VSeg *seg, int nseg, StateBufs b, const float *vec, hipStream_t s);
// part[j][chunk] = <w, V_j> over the chunk, j < nvec; row nvec: <w, w> if with_norm.
// skipc (or nullptr): per-slot coefficients [slot][cst] of a first projection
// pass with |w|^2 before it in row nvec; slots where that pass removed at most
// half of |w|^2 get zero in rows j < nvec (no second pass needed)
hipError_t launch_vdots(const VChunk *ch, int nch, const double *w, const double *V, long long ldv, int nvec,
                        int with_norm, double *part, const double *skipc, int cst, hipStream_t s);
hipError_t launch_vdots(const VChunk *ch, int nch, const double *w, const float *V, long long ldv, int nvec,
                        int with_norm, double *part, const double *skipc, int cst, hipStream_t s);
// out[slot][j] = sum of part[j][chunk] over the slot's chunks (fixed order)
hipError_t launch_vsum(const int *slot_chunk0, const int *slot_nchunk, int nslots, const double *part, int nch,
                       int nrows, double *out, int ostride, hipStream_t s);
// A run of the FP32 correction state (refinement): element offsets for
// sweeps that write parity 0 and parity 1 (moments: equal).
struct VSeg2 {
    long long off[2];
    long long vec_off;
    int len;
    int buf;             // 0 moments (FP64), 1 seams, 2 wrap state, 3 wall faces (FP32)
    int inst;
};
struct StateBufs32 {
    double *mom;
    float *b[3];         // seams, wrap state, wall faces
};
// The FP32 correction's add on one segment: state outputs of the sweep just
// run (parity par) += vec, elements i0, i0 + di, ...  FP32 values are added
// in FP64 and rounded once.
__device__ __forceinline__ void state32_add(const VSeg2 &sg, int par, StateBufs32 b, const double *vec, int i0,
                                            int di)
{
    const double *v = vec + sg.vec_off;
    const long long off = sg.off[par];
    if (sg.buf == 0) {
        double *m = b.mom + off;
        for (int i = i0; i < sg.len; i += di)
            m[i] += v[i];
    } else {
        float *f = b.b[sg.buf - 1] + off;
        for (int i = i0; i < sg.len; i += di)
            f[i] = (float)((double)f[i] + v[i]);
    }
}

// The same with the term in FP32 (the seam values of the FP32 correction
// iteration): an FP32 add.
__device__ __forceinline__ void state32_add(const VSeg2 &sg, int par, StateBufs32 b, const float *vec, int i0,
                                            int di)
{
    const float *v = vec + sg.vec_off;
    float *f = b.b[sg.buf - 1] + sg.off[par];
    for (int i = i0; i < sg.len; i += di)
        f[i] = f[i] + v[i];
}

// Blocks of source iterations of a batch as one cooperative launch (plain
// sweep modes: MODE_FIELD and MODE_XU only; 4 velocities per lane, 8 waves
// per workgroup).  Per iteration: the sweep's work items taken from a device
// counter, the moments, for the FP32 correction the add of rr (seg non-null),
// the records with the stop statistics and the stop rule, each phase behind a
// grid barrier; each phase computes what its separate kernel computes, in the
// same order, so the results are those of the separate launches.
template <typename T>
struct PersistArgs {
    SweepArgs<T> sw;
    MomArgs mom;
    RecArgs<T> rec;
    const VSeg2 *seg;         // FP32 correction: the state add (null: none)
    int nseg;
    StateBufs32 sb;
    const double *rr;
    const float *rr32;        // non-null: the add takes this FP32 term (FP32 segments only)
    SolveState *st;           // the stop rule's states (those of sw, mom, rec)
    int n_inst;
    int nitems;
    long long max_iter;
    double floor;
    unsigned int *ctr;        // work counter, 0 at entry
};
// iters iterations with the stop tolerance tol; dev_args in device memory,
// unchanged until the launch has run, nitems its sw work items.
// hipErrorNotSupported: mode outside the plain set, no cooperative launch on
// the device, or iters * (nitems + grid) >= 2^31.
template <typename T>
hipError_t launch_persist(const PersistArgs<T> *dev_args, int nitems, int iters, double tol, int mode,
                          hipStream_t s);

// what: 0 -- state outputs of the sweep just run (parity st.iter & 1) += vec
//            (instances that are not iterating are left alone)
//       1 -- state inputs of the next sweep (parity (st.iter & 1) ^ 1) = vec
//       2 -- vec = state inputs of the next sweep
//       3 -- vec = state outputs of the sweep just run
hipError_t launch_state32(const VSeg2 *seg, int nseg, const SolveState *st, StateBufs32 b, double *vec, int what,
                          hipStream_t s);
// the FP32 correction's constant term vec (segments of seg) into buffers in
// the layout of the moments and wrap buffers, and its seam part rounded to
// FP32 into rseam32 (same positions as in vec); wall-face segments are left
// out
hipError_t launch_rscatter(const VSeg2 *seg, int nseg, const double *vec, double *rmom, double *rwrap,
                           float *rseam32, hipStream_t s);
// FP32 state outputs of the sweep just run (parity st.iter & 1) += vec32, for
// the FP32 segments of seg (instances not iterating are left alone)
hipError_t launch_state32_add32(const VSeg2 *seg, int nseg, const SolveState *st, StateBufs32 b,
                                const float *vec32, hipStream_t s);
// mixed-precision Krylov steps: what 0 -- FP32 state inputs of the next
// sweep = v (an FP32 basis vector); what 1 -- w = v - FP32 state outputs of
// the sweep just run
hipError_t launch_state32_basis(const VSeg2 *seg, int nseg, const SolveState *st, StateBufs32 b, double *w,
                                const float *v, int what, hipStream_t s);
// y += a * x (n elements)
hipError_t launch_axpy(double *y, const double *x, double a, size_t n, hipStream_t s);
// w -= sum_j coef[slot][j] V_j; if vout: vout = w / hn, hn from coef[slot]
// (Pythagoras with the norm in coef[slot][nvec]); zero when hn == 0
hipError_t launch_vupdate(const VChunk *ch, int nch, double *w, const double *V, long long ldv, int nvec,
                          const double *coef, int cstride, double *vout, hipStream_t s);
// the same with the basis V (and vout) stored in FP32; w, coef and the sums
// stay FP64
hipError_t launch_vupdate(const VChunk *ch, int nch, double *w, const float *V, long long ldv, int nvec,
                          const double *coef, int cstride, float *vout, hipStream_t s);
// FP32-basis projections and updates with 16-byte loads: every chunk must
// start on a multiple of 4 elements and ldv be one (V, w, vout 16-byte
// aligned; checked where the pointers allow, hipErrorInvalidValue otherwise)
hipError_t launch_vdots4(const VChunk *ch, int nch, const double *w, const float *V, long long ldv, int nvec,
                         int with_norm, double *part, const double *skipc, int cst, hipStream_t s);
hipError_t launch_vupdate4(const VChunk *ch, int nch, double *w, const float *V, long long ldv, int nvec,
                           const double *coef, int cstride, float *vout, hipStream_t s);

} // namespace dvm
