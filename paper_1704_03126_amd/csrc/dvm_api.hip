// dvm_api.hip -- host side of the C ABI declared in include/dvm.h.
//
// Owns validation, geometry preprocessing (stencil codes, strips), the
// velocity tables of Eq. (nonuniform_v), device memory, and the iteration
// driver that replays captured blocks of source iterations and reads the
// per-instance stop flags back between blocks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <fstream>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dvm.h"
#include "dvm_eig.h"
#include "dvm_internal.h"
#include "dvm_krylov.h"

using namespace dvm;

static thread_local std::string g_err;

static int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(x)                                                                      \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess)                                                          \
            return fail(e_ == hipErrorOutOfMemory ? DVM_ENOMEM : DVM_EHIP,             \
                        std::string(#x) + ": " + hipGetErrorString(e_));               \
    } while (0)

namespace {

// Where device buffers come from: the caller's allocator hooks of dvm_create,
// or hipMalloc / hipFree.  The entry points that may allocate publish their
// context's hooks for the duration of the call (AllocScope); a buffer keeps
// the hooks it was allocated with, so that it is returned to the same place.
struct DevAlloc {
    dvm_alloc_fn alloc = nullptr;
    dvm_free_fn free = nullptr;
    void *ud = nullptr;
};
thread_local const DevAlloc *t_alloc = nullptr;

struct AllocScope {
    const DevAlloc *prev;
    explicit AllocScope(const DevAlloc *a) : prev(t_alloc) { t_alloc = a; }
    ~AllocScope() { t_alloc = prev; }
};

struct HostInst {
    bool has_geom = false;
    int nx = 0, ny = 0, periodic_y = 0;
    double cph = 1.0;
    std::vector<uint8_t> solid, codes;
    long long nfluid = 0;
    // wall faces: local id per (cell, side) (-1 none), cell-major order
    std::vector<int> face_of;
    int nfaces = 0;
    long long face_base = 0;  // first global face id (set by the layout)
    // last solve parameters
    bool field = false;
    double delta = 1.0, alpha = 1.0;
    std::vector<double> dfield;
    bool has_state = false;   // a converged/partial solution is on the device
    bool force_skew = false;  // DVM_SCHED_AUTO: this geometry needs the skewed order
    bool converged = false;   // the last solve met the stop rule
    // rows of unequal height across the channel (dvm_set_row_heights), in
    // units of H; empty: every row 1 / cells_per_H
    std::vector<double> rows;
};

template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevAlloc al{};
    hipError_t alloc(size_t count)
    {
        release();
        if (count == 0)
            return hipSuccess;
        if (t_alloc && t_alloc->alloc) {
            al = *t_alloc;
            p = static_cast<T *>(al.alloc(count * sizeof(T), al.ud));
            if (!p) {
                al = DevAlloc{};
                return hipErrorOutOfMemory;
            }
            n = count;
            return hipSuccess;
        }
        hipError_t e = hipMalloc((void **)&p, count * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        n = count;
        return hipSuccess;
    }
    void release()
    {
        if (p) {
            if (al.free)
                al.free(p, al.ud);
            else
                (void)hipFree(p);
        }
        p = nullptr;
        n = 0;
        al = DevAlloc{};
    }
};

// device workspace of the GMRES driver (grown on demand)
struct KrylovWork {
    DevBuf<float> V;    // GMRES basis, stored in FP32 (the residual, x, w and all sums are FP64)
    DevBuf<double> x, w, part, c1, c2, y;
    DevBuf<VSeg> gseg, sseg;
    DevBuf<VChunk> ch;
    DevBuf<int> c0, nc;
    DevBuf<VSeg2> seg2;  // FP32 correction state of the slots (mixed-precision steps)
    DevBuf<float> T;     // deflated restart: the next cycle's first basis vectors
    DevBuf<double> pc;   //                   and their combination coefficients
    DevBuf<int> vw;      // per slot: whether the Arnoldi step writes its next basis vector
    void release()
    {
        V.release(); x.release(); w.release(); part.release(); c1.release(); c2.release(); y.release();
        gseg.release(); sseg.release(); ch.release(); c0.release(); nc.release(); seg2.release();
        T.release(); pc.release(); vw.release();
    }
};

} // namespace

// Static device scratch of the allocation-free entry point
// (dvm_get_moments_noalloc): the density gauge (first 256 bytes) and the work
// items of the instance's shear-stress pass.  One copy per GPU, held until the
// process ends; every call on a GPU shares it.  Host code never uses the
// array's name as an address: ensure_device() looks up each device's copy
// with hipGetSymbolAddress (that device current) and keeps the pointer.
constexpr size_t SCRATCH_BYTES = 1u << 20;
constexpr size_t SCRATCH_HEAD = 256;
constexpr long long SCRATCH_ITEMS = (long long)((SCRATCH_BYTES - SCRATCH_HEAD) / sizeof(WorkItem));
constexpr int SCRATCH_MAX_DEV = 64;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[SCRATCH_MAX_DEV] = {};

struct dvm_ctx {
    int nv = 0, K = 0, n_inst = 0;
    dvm_config cfg{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = -1;             // current device at the first solve
    DevAlloc dalloc;             // allocator hooks of dvm_create (both null: hipMalloc)
    // flow rate of every instance, reduced on the device at the end of each
    // solve (dvm_flow_rate reads it from here)
    DevBuf<double> d_q;
    std::vector<double> qcache;
    std::vector<double> v, w1;
    double m0 = 0, m2 = 0, M2 = 0, M4 = 0, c2 = 0, c4 = 0, D = 0;
    std::vector<HostInst> inst;
    // what drives each instance's flow (dvm_set_driving): pressure-gradient
    // factor and x velocities of the outer bottom / top walls
    struct Driving {
        double drive = 1.0, u_bot = 0.0, u_top = 0.0;
    };
    std::vector<Driving> driving;

    // layout of the device buffers
    bool layout_ok = false;
    int V = 8, G = 8, gq = 0, kq = 0, kp4 = 0, max_cells = 0;
    int V32 = 4, G32 = 8;        // shape of the FP32 sweeps (same V * G)
    bool autotune = false;       // choose (V, G) by timing at the first solve
    bool tuned = false;
    std::string tune_path;       // copy of cfg.tune_cache (the caller's string is not kept)
    long long ncell = 0, seam_half = 0, wrap_total = 0;
    std::vector<InstDev> idev;
    std::vector<WorkItem> items;

    DevBuf<InstDev> d_inst;
    DevBuf<WorkItem> d_items;
    DevBuf<uint8_t> d_codes, d_scode;
    DevBuf<int> d_smap;
    DevBuf<long long> d_spos;
    DevBuf<FaceRec> d_sface;
    DevBuf<double> d_srec, d_vt, d_dfield, d_part, d_mom, d_u1prev, d_seam, d_wrap, d_aux, d_fb;
    DevBuf<double> d_rows;         // row heights of every instance, in units of H
    long long sk_total = 0, nfaces = 0;
    DevBuf<SolveState> d_st;

    // adjoint problem (allocated by the first dvm_grad)
    bool adj_ready = false;
    std::vector<uint8_t> h_scode_adj;
    std::vector<FaceRec> h_sface_adj;
    std::vector<FaceK> h_sfacek_adj;
    std::vector<int> h_wl_adj;            // wall-read lists of the adjoint sweep
    std::vector<int> h_face_cell, h_face_side, h_face_inst;
    DevBuf<uint8_t> d_scode_adj;
    DevBuf<FaceRec> d_sface_adj;
    DevBuf<FaceK> d_sfacek_adj;
    DevBuf<int> d_wl, d_wl_adj;
    DevBuf<int> d_face_cell, d_face_side, d_face_inst;
    DevBuf<double> d_srec_adj, d_mom_adj, d_u1prev_adj, d_seam_adj, d_wrap_adj, d_fb_adj;
    DevBuf<double> d_ckpt, d_part5, d_momg, d_dqda;
    DevBuf<SolveState> d_st_adj;

    KrylovWork kw;
    // warm-start continuation (cfg.warm_extrapolate): per instance the state
    // vectors of its last two converged solves at a uniform delta, in the
    // layout generation they were taken in
    DevBuf<double> whist[2];
    DevBuf<VSeg> wseg;
    DevBuf<double> wvec;
    std::vector<long long> whist_off, whist_len;
    std::vector<double> whist_d0, whist_d1, whist_par;   // deltas; alpha, drive, walls of the last one
    std::vector<int> whist_n;
    long long layout_gen = 0, whist_gen = -1;
    std::vector<long long> sweeps_done;   // per instance, last solve
    std::vector<long long> sweeps64_done; // of which FP64 sweeps
    std::vector<long long> gmres_s64;     // FP64 sweeps of the instance's last GMRES run
    std::vector<long long> sweeps_wasted;   // before a restart in the skewed order
    std::vector<long long> sweeps64_wasted; // of which FP64 sweeps
    // AUTO: a slow plain iteration is handed to GMRES on trial; per instance
    // the plain contraction per iteration, and the plain wall time per
    // iteration of the last block
    std::vector<double> trial_q;

    // FP32 correction state of the refinement (allocated by the first
    // DVM_FP32_REFINE solve)
    bool fp32_ready = false;
    DevBuf<float> d_srec32, d_seam32, d_wrap32, d_fb32, d_vt32;
    DevBuf<double> d_mom_d, d_u1prev_d, d_xr, d_rr, d_er;
    // the correction's constant term rr in the layout of the moments and
    // wrap buffers: the FP32 correction iteration adds it where it writes
    // those values (plain sweep modes); the seam part is added by a separate
    // pass over the seam segments only (d_seg32s)
    DevBuf<double> d_rb_mom, d_rb_wrap;
    DevBuf<float> d_rr32;       // the seam part of rr in FP32 (positions of rr)
    DevBuf<VSeg2> d_seg32s;
    int nseg32s = 0;
    DevBuf<SolveState> d_st32;
    DevBuf<VSeg2> d_seg32;
    int nseg32 = 0;

    // persistent blocks (cfg.persistent): their arguments in device memory
    // ([0] FP64 forward, [1] FP32 correction) with the host copy last sent,
    // and the work counter of the sweep phase
    DevBuf<unsigned char> d_pargs;
    std::vector<unsigned char> pargs_sent[2];
    DevBuf<unsigned int> d_ctr;
    // layout of the correction state vector of the live refinement slots
    // (offset and length per instance, -1 when not live; total length)
    std::vector<long long> dc_off, dc_len;
    long long dc_n = 0;

    // captured iteration blocks: [0] forward, [1] adjoint, [2] FP32 correction
    hipGraphExec_t graph[3] = {nullptr, nullptr, nullptr};
    int graph_iters[3] = {0, 0, 0};
    int graph_mode[3] = {-1, -1, -1};

    // profiling (cfg.profile): event pairs around sweep launches
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_sweep, ev_other;
    int ev_prec = 0;              // precision of the sweeps in ev_sweep: 0 FP64, 1 FP32
    size_t ev_next = 0;
    dvm_prof prof{};

    ~dvm_ctx()
    {
        for (auto &g : graph)
            if (g)
                (void)hipGraphExecDestroy(g);
        for (auto e : ev_pool)
            (void)hipEventDestroy(e);
        d_inst.release(); d_items.release(); d_codes.release(); d_srec.release();
        d_scode.release(); d_smap.release(); d_spos.release();
        d_vt.release(); d_dfield.release(); d_part.release(); d_mom.release(); d_rows.release();
        d_u1prev.release(); d_seam.release(); d_wrap.release(); d_aux.release();
        d_st.release(); d_sface.release(); d_fb.release(); d_wl.release(); d_wl_adj.release();
        d_scode_adj.release(); d_sface_adj.release(); d_sfacek_adj.release(); d_face_cell.release();
        d_face_side.release();
        d_face_inst.release(); d_srec_adj.release(); d_mom_adj.release(); d_u1prev_adj.release();
        d_seam_adj.release(); d_wrap_adj.release(); d_fb_adj.release(); d_ckpt.release();
        d_part5.release(); d_momg.release(); d_dqda.release(); d_st_adj.release();
        kw.release();
        whist[0].release(); whist[1].release(); wseg.release(); wvec.release();
        d_srec32.release(); d_seam32.release(); d_wrap32.release(); d_fb32.release(); d_vt32.release();
        d_mom_d.release(); d_u1prev_d.release(); d_xr.release(); d_rr.release(); d_er.release();
        d_rb_mom.release(); d_rb_wrap.release(); d_seg32s.release(); d_rr32.release();
        d_st32.release(); d_seg32.release(); d_q.release(); d_pargs.release(); d_ctr.release();
        if (own_stream && stream)
            (void)hipStreamDestroy(stream);
    }
};

// ------------------------------------------------------------ quadrature
// Eq. (nonuniform_v): v_j = 4 s_j^3, s_j = (2j - nv + 1)/(nv - 1); weights:
// trapezoid rule in s times dv/ds, halved at the ends; 2-D weight times the
// global Maxwellian exp(-|v|^2)/pi of the linearisation.
static void build_quadrature(dvm_ctx *c)
{
    const int nv = c->nv;
    c->v.assign(nv, 0.0);
    c->w1.assign(nv, 0.0);
    const double ds = 2.0 / (nv - 1);
    for (int j = 0; j < nv; ++j) {
        double s = (double)(2 * j - nv + 1) / (double)(nv - 1);
        c->v[j] = 4.0 * s * s * s;
        c->w1[j] = 12.0 * s * s * ds * ((j == 0 || j == nv - 1) ? 0.5 : 1.0);
    }
    double m0 = 0, m2 = 0, M2 = 0, M4 = 0, D = 0;
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) {
            double xi = c->v[i], eta = c->v[j];
            double W = c->w1[i] * c->w1[j] * std::exp(-xi * xi - eta * eta) / M_PI;
            double q = xi * xi + eta * eta;
            m0 += W;
            m2 += W * xi * xi;
            M2 += W * q;
            M4 += W * q * q;
            if (xi > 0)
                D += W * xi;
        }
    c->m0 = m0;
    c->m2 = m2;
    c->M2 = M2;
    c->M4 = M4;
    c->c2 = M2 / m0;
    c->c4 = M4 - M2 * M2 / m0;
    c->D = D;
}

// ------------------------------------------------------------- geometry
static bool solid_at(const HostInst &h, int x, int y)
{
    x = ((x % h.nx) + h.nx) % h.nx;
    if (y < 0 || y >= h.ny) {
        if (!h.periodic_y)
            return true;
        y = ((y % h.ny) + h.ny) % h.ny;
    }
    return h.solid[(size_t)y * h.nx + x] != 0;
}

// Staircase stencil codes (Sec. II.A "stair case"): per fluid cell and side,
// wall face on that side / upwind neighbour touches a wall / interior.
static void build_codes(HostInst &h)
{
    static const int ddx[4] = {-1, 1, 0, 0};
    static const int ddy[4] = {0, 0, -1, 1};
    h.codes.assign((size_t)h.nx * h.ny, 0xFF);
    h.nfluid = 0;
    for (int y = 0; y < h.ny; ++y)
        for (int x = 0; x < h.nx; ++x) {
            size_t c = (size_t)y * h.nx + x;
            if (h.solid[c])
                continue;
            ++h.nfluid;
            uint8_t b = 0;
            for (int d = 0; d < 4; ++d) {
                int code;
                if (d < 2 && h.nx == 1)
                    code = CODE_NONE;
                else if (solid_at(h, x + ddx[d], y + ddy[d]))
                    code = CODE_WALL;
                else if (solid_at(h, x + 2 * ddx[d], y + 2 * ddy[d]))
                    code = CODE_NEAR;
                else
                    code = CODE_INT;
                b |= (uint8_t)(code << (2 * d));
            }
            h.codes[c] = b;
        }
    h.face_of.assign((size_t)h.nx * h.ny * 4, -1);
    h.nfaces = 0;
    for (size_t c = 0; c < h.codes.size(); ++c)
        if (h.codes[c] != 0xFF)
            for (int d = 0; d < 4; ++d)
                if (((h.codes[c] >> (2 * d)) & 3) == CODE_WALL)
                    h.face_of[c * 4 + d] = h.nfaces++;
}

// neighbour cell on side d (x periodic; y periodic or -1 beyond the outer walls)
static long long neighbour(const HostInst &h, long long c, int d)
{
    int x = (int)(c % h.nx), y = (int)(c / h.nx);
    if (d == SIDE_W) x = (x + h.nx - 1) % h.nx;
    else if (d == SIDE_E) x = (x + 1) % h.nx;
    else if (d == SIDE_S) y -= 1;
    else y += 1;
    if (y < 0 || y >= h.ny) {
        if (!h.periodic_y)
            return -1;
        y = (y + h.ny) % h.ny;
    }
    return (long long)y * h.nx + x;
}

// Stencil nibble of the transposed transport along one axis for a velocity
// whose upwind side has forward code `up` and downstream side `down`:
// diagonal weight from the downstream code (the forward row of the cell for
// the reversed velocity), first-neighbour weight from the upwind neighbour's
// forward code facing the cell, second-neighbour weight when both upwind
// neighbours are fluid.
static uint8_t adjoint_nibble(int up, int down)
{
    if (up == CODE_NONE)
        return NIB_ZERO;
    const int ai = down == CODE_WALL ? 1 : 0;
    const int pi = up == CODE_WALL ? 2 : (down == CODE_WALL ? 1 : 0);   // w1 = 2, 1.5, 0
    const int qi = up == CODE_INT ? 0 : 1;                              // w2 = -0.5, 0
    return (uint8_t)(NIB_ONE * ai + 2 * pi + qi);
}

// Stencil nibble of the forward transport for the code of the upwind side.
static uint8_t forward_nibble(int up)
{
    switch (up) {
    case CODE_INT: return NIB_INT;
    case CODE_NEAR: return NIB_NEAR;
    case CODE_WALL: return NIB_ONE + NIB_ZERO;
    default: return NIB_ZERO;
    }
}

// Every fluid component must wrap around the x period (carry a net flux);
// each visited cell remembers the winding of its path from the seed.
static bool all_components_percolate(const HostInst &h, std::string &why)
{
    const int nx = h.nx, ny = h.ny;
    std::vector<int> lab((size_t)nx * ny, -1);
    std::vector<long long> wx((size_t)nx * ny, 0);
    std::deque<int> dq;
    int ncomp = 0;
    for (int s = 0; s < nx * ny; ++s) {
        if (h.solid[s] || lab[s] >= 0)
            continue;
        bool perc = false;
        lab[s] = ncomp;
        wx[s] = 0;
        dq.push_back(s);
        while (!dq.empty()) {
            int c = dq.front();
            dq.pop_front();
            int x = c % nx, y = c / nx;
            static const int ddx[4] = {1, -1, 0, 0}, ddy[4] = {0, 0, 1, -1};
            for (int d = 0; d < 4; ++d) {
                int xx = x + ddx[d], yy = y + ddy[d];
                long long w = wx[c];
                if (xx < 0) { xx += nx; w -= 1; }
                else if (xx >= nx) { xx -= nx; w += 1; }
                if (yy < 0 || yy >= ny) {
                    if (!h.periodic_y)
                        continue;
                    yy = (yy + ny) % ny;
                }
                int n = yy * nx + xx;
                if (h.solid[n])
                    continue;
                if (lab[n] < 0) {
                    lab[n] = ncomp;
                    wx[n] = w;
                    dq.push_back(n);
                } else if (wx[n] != w) {
                    perc = true;
                }
            }
        }
        if (!perc) {
            char msg[160];
            std::snprintf(msg, sizeof msg,
                          "fluid component containing cell (x=%d, y=%d) does not wrap around the x period",
                          s % nx, s / nx);
            why = msg;
            return false;
        }
        ++ncomp;
    }
    if (ncomp == 0) {
        why = "geometry has no fluid cell";
        return false;
    }
    return true;
}

static void strip_layout(int ny, int &nstrips, int &strip_h)
{
    nstrips = (ny + 63) / 64;
    for (;;) {
        strip_h = (ny + nstrips - 1) / nstrips;
        int last = ny - (nstrips - 1) * strip_h;
        if (strip_h <= 64 && last >= 2)
            return;
        ++nstrips;
    }
}

// The context touches the HIP runtime only from the first solve on, so the
// host-side checks run without a device.
static int ensure_device(dvm_ctx *c)
{
    if (c->device >= 0)
        return DVM_OK;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(DVM_EHIP, "no HIP device available");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_MAX_DEV)
        return fail(DVM_EINVAL, "device index beyond the library's table");
    {
        // this device's copy of the static scratch, looked up once per device
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void *p = nullptr;
            HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
            g_scratch_ptr[dev] = p;
        }
    }
    if (!c->stream) {
        HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    c->device = dev;
    return DVM_OK;
}

// -------------------------------------------------------------- layout
static void drop_graphs(dvm_ctx *c)
{
    for (int i = 0; i < 3; ++i) {
        if (c->graph[i])
            (void)hipGraphExecDestroy(c->graph[i]);
        c->graph[i] = nullptr;
        c->graph_mode[i] = -1;
    }
}

static int build_layout(dvm_ctx *c)
{
    // buffers are reallocated below: nothing queued may still use them
    HIPCHK(hipStreamSynchronize(c->stream));
    drop_graphs(c);
    c->adj_ready = false;
    c->fp32_ready = false;
    const int V = c->V, G = c->G, P = V * G;
    const std::vector<InstDev> prev = c->idev;
    const int prev_kp4 = c->kp4;
    const long long prev_faces = c->nfaces;
    c->gq = (c->K / 4 + P - 1) / P;
    c->kq = c->gq * P;
    c->kp4 = 4 * c->kq;
    c->idev.assign(c->n_inst, InstDev{});
    c->items.clear();
    long long cell = 0, seam = 0, wrap = 0, sk = 0, faces = 0, rows_total = 0;
    int maxc = 0;
    for (int i = 0; i < c->n_inst; ++i) {
        HostInst &h = c->inst[i];
        InstDev &d = c->idev[i];
        h.face_base = faces;
        faces += h.nfaces;
        d.nx = h.nx;
        d.ny = h.ny;
        const bool on_wrap = c->cfg.schedule == DVM_SCHED_WRAP ||
                             (c->cfg.schedule == DVM_SCHED_AUTO && !h.force_skew);
        d.tp = (on_wrap && h.nx >= WRAP_MIN) ? h.nx : h.nx + 63;
        strip_layout(h.ny, d.nstrips, d.strip_h);
        d.periodic_y = h.periodic_y;
        d.cell_off = cell;
        d.seam_off = seam;
        d.wrap_off = wrap;
        d.sk_off = sk;
        d.row_off = rows_total;
        d.nonuniform = h.rows.empty() ? 0 : 1;
        rows_total += h.ny;
        d.inv_dx = h.cph;
        d.delta = 1.0;
        d.alpha = 1.0;
        d.drive = 1.0;
        cell += (long long)h.nx * h.ny;
        seam += (long long)d.nstrips * h.nx * 2 * c->kp4;
        wrap += (long long)d.nstrips * c->kp4 * 64 * 3;
        sk += 4ll * d.nstrips * d.tp * 64;
        maxc = std::max(maxc, h.nx * h.ny);
        for (int s = 0; s < d.nstrips; ++s)
            for (int g = 0; g < 4 * c->gq; ++g)
                c->items.push_back(WorkItem{i, s, g, 0});
    }
    // longest passes first: the tail of the launch is then made of short items
    std::stable_sort(c->items.begin(), c->items.end(), [&](const WorkItem &a, const WorkItem &b) {
        return c->idev[a.inst].tp > c->idev[b.inst].tp;
    });
    for (int i = 0; i < c->n_inst; ++i) {
        if ((long long)c->inst[i].nx * 2 * c->kp4 >= (1ll << 31))
            return fail(DVM_EINVAL, "instance " + std::to_string(i) +
                                        ": nx too large for the velocity grid (nx * 2 * padded velocities >= 2^31)");
        if ((long long)c->inst[i].nx * c->inst[i].ny > SMAP_CELL)
            return fail(DVM_EINVAL, "instance " + std::to_string(i) + ": more than 2^29 - 1 cells");
    }
    // The solution state (moments, seam, wrap and wall-face buffers, delta
    // field) survives a new layout that keeps every instance's state where it
    // was: same velocity padding, same offsets -- only the sweep order of
    // some instance changed.
    bool keep = prev.size() == c->idev.size() && prev_kp4 == c->kp4 && prev_faces == faces &&
                c->d_mom.n == (size_t)cell * MOM_STRIDE && c->d_seam.n == (size_t)2 * seam &&
                c->d_wrap.n == (size_t)wrap;
    for (int i = 0; keep && i < c->n_inst; ++i) {
        const InstDev &a = prev[i], &b = c->idev[i];
        keep = a.nx == b.nx && a.ny == b.ny && a.cell_off == b.cell_off && a.seam_off == b.seam_off &&
               a.wrap_off == b.wrap_off && a.nstrips == b.nstrips;
    }
    if (keep)
        for (int i = 0; i < c->n_inst; ++i) {
            InstDev &d = c->idev[i];
            d.delta = prev[i].delta;
            d.alpha = prev[i].alpha;
            d.drive = prev[i].drive;
            d.u_bot = prev[i].u_bot;
            d.u_top = prev[i].u_top;
            d.field = prev[i].field;
        }
    c->ncell = cell;
    c->seam_half = seam;
    c->wrap_total = wrap;
    c->sk_total = sk;
    c->nfaces = faces;
    c->max_cells = maxc;

    HIPCHK(c->d_inst.alloc(c->n_inst));
    HIPCHK(c->d_items.alloc(c->items.size()));
    HIPCHK(c->d_codes.alloc(cell));
    HIPCHK(c->d_srec.alloc(sk * REC_STRIDE));
    HIPCHK(c->d_scode.alloc(sk));
    HIPCHK(c->d_smap.alloc(sk));
    HIPCHK(c->d_spos.alloc(cell * 4));
    HIPCHK(c->d_vt.alloc((size_t)c->n_inst * c->kp4 * VT_STRIDE));
    HIPCHK(c->d_part.alloc((size_t)4 * c->gq * cell * 4));
    if (!keep) {
        HIPCHK(c->d_dfield.alloc(cell));
        HIPCHK(c->d_mom.alloc(cell * MOM_STRIDE));
        HIPCHK(c->d_u1prev.alloc(cell));
        HIPCHK(c->d_seam.alloc(2 * seam));
        HIPCHK(c->d_wrap.alloc(wrap));
        HIPCHK(c->d_st.alloc(c->n_inst));
        HIPCHK(c->d_fb.alloc((size_t)2 * std::max<long long>(faces, 1) * c->kp4));
    }
    HIPCHK(c->d_aux.alloc(cell));
    HIPCHK(c->d_sface.alloc(sk));
    {
        std::vector<double> rows;
        rows.reserve(rows_total);
        for (const auto &h : c->inst)
            for (int y = 0; y < h.ny; ++y)
                rows.push_back(h.rows.empty() ? 1.0 / h.cph : h.rows[y]);
        HIPCHK(c->d_rows.alloc(std::max<size_t>(rows.size(), 1)));
        if (!rows.empty())
            HIPCHK(hipMemcpyAsync(c->d_rows.p, rows.data(), rows.size() * sizeof(double),
                                  hipMemcpyHostToDevice, c->stream));
    }
    HIPCHK(c->d_part5.alloc((size_t)4 * c->gq * cell));
    HIPCHK(c->d_q.alloc(c->n_inst));
    c->qcache.assign(c->n_inst, 0.0);

    std::vector<uint8_t> codes(cell);
    std::vector<double> vt((size_t)c->n_inst * c->kp4 * VT_STRIDE, 0.0);
    const int h2 = c->nv / 2;
    for (int i = 0; i < c->n_inst; ++i) {
        const HostInst &h = c->inst[i];
        std::copy(h.codes.begin(), h.codes.end(), codes.begin() + c->idev[i].cell_off);
        for (int q = 0; q < 4; ++q)
            for (int idx = 0; idx < c->K / 4; ++idx) {
                int ip = idx / h2, jp = idx % h2;
                int iv = (q & 1) ? h2 - 1 - ip : h2 + ip;   // node of xi
                int jv = (q & 2) ? h2 - 1 - jp : h2 + jp;   // node of eta
                double xi = c->v[iv], eta = c->v[jv];
                double *e = &vt[((size_t)i * c->kp4 + q * c->kq + idx) * VT_STRIDE];
                e[VT_XI] = xi;
                e[VT_ETA] = eta;
                e[VT_Q] = xi * xi + eta * eta;
                e[VT_W] = c->w1[iv] * c->w1[jv] * std::exp(-xi * xi - eta * eta) / M_PI;
                e[VT_CX] = h.nx == 1 ? 0.0 : std::fabs(xi) * h.cph;
                e[VT_CY] = std::fabs(eta) * h.cph;
            }
    }
    // skewed sweep order of every (instance, quadrant, strip): lane l treats
    // x_r = (t - l) mod tp at step t, rows run away from the upwind side.
    // Per entry: the fluid cell (-1 for none or solid), the x / y stencil
    // nibbles of the forward and the adjoint problem, and the wall faces each
    // problem reads and writes.
    const FaceRec none{-1, -1, -1, -1};
    std::vector<uint8_t> scode(sk, NIB_ZERO * 17), scode_adj(sk, NIB_ZERO * 17);
    std::vector<int> smap(sk, -1);
    std::vector<long long> spos(cell * 4, -1);
    std::vector<FaceRec> sface(sk, none), sface_adj(sk, none);
    std::vector<FaceK> sfacek_adj(sk, FaceK{0.0, 0.0});
    c->h_face_cell.assign(faces, 0);
    c->h_face_side.assign(faces, 0);
    c->h_face_inst.assign(faces, 0);
    for (int i = 0; i < c->n_inst; ++i) {
        const HostInst &h = c->inst[i];
        const InstDev &d = c->idev[i];
        auto gface = [&](long long cl, int side) -> int {
            const int f = h.face_of[cl * 4 + side];
            return f < 0 ? -1 : (int)(h.face_base + f);
        };
        for (long long cl = 0; cl < (long long)h.nx * h.ny; ++cl)
            for (int side = 0; side < 4; ++side) {
                const int f = gface(cl, side);
                if (f >= 0) {
                    c->h_face_cell[f] = (int)(d.cell_off + cl);
                    c->h_face_side[f] = side;
                    c->h_face_inst[f] = i;
                }
            }
        for (int q = 0; q < 4; ++q) {
            const bool xpos = (q & 1) == 0, ypos = (q & 2) == 0;
            const int dxs = xpos ? SIDE_W : SIDE_E, dys = ypos ? SIDE_S : SIDE_N;
            const int dxd = dxs ^ 1, dyd = dys ^ 1;
            for (int st = 0; st < d.nstrips; ++st) {
                const int y0 = st * d.strip_h;
                const int hs = std::min(d.strip_h, d.ny - y0);
                for (int t = 0; t < d.tp; ++t)
                    for (int l = 0; l < 64; ++l) {
                        const long long e = d.sk_off + (((long long)q * d.nstrips + st) * d.tp + t) * 64 + l;
                        const int xr = ((t - l) % d.tp + d.tp) % d.tp;
                        if (l >= hs || xr >= d.nx)
                            continue;
                        const int x = xpos ? xr : d.nx - 1 - xr;
                        const int row = ypos ? y0 + l : y0 + hs - 1 - l;
                        const long long cl = (long long)row * d.nx + x;
                        const uint8_t code = h.codes[cl];
                        if (code == 0xFF)
                            continue;
                        spos[(d.cell_off + cl) * 4 + q] = e;
                        const int cxu = (code >> (2 * dxs)) & 3, cxd = (code >> (2 * dxd)) & 3;
                        const int cyu = (code >> (2 * dys)) & 3, cyd = (code >> (2 * dyd)) & 3;
                        // wall terms: forward on WALL sides, adjoint also on NEAR sides
                        const bool wall = cxu == CODE_WALL || cxu == CODE_NEAR || cyu == CODE_WALL ||
                                          cyu == CODE_NEAR;
                        smap[e] = (int)cl | (wall ? SMAP_WALL : 0);
                        scode[e] = (uint8_t)(forward_nibble(cxu) | (forward_nibble(cyu) << 4));
                        scode_adj[e] = (uint8_t)(adjoint_nibble(cxu, cxd) | (adjoint_nibble(cyu, cyd) << 4));
                        // forward: the wall value on an upwind wall face has a
                        // specular share of that face's incident values; the
                        // cell sends incident values through downstream walls
                        FaceRec &fr = sface[e];
                        fr.rdx = cxu == CODE_WALL ? gface(cl, dxs) : -1;
                        fr.rdy = cyu == CODE_WALL ? gface(cl, dys) : -1;
                        fr.wrx = cxd == CODE_WALL ? gface(cl, dxd) : -1;
                        fr.wry = cyd == CODE_WALL ? gface(cl, dyd) : -1;
                        // adjoint: the upwind wall face of the cell (weight
                        // 1.5, or 1 with a wall on the far side too) or of its
                        // upwind neighbour (weight -0.5)
                        FaceRec &fa = sface_adj[e];
                        // (rows of unequal height, y faces: 1 + r and
                        // -r dy_c / dy_n, r the face-extrapolation ratio)
                        auto adj_face = [&](int up, int down, int side, int &rd, double &k) {
                            rd = -1;
                            k = 0.0;
                            const bool nu = !h.rows.empty() && side >= SIDE_S;
                            const double dyc = nu ? h.rows[cl / h.nx] : 0.0;
                            if (up == CODE_WALL) {
                                rd = gface(cl, side);
                                k = (down == CODE_WALL || down == CODE_NONE) ? 1.0 : 1.5;
                                if (nu && k == 1.5) {
                                    const double dyo = h.rows[neighbour(h, cl, side ^ 1) / h.nx];
                                    k = 1.0 + dyc / (dyc + dyo);
                                }
                            } else if (up == CODE_NEAR) {
                                const long long u1 = neighbour(h, cl, side);
                                rd = gface(u1, side);
                                k = -0.5;
                                if (nu) {
                                    const double dyn = h.rows[u1 / h.nx];
                                    k = -(dyn / (dyn + dyc)) * (dyc / dyn);
                                }
                            }
                        };
                        adj_face(cxu, cxd, dxs, fa.rdx, sfacek_adj[e].kx);
                        adj_face(cyu, cyd, dys, fa.rdy, sfacek_adj[e].ky);
                        fa.wrx = fr.wrx;
                        fa.wry = fr.wry;
                        if (fr.rdx >= 0 || fr.rdy >= 0 || fr.wrx >= 0 || fr.wry >= 0 || fa.rdx >= 0 || fa.rdy >= 0)
                            smap[e] |= SMAP_FACE;
                    }
            }
        }
    }
    // wall-read lists per chunk of every strip pass, and the slots in the
    // face records (forward and adjoint records read different faces)
    if (faces > SPEC_FACE_MASK)
        return fail(DVM_EINVAL, "too many wall faces (more than 2^25)");
    long long wl_total = 0;
    for (int i = 0; i < c->n_inst; ++i) {
        InstDev &d = c->idev[i];
        d.wl_off = wl_total;
        wl_total += 4ll * d.nstrips * ((d.tp + SWEEP_C - 1) / SWEEP_C) * SPEC_SLOTS;
    }
    std::vector<int> wl(wl_total, -1), wl_adj(wl_total, -1);
    auto assign_slots = [&](std::vector<FaceRec> &recs, std::vector<int> &list) {
        for (int i = 0; i < c->n_inst; ++i) {
            const InstDev &d = c->idev[i];
            const int nch = (d.tp + SWEEP_C - 1) / SWEEP_C;
            for (int ps = 0; ps < 4 * d.nstrips; ++ps)
                for (int k = 0; k < nch; ++k) {
                    int *lst = &list[d.wl_off + ((long long)ps * nch + k) * SPEC_SLOTS];
                    int n = 0;
                    for (int t = k * SWEEP_C; t < std::min((k + 1) * SWEEP_C, d.tp); ++t)
                        for (int l = 0; l < 64; ++l) {
                            FaceRec &f = recs[d.sk_off + ((long long)ps * d.tp + t) * 64 + l];
                            for (int axis = 0; axis < 2; ++axis) {
                                int &rd = axis ? f.rdy : f.rdx;
                                if (rd < 0)
                                    continue;
                                int slot = SPEC_SLOT_NONE;
                                if (n < SPEC_SLOTS) {
                                    lst[n] = 2 * rd + axis;
                                    slot = n++;
                                }
                                rd |= slot << SPEC_SLOT_SHIFT;
                            }
                        }
                }
        }
    };
    assign_slots(sface, wl);
    assign_slots(sface_adj, wl_adj);
    HIPCHK(c->d_wl.alloc(std::max<long long>(wl_total, 1)));
    if (wl_total > 0)
        HIPCHK(hipMemcpyAsync(c->d_wl.p, wl.data(), wl_total * sizeof(int), hipMemcpyHostToDevice, c->stream));
    c->h_wl_adj.swap(wl_adj);
    c->h_scode_adj.swap(scode_adj);
    c->h_sface_adj.swap(sface_adj);
    c->h_sfacek_adj.swap(sfacek_adj);
    HIPCHK(hipMemcpyAsync(c->d_codes.p, codes.data(), cell, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->d_scode.p, scode.data(), sk, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->d_smap.p, smap.data(), sk * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->d_spos.p, spos.data(), spos.size() * sizeof(long long), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipMemcpyAsync(c->d_sface.p, sface.data(), sk * sizeof(FaceRec), hipMemcpyHostToDevice, c->stream));
    if (!keep)
        HIPCHK(launch_zero(c->d_fb.p, c->d_fb.n, c->stream));
    HIPCHK(launch_zero(c->d_srec.p, c->d_srec.n, c->stream));
    HIPCHK(hipMemcpyAsync(c->d_vt.p, vt.data(), vt.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->d_items.p, c->items.data(), c->items.size() * sizeof(WorkItem),
                          hipMemcpyHostToDevice, c->stream));
    if (!keep) {
        HIPCHK(launch_zero(c->d_mom.p, c->d_mom.n, c->stream));
        HIPCHK(launch_zero(c->d_u1prev.p, c->d_u1prev.n, c->stream));
        HIPCHK(launch_zero(c->d_seam.p, c->d_seam.n, c->stream));
        HIPCHK(launch_zero(c->d_wrap.p, c->d_wrap.n, c->stream));
        HIPCHK(launch_zero(c->d_dfield.p, c->d_dfield.n, c->stream));
        for (auto &h : c->inst)
            h.has_state = false;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    c->layout_ok = true;
    c->layout_gen += 1;
    return DVM_OK;
}

// Arguments of the forward (adj = false) or adjoint iteration.
static SweepArgs<double> sweep_args(dvm_ctx *c, int force, bool adj = false)
{
    SweepArgs<double> a{};
    a.inst = c->d_inst.p;
    a.items = c->d_items.p;
    a.srec = adj ? c->d_srec_adj.p : c->d_srec.p;
    a.scode = adj ? c->d_scode_adj.p : c->d_scode.p;
    a.smap = c->d_smap.p;
    a.sface = adj ? c->d_sface_adj.p : c->d_sface.p;
    a.sfacek = adj ? c->d_sfacek_adj.p : nullptr;
    a.wl = adj ? c->d_wl_adj.p : c->d_wl.p;
    a.fb = adj ? c->d_fb_adj.p : c->d_fb.p;
    a.ckpt = c->d_ckpt.p;
    a.part5 = c->d_part5.p;
    a.vtab = c->d_vt.p;
    a.delta_field = c->d_dfield.p;
    a.part = c->d_part.p;
    a.seam = adj ? c->d_seam_adj.p : c->d_seam.p;
    a.wrap = adj ? c->d_wrap_adj.p : c->d_wrap.p;
    a.st = adj ? c->d_st_adj.p : c->d_st.p;
    a.ncell = c->ncell;
    a.seam_half = c->seam_half;
    a.fb_half = std::max<long long>(c->nfaces, 1) * c->kp4;
    a.gq = c->gq;
    a.kq = c->kq;
    a.kp4 = c->kp4;
    a.force = force;
    a.rows = c->d_rows.p;
    return a;
}

static MomArgs mom_args(dvm_ctx *c, bool adj = false, int force = 0)
{
    MomArgs a{};
    a.inst = c->d_inst.p;
    a.codes = c->d_codes.p;
    a.part = c->d_part.p;
    a.mom = adj ? c->d_mom_adj.p : c->d_mom.p;
    a.st = adj ? c->d_st_adj.p : c->d_st.p;
    a.ncell = c->ncell;
    a.gq = c->gq;
    a.force = force;
    return a;
}

// moments of the FP32 correction iteration: the FP32 sweep's partials into
// the correction's moments, stop states of the correction
static MomArgs mom_args32(dvm_ctx *c, int force = 0)
{
    MomArgs a = mom_args(c, false, force);
    a.part32 = reinterpret_cast<const float *>(c->d_part.p);
    a.mom = c->d_mom_d.p;
    a.st = c->d_st32.p;
    return a;
}

static int solve_mode(const dvm_ctx *c);

// The FP32 correction iteration adds its constant term where the sweep and
// the moments write the state (plain sweep modes); with wall-face buffers
// (specular walls) a separate pass adds it after the moments.
static bool fused_add32(const dvm_ctx *c)
{
    return (solve_mode(c) & MODE_SPEC) == 0 && c->d_rb_mom.p != nullptr;
}

static RecArgs<double> rec_args(dvm_ctx *c, bool adj = false)
{
    RecArgs<double> a{};
    a.adjoint = adj ? 1 : 0;
    a.homog = 0;
    a.monitor = 1;
    a.inst = c->d_inst.p;
    a.codes = c->d_codes.p;
    a.mom = adj ? c->d_mom_adj.p : c->d_mom.p;
    a.delta_field = c->d_dfield.p;
    a.u1prev = adj ? c->d_u1prev_adj.p : c->d_u1prev.p;
    a.srec = adj ? c->d_srec_adj.p : c->d_srec.p;
    a.spos = c->d_spos.p;
    a.st = adj ? c->d_st_adj.p : c->d_st.p;
    a.m0 = c->m0;
    a.m2 = c->m2;
    a.c2 = c->c2;
    a.c4 = c->c4;
    a.D = c->D;
    a.rows = c->d_rows.p;
    return a;
}

// MODE_XU when the V velocities of every wave share one xi node: velocities
// are ordered (|xi| index, |eta| index) within a quadrant, nv/2 per |xi|
static int xu_flag(const dvm_ctx *c, int V)
{
    return ((c->nv / 2) % V == 0) ? MODE_XU : 0;
}

// sweep mode of the instances being solved: per-cell delta, specular walls
static int solve_mode(const dvm_ctx *c)
{
    int m = 0;
    for (const auto &h : c->inst) {
        // rows of unequal height take the per-cell path (diagonal per cell)
        if (h.field || !h.rows.empty())
            m |= MODE_FIELD;
        if (h.alpha < 1.0)
            m |= MODE_SPEC;
    }
    return m;
}

static int next_event(dvm_ctx *c, hipEvent_t *e)
{
    if (c->ev_next == c->ev_pool.size()) {
        hipEvent_t n;
        HIPCHK(hipEventCreate(&n));
        c->ev_pool.push_back(n);
    }
    *e = c->ev_pool[c->ev_next++];
    return DVM_OK;
}

// Fold the recorded event pairs into the totals (the stream is idle).  Only
// the first `real` iterations of the block did work: the later launches found
// every instance stopped and returned at once, and are left out.  `updates`:
// fluid cell x velocity updates of those launches.
static int collect_profile(dvm_ctx *c, long long real, double updates)
{
    dvm_prof &p = c->prof;
    const bool f32 = c->ev_prec == 1;
    for (size_t i = 0; i < c->ev_sweep.size() && (long long)i < real; ++i) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->ev_sweep[i].first, c->ev_sweep[i].second));
        (f32 ? p.sweep32_ms : p.sweep_ms) += ms;
        ++(f32 ? p.n_sweeps32 : p.n_sweeps);
    }
    (f32 ? p.updates32 : p.updates) += updates;
    for (size_t i = 0; i < c->ev_other.size() && (long long)i < real; ++i) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->ev_other[i].first, c->ev_other[i].second));
        p.other_ms += ms;
    }
    c->ev_sweep.clear();
    c->ev_other.clear();
    c->ev_next = 0;
    return DVM_OK;
}

// Arguments of the FP32 correction iteration (refinement).
static SweepArgs<float> sweep_args32(dvm_ctx *c)
{
    SweepArgs<float> a{};
    a.inst = c->d_inst.p;
    a.items = c->d_items.p;
    a.srec = c->d_srec32.p;
    a.scode = c->d_scode.p;
    a.smap = c->d_smap.p;
    a.sface = c->d_sface.p;
    a.wl = c->d_wl.p;
    a.fb = c->d_fb32.p;
    a.vtab = c->d_vt32.p;
    a.delta_field = c->d_dfield.p;
    a.part = reinterpret_cast<float *>(c->d_part.p);      // FP32 partials, half the FP64 buffer
    a.part5 = c->d_part5.p;
    a.seam = c->d_seam32.p;
    a.wrap = c->d_wrap32.p;
    a.st = c->d_st32.p;
    a.ncell = c->ncell;
    a.seam_half = c->seam_half;
    a.fb_half = std::max<long long>(c->nfaces, 1) * c->kp4;
    a.gq = c->gq;
    a.kq = c->kq;
    a.kp4 = c->kp4;
    a.force = 0;
    a.rows = c->d_rows.p;
    return a;
}

// the FP32 correction iteration e <- L32 e + r with r added where the sweep
// and the moments write (fused_add32)
static SweepArgs<float> sweep_args32r(dvm_ctx *c)
{
    SweepArgs<float> a = sweep_args32(c);
    a.rwrap = c->d_rb_wrap.p;
    return a;
}

static MomArgs mom_args32r(dvm_ctx *c)
{
    MomArgs a = mom_args32(c);
    a.radd = c->d_rb_mom.p;
    return a;
}

static RecArgs<float> rec_args32(dvm_ctx *c)
{
    RecArgs<float> a{};
    a.adjoint = 0;
    a.homog = 1;
    a.monitor = 1;
    a.inst = c->d_inst.p;
    a.codes = c->d_codes.p;
    a.mom = c->d_mom_d.p;
    a.delta_field = c->d_dfield.p;
    a.u1prev = c->d_u1prev_d.p;
    a.srec = c->d_srec32.p;
    a.spos = c->d_spos.p;
    a.st = c->d_st32.p;
    a.m0 = c->m0;
    a.m2 = c->m2;
    a.c2 = c->c2;
    a.c4 = c->c4;
    a.D = c->D;
    a.rows = c->d_rows.p;
    return a;
}

static StateBufs32 state32(dvm_ctx *c)
{
    StateBufs32 b;
    b.mom = c->d_mom_d.p;
    b.b[0] = c->d_seam32.p;
    b.b[1] = c->d_wrap32.p;
    b.b[2] = c->d_fb32.p;
    return b;
}

static double refine_inner_tol(const dvm_ctx *c)
{
    return std::max(c->cfg.tol, 1e-4);
}

// One source iteration for every active instance: kind 0 forward, 1 adjoint,
// 2 FP32 correction iteration of the refinement (homogeneous sweep, then the
// FP64 residual added to the new state).
static int enqueue_iteration(dvm_ctx *c, int kind)
{
    const bool adj = kind == 1;
    const bool prof = c->cfg.profile != 0 && kind != 1;
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
    if (prof) {
        int rc = next_event(c, &e0);
        if (!rc) rc = next_event(c, &e1);
        if (!rc) rc = next_event(c, &e2);
        if (rc)
            return rc;
        HIPCHK(hipEventRecord(e0, c->stream));
        c->ev_prec = kind == 2 ? 1 : 0;
    }
    if (kind == 2) {
        const bool fused = fused_add32(c);
        HIPCHK(launch_sweep<float>(fused ? sweep_args32r(c) : sweep_args32(c), (int)c->items.size(), c->V32,
                                   c->G32, solve_mode(c) | xu_flag(c, c->V32), c->stream));
        if (prof) {
            HIPCHK(hipEventRecord(e1, c->stream));
            c->ev_sweep.emplace_back(e0, e1);
        }
        HIPCHK(launch_moments(fused ? mom_args32r(c) : mom_args32(c), c->max_cells, c->n_inst, c->stream));
        if (fused)
            HIPCHK(launch_state32_add32(c->d_seg32s.p, c->nseg32s, c->d_st32.p, state32(c), c->d_rr32.p,
                                        c->stream));
        else
            HIPCHK(launch_state32(c->d_seg32.p, c->nseg32, c->d_st32.p, state32(c), c->d_rr.p, 0, c->stream));
        HIPCHK(launch_record<float>(rec_args32(c), c->max_cells, c->n_inst, c->stream));
        HIPCHK(launch_status(c->d_st32.p, c->n_inst, refine_inner_tol(c), c->cfg.max_iter, STOP_FLOOR32,
                             c->stream));
        return DVM_OK;
    }
    const int mode = solve_mode(c) | (adj ? MODE_ADJ : xu_flag(c, c->V));
    HIPCHK(launch_sweep<double>(sweep_args(c, 0, adj), (int)c->items.size(), c->V, c->G, mode, c->stream));
    if (prof)
        HIPCHK(hipEventRecord(e1, c->stream));
    HIPCHK(launch_moments(mom_args(c, adj), c->max_cells, c->n_inst, c->stream));
    HIPCHK(launch_record<double>(rec_args(c, adj), c->max_cells, c->n_inst, c->stream));
    HIPCHK(launch_status(adj ? c->d_st_adj.p : c->d_st.p, c->n_inst, c->cfg.tol, c->cfg.max_iter, STOP_FLOOR64,
                         c->stream));
    if (prof) {
        HIPCHK(hipEventRecord(e2, c->stream));
        c->ev_sweep.emplace_back(e0, e1);
        c->ev_other.emplace_back(e1, e2);
    }
    return DVM_OK;
}

// PARG_SLOT bytes of device memory per argument block of a persistent launch
constexpr size_t PARG_SLOT = 1024;
static_assert(sizeof(PersistArgs<double>) <= PARG_SLOT && sizeof(PersistArgs<float>) <= PARG_SLOT,
              "persistent arguments exceed their slot");

template <typename T>
static int send_persist_args(dvm_ctx *c, int slot, const PersistArgs<T> &a, const PersistArgs<T> **dev)
{
    std::vector<unsigned char> &sent = c->pargs_sent[slot];
    const unsigned char *b = reinterpret_cast<const unsigned char *>(&a);
    if (sent.size() != sizeof(a) || std::memcmp(sent.data(), b, sizeof(a)) != 0) {
        // a launch still queued may read the old arguments
        if (!sent.empty())
            HIPCHK(hipStreamSynchronize(c->stream));
        sent.assign(b, b + sizeof(a));
        HIPCHK(hipMemcpyAsync(c->d_pargs.p + slot * PARG_SLOT, sent.data(), sizeof(a), hipMemcpyHostToDevice,
                              c->stream));
    }
    *dev = reinterpret_cast<const PersistArgs<T> *>(c->d_pargs.p + slot * PARG_SLOT);
    return DVM_OK;
}

// A block of iterations of kind 0 (FP64 forward) or 2 (FP32 correction) as one
// cooperative launch, where the sweep mode and shape allow it; *done false:
// the caller runs the block as separate launches.
static int enqueue_persist(dvm_ctx *c, int iters, int kind, bool *done)
{
    *done = false;
    const bool f32 = kind == 2;
    const int V = f32 ? c->V32 : c->V, G = f32 ? c->G32 : c->G;
    const int mode = solve_mode(c) | xu_flag(c, V);
    if (kind == 1 || V != 4 || G != 8 || (mode & ~(MODE_FIELD | MODE_XU)) != 0 || c->items.empty())
        return DVM_OK;
    if (!c->d_pargs.p) {
        HIPCHK(c->d_pargs.alloc(2 * PARG_SLOT));
        HIPCHK(c->d_ctr.alloc(1));
        c->pargs_sent[0].clear();
        c->pargs_sent[1].clear();
    }
    // the work counter starts every launch at 0 (these launches are never
    // captured into a graph)
    HIPCHK(hipMemsetAsync(c->d_ctr.p, 0, sizeof(unsigned int), c->stream));
    hipError_t e;
    if (f32) {
        PersistArgs<float> a;
        std::memset(&a, 0, sizeof(a));
        const bool fused = fused_add32(c);
        a.sw = fused ? sweep_args32r(c) : sweep_args32(c);
        a.mom = fused ? mom_args32r(c) : mom_args32(c);
        a.rec = rec_args32(c);
        a.seg = fused ? (c->nseg32s > 0 ? c->d_seg32s.p : nullptr) : (c->nseg32 > 0 ? c->d_seg32.p : nullptr);
        a.nseg = fused ? c->nseg32s : c->nseg32;
        a.sb = state32(c);
        a.rr = c->d_rr.p;
        a.rr32 = fused ? c->d_rr32.p : nullptr;
        a.st = c->d_st32.p;
        a.n_inst = c->n_inst;
        a.nitems = (int)c->items.size();
        a.max_iter = c->cfg.max_iter;
        a.floor = STOP_FLOOR32;
        a.ctr = c->d_ctr.p;
        const PersistArgs<float> *dev = nullptr;
        int rc = send_persist_args(c, 1, a, &dev);
        if (rc)
            return rc;
        e = launch_persist<float>(dev, a.nitems, iters, refine_inner_tol(c), mode, c->stream);
    } else {
        PersistArgs<double> a;
        std::memset(&a, 0, sizeof(a));
        a.sw = sweep_args(c, 0, false);
        a.mom = mom_args(c, false);
        a.rec = rec_args(c, false);
        a.st = c->d_st.p;
        a.n_inst = c->n_inst;
        a.nitems = (int)c->items.size();
        a.max_iter = c->cfg.max_iter;
        a.floor = STOP_FLOOR64;
        a.ctr = c->d_ctr.p;
        const PersistArgs<double> *dev = nullptr;
        int rc = send_persist_args(c, 0, a, &dev);
        if (rc)
            return rc;
        e = launch_persist<double>(dev, a.nitems, iters, c->cfg.tol, mode, c->stream);
    }
    if (e == hipErrorNotSupported)
        return DVM_OK;
    HIPCHK(e);
    *done = true;
    c->prof.persistent_blocks += 1;
    c->prof.persistent_iters += iters;
    return DVM_OK;
}

static int enqueue_block(dvm_ctx *c, int iters, int kind)
{
    if (c->cfg.persistent && !c->cfg.profile) {
        bool done = false;
        int rc = enqueue_persist(c, iters, kind, &done);
        if (rc || done)
            return rc;
    }
    if (!c->cfg.use_graphs || c->cfg.profile) {
        for (int i = 0; i < iters; ++i) {
            int rc = enqueue_iteration(c, kind);
            if (rc)
                return rc;
        }
        return DVM_OK;
    }
    const int slot = kind;
    const int mode = solve_mode(c);
    if (!c->graph[slot] || c->graph_iters[slot] != iters || c->graph_mode[slot] != mode) {
        if (c->graph[slot]) {
            (void)hipGraphExecDestroy(c->graph[slot]);
            c->graph[slot] = nullptr;
        }
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        int rc = DVM_OK;
        for (int i = 0; i < iters && rc == DVM_OK; ++i)
            rc = enqueue_iteration(c, kind);
        hipError_t e = hipStreamEndCapture(c->stream, &g);
        if (rc)
            return rc;
        HIPCHK(e);
        e = hipGraphInstantiate(&c->graph[slot], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(e);
        c->graph_iters[slot] = iters;
        c->graph_mode[slot] = mode;
    }
    HIPCHK(hipGraphLaunch(c->graph[slot], c->stream));
    return DVM_OK;
}

// diagnostics on stderr when DVM_DEBUG is set (not 0)
static bool debug_on()
{
    static int on = -1;
    if (on < 0) {
        const char *e = std::getenv("DVM_DEBUG");
        on = (e && *e && *e != '0') ? 1 : 0;
    }
    return on == 1;
}

static int gmres_run(dvm_ctx *c, int i0, int i1, bool adj, std::vector<SolveState> &st,
                     const std::vector<long long> &prior, const std::vector<char> *trial = nullptr,
                     std::vector<char> *reverted = nullptr, bool mixed = false);

static long long state_segments(const dvm_ctx *c, int i, int pw, long long voff, std::vector<VSeg> *g,
                                std::vector<VSeg> *sc);

// Vector extrapolation of the dominant mode (DVM_ACCEL_AUTO): where the
// plain iteration contracts at a settled rate q along one mode, the state
// x_k and one more iteration x_{k+1} give x_{k+1} + q/(1-q) (x_{k+1} - x_k),
// which removes that mode (Aitken's process on the whole iteration state:
// moments, lagged seam and wrap values, wall-face values).  One extra
// iteration for every instance; the candidates' stop statistics restart.
static int extrapolate(dvm_ctx *c, int kind, const std::vector<int> &cand, const std::vector<double> &q,
                       std::vector<SolveState> &st)
{
    const bool adj = kind == 1;
    StateBufs sb;
    sb.b[0] = adj ? c->d_mom_adj.p : c->d_mom.p;
    sb.b[1] = adj ? c->d_seam_adj.p : c->d_seam.p;
    sb.b[2] = adj ? c->d_wrap_adj.p : c->d_wrap.p;
    sb.b[3] = adj ? c->d_fb_adj.p : c->d_fb.p;
    SolveState *dst = adj ? c->d_st_adj.p : c->d_st.p;
    KrylovWork &kw = c->kw;
    std::vector<VSeg> gseg, sseg;
    std::vector<long long> off(cand.size()), len(cand.size());
    long long n = 0;
    for (size_t k = 0; k < cand.size(); ++k) {
        off[k] = n;
        len[k] = state_segments(c, cand[k], (int)(st[cand[k]].iter & 1), n, &gseg, &sseg);
        n += len[k];
    }
    if (n == 0)
        return DVM_OK;
    if (kw.x.n < (size_t)n)
        HIPCHK(kw.x.alloc(n));
    if (kw.w.n < (size_t)n)
        HIPCHK(kw.w.alloc(n));
    HIPCHK(kw.gseg.alloc(gseg.size()));
    HIPCHK(kw.sseg.alloc(sseg.size()));
    HIPCHK(hipMemcpyAsync(kw.gseg.p, gseg.data(), gseg.size() * sizeof(VSeg), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(kw.sseg.p, sseg.data(), sseg.size() * sizeof(VSeg), hipMemcpyHostToDevice, c->stream));
    // x_k: the state the next sweep reads; then x_{k+1} = F(x_k)
    HIPCHK(launch_gather(kw.sseg.p, (int)sseg.size(), sb, kw.x.p, nullptr, c->stream));
    double upd = 0.0;              // updates of the extra iteration (profiling)
    for (int i = 0; i < c->n_inst; ++i)
        if (st[i].active)
            upd += (double)c->inst[i].nfluid * c->K;
    int rc = enqueue_iteration(c, kind);
    if (rc)
        return rc;
    HIPCHK(launch_gather(kw.gseg.p, (int)gseg.size(), sb, kw.w.p, nullptr, c->stream));
    HIPCHK(hipMemcpyAsync(st.data(), dst, c->n_inst * sizeof(SolveState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->cfg.profile && kind != 1 && (rc = collect_profile(c, 1, upd)))
        return rc;
    for (size_t k = 0; k < cand.size(); ++k) {
        if (!st[cand[k]].active)
            continue;       // stopped in the extra iteration: keep F(x_k)
        const double f = q[k] / (1.0 - q[k]);
        HIPCHK(launch_axpy(kw.x.p + off[k], kw.w.p + off[k], -1.0, len[k], c->stream));   // x_k - x_{k+1}
        HIPCHK(launch_axpy(kw.w.p + off[k], kw.x.p + off[k], -f, len[k], c->stream));
    }
    HIPCHK(launch_scatter(kw.gseg.p, (int)gseg.size(), sb, kw.w.p, c->stream));
    // records of the next sweep from the extrapolated moments
    HIPCHK(launch_record<double>(rec_args(c, adj), c->max_cells, c->n_inst, c->stream));
    HIPCHK(hipMemcpyAsync(st.data(), dst, c->n_inst * sizeof(SolveState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (size_t k = 0; k < cand.size(); ++k) {
        SolveState &s = st[cand[k]];
        if (!s.active)
            continue;
        s.maxdiff_bits = s.maxabs_bits = 0ull;
        s.eps_prev = 0.0;
        s.npass = 0;
        s.qfloor = std::max(s.qfloor, q[k]);
    }
    HIPCHK(hipMemcpyAsync(dst, st.data(), c->n_inst * sizeof(SolveState), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return DVM_OK;
}

// The same extrapolation for the FP32 correction iteration of the
// refinement, e <- L32 e + r: its state (FP64 moments, FP32 seam, wrap and
// wall values) is read into FP64 vectors in the layout of the live
// refinement slots, combined there, and written back (FP32 parts rounded).
static int extrapolate32(dvm_ctx *c, const std::vector<int> &cand, const std::vector<double> &q,
                         std::vector<SolveState> &st)
{
    const long long n = c->dc_n;
    if (n == 0)
        return DVM_OK;
    KrylovWork &kw = c->kw;
    if (kw.x.n < (size_t)n)
        HIPCHK(kw.x.alloc(n));
    if (kw.w.n < (size_t)n)
        HIPCHK(kw.w.alloc(n));
    // x_k: the state the next sweep reads; then x_{k+1} = L32 x_k + r
    HIPCHK(launch_state32(c->d_seg32.p, c->nseg32, c->d_st32.p, state32(c), kw.x.p, 2, c->stream));
    double upd = 0.0;
    for (int i = 0; i < c->n_inst; ++i)
        if (st[i].active)
            upd += (double)c->inst[i].nfluid * c->K;
    int rc = enqueue_iteration(c, 2);
    if (rc)
        return rc;
    HIPCHK(launch_state32(c->d_seg32.p, c->nseg32, c->d_st32.p, state32(c), kw.w.p, 2, c->stream));
    HIPCHK(hipMemcpyAsync(st.data(), c->d_st32.p, c->n_inst * sizeof(SolveState), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->cfg.profile && (rc = collect_profile(c, 1, upd)))
        return rc;
    for (size_t k = 0; k < cand.size(); ++k) {
        const int i = cand[k];
        if (!st[i].active || c->dc_off[i] < 0)
            continue;       // stopped in the extra iteration: keep x_{k+1}
        const double f = q[k] / (1.0 - q[k]);
        const long long o = c->dc_off[i], len = c->dc_len[i];
        HIPCHK(launch_axpy(kw.x.p + o, kw.w.p + o, -1.0, len, c->stream));   // x_k - x_{k+1}
        HIPCHK(launch_axpy(kw.w.p + o, kw.x.p + o, -f, len, c->stream));
    }
    HIPCHK(launch_state32(c->d_seg32.p, c->nseg32, c->d_st32.p, state32(c), kw.w.p, 1, c->stream));
    // records of the next sweep from the extrapolated moments
    HIPCHK(launch_record<float>(rec_args32(c), c->max_cells, c->n_inst, c->stream));
    HIPCHK(hipMemcpyAsync(st.data(), c->d_st32.p, c->n_inst * sizeof(SolveState), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (size_t k = 0; k < cand.size(); ++k) {
        SolveState &s = st[cand[k]];
        if (!s.active)
            continue;
        s.maxdiff_bits = s.maxabs_bits = 0ull;
        s.eps_prev = 0.0;
        s.npass = 0;
        s.qfloor = std::max(s.qfloor, q[k]);
    }
    HIPCHK(hipMemcpyAsync(c->d_st32.p, st.data(), c->n_inst * sizeof(SolveState), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return DVM_OK;
}

// GMRES trial under AUTO: the plain iteration must be predicted to need more
// than this many further iterations.  FP64 solver: 150 (with deflated
// restarts GMRES pays off sooner; measured on the bench workloads: time to
// solution of the uneven batch in FP64 10.9 s at 1000, 7.5 s at 300, 7.3 s at
// 150; the porous sweep's step 11.8 / 9.8 / 8.4 s).  The FP64 tails of the
// refinement: 300 (the batch's refinement took 7.1 s at 150, 6.8 s at 300).
// FP32 correction iteration: 1000 (its GMRES adds an FP64 residual sweep per
// cycle; 6.8 s at 1000 and 6.9 s at 300).
constexpr double TRIAL_MIN_ITERS64 = 150.0;
constexpr double TRIAL_MIN_ITERS64_TAIL = 300.0;
constexpr double TRIAL_MIN_ITERS32 = 1000.0;

// Replay blocks of iterations until no instance of [i0, i1) is active.  A
// stalled instance is stopped and flagged in stalled[] (its state is that of
// a completed iteration).
// Stall test (when `stalled` is given), over the last 64 iterations: an
// instance whose relative change has not dropped by 5% while max |u1| grew
// by more than 10% runs away instead of creeping towards the fixed point
// (stalled = 2); one whose relative change has not dropped by 0.5% does not
// contract at all (stalled = 1).  A slow but contracting iteration (large
// delta) is not stopped by this test.  Instances with grow_only set stop only in the
// first case.
// With no_trial given (AUTO), an instance whose contraction per iteration has
// settled above 0.98 (no extrapolation there) with more than
// TRIAL_MIN_ITERS64 (refinement tails: TRIAL_MIN_ITERS64_TAIL) iterations
// still to go is stopped for a GMRES trial (stalled = 3); its rate is left in
// c->trial_q.
static int run_blocks(dvm_ctx *c, int i0, int i1, const std::vector<long long> &iter0, int kind,
                      std::vector<SolveState> &st, std::vector<char> *stalled = nullptr,
                      const std::vector<char> *grow_only = nullptr,
                      const std::vector<char> *no_trial = nullptr)
{
    const int B = c->cfg.block_iters > 0 ? c->cfg.block_iters : 32;
    const long long cap = c->cfg.max_iter;
    const long long W = 64;
    const double tol = c->cfg.tol;
    SolveState *dst = kind == 1 ? c->d_st_adj.p : kind == 2 ? c->d_st32.p : c->d_st.p;
    struct Hist {
        long long it;
        double eps, amax;
    };
    std::vector<std::vector<Hist>> hist(c->n_inst);
    std::vector<long long> before(c->n_inst);
    // relative change at block ends since the last extrapolation; an
    // instance whose relative change, a block after an extrapolation, is
    // above the one the extrapolation started from is not extrapolated again
    const bool extrap = c->cfg.accel == DVM_ACCEL_AUTO;
    // FP32 correction iterations (AUTO): one whose rate settles above 0.995
    // with more than 1000 iterations to go stops (stalled = 3); the
    // refinement continues that instance in FP64, where GMRES can take over
    const bool slow32 = c->cfg.accel == DVM_ACCEL_AUTO && kind == 2 && stalled;
    std::vector<std::vector<double>> eh(c->n_inst);
    std::vector<double> eps_at(c->n_inst, -1.0);
    std::vector<char> no_extrap(c->n_inst, 0);
    for (;;) {
        for (int i = 0; i < c->n_inst; ++i)
            before[i] = st[i].iter;
        int rc = enqueue_block(c, B, kind);
        if (rc)
            return rc;
        HIPCHK(hipMemcpyAsync(st.data(), dst, c->n_inst * sizeof(SolveState), hipMemcpyDeviceToHost,
                              c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (c->cfg.profile) {
            long long real = 0;
            double upd = 0.0;
            for (int i = 0; i < c->n_inst; ++i) {
                real = std::max(real, st[i].iter - before[i]);
                upd += (double)(st[i].iter - before[i]) * (double)c->inst[i].nfluid * c->K;
            }
            int prc = collect_profile(c, real, kind == 1 ? 0.0 : upd);
            if (prc)
                return prc;
        }
        bool running = false, stop = false;
        for (int i = i0; i < i1; ++i) {
            if (!(st[i].active && st[i].iter - iter0[i] < cap))
                continue;
            if (stalled) {
                auto &hv = hist[i];
                const long long it = st[i].iter - iter0[i];
                hv.push_back(Hist{it, st[i].eps, st[i].amax});
                const Hist *old = nullptr;
                for (const auto &e : hv)
                    if (e.it <= it - W)
                        old = &e;
                if (old && old->eps > 0.0 && st[i].eps > (st[i].tol > 0.0 ? st[i].tol : tol)) {
                    const bool runaway = !(st[i].eps < 0.95 * old->eps) && st[i].amax > 1.1 * old->amax;
                    const bool flat = !(st[i].eps < 0.995 * old->eps);
                    if (runaway || (flat && !(grow_only && (*grow_only)[i]))) {
                        st[i].active = 0;
                        (*stalled)[i] = runaway ? 2 : 1;
                        stop = true;
                        continue;
                    }
                }
            }
            running = true;
        }
        if (stop) {
            HIPCHK(hipMemcpyAsync(dst, st.data(), c->n_inst * sizeof(SolveState), hipMemcpyHostToDevice,
                                  c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
        }
        if (!running)
            return DVM_OK;
        if (extrap) {
            // a settled rate: per-iteration contraction over the last two
            // blocks agreeing to 5% of the gap 1 - q, and q <= 0.98 (the
            // factor q/(1-q) also multiplies the next mode's error: closer
            // to 1 it can amplify that mode more than it removes)
            std::vector<int> cand;
            std::vector<double> qs;
            bool trial_stop = false;
            for (int i = i0; i < i1; ++i) {
                if (!(st[i].active && st[i].iter - iter0[i] < cap) || no_extrap[i])
                    continue;
                auto &e = eh[i];
                e.push_back(st[i].eps);
                if (eps_at[i] > 0.0 && e.size() == 1 && !(st[i].eps < eps_at[i])) {
                    no_extrap[i] = 1;
                    continue;
                }
                const double tli = st[i].tol > 0.0 ? st[i].tol : tol;
                // what still separates the instance from its stop rule: the
                // change itself, or below the tolerance the a-posteriori
                // bound (a slow iteration spends most of its sweeps with a
                // change below the tolerance and a bound above it)
                const double err = std::min(std::max(st[i].eps, std::isnan(st[i].est) ? 0.0 : st[i].est), 1e300);
                if (e.size() < 3 || !(err > tli) || !(st[i].eps > 1e-13))
                    continue;
                const double e0 = e[e.size() - 3], e1 = e[e.size() - 2], e2 = e.back();
                if (!(e0 > 0.0 && e1 > 0.0 && e2 > 0.0))
                    continue;
                const double qa = std::pow(e2 / e1, 1.0 / B), qb = std::pow(e1 / e0, 1.0 / B);
                const bool settled = std::fabs(qa - qb) <= 0.05 * (1.0 - qa);
                if (debug_on())
                    std::fprintf(stderr, "[dvm rate] inst %d after %lld: eps %.3e q %.5f (previous block %.5f)%s\n",
                                 i, st[i].iter - iter0[i], st[i].eps, qa, qb, settled ? " settled" : "");
                // the FP32 correction iteration: extrapolating its state also
                // multiplies the state's FP32 rounding (about 6e-8 of it) by
                // q/(1-q); only where the correction's own tolerance stays far
                // above that
                const bool quiet = kind != 2 || tli >= 2e-6 * qa / (1.0 - qa);
                if (slow32 && !(no_trial && (*no_trial)[i]) && qa > 0.98 && qa < 1.0 && settled &&
                    std::log(tol / err) / std::log(qa) > TRIAL_MIN_ITERS32) {
                    // (the iterations predicted to the outer tolerance, as for
                    // the FP64 iteration's GMRES trial)
                    st[i].active = 0;
                    (*stalled)[i] = 3;
                    c->trial_q[i] = qa;
                    trial_stop = true;
                } else if (qa > 0.5 && qa <= 0.98 && settled && quiet) {
                    cand.push_back(i);
                    qs.push_back(qa);
                    eps_at[i] = st[i].eps;
                    e.clear();
                } else if (kind != 2 && stalled && no_trial && !(*no_trial)[i] && qa > 0.98 && qa < 1.0 &&
                           settled && std::log(tol / err) / std::log(qa) >
                                          (c->cfg.precision == DVM_FP32_REFINE ? TRIAL_MIN_ITERS64_TAIL
                                                                               : TRIAL_MIN_ITERS64)) {
                    st[i].active = 0;
                    (*stalled)[i] = 3;
                    c->trial_q[i] = qa;
                    trial_stop = true;
                }
            }
            if (trial_stop) {
                HIPCHK(hipMemcpyAsync(dst, st.data(), c->n_inst * sizeof(SolveState), hipMemcpyHostToDevice,
                                      c->stream));
                HIPCHK(hipStreamSynchronize(c->stream));
                bool left = false;
                for (int i = i0; i < i1; ++i)
                    left = left || (st[i].active && st[i].iter - iter0[i] < cap);
                if (!left)
                    return DVM_OK;
            }
            if (!cand.empty()) {
                rc = kind == 2 ? extrapolate32(c, cand, qs, st) : extrapolate(c, kind, cand, qs, st);
                if (rc)
                    return rc;
            }
        }
    }
}

// The iteration of [i0, i1) as configured: plain, GMRES, or plain with GMRES
// taking over stalled instances.  Leaves per-instance sweep counts in
// c->sweeps_done.
static int iterate(dvm_ctx *c, int i0, int i1, const std::vector<long long> &iter0_in, bool adj,
                   std::vector<SolveState> &st, std::vector<char> *need_skew = nullptr)
{
    if (c->cfg.accel == DVM_ACCEL_GMRES) {
        std::vector<long long> prior;
        return gmres_run(c, i0, i1, adj, st, prior);
    }
    // stall detection: for GMRES takeover (accel AUTO), and for instances on
    // the wrap-around diagonal under DVM_SCHED_AUTO, which move to the skewed
    // order when their iterates run away
    auto on_wrap = [&](int i) {
        return need_skew && c->cfg.schedule == DVM_SCHED_AUTO && !c->inst[i].force_skew &&
               c->inst[i].nx >= WRAP_MIN;
    };
    const bool gm = c->cfg.accel == DVM_ACCEL_AUTO;
    bool detect = gm;
    std::vector<char> grow_only(c->n_inst, gm ? 0 : 1);
    for (int i = i0; i < i1; ++i)
        detect = detect || on_wrap(i);
    // an instance whose GMRES trial lost to the plain iteration is not tried
    // again and stays plain; base = its sweeps before the current plain pass
    std::vector<char> no_trial(c->n_inst, gm ? 0 : 1);
    std::vector<int> ntrial(c->n_inst, 0);    // GMRES trials handed back so far
    std::vector<long long> iter0 = iter0_in, base(c->n_inst, 0);
    std::vector<char> counted(c->n_inst, 0);   // finished in GMRES: count final
    SolveState *dst = adj ? c->d_st_adj.p : c->d_st.p;
    for (;;) {
        std::vector<char> stalled(c->n_inst, 0);
        int rc = run_blocks(c, i0, i1, iter0, adj ? 1 : 0, st, detect ? &stalled : nullptr, &grow_only,
                            gm ? &no_trial : nullptr);
        if (rc)
            return rc;
        std::vector<long long> prior(c->n_inst, 0);
        std::vector<char> trial(c->n_inst, 0);
        bool any = false;
        for (int i = i0; i < i1; ++i) {
            if (counted[i])
                continue;
            prior[i] = base[i] + st[i].iter - iter0[i];
            c->sweeps_done[i] = prior[i];
            if (debug_on() && stalled[i])
                std::fprintf(stderr, "[dvm iterate] inst %d stopped (%d) after %lld sweeps, eps %.3e\n", i,
                             (int)stalled[i], prior[i], st[i].eps);
            if (on_wrap(i) && (stalled[i] == 2 || st[i].status == STATUS_DIVERGED)) {
                (*need_skew)[i] = 1;
            } else if (stalled[i]) {
                if (gm) {
                    st[i].active = 1;
                    st[i].status = STATUS_RUNNING;
                    trial[i] = stalled[i] == 3;
                    any = true;
                } else {
                    st[i].status = STATUS_DIVERGED;  // runs away: the plain iteration cannot converge
                }
            }
        }
        if (!any)
            return DVM_OK;
        HIPCHK(hipMemcpyAsync(dst, st.data(), c->n_inst * sizeof(SolveState), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        std::vector<char> reverted(c->n_inst, 0);
        if ((rc = gmres_run(c, i0, i1, adj, st, prior, &trial, &reverted)))
            return rc;
        // trial instances handed back: the plain iteration resumes from the
        // state GMRES reached (records from its moments, fresh stop history)
        bool again = false;
        for (int i = i0; i < i1; ++i) {
            if (stalled[i] && !reverted[i])
                counted[i] = 1;
            if (!reverted[i])
                continue;
            again = true;
            // a second trial once the plain iteration has shown its rate
            // again from the state GMRES reached (the rate measured before
            // the first trial can flatter it); after that, back for good:
            // neither another trial nor a takeover when the plain iteration
            // then creeps
            ntrial[i] += 1;
            no_trial[i] = ntrial[i] >= 2 ? 1 : 0;
            grow_only[i] = no_trial[i];
            base[i] = c->sweeps_done[i];
            iter0[i] = st[i].iter;
            // the stop rule's ratio is held at least at the rate measured
            // before the trial: the slow modes GMRES left still contract at
            // it, while two successive changes first show faster ones
            SolveState &s = st[i];
            s.active = 1;
            s.status = STATUS_RUNNING;
            s.npass = 0;
            s.eps_prev = 0.0;
            s.qfloor = std::max(s.qfloor, c->trial_q[i]);
            s.maxdiff_bits = s.maxabs_bits = 0ull;
        }
        if (!again)
            return DVM_OK;
        HIPCHK(hipMemcpyAsync(dst, st.data(), c->n_inst * sizeof(SolveState), hipMemcpyHostToDevice, c->stream));
        HIPCHK(launch_record<double>(rec_args(c, adj), c->max_cells, c->n_inst, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        for (int i = i0; i < i1; ++i)
            if (reverted[i])
                st[i].maxdiff_bits = st[i].maxabs_bits = 0ull;
        HIPCHK(hipMemcpyAsync(dst, st.data(), c->n_inst * sizeof(SolveState), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
}

// --------------------------------------------------------------- GMRES
// The source iteration is an affine map x -> F(x) = L x + b of its state x:
// the cell moments (they define the next collision gain and wall values),
// the values lagged across strip seams and the periodic x seam, and (for
// alpha < 1) the incident wall-face values.  Restarted GMRES solves
// (I - L) x = b with the same sweeps: L v is one sweep without the drive.
// Each cycle starts with one full iteration from the current x, which gives
// the residual x - F(x) and the relative change eps of u1; an instance is
// accepted when eps / sigma <= tol, sigma the smallest singular value of the
// last Krylov projection (clamped to [1e-3, 1]), or eps is at round-off.  The
// accepted state is F(x).

struct Slot {
    int inst;
    long long off, len;
    int pw;           // parity written by the sweeps while GMRES runs
};

static void add_seg(std::vector<VSeg> &v, int buf, long long boff, long long voff, long long len)
{
    while (len > 0) {
        const int l = (int)std::min<long long>(len, VCHUNK);
        v.push_back(VSeg{boff, voff, l, buf});
        boff += l;
        voff += l;
        len -= l;
    }
}

// Segments of one instance's state: outputs of a sweep (parity pw) for
// gather, inputs of the next sweep (parity pw ^ 1) for scatter.  Returns the
// state length.
static long long state_segments(const dvm_ctx *c, int i, int pw, long long voff, std::vector<VSeg> *g,
                                std::vector<VSeg> *sc)
{
    const HostInst &h = c->inst[i];
    const InstDev &d = c->idev[i];
    const int pr = pw ^ 1;
    long long v = voff;
    auto both = [&](int buf, long long off_w, long long off_r, long long len) {
        if (g)
            add_seg(*g, buf, off_w, v, len);
        if (sc)
            add_seg(*sc, buf, off_r, v, len);
        v += len;
    };
    const long long nmom = (long long)d.nx * d.ny * MOM_STRIDE;
    both(0, d.cell_off * MOM_STRIDE, d.cell_off * MOM_STRIDE, nmom);
    const long long kq = c->kq, kp4 = c->kp4;
    for (int st = 0; st < d.nstrips; ++st) {
        const bool up = st < d.nstrips - 1 || d.periodic_y;   // eta > 0 quadrants feed the strip above
        const bool dn = st > 0 || d.periodic_y;               // eta < 0 quadrants feed the strip below
        if (!up && !dn)
            continue;
        const long long k0 = up ? 0 : 2 * kq, k1 = dn ? 4 * kq : 2 * kq;
        for (int x = 0; x < d.nx; ++x)
            for (int sl = 0; sl < 2; ++sl) {
                const long long rel = d.seam_off + (((long long)st * d.nx + x) * 2 + sl) * kp4 + k0;
                both(1, pw * c->seam_half + rel, pr * c->seam_half + rel, k1 - k0);
            }
    }
    if (d.nx > 1)
        for (int st = 0; st < d.nstrips; ++st)
            for (int sl = 0; sl < 3; ++sl) {
                const long long off = d.wrap_off + ((long long)st * 3 + sl) * kp4 * 64;
                both(2, off, off, kp4 * 64);
            }
    if (h.alpha < 1.0 && h.nfaces > 0) {
        const long long fh = std::max<long long>(c->nfaces, 1) * kp4;
        const long long rel = h.face_base * kp4;
        both(3, pw * fh + rel, pr * fh + rel, (long long)h.nfaces * kp4);
    }
    return v - voff;
}

struct GmresSlotHost {
    std::vector<double> H, cs, sn, g;   // H: (m+1) x m column-major, rotated to R
    std::vector<double> Hr;             // the same unrotated (the cycle's Hessenberg Hb)
    std::vector<double> c;              // right-hand side of the cycle in its basis
    std::vector<double> Q0;             // deflated restart: orthogonal factor of the kept block
    std::vector<double> P, Hn;          //                   next cycle's basis map and block
    int kd = 0;                         // kept vectors this cycle starts from
    int kq = 0;                         // columns of this cycle so far
    bool done = false;                  // its Arnoldi process has stopped
    double beta = 0.0, sig = -1.0;
    bool live = true;
    long long sweeps = 0;
    long long sweeps64 = 0;             // of this run's sweeps, the FP64 ones
    double trial_red = 0.0;             // trial: -log of the residual reduction so far
    double trial_cost = 0.0;            //        and its work in sweep equivalents
    double beta_prev = 0.0;             // residual norm at the previous cycle's start
};

// smallest singular value of the k x k upper triangular R (column-major,
// leading dimension ld) by inverse iteration on R^T R
static double sigma_min_tri(const std::vector<double> &R, int ld, int k)
{
    if (k == 0)
        return 1.0;
    std::vector<double> z(k, 1.0 / std::sqrt((double)k)), t(k), u(k);
    double lam = 0.0;
    for (int it = 0; it < 40; ++it) {
        for (int i = 0; i < k; ++i) {           // R^T t = z
            double a = z[i];
            for (int j = 0; j < i; ++j)
                a -= R[(size_t)i * ld + j] * t[j];
            const double dg = R[(size_t)i * ld + i];
            if (dg == 0.0)
                return 0.0;
            t[i] = a / dg;
        }
        for (int i = k - 1; i >= 0; --i) {      // R u = t
            double a = t[i];
            for (int j = i + 1; j < k; ++j)
                a -= R[(size_t)j * ld + i] * u[j];
            u[i] = a / R[(size_t)i * ld + i];
        }
        double nrm = 0.0;
        for (double q : u)
            nrm += q * q;
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0) || !std::isfinite(nrm))
            return 0.0;
        lam = nrm;
        for (int i = 0; i < k; ++i)
            z[i] = u[i] / nrm;
    }
    return 1.0 / std::sqrt(lam);
}

// GMRES restart length with deflated restarts (dvm_config.krylov_dim = 0);
// a cycle then keeps a quarter of it (krylov_deflate = 0).  Time to solution
// of the uneven batch at 1e-6 (FP32 + refinement): 7.83 s at (64, 16), 6.73 s
// at (40, 10), 6.82 s at (48, 12), 6.87 s at (32, 8).
constexpr int KRYLOV_DIM_DEFLATED = 40;

// Work of one GMRES cycle of k Arnoldi steps on one instance, in sweeps of
// that instance: the cycle's k + 1 sweeps, plus the HBM traffic of the
// orthogonalisation over its state vector of len elements (step j reads the
// j FP32 basis vectors twice, dots and update, and w, the new basis vector
// and the gathered state a few times: about 8 j + 60 bytes per element)
// expressed at the bytes an FP64 sweep update costs in time (about 8 bytes
// at the vector kernels' bandwidth: 200 us per 1.07e8 updates against
// about 4.6 TB/s, measured on the rough channel; an FP32 sweep update costs
// about 5 such bytes, 0.6 of the FP64 one, measured on the uneven batch).
static double gmres_cycle_cost(int k, long long len, double updates_per_sweep, double bytes_per_update)
{
    const double bytes = (4.0 * k * (k + 1) + 60.0 * k) * (double)len;
    return (double)(k + 1) + bytes / (bytes_per_update * std::max(updates_per_sweep, 1.0));
}

static int gmres_run(dvm_ctx *c, int i0, int i1, bool adj, std::vector<SolveState> &st,
                     const std::vector<long long> &prior, const std::vector<char> *trial,
                     std::vector<char> *reverted, bool mixed)
{
    // restart length and the harmonic Ritz vectors a cycle hands to the next
    // (deflated restarts; defaults measured on the uneven batch, the porous
    // rarefaction sweep and the Couette channels)
    const bool deflate = c->cfg.krylov_deflate >= 0;
    const int m = c->cfg.krylov_dim > 0 ? std::min(c->cfg.krylov_dim, 64)
                                        : (deflate ? KRYLOV_DIM_DEFLATED : 64);
    const int want = !deflate ? 0 : std::min(c->cfg.krylov_deflate > 0 ? c->cfg.krylov_deflate : m / 4, m / 2 - 1);
    const int mode = solve_mode(c) | (adj ? MODE_ADJ : xu_flag(c, c->V));
    SolveState *dst = adj ? c->d_st_adj.p : c->d_st.p;
    StateBufs sb;
    sb.b[0] = adj ? c->d_mom_adj.p : c->d_mom.p;
    sb.b[1] = adj ? c->d_seam_adj.p : c->d_seam.p;
    sb.b[2] = adj ? c->d_wrap_adj.p : c->d_wrap.p;
    sb.b[3] = adj ? c->d_fb_adj.p : c->d_fb.p;

    std::vector<Slot> slots;
    long long n = 0;
    for (int i = i0; i < i1; ++i) {
        if (!st[i].active)
            continue;
        Slot sl{i, n, 0, (int)(st[i].iter & 1)};
        sl.len = state_segments(c, i, sl.pw, n, nullptr, nullptr);
        // slots (and with them every chunk) start on a multiple of 4
        // elements: the basis kernels load 4 at a time
        n += (sl.len + 3) & ~3LL;
        slots.push_back(sl);
    }
    const int ns = (int)slots.size();
    if (ns == 0)
        return DVM_OK;
    KrylovWork &kw = c->kw;
    auto grow = [&](auto &b, size_t cnt) -> hipError_t {
        return b.n >= cnt ? hipSuccess : b.alloc(cnt);
    };
    const long long nchmax = n / VCHUNK + ns + 1;
    if (kw.V.n < (size_t)(m + 1) * n) {
        // zeroed once: an instance whose Arnoldi process has stopped still
        // has the later basis columns scattered into its state (and its
        // results ignored), which must hold finite values
        HIPCHK(kw.V.alloc((size_t)(m + 1) * n));
        HIPCHK(launch_zero_f(kw.V.p, kw.V.n, c->stream));
    }
    HIPCHK(grow(kw.x, n));
    HIPCHK(grow(kw.w, n));
    HIPCHK(grow(kw.part, (size_t)(m + 2) * nchmax));
    HIPCHK(grow(kw.c1, (size_t)ns * (m + 2)));
    HIPCHK(grow(kw.c2, (size_t)ns * (m + 2)));
    HIPCHK(grow(kw.y, (size_t)ns * (m + 2)));
    const int cst = m + 2;
    const int pstr = VCOMB_IN * VCOMB_OUT;
    if (want > 0) {
        HIPCHK(grow(kw.T, (size_t)(want + 2) * n));
        HIPCHK(grow(kw.pc, (size_t)ns * pstr));
    }
    std::vector<double> hpc(want > 0 ? (size_t)ns * pstr : 0);

    std::vector<GmresSlotHost> hs(ns);
    for (int q = 0; q < ns; ++q)
        hs[q].sweeps = prior.empty() ? 0 : prior[slots[q].inst];
    for (auto &h : hs) {
        h.H.assign((size_t)(m + 1) * m, 0.0);
        h.Hr.assign((size_t)(m + 1) * m, 0.0);
        h.c.assign(m + 1, 0.0);
        h.cs.assign(m, 0.0);
        h.sn.assign(m, 0.0);
        h.g.assign(m + 1, 0.0);
    }
    // mixed: Krylov steps with FP32 sweeps on the FP32 correction state
    std::vector<SolveState> st32;
    int nseg2 = 0;
    if (mixed) {
        if (adj || !c->fp32_ready)
            return fail(DVM_ESTATE, "mixed-precision GMRES needs the FP32 state of the refinement");
        st32.resize(c->n_inst);
        HIPCHK(hipMemcpyAsync(st32.data(), c->d_st32.p, c->n_inst * sizeof(SolveState), hipMemcpyDeviceToHost,
                              c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        for (auto &s32 : st32)
            s32.active = 0;
    }
    // tables of the live slots (rebuilt when a slot finishes)
    std::vector<VSeg> gseg, sseg;
    std::vector<VChunk> chunks;
    std::vector<int> c0(ns), ncs(ns);
    auto rebuild = [&]() -> int {
        gseg.clear();
        sseg.clear();
        chunks.clear();
        for (int q = 0; q < ns; ++q) {
            c0[q] = (int)chunks.size();
            if (hs[q].live) {
                state_segments(c, slots[q].inst, slots[q].pw, slots[q].off, &gseg, &sseg);
                for (long long o = 0; o < slots[q].len; o += VCHUNK)
                    chunks.push_back(VChunk{slots[q].off + o, (int)std::min<long long>(VCHUNK, slots[q].len - o), q});
            }
            ncs[q] = (int)chunks.size() - c0[q];
        }
        HIPCHK(kw.gseg.alloc(std::max<size_t>(gseg.size(), 1)));
        HIPCHK(kw.sseg.alloc(std::max<size_t>(sseg.size(), 1)));
        HIPCHK(kw.ch.alloc(std::max<size_t>(chunks.size(), 1)));
        HIPCHK(kw.c0.alloc(ns));
        HIPCHK(kw.nc.alloc(ns));
        HIPCHK(hipMemcpyAsync(kw.gseg.p, gseg.data(), gseg.size() * sizeof(VSeg), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(kw.sseg.p, sseg.data(), sseg.size() * sizeof(VSeg), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(kw.ch.p, chunks.data(), chunks.size() * sizeof(VChunk), hipMemcpyHostToDevice,
                              c->stream));
        HIPCHK(hipMemcpyAsync(kw.c0.p, c0.data(), ns * sizeof(int), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(kw.nc.p, ncs.data(), ns * sizeof(int), hipMemcpyHostToDevice, c->stream));
        if (mixed) {
            // the Krylov steps run on the FP32 correction state: its segments
            // in this run's vector layout, and its active flags (the parity of
            // each instance's FP32 state is left where the refinement left it)
            std::vector<VSeg2> s2;
            for (int q = 0; q < ns; ++q) {
                st32[slots[q].inst].active = hs[q].live ? 1 : 0;
                if (!hs[q].live)
                    continue;
                std::vector<VSeg> g0, g1;
                state_segments(c, slots[q].inst, 0, slots[q].off, &g0, nullptr);
                state_segments(c, slots[q].inst, 1, slots[q].off, &g1, nullptr);
                for (size_t k = 0; k < g0.size(); ++k)
                    s2.push_back(VSeg2{{g0[k].buf_off, g1[k].buf_off}, g0[k].vec_off, g0[k].len, g0[k].buf,
                                       slots[q].inst});
            }
            nseg2 = (int)s2.size();
            HIPCHK(kw.seg2.alloc(std::max<size_t>(s2.size(), 1)));
            HIPCHK(hipMemcpyAsync(kw.seg2.p, s2.data(), s2.size() * sizeof(VSeg2), hipMemcpyHostToDevice,
                                  c->stream));
            HIPCHK(hipMemcpyAsync(c->d_st32.p, st32.data(), c->n_inst * sizeof(SolveState), hipMemcpyHostToDevice,
                                  c->stream));
        }
        HIPCHK(hipStreamSynchronize(c->stream));
        return DVM_OK;
    };
    int rc = rebuild();
    if (rc)
        return rc;
    const int nch = (int)chunks.size();
    (void)nch;
    // L v for the Krylov step from basis vector v (FP32): w = v - L v
    auto krylov_step = [&](const float *v) -> int {
        if (!mixed) {
            HIPCHK(launch_scatter(kw.sseg.p, (int)sseg.size(), sb, v, c->stream));
            RecArgs<double> ra = rec_args(c, adj);
            ra.homog = 1;
            ra.monitor = 0;
            HIPCHK(launch_record<double>(ra, c->max_cells, c->n_inst, c->stream));
            HIPCHK(launch_sweep<double>(sweep_args(c, 0, adj), (int)c->items.size(), c->V, c->G, mode, c->stream));
            HIPCHK(launch_moments(mom_args(c, adj), c->max_cells, c->n_inst, c->stream));
            HIPCHK(launch_gather_sub32(kw.gseg.p, (int)gseg.size(), sb, kw.w.p, v, c->stream));
            return DVM_OK;
        }
        HIPCHK(launch_state32_basis(kw.seg2.p, nseg2, c->d_st32.p, state32(c), nullptr, v, 0, c->stream));
        RecArgs<float> r32 = rec_args32(c);
        r32.monitor = 0;
        HIPCHK(launch_record<float>(r32, c->max_cells, c->n_inst, c->stream));
        HIPCHK(launch_sweep<float>(sweep_args32(c), (int)c->items.size(), c->V32, c->G32,
                                   solve_mode(c) | xu_flag(c, c->V32), c->stream));
        HIPCHK(launch_moments(mom_args32(c), c->max_cells, c->n_inst, c->stream));
        HIPCHK(launch_state32_basis(kw.seg2.p, nseg2, c->d_st32.p, state32(c), kw.w.p, v, 1, c->stream));
        return DVM_OK;
    };
    auto sweep_once = [&](bool homog, bool monitor) -> int {
        RecArgs<double> ra = rec_args(c, adj);
        ra.homog = homog ? 1 : 0;
        ra.monitor = monitor ? 1 : 0;
        HIPCHK(launch_record<double>(ra, c->max_cells, c->n_inst, c->stream));
        HIPCHK(launch_sweep<double>(sweep_args(c, 0, adj), (int)c->items.size(), c->V, c->G, mode, c->stream));
        HIPCHK(launch_moments(mom_args(c, adj), c->max_cells, c->n_inst, c->stream));
        return DVM_OK;
    };
    // dots of w against V_0..V_{nv-1} (and |w|^2) summed per slot into
    // out[slot][.]; with skip, slots whose first pass (skip's coefficients)
    // kept |w| above 1/sqrt(2) of its length get zero dots
    auto dots = [&](const double *w, int nv, bool norm, double *out, const double *skip = nullptr) -> int {
        const int nchl = (int)chunks.size();
        HIPCHK(launch_vdots4(kw.ch.p, nchl, w, kw.V.p, n, nv, norm ? 1 : 0, kw.part.p, skip, cst, c->stream));
        HIPCHK(launch_vsum(kw.c0.p, kw.nc.p, ns, kw.part.p, nchl, nv + (norm ? 1 : 0), out, cst, c->stream));
        return DVM_OK;
    };
    // synchronous: the host vector is modified again right after
    auto upload_st = [&]() -> int {
        HIPCHK(hipMemcpyAsync(dst, st.data(), c->n_inst * sizeof(SolveState), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        return DVM_OK;
    };
    const double tol = c->cfg.tol;
    const long long cap = c->cfg.max_iter;
    HIPCHK(launch_gather(kw.sseg.p, (int)sseg.size(), sb, kw.x.p, nullptr, c->stream));

    std::vector<double> hc1((size_t)ns * cst), hc2((size_t)ns * cst), hy((size_t)ns * cst), hz((size_t)ns * cst);
    std::vector<int> hvw(ns, 0);
    HIPCHK(grow(kw.vw, (size_t)ns));
    bool trials = false;
    for (int q = 0; q < ns; ++q)
        trials = trials || (trial && (*trial)[slots[q].inst]);
    for (;;) {
        // ---- one full iteration from x: residual w = x - F(x) and eps
        for (int q = 0; q < ns; ++q)
            if (hs[q].live)
                st[slots[q].inst].maxdiff_bits = st[slots[q].inst].maxabs_bits = 0ull;
        if ((rc = upload_st()))
            return rc;
        HIPCHK(launch_scatter(kw.sseg.p, (int)sseg.size(), sb, kw.x.p, c->stream));
        if ((rc = sweep_once(false, true)))
            return rc;
        HIPCHK(launch_gather(kw.gseg.p, (int)gseg.size(), sb, kw.w.p, kw.x.p, c->stream));
        {
            // statistics of u1(F(x)) - u1(x): the monitor of this record
            for (int q = 0; q < ns; ++q)
                if (hs[q].live)
                    st[slots[q].inst].maxdiff_bits = st[slots[q].inst].maxabs_bits = 0ull;
            if ((rc = upload_st()))
                return rc;
            RecArgs<double> ra = rec_args(c, adj);
            HIPCHK(launch_record<double>(ra, c->max_cells, c->n_inst, c->stream));
        }
        // with deflated restarts also the residual's coordinates in the kept bases
        int nkept = 0;
        for (int q = 0; q < ns; ++q)
            if (hs[q].live && hs[q].kd > 0)
                nkept = std::max(nkept, hs[q].kd + 1);
        if ((rc = dots(kw.w.p, nkept, true, kw.c1.p)))
            return rc;
        std::vector<SolveState> dev(c->n_inst);
        HIPCHK(hipMemcpyAsync(dev.data(), dst, c->n_inst * sizeof(SolveState), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(hc1.data(), kw.c1.p, hc1.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        bool changed = false, any = false;
        for (int q = 0; q < ns; ++q) {
            GmresSlotHost &h = hs[q];
            if (!h.live)
                continue;
            SolveState &s = st[slots[q].inst];
            h.sweeps += 1;
            h.sweeps64 += 1;
            const double dmax = __builtin_bit_cast(double, (long long)dev[slots[q].inst].maxdiff_bits);
            const double amax = __builtin_bit_cast(double, (long long)dev[slots[q].inst].maxabs_bits);
            const double eps = amax > 0.0 ? dmax / amax : (dmax == 0.0 ? 0.0 : INFINITY);
            const double sig = h.sig < 0.0 ? -1.0 : std::min(1.0, std::max(h.sig, 1e-3));
            const double est = sig > 0.0 ? eps / sig : INFINITY;
            s.eps = eps;
            s.est = est;
            h.beta = std::sqrt(std::max(hc1[(size_t)q * cst + nkept], 0.0));
            int fin = 0;
            if (!(amax < 1e30) || eps != eps || !std::isfinite(h.beta))
                fin = STATUS_DIVERGED;
            else if (eps <= STOP_FLOOR64 || est <= tol || h.beta == 0.0)
                fin = STATUS_CONVERGED;
            else if (h.sweeps >= cap)
                fin = STATUS_MAXITER;
            if (!fin && mixed && reverted && h.beta_prev > 0.0 && h.beta > 0.9 * h.beta_prev) {
                // FP32 Krylov steps no longer reduce the FP64 residual (the
                // FP32 operator's rounding floor, or a stagnating restart):
                // the instance goes back to its caller from x, marked 2
                if (debug_on())
                    std::fprintf(stderr, "[dvm gmres] inst %d mixed cycles stagnate (residual %.3e after %.3e)\n",
                                 slots[q].inst, h.beta, h.beta_prev);
                s.iter += 1;              // the state holds F(x), as for a finished slot
                s.maxdiff_bits = s.maxabs_bits = 0ull;
                h.live = false;
                s.active = 0;
                (*reverted)[slots[q].inst] = 2;
                c->sweeps_done[slots[q].inst] = h.sweeps;
                c->gmres_s64[slots[q].inst] = h.sweeps64;
                changed = true;
                continue;
            }
            h.beta_prev = h.beta;
            if (fin) {
                if (debug_on())
                    std::fprintf(stderr, "[dvm gmres] inst %d done (%d) after %lld sweeps, eps %.3e est %.3e\n",
                                 slots[q].inst, fin, h.sweeps, eps, est);
                // the state now holds F(x): advance the parity like an iteration
                s.iter += 1;
                s.status = fin;
                s.active = 0;
                s.maxdiff_bits = s.maxabs_bits = 0ull;
                h.live = false;
                changed = true;
                c->sweeps_done[slots[q].inst] = h.sweeps;
                c->gmres_s64[slots[q].inst] = h.sweeps64;
            } else {
                any = true;
            }
        }
        if ((rc = upload_st()))
            return rc;
        if (!any)
            break;
        if (changed && (rc = rebuild()))
            return rc;
        // ---- GMRES cycle.  Every instance runs its own Arnoldi process: it
        // starts from its kept basis (deflated restart, kd > 0) or from w
        // (kd = 0) and stops at its own column; the global step j only
        // shares the sweeps, so a batch gives each instance the arithmetic
        // of its own solve.
        bool plain_any = false;
        for (int q = 0; q < ns; ++q) {
            GmresSlotHost &h = hs[q];
            if (!h.live)
                continue;
            if (h.kd > 0) {
                // a deflated start needs the residual inside the kept span
                // (it is, up to the FP32 basis and, in the mixed steps, the
                // FP32 operator); otherwise this instance restarts plainly
                double in = 0.0;
                for (int i = 0; i <= h.kd; ++i)
                    in += hc1[(size_t)q * cst + i] * hc1[(size_t)q * cst + i];
                const double lost = h.beta * h.beta - in;
                if (!(lost <= 1e-4 * h.beta * h.beta)) {
                    if (debug_on())
                        std::fprintf(stderr, "[dvm gmres] inst %d: %.2e of the residual outside the kept basis, "
                                     "plain restart\n", slots[q].inst, std::sqrt(std::max(lost, 0.0)) / h.beta);
                    h.kd = 0;
                }
            }
            plain_any = plain_any || h.kd == 0;
        }
        int jmin = m;
        for (int q = 0; q < ns; ++q) {
            GmresSlotHost &h = hs[q];
            std::fill(h.H.begin(), h.H.end(), 0.0);
            std::fill(h.Hr.begin(), h.Hr.end(), 0.0);
            std::fill(h.g.begin(), h.g.end(), 0.0);
            std::fill(h.c.begin(), h.c.end(), 0.0);
            h.done = false;
            h.kq = 0;
            if (!h.live)
                continue;
            jmin = std::min(jmin, h.kd);
            if (h.kd == 0) {
                h.g[0] = h.beta;
                h.c[0] = h.beta;
                continue;
            }
            // kept block Hn = Q0 R: R opens the rotated matrix, Q0^T acts on
            // rows 0..kd of every later column and on c
            const int kd = h.kd;
            std::vector<double> R;
            dvm_eig::qr_small(h.Hn, kd + 1, kd, h.Q0, R);
            for (int j = 0; j < kd; ++j)
                for (int i = 0; i <= kd; ++i) {
                    h.Hr[(size_t)j * (m + 1) + i] = h.Hn[i + (size_t)j * (kd + 1)];
                    h.H[(size_t)j * (m + 1) + i] = R[i + (size_t)j * (kd + 1)];
                }
            for (int i = 0; i <= kd; ++i)
                h.c[i] = hc1[(size_t)q * cst + i];
            for (int i = 0; i <= kd; ++i) {
                double a = 0.0;
                for (int r = 0; r <= kd; ++r)
                    a += h.Q0[r + (size_t)i * (kd + 1)] * h.c[r];
                h.g[i] = a;
            }
        }
        if (plain_any) {
            // V_0 = w / beta for the instances that start plainly (coefficient
            // row |w|^2 with no vectors); the others keep their V_0
            std::fill(hz.begin(), hz.end(), 0.0);
            for (int q = 0; q < ns; ++q) {
                hvw[q] = hs[q].live && hs[q].kd == 0 ? 1 : 0;
                if (hvw[q])
                    hz[(size_t)q * cst] = hs[q].beta * hs[q].beta;
            }
            HIPCHK(hipMemcpyAsync(kw.c2.p, hz.data(), hz.size() * sizeof(double), hipMemcpyHostToDevice,
                                  c->stream));
            HIPCHK(hipMemcpyAsync(kw.vw.p, hvw.data(), ns * sizeof(int), hipMemcpyHostToDevice, c->stream));
            HIPCHK(launch_vupdate4_masked(kw.ch.p, (int)chunks.size(), kw.w.p, kw.V.p, n, 0, kw.c2.p, cst, kw.V.p,
                                          kw.vw.p, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
        }
        for (int j = jmin; j < m; ++j) {
            // the instances that take this step: live, not yet stopped, and
            // past their kept vectors
            bool pending = false, step = false;
            for (int q = 0; q < ns; ++q) {
                const GmresSlotHost &h = hs[q];
                pending = pending || (h.live && !h.done);
                hvw[q] = h.live && !h.done && j >= h.kd ? 1 : 0;
                step = step || hvw[q];
            }
            if (!pending)
                break;
            if (!step)
                continue;
            HIPCHK(hipMemcpyAsync(kw.vw.p, hvw.data(), ns * sizeof(int), hipMemcpyHostToDevice, c->stream));
            float *Vj = kw.V.p + (size_t)j * n;
            if ((rc = krylov_step(Vj)))
                return rc;
            // classical Gram-Schmidt; the second pass only where the first
            // one cancelled more than half of |w|^2
            if ((rc = dots(kw.w.p, j + 1, true, kw.c1.p)))
                return rc;
            HIPCHK(launch_vupdate4(kw.ch.p, (int)chunks.size(), kw.w.p, kw.V.p, n, j + 1, kw.c1.p, cst, nullptr,
                                  c->stream));
            if ((rc = dots(kw.w.p, j + 1, true, kw.c2.p, kw.c1.p)))
                return rc;
            HIPCHK(launch_vupdate4_masked(kw.ch.p, (int)chunks.size(), kw.w.p, kw.V.p, n, j + 1, kw.c2.p, cst,
                                          kw.V.p + (size_t)(j + 1) * n, kw.vw.p, c->stream));
            HIPCHK(hipMemcpyAsync(hc1.data(), kw.c1.p, hc1.size() * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream));
            HIPCHK(hipMemcpyAsync(hc2.data(), kw.c2.p, hc2.size() * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            for (int q = 0; q < ns; ++q) {
                GmresSlotHost &h = hs[q];
                if (!hvw[q])
                    continue;
                h.sweeps += 1;
                double *col = &h.H[(size_t)j * (m + 1)];
                double n2 = hc2[(size_t)q * cst + j + 1];
                for (int i = 0; i <= j; ++i) {
                    col[i] = hc1[(size_t)q * cst + i] + hc2[(size_t)q * cst + i];
                    n2 -= hc2[(size_t)q * cst + i] * hc2[(size_t)q * cst + i];
                }
                col[j + 1] = std::sqrt(std::max(n2, 0.0));
                std::copy(col, col + j + 2, &h.Hr[(size_t)j * (m + 1)]);
                const int kd = h.kd;
                if (kd > 0) {
                    double t[VCOMB_OUT];
                    for (int i = 0; i <= kd; ++i) {
                        double a = 0.0;
                        for (int r = 0; r <= kd; ++r)
                            a += h.Q0[r + (size_t)i * (kd + 1)] * col[r];
                        t[i] = a;
                    }
                    std::copy(t, t + kd + 1, col);
                }
                for (int i = kd; i < j; ++i) {
                    const double a = h.cs[i] * col[i] + h.sn[i] * col[i + 1];
                    col[i + 1] = -h.sn[i] * col[i] + h.cs[i] * col[i + 1];
                    col[i] = a;
                }
                const double r = std::hypot(col[j], col[j + 1]);
                h.cs[j] = r > 0.0 ? col[j] / r : 1.0;
                h.sn[j] = r > 0.0 ? col[j + 1] / r : 0.0;
                col[j] = r;
                col[j + 1] = 0.0;
                h.g[j + 1] = -h.sn[j] * h.g[j];
                h.g[j] = h.cs[j] * h.g[j];
                h.kq = j + 1;
                const double res = std::fabs(h.g[j + 1]);
                if (res <= 1e-3 * h.beta || h.sweeps >= cap)
                    h.done = true;
            }
        }
        // x -= V y per slot, y from the triangular system of its cycle
        std::fill(hy.begin(), hy.end(), 0.0);
        int kmax = 0;
        for (int q = 0; q < ns; ++q) {
            GmresSlotHost &h = hs[q];
            if (!h.live)
                continue;
            const int kq = h.kq;
            kmax = std::max(kmax, kq);
            std::vector<double> y(kq, 0.0);
            for (int i = kq - 1; i >= 0; --i) {
                double a = h.g[i];
                for (int jj = i + 1; jj < kq; ++jj)
                    a -= h.H[(size_t)jj * (m + 1) + i] * y[jj];
                const double dg = h.H[(size_t)i * (m + 1) + i];
                y[i] = dg != 0.0 ? a / dg : 0.0;
            }
            for (int i = 0; i < kq; ++i)
                hy[(size_t)q * cst + i] = y[i];
            h.sig = sigma_min_tri(h.H, m + 1, kq);
        }
        HIPCHK(hipMemcpyAsync(kw.y.p, hy.data(), hy.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIPCHK(launch_vupdate4(kw.ch.p, (int)chunks.size(), kw.x.p, kw.V.p, n, kmax, kw.y.p, cst, nullptr,
                              c->stream));
        if (trials && kmax > 0) {
            // a trial instance stays with GMRES while its cycles together
            // have reduced its residual at least 1.5 times faster per unit of
            // work than the plain iteration, both counted in sweeps of the
            // instance (a single stagnating cycle after a good one does not
            // end the trial; the rule is deterministic, so the path a solve
            // takes does not depend on
            // machine load or on the other instances of the batch)
            HIPCHK(hipStreamSynchronize(c->stream));
            bool back = false, left = false;
            for (int q = 0; q < ns; ++q) {
                GmresSlotHost &h = hs[q];
                const int inst = slots[q].inst;
                if (!h.live)
                    continue;
                if ((*trial)[inst] && h.beta > 0.0 && h.kq > 0) {
                    const double red = std::max(std::fabs(h.g[h.kq]) / h.beta, 1e-300);
                    const double cost = gmres_cycle_cost(h.kq, slots[q].len, c->inst[inst].nfluid * (double)c->K,
                                                         mixed ? 5.0 : 8.0) - h.kd;
                    h.trial_red += -std::log(red);
                    h.trial_cost += cost;
                    const double rate_g = h.trial_red / h.trial_cost;
                    const double rate_p = -std::log(c->trial_q[inst]);
                    if (debug_on())
                        std::fprintf(stderr, "[dvm trial] inst %d cycle of %d: residual x %.3e over %.1f "
                                     "sweep-equivalents (trial so far %.3g per sweep) vs plain q %.5f (%.3g per "
                                     "sweep)\n", inst, h.kq, red, cost, rate_g, c->trial_q[inst], rate_p);
                    if (rate_g < 1.5 * rate_p) {
                        h.live = false;
                        st[inst].active = 0;
                        (*reverted)[inst] = 1;
                        c->sweeps_done[inst] = h.sweeps;
                        c->gmres_s64[inst] = h.sweeps64;
                        back = true;
                        continue;
                    }
                }
                left = true;
            }
            if (back) {
                // the cycle's result goes back to the state the plain
                // iteration reads (harmless for the others: every cycle
                // starts by scattering x)
                HIPCHK(launch_scatter(kw.sseg.p, (int)sseg.size(), sb, kw.x.p, c->stream));
                if ((rc = upload_st()))
                    return rc;
                if (!left)
                    break;
                if ((rc = rebuild()))
                    return rc;
            }
        }
        // ---- deflated restart: each instance's next cycle starts from the
        // harmonic Ritz vectors of its smallest harmonic Ritz values and its
        // cycle's residual (csrc/dvm_eig.h)
        int dmax = 0, kin = 0;
        for (int q = 0; q < ns; ++q) {
            GmresSlotHost &h = hs[q];
            const int kd_prev = h.kd;
            h.kd = 0;
            if (!h.live || want <= 0 || h.kq < want + 2)
                continue;
            const int kq = h.kq;
            std::vector<double> rho(h.c.begin(), h.c.begin() + kq + 1);
            for (int j = 0; j < kq; ++j) {
                const double yj = hy[(size_t)q * cst + j];
                for (int i = 0; i <= kq; ++i)
                    rho[i] -= h.Hr[(size_t)j * (m + 1) + i] * yj;
            }
            h.kd = std::max(dvm_eig::deflate(h.Hr, m + 1, kq, rho, want, h.P, h.Hn), 0);
            if (h.kd > 0) {
                dmax = std::max(dmax, h.kd);
                kin = std::max(kin, kq + 1);
            }
            if (debug_on())
                std::fprintf(stderr, "[dvm gmres] inst %d: cycle of %d columns (%d kept): next cycle keeps %d\n",
                             slots[q].inst, kq, kd_prev, h.kd);
        }
        if (dmax > 0) {
            // V_0..V_dmax <- V P per slot (zero columns past a slot's own
            // count: its Arnoldi steps rewrite them)
            std::fill(hpc.begin(), hpc.end(), 0.0);
            for (int q = 0; q < ns; ++q) {
                const GmresSlotHost &h = hs[q];
                if (!h.live || h.kd == 0)
                    continue;
                double *pq = hpc.data() + (size_t)q * pstr;
                for (int j = 0; j <= h.kq; ++j)
                    for (int o = 0; o <= h.kd; ++o)
                        pq[j * (dmax + 1) + o] = h.P[j + (size_t)o * (h.kq + 1)];
            }
            HIPCHK(hipMemcpyAsync(kw.pc.p, hpc.data(), hpc.size() * sizeof(double), hipMemcpyHostToDevice,
                                  c->stream));
            HIPCHK(launch_vcombine(kw.ch.p, (int)chunks.size(), kw.V.p, n, kin, dmax + 1, kw.pc.p, pstr, kw.T.p,
                                   c->stream));
            HIPCHK(hipMemcpyAsync(kw.V.p, kw.T.p, (size_t)(dmax + 1) * n * sizeof(float), hipMemcpyDeviceToDevice,
                                  c->stream));
            // hpc is rewritten only after the next cycle's synchronisations
        }
    }
    if (mixed) {
        // the FP32 correction state is idle again
        for (auto &s32 : st32)
            s32.active = 0;
        HIPCHK(hipMemcpyAsync(c->d_st32.p, st32.data(), c->n_inst * sizeof(SolveState), hipMemcpyHostToDevice,
                              c->stream));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return DVM_OK;
}

// ---------------------------------------------------------- refinement
// DVM_FP32_REFINE: outer defect correction in FP64 around FP32 sweeps.
//   r = x - F64(x)   (one FP64 iteration from the FP64 state x; eps64 is its
//                     relative change of u1)
//   solve (I - L) e = r with the FP32 source iteration e <- L32 e + r
//                    (FP32 records, seams, wrap and wall values; moments
//                     accumulated in FP64), to relative change 1e-4
//   x <- x - e
// An instance is accepted when eps64 * q / (1 - q) <= tol, q the contraction
// observed in the last FP32 solve (the a-posteriori bound of the stop rule);
// the accepted state is F64(x).  An instance whose FP32 iteration stalls or
// diverges continues with the FP64 iteration.

static int ensure_fp32(dvm_ctx *c)
{
    if (c->fp32_ready)
        return DVM_OK;
    // (re)allocation below: nothing queued may still use the old buffers
    HIPCHK(hipStreamSynchronize(c->stream));
    const long long sk = c->sk_total, fh = std::max<long long>(c->nfaces, 1) * c->kp4;
    HIPCHK(c->d_srec32.alloc(sk * REC_STRIDE));
    HIPCHK(c->d_seam32.alloc(2 * c->seam_half));
    HIPCHK(c->d_wrap32.alloc(c->wrap_total));
    HIPCHK(c->d_fb32.alloc(2 * fh));
    HIPCHK(c->d_vt32.alloc((size_t)c->n_inst * c->kp4 * VT_STRIDE));
    HIPCHK(c->d_mom_d.alloc(c->ncell * MOM_STRIDE));
    HIPCHK(c->d_u1prev_d.alloc(c->ncell));
    HIPCHK(c->d_st32.alloc(c->n_inst));
    HIPCHK(c->d_rb_mom.alloc(c->ncell * MOM_STRIDE));
    HIPCHK(c->d_rb_wrap.alloc(c->wrap_total));
    // values outside every instance's state stay 0
    HIPCHK(launch_zero(c->d_rb_mom.p, c->d_rb_mom.n, c->stream));
    HIPCHK(launch_zero(c->d_rb_wrap.p, c->d_rb_wrap.n, c->stream));
    HIPCHK(launch_zero_f(c->d_srec32.p, c->d_srec32.n, c->stream));
    HIPCHK(launch_zero_f(c->d_seam32.p, c->d_seam32.n, c->stream));
    HIPCHK(launch_zero_f(c->d_wrap32.p, c->d_wrap32.n, c->stream));
    HIPCHK(launch_zero_f(c->d_fb32.p, c->d_fb32.n, c->stream));
    HIPCHK(launch_zero(c->d_mom_d.p, c->d_mom_d.n, c->stream));
    HIPCHK(launch_zero(c->d_u1prev_d.p, c->d_u1prev_d.n, c->stream));
    std::vector<double> vt(c->d_vt.n);
    HIPCHK(hipMemcpyAsync(vt.data(), c->d_vt.p, vt.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::vector<float> vt32(vt.begin(), vt.end());
    std::vector<SolveState> st(c->n_inst);
    HIPCHK(hipMemcpyAsync(c->d_vt32.p, vt32.data(), vt32.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->d_st32.p, st.data(), st.size() * sizeof(SolveState), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->fp32_ready = true;
    return DVM_OK;
}


// The refinement of the active instances of [i0, i1).  Under AUTO an
// instance whose FP32 correction iteration is slow goes on in GMRES with
// FP32 Krylov steps, on trial; one that does not contract is taken over by
// it.  What GMRES hands back (slower than the plain rate, or FP32 steps that
// stagnate) continues in FP64 under AUTO, which has its own trials and
// takeover: the FP32 correction iteration of such an instance has already
// shown its rate.
static int dc_run(dvm_ctx *c, int i0, int i1, std::vector<SolveState> &st, std::vector<char> *need_skew)
{
    int rc = ensure_fp32(c);
    if (rc)
        return rc;
    const int mode = solve_mode(c);
    const double tol = c->cfg.tol;
    const long long cap = c->cfg.max_iter;
    StateBufs sb;
    sb.b[0] = c->d_mom.p;
    sb.b[1] = c->d_seam.p;
    sb.b[2] = c->d_wrap.p;
    sb.b[3] = c->d_fb.p;

    struct DSlot {
        int inst;
        long long off, len;
        int pw;
        bool live;
        double q;
        long long s32, s64;
        bool fallback;
        bool drop_e = false;   // this step's correction did not converge: not applied
        bool slow = false;     // fell back for being slow (GMRES on trial)
    };
    std::vector<DSlot> slots;
    long long n = 0;
    for (int i = i0; i < i1; ++i) {
        if (!st[i].active)
            continue;
        DSlot d{i, n, 0, (int)(st[i].iter & 1), true, -1.0, 0, 0, false};
        d.len = state_segments(c, i, d.pw, n, nullptr, nullptr);
        n += d.len;
        slots.push_back(d);
    }
    if (slots.empty())
        return DVM_OK;
    HIPCHK(c->d_xr.alloc(n));
    HIPCHK(c->d_rr.alloc(n));
    HIPCHK(c->d_rr32.alloc(n));
    HIPCHK(c->d_er.alloc(n));
    KrylovWork &kw = c->kw;
    std::vector<VSeg> gseg, sseg;
    auto rebuild = [&]() -> int {
        gseg.clear();
        sseg.clear();
        std::vector<VSeg2> s2;
        c->dc_off.assign(c->n_inst, -1);
        c->dc_len.assign(c->n_inst, 0);
        c->dc_n = n;
        for (const auto &d : slots) {
            if (!d.live)
                continue;
            c->dc_off[d.inst] = d.off;
            c->dc_len[d.inst] = d.len;
            state_segments(c, d.inst, d.pw, d.off, &gseg, &sseg);
            std::vector<VSeg> g0, g1;
            state_segments(c, d.inst, 0, d.off, &g0, nullptr);
            state_segments(c, d.inst, 1, d.off, &g1, nullptr);
            for (size_t k = 0; k < g0.size(); ++k)
                s2.push_back(VSeg2{{g0[k].buf_off, g1[k].buf_off}, g0[k].vec_off, g0[k].len, g0[k].buf, d.inst});
        }
        HIPCHK(kw.gseg.alloc(std::max<size_t>(gseg.size(), 1)));
        HIPCHK(kw.sseg.alloc(std::max<size_t>(sseg.size(), 1)));
        std::vector<VSeg2> s2s;                // the seam segments alone
        for (const VSeg2 &g : s2)
            if (g.buf == 1)
                s2s.push_back(g);
        HIPCHK(c->d_seg32.alloc(std::max<size_t>(s2.size(), 1)));
        HIPCHK(c->d_seg32s.alloc(std::max<size_t>(s2s.size(), 1)));
        HIPCHK(hipMemcpyAsync(kw.gseg.p, gseg.data(), gseg.size() * sizeof(VSeg), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(kw.sseg.p, sseg.data(), sseg.size() * sizeof(VSeg), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(c->d_seg32.p, s2.data(), s2.size() * sizeof(VSeg2), hipMemcpyHostToDevice, c->stream));
        if (!s2s.empty())
            HIPCHK(hipMemcpyAsync(c->d_seg32s.p, s2s.data(), s2s.size() * sizeof(VSeg2), hipMemcpyHostToDevice,
                                  c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        c->nseg32 = (int)s2.size();
        c->nseg32s = (int)s2s.size();
        if (c->graph[2]) {                 // the captured block holds the old table
            (void)hipGraphExecDestroy(c->graph[2]);
            c->graph[2] = nullptr;
        }
        return DVM_OK;
    };
    if ((rc = rebuild()))
        return rc;
    auto upload = [&](SolveState *dst, std::vector<SolveState> &v) -> int {
        HIPCHK(hipMemcpyAsync(dst, v.data(), c->n_inst * sizeof(SolveState), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        return DVM_OK;
    };
    std::vector<SolveState> st32(c->n_inst);
    HIPCHK(hipMemcpyAsync(st32.data(), c->d_st32.p, c->n_inst * sizeof(SolveState), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(launch_gather(kw.sseg.p, (int)sseg.size(), sb, c->d_xr.p, nullptr, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));

    for (;;) {
        // ---- FP64 residual r = x - F64(x) and eps64
        for (auto &d : slots)
            if (d.live)
                st[d.inst].maxdiff_bits = st[d.inst].maxabs_bits = 0ull;
        if ((rc = upload(c->d_st.p, st)))
            return rc;
        HIPCHK(launch_scatter(kw.sseg.p, (int)sseg.size(), sb, c->d_xr.p, c->stream));
        HIPCHK(launch_record<double>(rec_args(c), c->max_cells, c->n_inst, c->stream));
        hipEvent_t pe0 = nullptr, pe1 = nullptr;
        double pupd = 0.0;
        if (c->cfg.profile) {
            if ((rc = next_event(c, &pe0)) || (rc = next_event(c, &pe1)))
                return rc;
            HIPCHK(hipEventRecord(pe0, c->stream));
            for (const auto &d : slots)
                if (d.live)
                    pupd += (double)c->inst[d.inst].nfluid * c->K;
        }
        HIPCHK(launch_sweep<double>(sweep_args(c, 0, false), (int)c->items.size(), c->V, c->G,
                                    mode | xu_flag(c, c->V), c->stream));
        if (c->cfg.profile) {
            HIPCHK(hipEventRecord(pe1, c->stream));
            c->ev_prec = 0;
            c->ev_sweep.emplace_back(pe0, pe1);
            HIPCHK(hipStreamSynchronize(c->stream));
            if ((rc = collect_profile(c, 1, pupd)))
                return rc;
        }
        HIPCHK(launch_moments(mom_args(c), c->max_cells, c->n_inst, c->stream));
        HIPCHK(launch_gather(kw.gseg.p, (int)gseg.size(), sb, c->d_rr.p, c->d_xr.p, c->stream));
        if ((rc = upload(c->d_st.p, st)))
            return rc;
        HIPCHK(launch_record<double>(rec_args(c), c->max_cells, c->n_inst, c->stream));
        std::vector<SolveState> dev(c->n_inst);
        HIPCHK(hipMemcpyAsync(dev.data(), c->d_st.p, c->n_inst * sizeof(SolveState), hipMemcpyDeviceToHost,
                              c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        bool changed = false, any = false;
        for (auto &d : slots) {
            if (!d.live)
                continue;
            SolveState &s = st[d.inst];
            d.s64 += 1;
            const double dmax = __builtin_bit_cast(double, (long long)dev[d.inst].maxdiff_bits);
            const double amax = __builtin_bit_cast(double, (long long)dev[d.inst].maxabs_bits);
            const double eps = amax > 0.0 ? dmax / amax : (dmax == 0.0 ? 0.0 : INFINITY);
            const double est = d.q >= 0.0 ? eps * d.q / (1.0 - d.q) : INFINITY;
            s.eps = eps;
            s.est = est;
            if (debug_on())
                std::fprintf(stderr, "[dvm refine] inst %d fp64 step %lld: eps64 %.3e amax %.3e q %.4f est %.3e\n",
                             d.inst, d.s64, eps, amax, d.q, est);
            int fin = 0;
            if (!(amax < 1e30) || eps != eps)
                fin = STATUS_DIVERGED;
            else if (eps <= STOP_FLOOR64 || est <= tol)
                fin = STATUS_CONVERGED;
            else if (d.s32 + d.s64 >= cap)
                fin = STATUS_MAXITER;
            if (fin) {
                s.iter += 1;              // the state holds F64(x)
                s.status = fin;
                s.active = 0;
                s.maxdiff_bits = s.maxabs_bits = 0ull;
                d.live = false;
                changed = true;
            } else {
                any = true;
            }
        }
        if ((rc = upload(c->d_st.p, st)))
            return rc;
        if (!any)
            break;
        if (changed && (rc = rebuild()))
            return rc;
        if (debug_on() && std::getenv("DVM_DEBUG_CMP")) {
            // one homogeneous map of the residual vector in both precisions
            std::vector<double> a64(n), a32(n);
            HIPCHK(launch_scatter(kw.sseg.p, (int)sseg.size(), sb, c->d_rr.p, c->stream));
            RecArgs<double> ra = rec_args(c);
            ra.homog = 1;
            ra.monitor = 0;
            HIPCHK(launch_record<double>(ra, c->max_cells, c->n_inst, c->stream));
            HIPCHK(launch_sweep<double>(sweep_args(c, 0, false), (int)c->items.size(), c->V, c->G, mode, c->stream));
            HIPCHK(launch_moments(mom_args(c), c->max_cells, c->n_inst, c->stream));
            HIPCHK(launch_gather(kw.gseg.p, (int)gseg.size(), sb, c->d_er.p, nullptr, c->stream));
            HIPCHK(hipMemcpyAsync(a64.data(), c->d_er.p, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            for (auto &d : slots)
                st32[d.inst].active = d.live ? 1 : 0;
            if ((rc = upload(c->d_st32.p, st32)))
                return rc;
            HIPCHK(launch_state32(c->d_seg32.p, c->nseg32, c->d_st32.p, state32(c), c->d_rr.p, 1, c->stream));
            RecArgs<float> r32 = rec_args32(c);
            r32.monitor = 0;
            HIPCHK(launch_record<float>(r32, c->max_cells, c->n_inst, c->stream));
            HIPCHK(launch_sweep<float>(sweep_args32(c), (int)c->items.size(), c->V32, c->G32, mode, c->stream));
            HIPCHK(launch_moments(mom_args32(c), c->max_cells, c->n_inst, c->stream));
            HIPCHK(launch_state32(c->d_seg32.p, c->nseg32, c->d_st32.p, state32(c), c->d_er.p, 3, c->stream));
            HIPCHK(hipMemcpyAsync(a32.data(), c->d_er.p, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            double dmax = 0, amax64 = 0, amax32 = 0;
            long long imax = 0;
            for (long long k = 0; k < n; ++k) {
                if (std::fabs(a64[k] - a32[k]) > dmax) {
                    dmax = std::fabs(a64[k] - a32[k]);
                    imax = k;
                }
                amax64 = std::max(amax64, std::fabs(a64[k]));
                amax32 = std::max(amax32, std::fabs(a32[k]));
            }
            std::fprintf(stderr, "[dvm refine] L64 r vs L32 r: max|diff| %.3e at %lld (%.6e vs %.6e), max %.3e / %.3e\n",
                         dmax, imax, a64[imax], a32[imax], amax64, amax32);
            for (long long k = 0; k < std::min<long long>(n, 16); ++k)
                std::fprintf(stderr, "   %lld: %.6e %.6e\n", k, a64[k], a32[k]);
        }
        // ---- FP32 correction: (I - L) e = r
        std::vector<long long> iter0(c->n_inst, 0);
        for (int i = 0; i < c->n_inst; ++i) {
            SolveState &s = st32[i];
            s.active = 0;
            iter0[i] = s.iter;
        }
        for (auto &d : slots) {
            if (!d.live)
                continue;
            SolveState &s = st32[d.inst];
            s.active = 1;
            s.status = STATUS_RUNNING;
            s.npass = 0;
            s.qfloor = 0.0;
            s.eps_prev = 0.0;
            s.iter0 = s.iter;
            s.maxdiff_bits = s.maxabs_bits = 0ull;
            // relative accuracy this correction needs: the error estimate of
            // x must drop below tol (with a margin), within what FP32
            // resolves.  Before any contraction has been measured the error
            // is taken as eps64 q/(1 - q) with q = 0.99 and the correction is
            // solved to 1e-4 at most (a later FP64 step with the measured
            // rate asks for another correction if either was optimistic)
            double est = st[d.inst].est;
            const bool first = !std::isfinite(est);
            if (first)
                est = st[d.inst].eps * 99.0;
            const double need = est > 0.0 ? 0.3 * tol / est : 1e-4;
            s.tol = std::min(0.1, std::max(need, first ? 1e-4 : 1e-5));
        }
        if ((rc = upload(c->d_st32.p, st32)))
            return rc;
        HIPCHK(launch_state32(c->d_seg32.p, c->nseg32, c->d_st32.p, state32(c), c->d_rr.p, 1, c->stream));
        HIPCHK(launch_rscatter(c->d_seg32.p, c->nseg32, c->d_rr.p, c->d_rb_mom.p, c->d_rb_wrap.p, c->d_rr32.p,
                               c->stream));
        HIPCHK(launch_record<float>(rec_args32(c), c->max_cells, c->n_inst, c->stream));
        for (auto &d : slots)
            if (d.live)
                st32[d.inst].maxdiff_bits = st32[d.inst].maxabs_bits = 0ull;
        if ((rc = upload(c->d_st32.p, st32)))
            return rc;
        std::vector<char> stalled(c->n_inst, 0);
        if ((rc = run_blocks(c, i0, i1, iter0, 2, st32, &stalled)))
            return rc;
        bool fb = false;
        for (auto &d : slots) {
            if (!d.live)
                continue;
            const SolveState &s = st32[d.inst];
            d.s32 += s.iter - iter0[d.inst];
            if (debug_on())
                std::fprintf(stderr, "[dvm refine] inst %d fp32 solve: %lld iterations status %d eps %.3e "
                             "eps_prev %.3e stalled %d\n", d.inst, s.iter - iter0[d.inst], s.status, s.eps,
                             s.eps_prev, (int)stalled[d.inst]);
            // contraction of the last FP32 iterations: the stop rule's bound
            // est = eps q / (1 - q) (the status kernel has already replaced
            // eps_prev by eps).  Every correction iterates the same operator,
            // so the slowest rate seen so far is kept: a short, loosely
            // solved correction can end before its ratio shows the slowest
            // mode.
            double qn = 0.9999;
            if (s.status == STATUS_CONVERGED && s.eps > 0.0 && std::isfinite(s.est) && s.est > 0.0)
                qn = std::min(s.est / (s.eps + s.est), 0.9999);
            d.q = std::max(d.q, qn);
            // a slow correction iteration (under AUTO: rate settled above
            // 0.98 with over 1000 iterations predicted, or q > 0.995 seen at
            // convergence) goes on in GMRES with FP32 Krylov steps, on trial
            // as in the FP64 iteration; one that does not contract at all
            // (stalled) or diverges is taken over by it
            // (stalled = 3: stopped early for being slow; its partial
            // correction is applied like a converged one)
            const bool slow = c->cfg.accel == DVM_ACCEL_AUTO &&
                              ((s.status == STATUS_CONVERGED && qn > 0.995) || stalled[d.inst] == 3);
            if (stalled[d.inst] || s.status == STATUS_DIVERGED || slow) {
                d.fallback = true;
                d.live = false;
                d.drop_e = !slow;
                d.slow = slow;
                if (slow && stalled[d.inst] != 3)      // (stalled = 3 left its measured rate)
                    c->trial_q[d.inst] = std::min(d.q, 0.9999);
                fb = true;
            }
        }
        // ---- x <- x - e
        HIPCHK(launch_state32(c->d_seg32.p, c->nseg32, c->d_st32.p, state32(c), c->d_er.p, 2, c->stream));
        for (auto &d : slots)
            if (d.drop_e) {
                HIPCHK(launch_zero(c->d_er.p + d.off, (size_t)d.len, c->stream));
                d.drop_e = false;
            }
        HIPCHK(launch_axpy(c->d_xr.p, c->d_er.p, -1.0, n, c->stream));
        if (fb) {
            // back to the FP64 state x for the instances that leave
            HIPCHK(launch_scatter(kw.sseg.p, (int)sseg.size(), sb, c->d_xr.p, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            if ((rc = rebuild()))
                return rc;
        }
    }
    for (const auto &d : slots) {
        c->sweeps_done[d.inst] = d.s32 + d.s64;
        c->sweeps64_done[d.inst] = d.s64;
    }
    // instances whose FP32 iteration did not contract: FP64 from x
    bool any_fb = false;
    std::vector<long long> iter0(c->n_inst, 0);
    for (int i = 0; i < c->n_inst; ++i)
        iter0[i] = st[i].iter;
    for (const auto &d : slots)
        if (d.fallback) {
            SolveState &s = st[d.inst];
            s.active = 1;
            s.status = STATUS_RUNNING;
            s.npass = 0;
            s.eps_prev = 0.0;
            any_fb = true;
        }
    if (!any_fb)
        return DVM_OK;
    HIPCHK(launch_record<double>(rec_args(c), c->max_cells, c->n_inst, c->stream));
    for (const auto &d : slots)
        if (d.fallback)
            st[d.inst].maxdiff_bits = st[d.inst].maxabs_bits = 0ull;
    if ((rc = upload(c->d_st.p, st)))
        return rc;
    std::vector<long long> before(c->n_inst);
    for (const auto &d : slots)
        before[d.inst] = c->sweeps_done[d.inst];
    if (c->cfg.accel == DVM_ACCEL_AUTO) {
        // GMRES from x with FP32 Krylov steps: each cycle starts from the
        // FP64 residual of one full FP64 iteration, so the FP32 steps limit
        // only what one cycle gains (the same defect correction, in Krylov
        // form).  Slow instances are on trial; what GMRES hands back goes on
        // with the FP64 iteration below.
        std::vector<char> trial(c->n_inst, 0), reverted(c->n_inst, 0);
        std::vector<long long> prior(c->n_inst, 0);
        for (const auto &d : slots)
            if (d.fallback) {
                trial[d.inst] = d.slow ? 1 : 0;
                prior[d.inst] = before[d.inst];
                c->gmres_s64[d.inst] = 0;
            }
        if ((rc = gmres_run(c, i0, i1, false, st, prior, &trial, &reverted, true)))
            return rc;
        bool any_rev = false;
        for (auto &d : slots) {
            if (!d.fallback)
                continue;
            c->sweeps64_done[d.inst] += c->gmres_s64[d.inst];
            before[d.inst] = c->sweeps_done[d.inst];
            if (reverted[d.inst]) {
                SolveState &s = st[d.inst];
                s.active = 1;
                s.status = STATUS_RUNNING;
                s.npass = 0;
                s.eps_prev = 0.0;
                s.qfloor = std::max(s.qfloor, c->trial_q[d.inst]);
                any_rev = true;
            } else {
                d.fallback = false;     // finished in GMRES: counts are final
            }
        }
        if (!any_rev) {
            for (const auto &d : slots)
                c->sweeps_done[d.inst] = before[d.inst];
            return DVM_OK;
        }
        for (int i = 0; i < c->n_inst; ++i)
            iter0[i] = st[i].iter;
        HIPCHK(launch_record<double>(rec_args(c), c->max_cells, c->n_inst, c->stream));
        for (const auto &d : slots)
            if (d.fallback)
                st[d.inst].maxdiff_bits = st[d.inst].maxabs_bits = 0ull;
        if ((rc = upload(c->d_st.p, st)))
            return rc;
    }
    rc = iterate(c, i0, i1, iter0, false, st, need_skew);
    // iterate() recounts every instance of [i0, i1): the ones that did not
    // fall back keep their refinement counts
    for (const auto &d : slots)
        if (d.fallback) {
            c->sweeps64_done[d.inst] += c->sweeps_done[d.inst];
            c->sweeps_done[d.inst] += before[d.inst];
        } else {
            c->sweeps_done[d.inst] = before[d.inst];
        }
    return rc;
}

// ------------------------------------------------------------ autotuner
// The sweep shape (V velocities per lane, G waves per workgroup) is chosen
// by timing a few sweeps of the actual geometries: the FP64 shape, and for
// DVM_FP32_REFINE the FP32 shape among those with the same V * G (the
// layout of partials and seams depends only on V * G).  Results are kept per
// process and, with cfg.tune_cache, in a text file (one line per problem:
// key, then V G V32 G32), so the choice is stable across contexts.

struct TuneResult {
    int V, G, V32, G32;
};

static std::mutex g_tune_mu;
static std::map<std::string, TuneResult> g_tune;

static std::string tune_key(const dvm_ctx *c)
{
    std::string k = "nv" + std::to_string(c->nv) + " p" + std::to_string(c->cfg.precision) + " s" +
                    std::to_string(c->cfg.schedule);
    for (const auto &h : c->inst)
        k += " " + std::to_string(h.nx) + "x" + std::to_string(h.ny) + (h.periodic_y ? "p" : "w") +
             (h.force_skew ? "s" : "");
    return k;
}

static bool tune_file_read(const std::string &path, const std::string &key, TuneResult &r)
{
    if (path.empty())
        return false;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t bar = line.rfind('|');
        if (bar == std::string::npos || line.substr(0, bar) != key)
            continue;
        TuneResult t{};
        if (std::sscanf(line.c_str() + bar + 1, "%d %d %d %d", &t.V, &t.G, &t.V32, &t.G32) == 4) {
            r = t;
            return true;
        }
    }
    return false;
}

// file first (a cache written by another process wins), then this process
static bool tune_lookup(dvm_ctx *c, const std::string &key, TuneResult &r)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (tune_file_read(c->tune_path, key, r)) {
        g_tune[key] = r;
        return true;
    }
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
        r = it->second;
        return true;
    }
    return false;
}

// remember the choice in this process and in the cache file (once per key)
static void tune_store(dvm_ctx *c, const std::string &key, const TuneResult &r)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = r;
    TuneResult old{};
    if (!c->tune_path.empty() && !tune_file_read(c->tune_path, key, old)) {
        std::ofstream f(c->tune_path, std::ios::app);
        f << key << "|" << r.V << " " << r.G << " " << r.V32 << " " << r.G32 << "\n";
    }
}

static int upload_inst(dvm_ctx *c)
{
    HIPCHK(hipMemcpyAsync(c->d_inst.p, c->idev.data(), c->n_inst * sizeof(InstDev), hipMemcpyHostToDevice,
                          c->stream));
    return DVM_OK;
}

// average milliseconds of one sweep launch of every instance in shape (V, G)
template <typename T>
static int time_sweep(dvm_ctx *c, int V, int G, double *ms)
{
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    hipError_t err = hipSuccess;
    for (int rep = 0; rep < 4 && err == hipSuccess; ++rep) {
        if (rep == 1)
            err = hipEventRecord(e0, c->stream);
        if (err == hipSuccess) {
            // sweep + group sum: the velocity-group size sets both costs
            if constexpr (sizeof(T) == 8)
                err = launch_sweep<double>(sweep_args(c, 1, false), (int)c->items.size(), V, G, xu_flag(c, V),
                                           c->stream);
            else {
                SweepArgs<float> a = sweep_args32(c);
                a.force = 1;
                err = launch_sweep<float>(a, (int)c->items.size(), V, G, xu_flag(c, V), c->stream);
            }
            if (err == hipSuccess) {
                MomArgs m = mom_args(c, false, 1);
                if constexpr (sizeof(T) == 4)
                    m.part32 = reinterpret_cast<const float *>(c->d_part.p);
                err = launch_moments(m, c->max_cells, c->n_inst, c->stream);
            }
        }
    }
    if (err == hipSuccess)
        err = hipEventRecord(e1, c->stream);
    if (err == hipSuccess)
        err = hipEventSynchronize(e1);
    float t = 0.f;
    if (err == hipSuccess)
        err = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(err);
    *ms = t / 3.0;
    return DVM_OK;
}

static int autotune(dvm_ctx *c)
{
    c->tuned = true;
    const std::string key = tune_key(c);
    TuneResult best{c->V, c->G, c->V32, c->G32};
    if (!tune_lookup(c, key, best)) {
        static const int shapes[4][2] = {{4, 8}, {8, 4}, {4, 4}, {2, 8}};
        const bool r32 = c->cfg.precision == DVM_FP32_REFINE;
        double best_t = INFINITY;
        for (int P : {32, 16}) {
            int v0 = 0, g0 = 0;
            for (auto &sh : shapes)
                if (sh[0] * sh[1] == P && !v0) {
                    v0 = sh[0];
                    g0 = sh[1];
                }
            c->V = v0;
            c->G = g0;
            int rc = build_layout(c);
            if (!rc) rc = upload_inst(c);
            if (!rc && r32) rc = ensure_fp32(c);
            if (rc)
                return rc;
            double t64 = INFINITY, t32 = INFINITY;
            int bv = v0, bg = g0, bv32 = v0, bg32 = g0;
            for (auto &sh : shapes) {
                if (sh[0] * sh[1] != P)
                    continue;
                double t = 0.0;
                if ((rc = time_sweep<double>(c, sh[0], sh[1], &t)))
                    return rc;
                if (t < t64) {
                    t64 = t;
                    bv = sh[0];
                    bg = sh[1];
                }
                if (r32) {
                    if ((rc = time_sweep<float>(c, sh[0], sh[1], &t)))
                        return rc;
                    if (t < t32) {
                        t32 = t;
                        bv32 = sh[0];
                        bg32 = sh[1];
                    }
                }
            }
            // refinement: nearly all sweeps are FP32
            const double score = r32 ? t32 : t64;
            if (score < best_t) {
                best_t = score;
                best = TuneResult{bv, bg, bv32, bg32};
            }
        }
    }
    tune_store(c, key, best);
    c->V = best.V;
    c->G = best.G;
    c->V32 = best.V32;
    c->G32 = best.G32;
    c->layout_ok = false;
    return DVM_OK;
}

static int check_instance(const dvm_ctx *c, int instance)
{
    if (!c)
        return fail(DVM_EINVAL, "context is NULL");
    if (instance < 0 || instance >= c->n_inst)
        return fail(DVM_EINVAL, "instance index out of range");
    return DVM_OK;
}

// ------------------------------------------------ warm-start continuation
// cfg.warm_extrapolate: a warm solve at a new uniform delta starts from the
// state extrapolated linearly in log(delta) through the instance's last two
// converged solves (same alpha, drive and walls, same layout):
//   x0 = x + theta (x_1 - x_2),  theta = log(delta / d_1) / log(d_1 / d_2),
// x the current state (normally x_1, the last solution), for
// 0 < theta <= 2 (forward along the sweep, at most twice its last step).
// The fixed point is the plain warm start's; only the start is closer.  The
// state vector is the GMRES one: moments, lagged seam, wrap and wall values.

static StateBufs fwd_state_bufs(dvm_ctx *c)
{
    StateBufs sb;
    sb.b[0] = c->d_mom.p;
    sb.b[1] = c->d_seam.p;
    sb.b[2] = c->d_wrap.p;
    sb.b[3] = c->d_fb.p;
    return sb;
}

// history slots for the current layout (a new layout drops the history)
static int whist_ensure(dvm_ctx *c)
{
    if (c->whist_gen == c->layout_gen)
        return DVM_OK;
    c->whist_off.assign(c->n_inst, 0);
    c->whist_len.assign(c->n_inst, 0);
    c->whist_n.assign(c->n_inst, 0);
    c->whist_d0.assign(c->n_inst, 0.0);
    c->whist_d1.assign(c->n_inst, 0.0);
    c->whist_par.assign((size_t)c->n_inst * 4, 0.0);
    long long tot = 0, lmax = 1;
    for (int i = 0; i < c->n_inst; ++i) {
        c->whist_off[i] = tot;
        c->whist_len[i] = c->inst[i].has_geom ? state_segments(c, i, 0, 0, nullptr, nullptr) : 0;
        tot += c->whist_len[i];
        lmax = std::max(lmax, c->whist_len[i]);
    }
    for (auto &b : c->whist)
        HIPCHK(b.alloc((size_t)std::max<long long>(tot, 1)));
    HIPCHK(c->wvec.alloc((size_t)lmax));
    c->whist_gen = c->layout_gen;
    return DVM_OK;
}

// segment table of instance i's current state (the inputs of its next sweep)
static int whist_segs(dvm_ctx *c, int i, const SolveState &s, long long *len, int *nseg)
{
    std::vector<VSeg> sc;
    *len = state_segments(c, i, (int)(s.iter & 1), 0, nullptr, &sc);
    *nseg = (int)sc.size();
    if (c->wseg.n < sc.size())
        HIPCHK(c->wseg.alloc(sc.size()));
    if (!sc.empty())
        HIPCHK(hipMemcpyAsync(c->wseg.p, sc.data(), sc.size() * sizeof(VSeg), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return DVM_OK;
}

static void whist_params(const dvm_ctx *c, int i, double *par)
{
    par[0] = c->inst[i].alpha;
    par[1] = c->driving[i].drive;
    par[2] = c->driving[i].u_bot;
    par[3] = c->driving[i].u_top;
}

// after a converged uniform-delta solve: its state becomes x_1
static int whist_save(dvm_ctx *c, int i, const SolveState &s)
{
    int rc = whist_ensure(c);
    if (rc)
        return rc;
    long long len = 0;
    int nseg = 0;
    if ((rc = whist_segs(c, i, s, &len, &nseg)))
        return rc;
    if (len != c->whist_len[i] || len == 0) {
        c->whist_n[i] = 0;
        return DVM_OK;
    }
    double par[4];
    whist_params(c, i, par);
    if (c->whist_n[i] > 0 && !std::equal(par, par + 4, &c->whist_par[(size_t)i * 4]))
        c->whist_n[i] = 0;                    // other parameters: start a new history
    double *h0 = c->whist[0].p + c->whist_off[i], *h1 = c->whist[1].p + c->whist_off[i];
    if (c->whist_n[i] > 0)
        HIPCHK(hipMemcpyAsync(h1, h0, (size_t)len * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(launch_gather(c->wseg.p, nseg, fwd_state_bufs(c), h0, nullptr, c->stream));
    c->whist_d1[i] = c->whist_d0[i];
    c->whist_d0[i] = c->inst[i].delta;
    c->whist_n[i] = std::min(c->whist_n[i] + 1, 2);
    std::copy(par, par + 4, &c->whist_par[(size_t)i * 4]);
    return DVM_OK;
}

// before a warm solve at delta: x <- x + theta (x_1 - x_2) where it applies
static int whist_start(dvm_ctx *c, int i, const SolveState &s, double delta)
{
    if (c->whist_gen != c->layout_gen || c->whist_n[i] < 2)
        return DVM_OK;
    double par[4];
    whist_params(c, i, par);
    const double d1 = c->whist_d0[i], d2 = c->whist_d1[i];
    if (!std::equal(par, par + 4, &c->whist_par[(size_t)i * 4]) || !(d1 > 0.0 && d2 > 0.0 && delta > 0.0) ||
        d1 == d2 || delta == d1)
        return DVM_OK;
    const double theta = std::log(delta / d1) / std::log(d1 / d2);
    if (!(theta > 0.0 && theta <= 2.0))
        return DVM_OK;
    long long len = 0;
    int nseg = 0;
    int rc = whist_segs(c, i, s, &len, &nseg);
    if (rc)
        return rc;
    if (len != c->whist_len[i])
        return DVM_OK;
    const StateBufs sb = fwd_state_bufs(c);
    const double *h0 = c->whist[0].p + c->whist_off[i], *h1 = c->whist[1].p + c->whist_off[i];
    HIPCHK(launch_gather(c->wseg.p, nseg, sb, c->wvec.p, nullptr, c->stream));
    HIPCHK(launch_axpy(c->wvec.p, h0, theta, (size_t)len, c->stream));
    HIPCHK(launch_axpy(c->wvec.p, h1, -theta, (size_t)len, c->stream));
    HIPCHK(launch_scatter(c->wseg.p, nseg, sb, c->wvec.p, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (debug_on())
        std::fprintf(stderr, "[dvm continuation] inst %d: delta %.4g from %.4g and %.4g, theta %.3f\n", i, delta,
                     d1, d2, theta);
    return DVM_OK;
}

static int do_solve(dvm_ctx *c, int instance, const double *delta, int delta_is_field,
                    double alpha, dvm_info *info, bool warm, int depth = 0)
{
    if (!c)
        return fail(DVM_EINVAL, "context is NULL");
    AllocScope scope(&c->dalloc);
    if (instance < -1 || instance >= c->n_inst)
        return fail(DVM_EINVAL, "instance index out of range");
    if (!delta)
        return fail(DVM_EINVAL, "delta is NULL");
    if (!(alpha > 0.0 && alpha <= 1.0))
        return fail(DVM_EINVAL, "alpha must lie in (0, 1]");
    const int i0 = instance < 0 ? 0 : instance, i1 = instance < 0 ? c->n_inst : instance + 1;
    for (int i = i0; i < i1; ++i) {
        if (!c->inst[i].has_geom)
            return fail(DVM_ESTATE, "dvm_set_geometry has not been called for instance " + std::to_string(i));
        if (c->inst[i].periodic_y && (c->driving[i].u_bot != 0.0 || c->driving[i].u_top != 0.0))
            return fail(DVM_EINVAL, "instance " + std::to_string(i) +
                                        ": sliding walls need a walled channel (periodic_y = 0)");
    }
    // validate delta on the host before any device work
    {
        size_t off = 0;
        for (int i = i0; i < i1; ++i) {
            const HostInst &h = c->inst[i];
            if (delta_is_field) {
                for (size_t k = 0; k < (size_t)h.nx * h.ny; ++k)
                    if (!h.solid[k] && !(std::isfinite(delta[off + k]) && delta[off + k] >= 0.0))
                        return fail(DVM_EINVAL, "delta field must be finite and >= 0 in fluid cells");
                off += (size_t)h.nx * h.ny;
            } else {
                double d = delta[instance < 0 ? i : 0];
                if (!(std::isfinite(d) && d >= 0.0))
                    return fail(DVM_EINVAL, "delta must be finite and >= 0");
            }
        }
    }
    {
        int rc = ensure_device(c);
        if (rc)
            return rc;
    }
    if (c->autotune && !c->tuned) {
        int rc = autotune(c);
        if (rc)
            return rc;
    }
    if (!c->layout_ok) {
        int rc = build_layout(c);
        if (rc)
            return rc;
    }
    // parameters
    std::vector<double> dcat;
    size_t off = 0;
    for (int i = i0; i < i1; ++i) {
        HostInst &h = c->inst[i];
        InstDev &d = c->idev[i];
        h.alpha = alpha;
        h.field = delta_is_field != 0;
        d.alpha = alpha;
        d.field = h.field ? 1 : 0;
        d.drive = c->driving[i].drive;
        d.u_bot = c->driving[i].u_bot;
        d.u_top = c->driving[i].u_top;
        if (h.field) {
            size_t n = (size_t)h.nx * h.ny;
            h.dfield.assign(delta + off, delta + off + n);
            h.delta = NAN;
            d.delta = 0.0;
            HIPCHK(hipMemcpyAsync(c->d_dfield.p + d.cell_off, delta + off, n * sizeof(double),
                                  hipMemcpyHostToDevice, c->stream));
            off += n;
        } else {
            h.delta = delta[instance < 0 ? i : 0];
            d.delta = h.delta;
        }
    }
    HIPCHK(hipMemcpyAsync(c->d_inst.p, c->idev.data(), c->n_inst * sizeof(InstDev),
                          hipMemcpyHostToDevice, c->stream));
    // per-instance state: solve [i0, i1), freeze the others
    std::vector<SolveState> st(c->n_inst);
    HIPCHK(hipMemcpyAsync(st.data(), c->d_st.p, c->n_inst * sizeof(SolveState), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::vector<long long> iter0(c->n_inst, 0);
    std::vector<char> kept(c->n_inst, 0);
    for (int i = 0; i < c->n_inst; ++i) {
        SolveState &s = st[i];
        bool mine = i >= i0 && i < i1;
        if (!c->inst[i].has_state && !mine)
            s = SolveState{};
        if (mine) {
            bool keep = warm && c->inst[i].has_state;
            kept[i] = keep ? 1 : 0;
            if (!keep) {
                const InstDev &d = c->idev[i];
                size_t n = (size_t)d.nx * d.ny;
                HIPCHK(launch_zero(c->d_mom.p + d.cell_off * MOM_STRIDE, n * MOM_STRIDE, c->stream));
                HIPCHK(launch_zero(c->d_u1prev.p + d.cell_off, n, c->stream));
                size_t sn = (size_t)d.nstrips * d.nx * 2 * c->kp4;
                HIPCHK(launch_zero(c->d_seam.p + d.seam_off, sn, c->stream));
                HIPCHK(launch_zero(c->d_seam.p + c->seam_half + d.seam_off, sn, c->stream));
                HIPCHK(launch_zero(c->d_wrap.p + d.wrap_off, (size_t)d.nstrips * c->kp4 * 64 * 3,
                                   c->stream));
                const HostInst &h = c->inst[i];
                const size_t fh = (size_t)std::max<long long>(c->nfaces, 1) * c->kp4;
                for (int par = 0; par < 2; ++par)
                    HIPCHK(launch_zero(c->d_fb.p + par * fh + (size_t)h.face_base * c->kp4,
                                       (size_t)h.nfaces * c->kp4, c->stream));
                s = SolveState{};
            }
            s.active = 1;
            s.status = STATUS_RUNNING;
            s.npass = 0;
            s.eps_prev = 0.0;
            s.qfloor = 0.0;
            s.maxdiff_bits = s.maxabs_bits = 0ull;
            s.iter0 = s.iter;
            iter0[i] = s.iter;
        } else {
            s.active = 0;
        }
    }
    HIPCHK(hipMemcpyAsync(c->d_st.p, st.data(), c->n_inst * sizeof(SolveState), hipMemcpyHostToDevice,
                          c->stream));
    if (c->cfg.warm_extrapolate > 0 && !delta_is_field)
        for (int i = i0; i < i1; ++i)
            if (kept[i]) {
                int rc = whist_start(c, i, st[i], c->inst[i].delta);
                if (rc)
                    return rc;
            }
    // the record of the first sweep (from zero or the warm moments); the stop
    // statistics it gathers are discarded
    HIPCHK(launch_record<double>(rec_args(c), c->max_cells, c->n_inst, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int i = i0; i < i1; ++i) {
        st[i].maxdiff_bits = st[i].maxabs_bits = 0ull;
    }
    // u1prev was refreshed by the record kernel; reset the max slots only
    HIPCHK(hipMemcpyAsync(c->d_st.p, st.data(), c->n_inst * sizeof(SolveState), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int i = i0; i < i1; ++i)
        c->inst[i].has_state = true;

    if (depth == 0) {
        std::fill(c->sweeps_wasted.begin(), c->sweeps_wasted.end(), 0);
        std::fill(c->sweeps64_wasted.begin(), c->sweeps64_wasted.end(), 0);
    }
    {
        std::vector<char> need_skew(c->n_inst, 0);
        int rc = c->cfg.precision == DVM_FP32_REFINE ? dc_run(c, i0, i1, st, &need_skew)
                                                     : iterate(c, i0, i1, iter0, false, st, &need_skew);
        if (rc)
            return rc;
        bool restart = false;
        for (int i = i0; i < i1; ++i)
            if (need_skew[i]) {
                // the wrap-around diagonal stopped contracting on this geometry:
                // skewed order from now on, and the solve starts over
                c->inst[i].force_skew = true;
                restart = true;
            }
        if (restart && depth == 0) {
            // the new layout keeps the other instances' states: they restart
            // warm from what this pass reached, the moved ones from zero
            for (int i = i0; i < i1; ++i) {
                c->sweeps_wasted[i] += c->sweeps_done[i];
                c->sweeps64_wasted[i] += c->cfg.precision == DVM_FP32_REFINE ? c->sweeps64_done[i]
                                                                             : c->sweeps_done[i];
                if (need_skew[i])
                    c->inst[i].has_state = false;
            }
            c->layout_ok = false;
            return do_solve(c, instance, delta, delta_is_field, alpha, info, true, depth + 1);
        }
    }
    // flow rate of Sec. III of every instance with a state, reduced on the
    // device in a fixed order; kept for dvm_flow_rate
    HIPCHK(launch_flow(c->d_inst.p, c->d_codes.p, c->d_mom.p, c->d_rows.p, c->d_q.p, c->n_inst, c->stream));
    HIPCHK(hipMemcpyAsync(c->qcache.data(), c->d_q.p, c->n_inst * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    int rc = DVM_OK;
    for (int i = i0; i < i1; ++i) {
        const SolveState &s = st[i];
        if (info) {
            dvm_info &o = info[instance < 0 ? i : 0];
            o.iters = c->sweeps_done[i] + c->sweeps_wasted[i];
            o.sweeps_fp64 = c->sweeps64_wasted[i] +
                            (c->cfg.precision == DVM_FP32_REFINE ? c->sweeps64_done[i] : c->sweeps_done[i]);
            o.rel_change = s.eps;
            o.est_error = s.est;
            o.status = s.status;
            o.schedule = c->idev[i].tp == c->idev[i].nx && c->idev[i].nx > 1 ? DVM_SCHED_WRAP : DVM_SCHED_SKEW;
        }
        c->inst[i].converged = s.status == STATUS_CONVERGED;
        if (c->cfg.warm_extrapolate > 0 && !delta_is_field && s.status == STATUS_CONVERGED) {
            int rs = whist_save(c, i, s);
            if (rs)
                return rs;
        }
        if (s.status == STATUS_DIVERGED)
            rc = fail(DVM_EDIVERGED, "instance " + std::to_string(i) + " produced non-finite iterates");
        else if (rc == DVM_OK && s.status != STATUS_CONVERGED)
            rc = fail(DVM_ENOCONV, "instance " + std::to_string(i) + " reached max_iter");
    }
    return rc;
}

// ------------------------------------------------------------- adjoint
static int ensure_adjoint(dvm_ctx *c)
{
    if (c->adj_ready)
        return DVM_OK;
    // (re)allocation below: nothing queued may still use the old buffers
    HIPCHK(hipStreamSynchronize(c->stream));
    const long long sk = c->sk_total, cell = c->ncell, nf = std::max<long long>(c->nfaces, 1);
    HIPCHK(c->d_scode_adj.alloc(sk));
    HIPCHK(c->d_sface_adj.alloc(sk));
    HIPCHK(c->d_sfacek_adj.alloc(sk));
    HIPCHK(c->d_face_cell.alloc(nf));
    HIPCHK(c->d_face_side.alloc(nf));
    HIPCHK(c->d_face_inst.alloc(nf));
    HIPCHK(c->d_srec_adj.alloc(sk * REC_STRIDE));
    HIPCHK(c->d_mom_adj.alloc(cell * MOM_STRIDE));
    HIPCHK(c->d_u1prev_adj.alloc(cell));
    HIPCHK(c->d_seam_adj.alloc(2 * c->seam_half));
    HIPCHK(c->d_wrap_adj.alloc(c->wrap_total));
    HIPCHK(c->d_fb_adj.alloc((size_t)2 * nf * c->kp4));
    HIPCHK(c->d_ckpt.alloc((size_t)cell * c->kp4));
    HIPCHK(c->d_momg.alloc(cell * MOM_STRIDE));
    HIPCHK(c->d_dqda.alloc(nf));
    HIPCHK(c->d_st_adj.alloc(c->n_inst));
    HIPCHK(hipMemcpyAsync(c->d_scode_adj.p, c->h_scode_adj.data(), sk, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->d_sface_adj.p, c->h_sface_adj.data(), sk * sizeof(FaceRec), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipMemcpyAsync(c->d_sfacek_adj.p, c->h_sfacek_adj.data(), sk * sizeof(FaceK), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(c->d_wl_adj.alloc(std::max<size_t>(c->h_wl_adj.size(), 1)));
    if (!c->h_wl_adj.empty())
        HIPCHK(hipMemcpyAsync(c->d_wl_adj.p, c->h_wl_adj.data(), c->h_wl_adj.size() * sizeof(int),
                              hipMemcpyHostToDevice, c->stream));
    if (c->nfaces > 0) {
        HIPCHK(hipMemcpyAsync(c->d_face_cell.p, c->h_face_cell.data(), c->nfaces * sizeof(int),
                              hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(c->d_face_side.p, c->h_face_side.data(), c->nfaces * sizeof(int),
                              hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(c->d_face_inst.p, c->h_face_inst.data(), c->nfaces * sizeof(int),
                              hipMemcpyHostToDevice, c->stream));
    }
    HIPCHK(launch_zero(c->d_srec_adj.p, c->d_srec_adj.n, c->stream));
    HIPCHK(launch_zero(c->d_ckpt.p, c->d_ckpt.n, c->stream));
    std::vector<SolveState> st(c->n_inst);
    HIPCHK(hipMemcpyAsync(c->d_st_adj.p, st.data(), c->n_inst * sizeof(SolveState), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->adj_ready = true;
    return DVM_OK;
}

// Discrete adjoint of the flow rate at the converged state of one instance:
//  1. one more forward sweep that keeps h (all velocities) and the incident
//     wall-face values, and the moments of that h;
//  2. source iteration of the transposed problem for nu(c, v) =
//     lambda(c, -v) / W(v), driven by -(dx / nx) xi -- the same sweeps with
//     transposed stencil weights and wall couplings;
//  3. one more adjoint sweep that accumulates sum_v W nu h(-v) per cell and
//     keeps nu on the wall faces; then the per-cell and per-face assembly.
static int grad_instance(dvm_ctx *c, int instance, double *dqdd_out, double *dqda_out)
{
    int rc = ensure_adjoint(c);
    if (rc)
        return rc;
    const HostInst &h = c->inst[instance];
    const InstDev &d = c->idev[instance];
    const size_t n = (size_t)d.nx * d.ny;
    const size_t fh = (size_t)std::max<long long>(c->nfaces, 1) * c->kp4;
    std::vector<WorkItem> mine;
    for (const auto &it : c->items)
        if (it.inst == instance)
            mine.push_back(it);
    DevBuf<WorkItem> ditems;
    HIPCHK(ditems.alloc(mine.size()));
    HIPCHK(hipMemcpyAsync(ditems.p, mine.data(), mine.size() * sizeof(WorkItem), hipMemcpyHostToDevice,
                          c->stream));
    const int base = (h.field ? MODE_FIELD : 0) | (h.alpha < 1.0 ? MODE_SPEC : 0);
    std::vector<SolveState> st(c->n_inst);
    HIPCHK(hipMemcpyAsync(st.data(), c->d_st.p, c->n_inst * sizeof(SolveState), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int par_f = (int)(st[instance].iter & 1);

    // 1. forward checkpoint
    {
        SweepArgs<double> a = sweep_args(c, 1, false);
        a.items = ditems.p;
        HIPCHK(launch_sweep<double>(a, (int)mine.size(), c->V, c->G, MODE_CKPT | base, c->stream));
        MomArgs m = mom_args(c, false, 1);
        m.mom = c->d_momg.p;
        HIPCHK(launch_moments(m, c->max_cells, c->n_inst, c->stream));
    }
    // 2. adjoint source iteration (cold start)
    HIPCHK(launch_zero(c->d_mom_adj.p + d.cell_off * MOM_STRIDE, n * MOM_STRIDE, c->stream));
    HIPCHK(launch_zero(c->d_u1prev_adj.p + d.cell_off, n, c->stream));
    {
        size_t sn = (size_t)d.nstrips * d.nx * 2 * c->kp4;
        HIPCHK(launch_zero(c->d_seam_adj.p + d.seam_off, sn, c->stream));
        HIPCHK(launch_zero(c->d_seam_adj.p + c->seam_half + d.seam_off, sn, c->stream));
        HIPCHK(launch_zero(c->d_wrap_adj.p + d.wrap_off, (size_t)d.nstrips * c->kp4 * 64 * 3, c->stream));
        for (int par = 0; par < 2; ++par)
            HIPCHK(launch_zero(c->d_fb_adj.p + par * fh + (size_t)h.face_base * c->kp4,
                               (size_t)h.nfaces * c->kp4, c->stream));
    }
    std::vector<SolveState> sa(c->n_inst);
    sa[instance].active = 1;
    sa[instance].status = STATUS_RUNNING;
    HIPCHK(hipMemcpyAsync(c->d_st_adj.p, sa.data(), c->n_inst * sizeof(SolveState), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(launch_record<double>(rec_args(c, true), c->max_cells, c->n_inst, c->stream));
    HIPCHK(hipMemcpyAsync(c->d_st_adj.p, sa.data(), c->n_inst * sizeof(SolveState), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    {
        std::vector<long long> iter0(c->n_inst, 0);
        rc = iterate(c, instance, instance + 1, iter0, true, sa);
        if (rc)
            return rc;
    }
    if (sa[instance].status == STATUS_DIVERGED)
        return fail(DVM_EDIVERGED, "adjoint iteration produced non-finite iterates");
    if (sa[instance].status != STATUS_CONVERGED)
        return fail(DVM_ENOCONV, "adjoint iteration reached max_iter");
    const int par_a = (int)(sa[instance].iter & 1);

    // 3. gradient sweep and assembly
    {
        SweepArgs<double> a = sweep_args(c, 1, true);
        a.items = ditems.p;
        HIPCHK(launch_sweep<double>(a, (int)mine.size(), c->V, c->G, MODE_ADJ | MODE_GRAD | base, c->stream));
        HIPCHK(launch_moments(mom_args(c, true, 1), c->max_cells, c->n_inst, c->stream));
    }
    GradArgs g{};
    g.inst = c->d_inst.p;
    g.codes = c->d_codes.p;
    g.mom_fwd = c->d_momg.p;
    g.mom_adj = c->d_mom_adj.p;
    g.part5 = c->d_part5.p;
    g.dqdd = c->d_aux.p;
    g.face_cell = c->d_face_cell.p;
    g.rows = c->d_rows.p;
    g.face_side = c->d_face_side.p;
    g.face_inst = c->d_face_inst.p;
    g.fb_fwd = c->d_fb.p + par_f * fh;
    g.fb_adj = c->d_fb_adj.p + par_a * fh;
    g.vtab = c->d_vt.p;
    g.dqda_face = c->d_dqda.p;
    g.ncell = c->ncell;
    g.ngroups = 4 * c->gq;
    g.kq = c->kq;
    g.kp4 = c->kp4;
    g.face0 = (int)h.face_base;
    g.nfaces = h.nfaces;
    g.m0 = c->m0;
    g.m2 = c->m2;
    g.c2 = c->c2;
    g.c4 = c->c4;
    g.D = c->D;
    HIPCHK(launch_grad(g, instance, (int)n, c->stream));
    std::vector<double> dqdd(n), dqda(h.nfaces);
    HIPCHK(hipMemcpyAsync(dqdd.data(), c->d_aux.p + d.cell_off, n * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
    if (h.nfaces > 0)
        HIPCHK(hipMemcpyAsync(dqda.data(), c->d_dqda.p + h.face_base, h.nfaces * sizeof(double),
                              hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    ditems.release();
    if (dqdd_out)
        std::copy(dqdd.begin(), dqdd.end(), dqdd_out);
    if (dqda_out) {
        double sum = 0.0;
        for (double v : dqda)
            sum += v;
        *dqda_out = sum;
    }
    return DVM_OK;
}

// ================================================================ C ABI
extern "C" {

const char *dvm_last_error(void) { return g_err.c_str(); }

const char *dvm_version(void) { return "dvm-gfx950 0.1"; }

int dvm_create(dvm_ctx **out, int nv, int n_instances, const dvm_config *cfg, void *hip_stream,
               dvm_alloc_fn alloc, dvm_free_fn free_, void *alloc_ud)
{
    if (!out)
        return fail(DVM_EINVAL, "out is NULL");
    *out = nullptr;
    if ((alloc == nullptr) != (free_ == nullptr))
        return fail(DVM_EINVAL, "alloc and free_ must both be given or both be NULL");
    if (nv < 4 || nv > 128 || (nv % 2) != 0)
        return fail(DVM_EINVAL, "nv must be even and in [4, 128]");
    if (n_instances < 1 || n_instances > 65535)
        return fail(DVM_EINVAL, "n_instances must be in [1, 65535]");
    dvm_config c{};
    if (cfg)
        c = *cfg;
    if (c.precision != DVM_FP64 && c.precision != DVM_FP32_REFINE)
        return fail(DVM_EINVAL, "unknown precision mode");
    if (c.tol == 0.0)
        c.tol = 1e-8;
    if (!(c.tol > 0.0))
        return fail(DVM_EINVAL, "tol must be > 0");
    if (c.max_iter == 0)
        c.max_iter = 200000;
    if (c.max_iter < 0)
        return fail(DVM_EINVAL, "max_iter must be > 0");
    if (c.block_iters < 0 || c.block_iters > 4096)
        return fail(DVM_EINVAL, "block_iters must be in [0, 4096]");
    if (c.schedule != DVM_SCHED_AUTO && c.schedule != DVM_SCHED_SKEW && c.schedule != DVM_SCHED_WRAP)
        return fail(DVM_EINVAL, "unknown schedule");
    if (c.accel != DVM_ACCEL_AUTO && c.accel != DVM_ACCEL_NONE && c.accel != DVM_ACCEL_GMRES)
        return fail(DVM_EINVAL, "unknown acceleration");
    if (c.krylov_dim < 0 || c.krylov_dim > 64)
        return fail(DVM_EINVAL, "krylov_dim must be in [0, 64]");
    if (c.persistent != 0 && c.persistent != 1)
        return fail(DVM_EINVAL, "persistent must be 0 or 1");
    if (c.krylov_deflate > VCOMB_OUT - 2)
        return fail(DVM_EINVAL, "krylov_deflate must be at most 31");
    if (c.warm_extrapolate != 0 && c.warm_extrapolate != 1)
        return fail(DVM_EINVAL, "warm_extrapolate must be 0 or 1");
    int V = c.vel_per_lane ? c.vel_per_lane : 4;
    int G = c.waves_per_block ? c.waves_per_block : 8;
    bool okvg = (V == 4 && G == 8) || (V == 8 && G == 4) || (V == 4 && G == 4) || (V == 2 && G == 8);
    if (!okvg)
        return fail(DVM_EINVAL, "unsupported (vel_per_lane, waves_per_block) combination");
    dvm_ctx *ctx = new (std::nothrow) dvm_ctx();
    if (!ctx)
        return fail(DVM_ENOMEM, "out of host memory");
    ctx->nv = nv;
    ctx->K = nv * nv;
    ctx->n_inst = n_instances;
    ctx->cfg = c;
    ctx->V = V;
    ctx->V32 = V;
    ctx->G32 = G;
    ctx->autotune = c.vel_per_lane == 0 && c.waves_per_block == 0;
    if (c.tune_cache)
        ctx->tune_path = c.tune_cache;
    ctx->cfg.tune_cache = nullptr;
    ctx->G = G;
    ctx->inst.assign(n_instances, HostInst{});
    ctx->sweeps_done.assign(n_instances, 0);
    ctx->trial_q.assign(n_instances, 0.0);
    ctx->sweeps64_done.assign(n_instances, 0);
    ctx->gmres_s64.assign(n_instances, 0);
    ctx->sweeps_wasted.assign(n_instances, 0);
    ctx->driving.assign(n_instances, dvm_ctx::Driving{});
    ctx->sweeps64_wasted.assign(n_instances, 0);
    ctx->stream = (hipStream_t)hip_stream;   // NULL: a stream is made on first use
    ctx->dalloc.alloc = alloc;
    ctx->dalloc.free = free_;
    ctx->dalloc.ud = alloc_ud;
    build_quadrature(ctx);
    *out = ctx;
    return DVM_OK;
}

int dvm_set_geometry(dvm_ctx *ctx, int instance, int nx, int ny, const uint8_t *solid, int periodic_y,
                     double cells_per_H)
{
    int rc = check_instance(ctx, instance);
    if (rc)
        return rc;
    if (!solid)
        return fail(DVM_EINVAL, "solid is NULL");
    if (!(nx == 1 || nx >= 4) || ny < 4)
        return fail(DVM_EINVAL, "need nx == 1 or nx >= 4, and ny >= 4");
    if ((long long)nx * ny > (1ll << 30))
        return fail(DVM_EINVAL, "grid too large");
    if (!(cells_per_H > 0.0) || !std::isfinite(cells_per_H))
        return fail(DVM_EINVAL, "cells_per_H must be finite and > 0");
    HostInst h;
    h.nx = nx;
    h.ny = ny;
    h.periodic_y = periodic_y ? 1 : 0;
    h.cph = cells_per_H;
    h.solid.resize((size_t)nx * ny);
    for (size_t k = 0; k < h.solid.size(); ++k) {
        if (solid[k] > 1)
            return fail(DVM_EINVAL, "solid mask values must be 0 or 1");
        h.solid[k] = solid[k];
    }
    std::string why;
    if (!all_components_percolate(h, why))
        return fail(DVM_EINVAL, why);
    build_codes(h);
    h.has_geom = true;
    ctx->inst[instance] = std::move(h);
    ctx->layout_ok = false;
    ctx->tuned = false;
    return DVM_OK;
}

int dvm_set_row_heights(dvm_ctx *ctx, int instance, const double *dy)
{
    int rc = check_instance(ctx, instance);
    if (rc)
        return rc;
    HostInst &h = ctx->inst[instance];
    if (!h.has_geom)
        return fail(DVM_ESTATE, "dvm_set_geometry has not been called for this instance");
    std::vector<double> rows;
    if (dy) {
        rows.assign(dy, dy + h.ny);
        for (double v : rows)
            if (!(std::isfinite(v) && v > 0.0))
                return fail(DVM_EINVAL, "row heights must be finite and > 0");
    }
    h.rows.swap(rows);
    h.has_state = false;
    ctx->layout_ok = false;
    return DVM_OK;
}

int dvm_set_driving(dvm_ctx *ctx, int instance, double pressure_gradient, double wall_velocity_bottom,
                    double wall_velocity_top)
{
    int rc = check_instance(ctx, instance);
    if (rc)
        return rc;
    if (!std::isfinite(pressure_gradient) || !std::isfinite(wall_velocity_bottom) ||
        !std::isfinite(wall_velocity_top))
        return fail(DVM_EINVAL, "driving parameters must be finite");
    auto &dr = ctx->driving[instance];
    dr.drive = pressure_gradient;
    dr.u_bot = wall_velocity_bottom;
    dr.u_top = wall_velocity_top;
    return DVM_OK;
}

int dvm_solve(dvm_ctx *ctx, int instance, const double *delta, int delta_is_field, double alpha,
              dvm_info *info)
{
    return do_solve(ctx, instance, delta, delta_is_field, alpha, info, false);
}

int dvm_solve_warm(dvm_ctx *ctx, int instance, const double *delta, int delta_is_field, double alpha,
                   dvm_info *info)
{
    return do_solve(ctx, instance, delta, delta_is_field, alpha, info, true);
}

int dvm_flow_rate(const dvm_ctx *cc, int instance, double *Q, double *k_a)
{
    dvm_ctx *ctx = const_cast<dvm_ctx *>(cc);
    int rc = check_instance(ctx, instance);
    if (rc)
        return rc;
    if (!Q)
        return fail(DVM_EINVAL, "Q is NULL");
    const HostInst &h = ctx->inst[instance];
    if (!ctx->layout_ok || !h.has_state || (size_t)instance >= ctx->qcache.size())
        return fail(DVM_ESTATE, "instance has not been solved");
    // reduced on the device at the end of the last solve
    *Q = ctx->qcache[instance];
    if (k_a)
        *k_a = h.field ? NAN : *Q / h.delta;
    return DVM_OK;
}

int dvm_permeability(int n, const double *delta, const double *Q, double phi, double *k_inf, double *H_star,
                     double *Kn_star, double *ka_ratio, double *Kn, double *k_a)
{
    if (n < 3 || !delta || !Q)
        return fail(DVM_EINVAL, "need n >= 3 samples (delta, Q)");
    if (!(phi > 0.0 && phi <= 1.0))
        return fail(DVM_EINVAL, "porosity must lie in (0, 1]");
    std::vector<double> kn(n), ka(n);
    for (int i = 0; i < n; ++i) {
        if (!(std::isfinite(delta[i]) && delta[i] > 0.0 && std::isfinite(Q[i])))
            return fail(DVM_EINVAL, "delta must be finite and > 0, Q finite");
        kn[i] = std::sqrt(M_PI) / (2.0 * delta[i]);    // delta = sqrt(pi) / (2 Kn)
        ka[i] = Q[i] / delta[i];                         // k_a = sqrt(4/pi) Q Kn
    }
    // the three samples closest to the continuum limit
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i)
        idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return kn[a] < kn[b]; });
    for (int i = 0; i + 1 < n; ++i)
        if (kn[idx[i]] == kn[idx[i + 1]])
            return fail(DVM_EINVAL, "two samples share the same delta");
    // Lagrange form of the interpolating quadratic, evaluated at Kn = 0
    double k0 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double l = 1.0;
        for (int b = 0; b < 3; ++b)
            if (b != a)
                l *= (0.0 - kn[idx[b]]) / (kn[idx[a]] - kn[idx[b]]);
        k0 += ka[idx[a]] * l;
    }
    if (!(k0 > 0.0 && std::isfinite(k0)))
        return fail(DVM_EINVAL, "the extrapolated intrinsic permeability is not positive");
    const double hs = std::sqrt(12.0 * k0 / phi);       // H* / H
    if (k_inf)
        *k_inf = k0;
    if (H_star)
        *H_star = hs;
    for (int i = 0; i < n; ++i) {
        if (Kn_star)
            Kn_star[i] = kn[i] / hs;
        if (ka_ratio)
            ka_ratio[i] = ka[i] / k0;
        if (Kn)
            Kn[i] = kn[i];
        if (k_a)
            k_a[i] = ka[i];
    }
    return DVM_OK;
}

int dvm_get_moments(const dvm_ctx *cc, int instance, double *rho, double *u1, double *u2, double *tau,
                    double *p12)
{
    dvm_ctx *ctx = const_cast<dvm_ctx *>(cc);
    int rc = check_instance(ctx, instance);
    if (rc)
        return rc;
    AllocScope scope(&ctx->dalloc);
    const HostInst &h = ctx->inst[instance];
    if (!ctx->layout_ok || !h.has_state)
        return fail(DVM_ESTATE, "instance has not been solved");
    const InstDev &d = ctx->idev[instance];
    size_t n = (size_t)d.nx * d.ny;
    std::vector<double> mom(n * MOM_STRIDE);
    HIPCHK(hipMemcpyAsync(mom.data(), ctx->d_mom.p + d.cell_off * MOM_STRIDE, mom.size() * sizeof(double),
                          hipMemcpyDeviceToHost, ctx->stream));
    std::vector<double> shear;
    if (p12) {
        // the shear stress is not carried by the iteration: one extra
        // diagnostic sweep from the current state accumulates it
        SweepArgs<double> a = sweep_args(ctx, 1);
        std::vector<WorkItem> mine;
        for (const auto &it : ctx->items)
            if (it.inst == instance)
                mine.push_back(it);
        DevBuf<WorkItem> ditems;
        HIPCHK(ditems.alloc(mine.size()));
        HIPCHK(hipMemcpyAsync(ditems.p, mine.data(), mine.size() * sizeof(WorkItem), hipMemcpyHostToDevice,
                              ctx->stream));
        a.items = ditems.p;
        const int mode = MODE_P12 | (h.field ? MODE_FIELD : 0) | (h.alpha < 1.0 ? MODE_SPEC : 0);
        HIPCHK(launch_sweep<double>(a, (int)mine.size(), ctx->V, ctx->G, mode, ctx->stream));
        MomArgs m = mom_args(ctx);
        HIPCHK(launch_sum1(m, ctx->d_part5.p, ctx->d_aux.p, 2.0, ctx->max_cells, ctx->n_inst, ctx->stream));
        shear.resize(n);
        HIPCHK(hipMemcpyAsync(shear.data(), ctx->d_aux.p + d.cell_off, n * sizeof(double),
                              hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        ditems.release();
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    double rmean = 0.0;
    long long nf = 0;
    for (size_t k = 0; k < n; ++k)
        if (!h.solid[k]) {
            rmean += mom[k * MOM_STRIDE + MOM_RHO];
            ++nf;
        }
    rmean /= (double)nf;
    for (size_t k = 0; k < n; ++k) {
        bool f = !h.solid[k];
        const double *m = &mom[k * MOM_STRIDE];
        double r = f ? m[MOM_RHO] - rmean : 0.0;
        double e = f ? m[MOM_E] - rmean * ctx->M2 / ctx->m0 : 0.0;
        if (rho) rho[k] = r;
        if (u1) u1[k] = f ? m[MOM_U1] : 0.0;
        if (u2) u2[k] = f ? m[MOM_U2] : 0.0;
        if (tau) tau[k] = f ? e - r : 0.0;
        if (p12) p12[k] = f ? shear[k] : 0.0;
    }
    return DVM_OK;
}

int dvm_get_moments_noalloc(const dvm_ctx *cc, int instance, double *rho, double *u1, double *u2, double *tau,
                            double *p12)
{
    dvm_ctx *ctx = const_cast<dvm_ctx *>(cc);
    int rc = check_instance(ctx, instance);
    if (rc)
        return rc;
    const HostInst &h = ctx->inst[instance];
    if (!ctx->layout_ok || !h.has_state || ctx->device < 0)
        return fail(DVM_ESTATE, "instance has not been solved");
    void *sp = g_scratch_ptr[ctx->device];
    if (!sp)
        return fail(DVM_ESTATE, "static scratch of the device not set up");
    const InstDev &d = ctx->idev[instance];
    const long long nitems = (long long)d.nstrips * 4 * ctx->gq;
    if (nitems > SCRATCH_ITEMS)
        return fail(DVM_EINVAL, "instance needs " + std::to_string(nitems) + " work items for the shear-stress pass; "
                                "the static scratch holds " + std::to_string(SCRATCH_ITEMS));
    double *mean = static_cast<double *>(sp);
    WorkItem *items = reinterpret_cast<WorkItem *>(static_cast<unsigned char *>(sp) + SCRATCH_HEAD);
    if (p12) {
        // one diagnostic sweep from the current state accumulates the shear
        // stress; its work items are written into the scratch on the device
        HIPCHK(launch_items(items, instance, d.nstrips, 4 * ctx->gq, ctx->stream));
        SweepArgs<double> a = sweep_args(ctx, 1);
        a.items = items;
        const int mode = MODE_P12 | (h.field ? MODE_FIELD : 0) | (h.alpha < 1.0 ? MODE_SPEC : 0);
        HIPCHK(launch_sweep<double>(a, (int)nitems, ctx->V, ctx->G, mode, ctx->stream));
        HIPCHK(launch_sum1(mom_args(ctx), ctx->d_part5.p, ctx->d_aux.p, 2.0, ctx->max_cells, ctx->n_inst,
                           ctx->stream));
    }
    HIPCHK(launch_moments_out(ctx->d_inst.p, instance, d.nx * d.ny, ctx->d_codes.p, ctx->d_mom.p, ctx->d_aux.p,
                              mean, ctx->M2 / ctx->m0, rho, u1, u2, tau, p12, ctx->stream));
    return DVM_OK;
}

int dvm_grad(dvm_ctx *ctx, int instance, double *dQ_ddelta, double *dQ_dalpha)
{
    int rc = check_instance(ctx, instance);
    if (rc)
        return rc;
    const HostInst &h = ctx->inst[instance];
    if (!ctx->layout_ok || !h.has_state || !h.converged)
        return fail(DVM_ESTATE, "instance has no converged solution (call dvm_solve first)");
    AllocScope scope(&ctx->dalloc);
    return grad_instance(ctx, instance, dQ_ddelta, dQ_dalpha);
}

int dvm_profile(dvm_ctx *ctx, dvm_prof *out)
{
    if (!ctx || !out)
        return fail(DVM_EINVAL, "context or out is NULL");
    *out = ctx->prof;
    ctx->prof = dvm_prof{};
    return DVM_OK;
}

int dvm_launch_shape(const dvm_ctx *ctx, int *vel_per_lane, int *waves_per_block, int *vel_per_lane32,
                     int *waves_per_block32)
{
    if (!ctx)
        return fail(DVM_EINVAL, "context is NULL");
    const bool known = !ctx->autotune || ctx->tuned;
    if (vel_per_lane)
        *vel_per_lane = known ? ctx->V : 0;
    if (waves_per_block)
        *waves_per_block = known ? ctx->G : 0;
    if (vel_per_lane32)
        *vel_per_lane32 = known ? ctx->V32 : 0;
    if (waves_per_block32)
        *waves_per_block32 = known ? ctx->G32 : 0;
    return DVM_OK;
}

void dvm_destroy(dvm_ctx *ctx)
{
    if (!ctx)
        return;
    if (ctx->stream)
        (void)hipStreamSynchronize(ctx->stream);
    delete ctx;   // every buffer goes back through the hooks it came from
}

} // extern "C"
